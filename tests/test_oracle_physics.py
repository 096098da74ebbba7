"""Physics pins of the FP64 oracle: closed forms and the paper's calibration numbers.

Each case runs the oracle to a steady state and compares it with something
fixed independently of the oracle: a textbook flow profile, a mean-field
coexistence law, the paper's surface tension (Sec. 3.1) or its fitted
contact-angle cubic (Sec. 3.2).  Quasi-2D cases (one lattice plane in z,
periodic) reduce D3Q19 exactly to a 2D lattice and keep the suite fast; the
flat-interface physics they probe is the same as in 3D.
"""
import json
import os

import numpy as np
import pytest

from oracle.oracle import Oracle, OracleParams
from paper_2207_01534_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PAPER = json.load(open(os.path.join(GOLDEN, "paper_values.json")))


def _channel(H, taus, g, rho_profile, G=3.5, shift=True):
    """Channel of H fluid rows y = 1..H; solid row y = 0 (periodic in y, so both
    walls are the same row; halfway walls at y = 0.5 and y = H + 0.5)."""
    shape = (1, H + 1, 1)
    solid = np.zeros((1, H + 1, 1), np.uint8)
    solid[:, 0, :] = 1
    rho = np.zeros((2, 1, H + 1, 1))
    rho[0, 0, :, 0], rho[1, 0, :, 0] = rho_profile
    rho[:, solid != 0] = 0
    p = OracleParams(shape, tau=taus, G=G, g=g, half_force_shift=shift)
    o = Oracle(p, solid)
    o.init_equilibrium(rho)
    return o


@pytest.mark.parametrize("shift", [True, False])
def test_single_fluid_poiseuille(shift):
    """u(y) = g (y - 1/2)(H + 1/2 - y) / (2 nu), nu = (tau - 1/2)/3 (Eq. 7 minus-sign reading).
    The as-printed velocity (no half-force shift) reaches only half the amplitude at tau = 1."""
    H, g = 32, 1e-6
    ones = np.ones(H + 1)
    o = _channel(H, (1.0, 1.0), ((g, 0, 0), (0, 0, 0)), (ones, 0 * ones), shift=shift)
    o.run(8000)
    _, _, _, u = o.fields()
    y = np.arange(1, H + 1)
    nu = (1.0 - 0.5) / 3.0
    ua = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y)
    un = u[0, 0, 1:, 0]
    err = np.linalg.norm(un - ua) / np.linalg.norm(ua)
    if shift:
        assert err < 1e-2
    else:
        assert un.max() / ua.max() == pytest.approx(0.5, rel=2e-2)


def _nu_mix(taus, r1, r2):
    """Eq. (6) with Eq. (7): mixture kinematic viscosity (tau_s - 1/2)/3."""
    return (r1 * (taus[0] - 0.5) + r2 * (taus[1] - 0.5)) / (r1 + r2) / 3.0


def test_layered_two_fluid_poiseuille():
    """Core of component 1 between wall layers of component 2, M = 10, same g on both.

    Steady x-momentum in a channel: d/dy(rho nu du/dy) = -rho g, so the shear
    stress at height y equals g times the mass between y and the centre line.
    Integrating du/dy = stress / (rho nu) from the halfway wall with the
    measured densities and the Eq. (6) viscosity gives the exact profile of
    the diffuse-interface flow; the textbook piecewise parabola with the two
    bulk viscosities is checked more loosely.
    """
    H, g, taus = 64, 1e-6, (1.5, 0.6)
    y = np.arange(H + 1).astype(float)
    c, a = (H + 1) / 2.0, 16.0
    t = np.tanh(2 * (np.abs(y - c) - a) / 5.0)
    r1 = 0.5 * (1 + 0.03) - 0.5 * (1 - 0.03) * t
    o = _channel(H, taus, ((g, 0, 0), (g, 0, 0)), (r1, 1.03 - r1))
    o.run(60000)
    r, _, _, u = o.fields()
    ux = u[0, 0, 1:, 0]
    R1, R2 = r[0, 0, 1:, 0], r[1, 0, 1:, 0]
    rt = R1 + R2
    mu = rt * _nu_mix(taus, R1, R2)
    cum = np.concatenate([[0.0], np.cumsum(rt)])
    stress = g * (rt.sum() / 2 - cum)                 # at y = 0.5, 1.5, ..., H + 0.5
    mu_half = np.concatenate([[mu[0]], 0.5 * (mu[:-1] + mu[1:]), [mu[-1]]])
    dudy = stress / mu_half
    u_ode = np.zeros(H)
    u_ode[0] = 0.25 * (dudy[0] + dudy[1])
    for k in range(1, H):
        u_ode[k] = u_ode[k - 1] + dudy[k]
    assert np.linalg.norm(ux - u_ode) / np.linalg.norm(u_ode) < 1.5e-2
    # textbook two-layer parabola with the bulk mixture viscosities
    yy = y[1:]
    s = np.abs(yy - c)
    L = H / 2.0
    n1 = _nu_mix(taus, R1[int(c) - 1], R2[int(c) - 1])
    n2 = _nu_mix(taus, R1[7], R2[7])
    C1 = g * (L * L - a * a) / (2 * n2) + g * a * a / (2 * n1)
    ub = np.where(s < a, -g * s * s / (2 * n1) + C1, g * (L * L - s * s) / (2 * n2))
    assert np.linalg.norm(ux - ub) / np.linalg.norm(ub) < 8e-2


@pytest.mark.parametrize("shift", [True, False])
def test_flat_interface_coexistence(shift):
    """Flat interfaces in a periodic 1D box relax to rest, with bulk densities on the
    mean-field coexistence line ln(a/b) = G (a - b) (from ln rho + G rho_bar = const,
    Eqs. 11 and 12).  Without the half-force shift the box never comes to rest."""
    n, G = 64, 3.5
    x = np.arange(n)
    a0 = np.where((x >= 16) & (x < 48), 1.0, 0.03)
    rho = np.zeros((2, 1, 1, n))
    rho[0, 0, 0], rho[1, 0, 0] = a0, 1.03 - a0
    o = Oracle(OracleParams((n, 1, 1), tau=(1.0, 1.0), G=G, half_force_shift=shift),
               np.zeros((1, 1, n), np.uint8))
    o.init_equilibrium(rho)
    o.run(20000)
    r, _, _, u = o.fields()
    if not shift:
        assert np.abs(u).max() > 1e-3
        return
    assert np.abs(u).max() < 1e-12
    a, b = r[0, 0, 0, 32], r[1, 0, 0, 32]
    assert r[1, 0, 0, 0] == pytest.approx(a, rel=1e-10)   # phases are mirror images
    assert np.log(a / b) / (a - b) == pytest.approx(G, rel=0.10)


def _cylinder_laplace(R, taus, n=64, steps=3000):
    shape = (n, n, 1)
    lv = PAPER["laplace_densities"]
    rho = wl.tanh_droplet(shape, R, center=((n - 1) / 2, (n - 1) / 2, 0.0),
                          rho_in=lv["rho_in"], rho_out=lv["rho_out"], width=lv["W"])
    o = Oracle(OracleParams(shape, tau=taus, G=PAPER["G_coh"]["value"]),
               np.zeros((1, n, n), np.uint8))
    o.init_equilibrium(rho)
    o.run(steps)
    r, _, _, _ = o.fields()
    P = o.pressure()                       # Eq. (12)
    d = r[0, 0, n // 2, :] - r[1, 0, n // 2, :]
    k = [i for i in range(n // 2, n - 1) if d[i] > 0 and d[i + 1] <= 0][0]
    radius = k + d[k] / (d[k] - d[k + 1]) - (n - 1) / 2.0
    return P[0, n // 2, n // 2] - P[0, 0, 0], radius


@pytest.mark.parametrize("taus", [(1.0, 1.0), (3.5, 0.62)], ids=["M1", "M25"])
def test_laplace_law_surface_tension(taus):
    """Sec. 3.1: dP is linear in the curvature with gamma = 0.071 at G = 3.5 for every M.
    Cylindrical drops (quasi-2D) obey dP = gamma / R with the same flat-interface gamma."""
    pts = [_cylinder_laplace(R, taus) for R in (10, 14, 18, 22)]
    inv_r = np.array([1.0 / rad for _, rad in pts])
    dp = np.array([d for d, _ in pts])
    A = np.vstack([inv_r, np.ones_like(inv_r)]).T
    (gamma, icpt), res, _, _ = np.linalg.lstsq(A, dp, rcond=None)
    assert gamma == pytest.approx(PAPER["laplace_gamma"]["value"], rel=0.15)
    # linear in 1/R: residuals small against the spread of dP
    assert np.sqrt(res[0] / len(dp)) < 0.02 * (dp.max() - dp.min())
    assert abs(icpt) < 0.05 * dp.max()


def _wall_drop_angle(xi0, nx=120, ny=60, R0=22, steps=8000, tau=(1.0, 1.0)):
    """Half-drop of component 1 on a flat wall; angle through component 2 (the 'water')."""
    shape = (nx, ny, 1)
    solid = np.zeros((1, ny, nx), np.uint8)
    solid[0, 0, :] = 1
    solid[0, ny - 1, :] = 1
    xi = np.where(solid != 0, xi0, 0.0)
    lv = PAPER["laplace_densities"]
    rho = wl.tanh_droplet(shape, R0, center=((nx - 1) / 2, 0.5, 0.0), rho_in=lv["rho_in"],
                          rho_out=lv["rho_out"], width=lv["W"])
    rho[:, solid != 0] = 0
    o = Oracle(OracleParams(shape, tau=tau, G=3.5), solid, xi)
    o.init_equilibrium(rho)
    o.run(steps)
    r, _, _, _ = o.fields()
    d = r[0, 0] - r[1, 0]
    yw = 0.5                                   # halfway wall plane
    pts = []
    for y in range(1, ny - 1):                 # row crossings at least 5 l.u. above the wall
        if y - yw < 5:
            continue
        for x in range(nx - 1):
            if (d[y, x] > 0) != (d[y, x + 1] > 0):
                pts.append((x + d[y, x] / (d[y, x] - d[y, x + 1]), y))
    for x in range(nx):                        # column crossings
        for y in range(1, ny - 2):
            if y - yw < 5:
                continue
            if (d[y, x] > 0) != (d[y + 1, x] > 0):
                pts.append((x, y + d[y, x] / (d[y, x] - d[y + 1, x])))
    pts = np.array(pts)
    A = np.c_[2 * pts[:, 0], 2 * pts[:, 1], np.ones(len(pts))]
    cx, cy, k = np.linalg.lstsq(A, (pts ** 2).sum(1), rcond=None)[0]
    rc = np.sqrt(k + cx * cx + cy * cy)
    theta_drop = np.degrees(np.arccos(-(cy - yw) / rc))
    return 180.0 - theta_drop


@pytest.mark.parametrize("xi0", [-0.2, 0.2])
def test_contact_angle_matches_paper_cubic(xi0):
    """Sec. 3.2 cubic theta(xi) (through the water, component 2): 71.96 deg at xi = -0.2,
    108.63 deg at xi = +0.2; component 1 is non-wetting for xi < 0."""
    c = PAPER["contact_angle_cubic"]["coeffs_deg"]
    expect = np.polyval(c, xi0)
    theta = _wall_drop_angle(xi0)
    assert theta == pytest.approx(expect, abs=4.0)
    spot = PAPER["contact_angle_spot"]["xi_%g" % xi0]
    assert theta == pytest.approx(spot, abs=6.0)


def test_xi_for_45_degrees_recalibrated_at_viscosity_ratio_10():
    """The porous workloads run at M = 10 (tau = 1.5, 0.6) with the wetting
    phase at a 45 degree contact angle.  The flat-wall half drop at that M
    reaches 45 degrees at the recalibrated xi (workloads.XI45_M10); the root of
    the paper's Sec. 3.2 cubic (fitted at M = 25 on a 3D drop) lands about
    5 degrees higher on this quasi-2D drop."""
    theta = _wall_drop_angle(wl.XI45_M10, tau=(1.5, 0.6))
    assert theta == pytest.approx(45.0, abs=1.0)
    assert wl.xi_for_angle(45.0) == pytest.approx(-0.426, abs=1e-3)
