"""Pins of the oracle's open inlet/outlet planes (Sec. 2, the inlet and outlet
conditions; Sec. 4.1, the drainage drive).  CPU only.

What fixes the result, independent of the oracle's own code:
  * psi-hat mirror (the pairing printed after Eq. 11): every missing neighbour
    at an open plane takes the psi-hat of its mirror image, so the x component
    of the interaction force cancels pairwise there, for any state;
  * NEEM conserves the zeroth moment exactly: the imposed component's density
    at its boundary plane equals the imposed value after every step, and its
    first moment moves by (rho_b - rho_f) u_f (the moments of Eq. 2);
  * the entering populations of the other component keep their initial
    values (the paper's statement that they keep the initial condition);
  * a uniform state with matching imposed densities is a fixed point;
  * at steady state the component-1 mass flux is the same through every
    cross-section of a pressure-driven channel.
"""
import numpy as np

from oracle import oracle as orc

E, W, OPP = orc.lattice_tables()
EX = E[:, 0]


def _oracle(shape, solid=None, G=3.5, tau=(1.0, 1.0)):
    nx, ny, nz = shape
    if solid is None:
        solid = np.zeros((nz, ny, nx), np.uint8)
    return orc.Oracle(orc.OracleParams(shape, tau=tau, G=G), solid)


def test_interaction_force_normal_component_vanishes_on_open_planes():
    shape = (10, 7, 6)
    o = _oracle(shape)
    rng = np.random.default_rng(21)
    rho = np.stack([0.4 + rng.random(o.dims), 0.1 + rng.random(o.dims)])
    o.init_equilibrium(rho)
    _, _, F_per, _ = o.fields()
    o.set_open_x(1.0, 0.5)
    _, _, F, _ = o.fields()
    nx = shape[0]
    for xb in (0, nx - 1):
        assert np.abs(F[:, 0, :, :, xb]).max() < 1e-14
        assert np.abs(F_per[:, 0, :, :, xb]).max() > 1e-3      # periodic wrap: generic nonzero
    # interior planes do not see the open planes' mirror
    assert np.array_equal(F[:, :, :, :, 2:nx - 2], F_per[:, :, :, :, 2:nx - 2])
    assert np.abs(F[:, 0, :, :, 1:nx - 1]).max() > 1e-3


def _reservoir_case(shape=(16, 10, 8)):
    nx, ny, nz = shape
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 3:7, 6:10] = 1                                   # obstacle away from the open planes
    o = _oracle(shape, solid, tau=(1.5, 0.6))
    x = np.arange(nx)[None, None, :] * np.ones(o.dims)
    r1 = np.where(x < 3, 1.0, 0.03)
    r2 = np.where(x < 3, 0.03, 1.0)
    o.init_equilibrium(np.stack([r1, r2]))
    return o


def test_imposed_densities_exact_and_entering_populations_held():
    o = _reservoir_case()
    nx = o.dims[2]
    f0 = o.f.copy()
    o.set_open_x(1.02, 1.0)
    o.run(40)
    f = o.f
    fluid_in = o.solid[:, :, 0] == 0
    fluid_out = o.solid[:, :, nx - 1] == 0
    assert fluid_in.all() and fluid_out.all()
    np.testing.assert_allclose(f[0, :, :, :, 0].sum(0), 1.02, rtol=0, atol=1e-13)
    np.testing.assert_allclose(f[1, :, :, :, nx - 1].sum(0), 1.0, rtol=0, atol=1e-13)
    for i in range(19):
        if EX[i] == +1:
            assert np.array_equal(f[1, i, :, :, 0], f0[1, i, :, :, 0])
        if EX[i] == -1:
            assert np.array_equal(f[0, i, :, :, nx - 1], f0[0, i, :, :, nx - 1])
    # first moment of the imposed component: j(x_b) - j(x_f) = (rho_b - rho_f) u_f
    for side, (xb, xf, s, rb) in enumerate(((0, 1, 0, 1.02), (nx - 1, nx - 2, 1, 1.0))):
        ff = f[:, :, :, :, xf]                                # (2, 19, nz, ny)
        rho_f = ff.sum(1)
        u_f = np.einsum("ia,sizy->azy", E.astype(float), ff) / rho_f.sum(0)
        j_b = np.einsum("ia,izy->azy", E.astype(float), f[s, :, :, :, xb])
        j_f = np.einsum("ia,izy->azy", E.astype(float), ff[s])
        np.testing.assert_allclose(j_b - j_f, (rb - rho_f[s]) * u_f, rtol=0, atol=1e-13)


def test_uniform_state_with_matching_densities_is_stationary():
    o = _oracle((12, 6, 5))
    rho = np.stack([np.full(o.dims, 1.0), np.full(o.dims, 0.03)])
    o.init_equilibrium(rho)
    f0 = o.f.copy()
    o.set_open_x(1.0, 0.03)
    o.run(50)
    r, _, _, u = o.fields()
    assert np.abs(u).max() < 1e-13
    np.testing.assert_allclose(o.f, f0, rtol=0, atol=1e-13)


def test_pressure_driven_channel_reaches_a_constant_flux():
    nx, ny, nz = 24, 9, 3
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    o = _oracle((nx, ny, nz), solid)
    rho = np.stack([np.full(o.dims, 1.0), np.full(o.dims, 0.03)]) * (solid == 0)
    o.init_equilibrium(rho)
    o.set_open_x(1.01, 0.03)
    o.run(3000)
    _, _, F, _ = o.fields()
    f1 = o.f[0]
    jx = np.einsum("i,izyx->zyx", EX.astype(float), f1) + 0.5 * F[0, 0]
    flux = (jx * (solid == 0)).sum(axis=(0, 1))              # per x plane
    assert flux.min() > 0                                     # inlet -> outlet
    spread = (flux.max() - flux.min()) / flux.mean()
    assert spread < 5e-3, (spread, flux)
    # plane Poiseuille between the halfway walls (H = ny - 2), driven by the
    # measured pressure gradient of Eq. (12), nu = c_s^2 (tau - 1/2) = 1/6
    r, _, _, u = o.fields()
    P = o.pressure()
    dpdx = (P[1, ny // 2, 16] - P[1, ny // 2, 8]) / 8.0
    H = ny - 2.0
    yy = np.arange(1, ny - 1) - 0.5
    rt = (r[0] + r[1])[1, ny // 2, 12]
    ua = -dpdx / (2.0 * rt * (1.0 / 6.0)) * yy * (H - yy)
    un = u[0, 1, 1:ny - 1, 12]
    assert abs(un.max() / ua.max() - 1.0) < 0.02
    assert np.linalg.norm(un - ua) / np.linalg.norm(ua) < 0.02
