"""Open inlet/outlet planes on the HIP path against the FP64 oracle (Sec. 2,
the inlet and outlet conditions; Sec. 4.1, the drainage drive).

The oracle runs the physical domain of nx - 2 planes with the open
conditions applied directly; the GPU lattice carries one ghost plane at each
x end, so GPU planes 1 .. nx-2 are compared with oracle planes 0 .. nx-3.
"""
import numpy as np
import pytest

from parity_util import field_errors, gpu_case, gpu_fields

from oracle.oracle import Oracle, OracleParams

pytestmark = pytest.mark.gpu

TAU = (1.5, 0.6)
G = 3.5
RHO_IN, RHO_OUT = 1.02, 1.0


def _case(nxp=22, ny=12, nz=10, seed=7):
    """Physical domain nxp x ny x nz: reservoir of component 1 at the inlet
    (tanh interface, W = 5), component 2 elsewhere, two spherical grains in
    the middle; returns the GPU lattice arrays (with ghost planes) and the
    oracle arrays."""
    rng = np.random.default_rng(seed)
    x = np.arange(nxp)[None, None, :]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nxp), indexing="ij")
    solid = np.zeros((nz, ny, nxp), np.uint8)
    for c in rng.uniform([8, 2, 2], [14, ny - 2, nz - 2], size=(2, 3)):
        solid[(xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2 <= 9.0] = 1
    solid[:, :, :2] = 0
    solid[:, :, nxp - 2:] = 0
    phi = 0.5 * (1.0 + np.tanh((5.0 - x) / 2.5)) * np.ones((nz, ny, nxp))
    r1 = 0.03 + (1.0 - 0.03) * phi
    r2 = 0.03 + (1.0 - 0.03) * (1.0 - phi)
    rho = np.stack([r1, r2]).astype(np.float32)
    xi = np.where(solid != 0, -0.2, 0.0).astype(np.float32)
    pad = lambda a: np.concatenate([a[..., :1], a, a[..., -1:]], axis=-1)
    g_solid = pad(solid)
    g_rho = np.stack([pad(rho[0]), pad(rho[1])])
    g_xi = pad(xi)
    return (nxp + 2, ny, nz), g_solid, g_xi, g_rho, (nxp, ny, nz), solid, xi, rho


def _case_ragged(nxp=20, ny=37, nz=21, seed=11):
    """Boundary planes wider than one 16 x 16 patch of rows in y and z, with a
    ragged last patch in both, and grains that reach the plane next to the
    boundary plane (physical x = 2 and nxp - 3), so that the rebuild meets
    wall slots there; otherwise as _case."""
    rng = np.random.default_rng(seed)
    x = np.arange(nxp)[None, None, :]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nxp), indexing="ij")
    solid = np.zeros((nz, ny, nxp), np.uint8)
    for cx in (4.5, nxp - 5.5, 4.5, nxp - 5.5, nxp / 2.0):
        cy, cz = rng.uniform(0, ny), rng.uniform(0, nz)
        dy = (yy - cy + ny / 2.0) % ny - ny / 2.0             # periodic in y and z
        dz = (zz - cz + nz / 2.0) % nz - nz / 2.0
        solid[(xx - cx) ** 2 + dy ** 2 + dz ** 2 <= 2.6 ** 2] = 1
    solid[:, :, :2] = 0
    solid[:, :, nxp - 2:] = 0
    assert solid[:, :, 2].any() and solid[:, :, nxp - 3].any()
    phi = 0.5 * (1.0 + np.tanh((5.0 - x) / 2.5)) * np.ones((nz, ny, nxp))
    r1 = 0.03 + (1.0 - 0.03) * phi
    r2 = 0.03 + (1.0 - 0.03) * (1.0 - phi)
    rho = np.stack([r1, r2]).astype(np.float32)
    xi = np.where(solid != 0, -0.2, 0.0).astype(np.float32)
    pad = lambda a: np.concatenate([a[..., :1], a, a[..., -1:]], axis=-1)
    return ((nxp + 2, ny, nz), pad(solid), pad(xi), np.stack([pad(rho[0]), pad(rho[1])]),
            (nxp, ny, nz), solid, xi, rho)


def _oracle(shape, solid, xi, rho):
    o = Oracle(OracleParams(shape, tau=TAU, G=G), solid, xi.astype(np.float64))
    r = rho.astype(np.float64)
    r[:, solid != 0] = 0.0
    o.init_equilibrium(r)
    return o


def _interior(fields):
    r, u, F, P = fields
    return r[..., 1:-1], u[..., 1:-1], F[..., 1:-1], P[..., 1:-1]


def _oracle_fields(o):
    r, _, F, u = o.fields()
    return r, u, F, o.pressure()


@pytest.mark.parametrize("storage,e_rho_bar,e_u_bar", [(0, 1e-5, 1e-4), (1, 2e-3, 2e-3), (2, 2e-2, 2e-2)],
                         ids=["f32", "f16", "bf16"])
def test_open_planes_match_oracle_with_inlet_ramp(storage, e_rho_bar, e_u_bar):
    gshape, gsolid, gxi, grho, oshape, osolid, oxi, orho = _case()
    print(f"[case] open planes {oshape} (+2 ghost planes) storage={storage}", flush=True)
    lat = gpu_case(gshape, gsolid, gxi, grho, TAU, G, ((0, 0, 0), (0, 0, 0)), storage=storage)
    o = _oracle(oshape, osolid, oxi, orho)
    lat.set_open_x(RHO_IN, RHO_OUT)
    o.set_open_x(RHO_IN, RHO_OUT)
    lat.step(120)
    o.run(120)
    lat.set_open_x(RHO_IN + 0.02, RHO_OUT)                   # inlet-density ramp
    o.set_open_x(RHO_IN + 0.02, RHO_OUT)
    lat.step(80)
    o.run(80)
    e = field_errors(_interior(gpu_fields(lat)), _oracle_fields(o), osolid)
    print(f"[open] storage={storage} e_rho={e['e_rho']:.3e} e_u={e['e_u']:.3e} e_F={e['e_F']:.3e} "
          f"u_max={e['u_max']:.3e}", flush=True)
    assert e["u_max"] > 1e-4                                  # the drive moves the fluid
    assert e["e_rho"] <= e_rho_bar and e["e_u"] <= e_u_bar, e
    # imposed densities on the boundary planes
    r = lat.density().cpu().numpy()
    np.testing.assert_allclose(r[0][:, :, 1], RHO_IN + 0.02, rtol=0, atol=2e-6)
    np.testing.assert_allclose(r[1][:, :, -2], RHO_OUT, rtol=0, atol=2e-6)


@pytest.mark.parametrize("storage,e_rho_bar,e_u_bar", [(0, 1e-5, 1e-4), (1, 2e-3, 2e-3)], ids=["f32", "f16"])
def test_open_planes_over_several_ragged_row_patches(storage, e_rho_bar, e_u_bar):
    gshape, gsolid, gxi, grho, oshape, osolid, oxi, orho = _case_ragged()
    print(f"[case] open planes ragged {oshape} (+2 ghost planes) storage={storage}", flush=True)
    lat = gpu_case(gshape, gsolid, gxi, grho, TAU, G, ((0, 0, 0), (0, 0, 0)), storage=storage)
    o = _oracle(oshape, osolid, oxi, orho)
    lat.set_open_x(RHO_IN, RHO_OUT)
    o.set_open_x(RHO_IN, RHO_OUT)
    lat.step(101)                                            # ends on an odd level
    o.run(101)
    e = field_errors(_interior(gpu_fields(lat)), _oracle_fields(o), osolid)
    print(f"[open] ragged storage={storage} e_rho={e['e_rho']:.3e} e_u={e['e_u']:.3e} e_F={e['e_F']:.3e} "
          f"u_max={e['u_max']:.3e}", flush=True)
    assert e["u_max"] > 1e-4
    assert e["e_rho"] <= e_rho_bar and e["e_u"] <= e_u_bar, e
    r = lat.density().cpu().numpy()
    fl_in, fl_out = gsolid[:, :, 1] == 0, gsolid[:, :, -2] == 0
    np.testing.assert_allclose(r[0][:, :, 1][fl_in], RHO_IN, rtol=0, atol=2e-6)
    np.testing.assert_allclose(r[1][:, :, -2][fl_out], RHO_OUT, rtol=0, atol=2e-6)


def test_open_pressure_readout_matches_oracle():
    gshape, gsolid, gxi, grho, oshape, osolid, oxi, orho = _case()
    lat = gpu_case(gshape, gsolid, gxi, grho, TAU, G, ((0, 0, 0), (0, 0, 0)))
    o = _oracle(oshape, osolid, oxi, orho)
    lat.set_open_x(RHO_IN, RHO_OUT)
    o.set_open_x(RHO_IN, RHO_OUT)
    lat.step(60)
    o.run(60)
    pc = lat.open_x_pressure()
    P = o.pressure()
    fl = osolid == 0
    p_in = P[..., 0][fl[..., 0]].mean()
    p_out = P[..., -1][fl[..., -1]].mean()
    print(f"[open] P_in={pc['P_in']:.6f} ({p_in:.6f}) P_out={pc['P_out']:.6f} ({p_out:.6f})", flush=True)
    assert pc["P_in"] == pytest.approx(p_in, abs=1e-5)
    assert pc["P_out"] == pytest.approx(p_out, abs=1e-5)
    assert pc["P_c"] == pytest.approx(p_in - p_out, abs=2e-5)


def test_open_planes_refuse_solid_on_required_planes():
    from paper_2207_01534_amd.lattice import MclbmError
    gshape, gsolid, gxi, grho, _, _, _, _ = _case()
    gsolid = gsolid.copy()
    gsolid[3, 4, 2] = 1                                       # plane x = 2 must stay fluid
    lat = gpu_case(gshape, gsolid, gxi, grho, TAU, G, ((0, 0, 0), (0, 0, 0)))
    with pytest.raises(MclbmError):
        lat.set_open_x(RHO_IN, RHO_OUT)
    lat.step(2)                                               # still periodic and usable


def test_new_geometry_state_or_load_returns_x_to_periodic():
    """Open planes hold populations captured from one state: set_geometry,
    init_equilibrium and load_state return x to periodic, so the adjoint (which
    refuses open planes) accepts the lattice again, and reopening checks the
    planes of the new geometry before anything is captured."""
    import torch
    from paper_2207_01534_amd.lattice import MclbmError
    gshape, gsolid, gxi, grho, _, _, _, _ = _case()
    lat = gpu_case(gshape, gsolid, gxi, grho, TAU, G, ((0, 0, 0), (0, 0, 0)))
    saved = lat.save()
    rho32 = torch.as_tensor(np.asarray(grho, np.float32))
    for reset in ("geometry", "init", "load"):
        print(f"[case] open planes then {reset}", flush=True)
        lat.set_open_x(RHO_IN, RHO_OUT)
        with pytest.raises(MclbmError):
            lat.step_checkpointed(2, 1)
        if reset == "geometry":
            lat.set_geometry(torch.as_tensor(gsolid), torch.as_tensor(np.asarray(gxi, np.float32)))
            lat.init_equilibrium(rho32)
        elif reset == "init":
            lat.init_equilibrium(rho32)
        else:
            lat.load(saved)
        lat.step_checkpointed(2, 1)                           # periodic again
        assert lat.diagnostics()["nonfinite"] == 0
    blocked = gsolid.copy()
    blocked[3, 4, 1] = 1                                      # the inlet plane x = 1 must be fluid
    lat.set_open_x(RHO_IN, RHO_OUT)
    lat.set_geometry(torch.as_tensor(blocked), torch.as_tensor(np.asarray(gxi, np.float32)))
    lat.init_equilibrium(rho32)
    with pytest.raises(MclbmError):
        lat.set_open_x(RHO_IN, RHO_OUT)                      # checked again on the new geometry
    lat.step(2)
    assert lat.diagnostics()["nonfinite"] == 0
