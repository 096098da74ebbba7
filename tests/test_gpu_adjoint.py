"""Hand-written adjoint (HIP, FP32) against central finite differences of the
FP64 oracle, for the smooth non-wetting saturation loss (over the sample, or
over the trapped ganglia) and the outlet flux, with respect to the per-voxel
adhesion parameter xi.  Bars (fd_gate): |g_adj - g_fd| <= 1e-3 max |g_fd| over
the sampled voxels, and at every sampled voxel |g_adj - g_fd| <= 1e-3 |g_fd| +
2e-5 max |g_fd|, so that a wrong sign or a wrong value at a voxel whose
derivative is small against the largest one is caught as well."""
import json
import os

import numpy as np
import pytest

from oracle.oracle import Oracle, OracleParams, lattice_tables
from paper_2207_01534_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adjoint64_fd.json")
GOLDEN_TRAPPED = os.path.join(os.path.dirname(__file__), "golden", "adjoint64_trapped_fd.json")


def _boundary_solid(solid):
    e, _, _ = lattice_tables()
    fluid = solid == 0
    touch = np.zeros_like(fluid)
    for i in range(1, 19):
        touch |= np.roll(fluid, shift=(-e[i][2], -e[i][1], -e[i][0]), axis=(0, 1, 2))
    return (solid != 0) & touch


def fd_gate(adj, fd, label):
    """The two gradient bars against central differences (module docstring);
    prints the per-voxel relative errors of the voxels with |fd| >= 1e-2 max."""
    adj, fd = np.asarray(adj, np.float64), np.asarray(fd, np.float64)
    scale = np.abs(fd).max()
    assert scale > 0
    err = np.abs(adj - fd)
    big = np.abs(fd) >= 1e-2 * scale
    rel_big = (err[big] / np.abs(fd[big])).max()
    print(f"[{label}] max|fd|={scale:.3e} max-normalised err={err.max() / scale:.3e} "
          f"per-voxel rel err (|fd| >= 1e-2 max, {int(big.sum())} voxels)={rel_big:.3e}", flush=True)
    assert err.max() <= 1e-3 * scale
    bad = err > 1e-3 * np.abs(fd) + 2e-5 * scale
    assert not bad.any(), [(float(a), float(f)) for a, f in zip(adj[bad], fd[bad])]
    return err.max() / scale


def _oracle_loss(shape, solid, xi64, rho, tau, G, g, steps, region):
    o = Oracle(OracleParams(shape, tau=tau, G=G, g=g), solid, xi64)
    o.init_equilibrium(rho.astype(np.float32).astype(np.float64))
    o.run(steps)
    return o.loss_snw(region)


def _gpu_gradient(shape, solid, xi, rho, tau, G, g, steps, every, region):
    import torch
    from paper_2207_01534_amd.autograd import WettabilityLoss
    from paper_2207_01534_amd.lattice import Lattice, LatticeParams
    lat = Lattice(LatticeParams(shape=shape, tau=tau, G=G, g=g), torch.as_tensor(solid),
                  torch.as_tensor(xi), None)
    xi_t = torch.tensor(xi, device="cuda", requires_grad=True)
    rho_t = torch.as_tensor(rho.astype(np.float32), device="cuda")
    reg_t = torch.as_tensor(region, device="cuda")
    L = WettabilityLoss.apply(xi_t, lat, rho_t, reg_t, steps, every)
    L.backward()
    torch.cuda.synchronize()
    return float(L.detach()), xi_t.grad.double().cpu().numpy(), lat


@pytest.mark.parametrize("steps,every", [(1, 1), (2, 1), (9, 4), (30, 7)])
def test_small_gradient_against_oracle_fd(steps, every):
    shape = (12, 10, 8)
    nx, ny, nz = shape
    print(f"[case] adjoint small {shape} steps={steps} every={every}", flush=True)
    solid = wl.random_mask(shape, 0.25, seed=77)
    xi = wl.uniform_xi(solid, -0.4, 0.4, seed=78)
    rho = wl.tanh_droplet(shape, 3.0)
    rho[:, solid != 0] = 0
    tau, G, g = (1.5, 0.6), 3.5, ((2e-4, 0.0, 0.0), (0.0, 0.0, 0.0))
    region = np.ones((nz, ny, nx), np.uint8)
    L_gpu, grad, lat = _gpu_gradient(shape, solid, xi, rho, tau, G, g, steps, every, region)
    xi64 = xi.astype(np.float64)
    L_orc = _oracle_loss(shape, solid, xi64, rho, tau, G, g, steps, region)
    assert L_gpu == pytest.approx(L_orc, rel=1e-5, abs=1e-7)
    bs = _boundary_solid(solid)
    assert lat.boundary_count() == int(bs.sum())
    assert np.all(grad[~bs] == 0.0)                       # structural zeros
    rng = np.random.default_rng(steps)
    cand = np.argwhere(bs)
    pick = cand[rng.choice(len(cand), size=10, replace=False)]
    eps = 1e-3
    fd = []
    for z, y, x in pick:
        xp, xm = xi64.copy(), xi64.copy()
        xp[z, y, x] += eps
        xm[z, y, x] -= eps
        fd.append((_oracle_loss(shape, solid, xp, rho, tau, G, g, steps, region)
                   - _oracle_loss(shape, solid, xm, rho, tau, G, g, steps, region)) / (2 * eps))
    fd = np.array(fd)
    adj = np.array([grad[z, y, x] for z, y, x in pick])
    scale = np.abs(fd).max()
    fd_gate(adj, fd, f"adjoint steps={steps}")
    # directional derivative along a random direction over all boundary voxels
    v = np.where(bs, rng.standard_normal(bs.shape), 0.0)
    v /= np.abs(v).max()
    def directional(e):
        return (_oracle_loss(shape, solid, xi64 + e * v, rho, tau, G, g, steps, region)
                - _oracle_loss(shape, solid, xi64 - e * v, rho, tau, G, g, steps, region)) / (2 * e)
    dd, dd_half = directional(eps), directional(eps / 2)
    # the finite difference itself is converged: halving the step changes it
    # by the O(eps^2) truncation term only
    assert dd_half == pytest.approx(dd, rel=1e-5, abs=1e-6 * scale)
    assert float((grad * v).sum()) == pytest.approx(dd_half, rel=1e-3, abs=1e-3 * scale)


def test_trapped_saturation_gradient_against_oracle_fd():
    """The trapped variant of the loss: the smooth non-wetting saturation over
    the non-wetting ganglia cut off from the inlet reservoir in the
    unperturbed run at T (found on the oracle's own run, then frozen), on a
    porous lattice seeded with dispersed ganglia."""
    shape, steps, every = (20, 14, 12), 30, 7
    print(f"[case] adjoint trapped {shape} steps={steps} every={every}", flush=True)
    solid, _ = wl.sphere_pack(shape, 2.0, 0.6, seed=91)
    rho = wl.ganglia_rho(solid, 4, 2.0, seed=92)
    xi = wl.uniform_xi(solid, -0.4, 0.4, seed=93)
    tau, G, g = (1.5, 0.6), 3.5, ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    xi64 = xi.astype(np.float64)
    o = Oracle(OracleParams(shape, tau=tau, G=G, g=g), solid, xi64)
    o.init_equilibrium(rho.astype(np.float32).astype(np.float64))
    o.run(steps)
    region = wl.trapped_region(o.fields()[0], solid)
    assert region.sum() > 50
    L_orc = o.loss_snw(region)
    L_gpu, grad, _ = _gpu_gradient(shape, solid, xi, rho, tau, G, g, steps, every, region)
    assert L_gpu == pytest.approx(L_orc, rel=1e-5, abs=1e-7)
    bs = _boundary_solid(solid)
    rng = np.random.default_rng(94)
    cand = np.argwhere(bs)
    pick = cand[rng.choice(len(cand), size=10, replace=False)]
    eps = 1e-3
    fd = []
    for z, y, x in pick:
        xp, xm = xi64.copy(), xi64.copy()
        xp[z, y, x] += eps
        xm[z, y, x] -= eps
        fd.append((_oracle_loss(shape, solid, xp, rho, tau, G, g, steps, region)
                   - _oracle_loss(shape, solid, xm, rho, tau, G, g, steps, region)) / (2 * eps))
    fd = np.array(fd)
    adj = np.array([grad[z, y, x] for z, y, x in pick])
    scale = np.abs(fd).max()
    print(f"[adjoint-trapped] region={int(region.sum())} L={L_gpu:.6f}", flush=True)
    fd_gate(adj, fd, "adjoint-trapped")
    v = np.where(bs, rng.standard_normal(bs.shape), 0.0)
    v /= np.abs(v).max()
    dd = (_oracle_loss(shape, solid, xi64 + eps * v, rho, tau, G, g, steps, region)
          - _oracle_loss(shape, solid, xi64 - eps * v, rho, tau, G, g, steps, region)) / (2 * eps)
    assert float((grad * v).sum()) == pytest.approx(dd, rel=1e-3, abs=1e-3 * scale)


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden finite differences not generated")
def test_adjoint64_full_against_golden_fd():
    """64^3 sphere pack, xi ~ U[-0.4, 0.4], 500 steps, checkpoint every 25;
    20 voxels against FP64 oracle central differences stored by
    tests/golden/make_adjoint64_fd.py."""
    rec = json.load(open(GOLDEN))
    w = wl.workload("adjoint64")
    assert wl.sha256(w.solid) == rec["solid_sha256"] and wl.sha256(w.xi) == rec["xi_sha256"]
    nx, ny, nz = w.shape
    region = np.zeros((nz, ny, nx), np.uint8)
    region[:, :, 3:nx - 3] = 1
    print(f"[case] adjoint64 full steps={rec['steps']}", flush=True)
    L, grad, _ = _gpu_gradient(w.shape, w.solid, w.xi, w.rho, w.tau, w.G, w.g, rec["steps"], 25, region)
    assert L == pytest.approx(rec["loss"], rel=1e-5)
    fd = np.array([v["fd"] for v in rec["voxels"]])
    adj = np.array([grad[tuple(v["zyx"])] for v in rec["voxels"]])
    for v, a in zip(rec["voxels"], adj):
        print(f"   {v['zyx']} fd={v['fd']:.6e} adj={a:.6e}", flush=True)
    fd_gate(adj, fd, "adjoint64")


@pytest.mark.skipif(not os.path.exists(GOLDEN_TRAPPED), reason="golden finite differences not generated")
def test_adjoint64_trapped_against_golden_fd():
    """The 64^3 adjoint workload as specified for the trapped saturation: the
    non-wetting phase seeded as dispersed ganglia, the loss the smooth
    non-wetting saturation over the ganglia still cut off from the inlet in
    the oracle's unperturbed run after 500 steps (frozen), checkpoint every
    25; 20 voxels against the FP64 oracle's central differences stored by
    tests/golden/make_adjoint64_trapped_fd.py."""
    rec = json.load(open(GOLDEN_TRAPPED))
    w = wl.workload("adjoint64")
    gp = rec["initial"]["ganglia"]
    rho = wl.ganglia_rho(w.solid, gp["n_blobs"], gp["radius"], seed=gp["seed"])
    assert wl.sha256(w.solid) == rec["solid_sha256"] and wl.sha256(w.xi) == rec["xi_sha256"]
    assert wl.sha256(rho.astype(np.float32)) == rec["rho_sha256"]
    region = np.zeros(w.solid.size, np.uint8)
    region[np.asarray(rec["region_flat_indices"], np.int64)] = 1
    region = region.reshape(w.solid.shape)
    print(f"[case] adjoint64 trapped steps={rec['steps']} region={int(region.sum())}", flush=True)
    L, grad, _ = _gpu_gradient(w.shape, w.solid, w.xi, rho, w.tau, w.G, w.g, rec["steps"], 25, region)
    assert L == pytest.approx(rec["loss"], rel=1e-5)
    fd = np.array([v["fd"] for v in rec["voxels"]])
    adj = np.array([grad[tuple(v["zyx"])] for v in rec["voxels"]])
    for v, a in zip(rec["voxels"], adj):
        print(f"   {v['zyx']} fd={v['fd']:.6e} adj={a:.6e}", flush=True)
    fd_gate(adj, fd, "adjoint64-trapped")


def test_adjoint_entry_points_refuse_unsupported_lattices():
    """The adjoint covers FP32 storage with periodic x: FP16 storage and open
    planes are refused with an error, and the lattice stays usable."""
    import torch
    from paper_2207_01534_amd.lattice import Lattice, LatticeParams, MclbmError, Storage
    shape = (12, 10, 8)
    nx, ny, nz = shape
    solid = wl.random_mask(shape, 0.25, seed=77)
    xi = wl.uniform_xi(solid, -0.4, 0.4, seed=78)
    rho = wl.tanh_droplet(shape, 3.0)
    rho[:, solid != 0] = 0
    half = Lattice(LatticeParams(shape=shape, storage=Storage.F16), torch.as_tensor(solid), torch.as_tensor(xi),
                   torch.as_tensor(rho.astype(np.float32)))
    with pytest.raises(MclbmError):
        half.step_checkpointed(4, 2)
    half.step(2)
    opened = Lattice(LatticeParams(shape=(nx + 2, ny, nz)), torch.zeros((nz, ny, nx + 2), dtype=torch.uint8),
                     None, torch.full((2, nz, ny, nx + 2), 0.5))
    opened.set_open_x(0.52, 0.5)
    with pytest.raises(MclbmError):
        opened.step_checkpointed(4, 2)
    opened.step(2)
    assert opened.time == 2


def _oracle_flux(shape, solid, xi64, rho, tau, G, g, steps, region):
    o = Oracle(OracleParams(shape, tau=tau, G=G, g=g), solid, xi64)
    o.init_equilibrium(rho.astype(np.float32).astype(np.float64))
    o.run(steps)
    r, _, _, u = o.fields()
    sel = (solid == 0) & (region != 0)
    return float((r[0] * u[0])[sel].sum())


@pytest.mark.parametrize("steps,every", [(1, 1), (2, 1), (9, 4)])
def test_flux_gradient_against_oracle_fd(steps, every):
    """Outlet flux sum rho1 u_x over the plane x = nx - 3: loss against the
    oracle's fields, gradient against its central differences at sampled
    boundary voxels and along a random direction over all of them."""
    import torch
    from paper_2207_01534_amd.autograd import OutletFluxLoss
    from paper_2207_01534_amd.lattice import Lattice, LatticeParams
    shape = (12, 10, 8)
    nx, ny, nz = shape
    print(f"[case] flux adjoint {shape} steps={steps} every={every}", flush=True)
    solid = wl.random_mask(shape, 0.25, seed=91)
    xi = wl.uniform_xi(solid, -0.4, 0.4, seed=92)
    rho = wl.tanh_droplet(shape, 3.0)
    rho[:, solid != 0] = 0
    tau, G, g = (1.5, 0.6), 3.5, ((3e-4, 0.0, 0.0), (1e-4, 0.0, 0.0))
    region = np.zeros((nz, ny, nx), np.uint8)
    region[:, :, nx - 3] = 1
    lat = Lattice(LatticeParams(shape=shape, tau=tau, G=G, g=g), torch.as_tensor(solid), torch.as_tensor(xi), None)
    xi_t = torch.tensor(xi, device="cuda", requires_grad=True)
    L = OutletFluxLoss.apply(xi_t, lat, torch.as_tensor(rho.astype(np.float32), device="cuda"),
                             torch.as_tensor(region, device="cuda"), steps, every)
    L.backward()
    torch.cuda.synchronize()
    grad = xi_t.grad.double().cpu().numpy()
    xi64 = xi.astype(np.float64)
    L_orc = _oracle_flux(shape, solid, xi64, rho, tau, G, g, steps, region)
    L_gpu = float(L.detach())
    print(f"[flux] L_gpu={L_gpu:.6e} L_orc={L_orc:.6e}", flush=True)
    assert L_gpu == pytest.approx(L_orc, rel=1e-4, abs=1e-7 * max(abs(L_orc), 1e-3))
    bs = _boundary_solid(solid)
    assert np.all(grad[~bs] == 0.0)
    rng = np.random.default_rng(100 + steps)
    cand = np.argwhere(bs)
    pick = cand[rng.choice(len(cand), size=10, replace=False)]
    eps = 1e-3
    fd = []
    for z, y, x in pick:
        xp, xm = xi64.copy(), xi64.copy()
        xp[z, y, x] += eps
        xm[z, y, x] -= eps
        fd.append((_oracle_flux(shape, solid, xp, rho, tau, G, g, steps, region)
                   - _oracle_flux(shape, solid, xm, rho, tau, G, g, steps, region)) / (2 * eps))
    fd = np.array(fd)
    adj = np.array([grad[z, y, x] for z, y, x in pick])
    scale = np.abs(fd).max()
    fd_gate(adj, fd, f"flux-adjoint steps={steps}")
    v = np.where(bs, rng.standard_normal(bs.shape), 0.0)
    v /= np.abs(v).max()

    def directional(e):
        return (_oracle_flux(shape, solid, xi64 + e * v, rho, tau, G, g, steps, region)
                - _oracle_flux(shape, solid, xi64 - e * v, rho, tau, G, g, steps, region)) / (2 * e)
    dd, dd_half = directional(eps), directional(eps / 2)
    assert dd_half == pytest.approx(dd, rel=1e-5, abs=1e-6 * scale)
    assert float((grad * v).sum()) == pytest.approx(dd_half, rel=1e-3, abs=1e-3 * scale)


def test_reverse_sweep_refuses_a_state_it_was_not_recorded_for():
    """The reverse sweep differentiates the run recorded by the last
    step_checkpointed: a step, a re-initialisation or a second recording in
    between, other nsteps / every, another checkpoint buffer or one smaller
    than nsteps / every need are refused, and an untouched record still gives
    the same gradient bit for bit (twice in a row)."""
    import torch
    from paper_2207_01534_amd.lattice import Lattice, LatticeParams, MclbmError
    shape = (12, 10, 8)
    solid = wl.random_mask(shape, 0.25, seed=91)
    xi = wl.uniform_xi(solid, -0.4, 0.4, seed=92)
    rho = wl.tanh_droplet(shape, 3.0)
    rho[:, solid != 0] = 0
    rho_t = torch.as_tensor(rho.astype(np.float32), device="cuda")
    lat = Lattice(LatticeParams(shape=shape, tau=(1.5, 0.6)), torch.as_tensor(solid), torch.as_tensor(xi), rho_t)
    reg = torch.ones(shape[::-1], dtype=torch.uint8, device="cuda")
    ck = lat.step_checkpointed(6, 2)
    g1 = lat.gradient_snw(6, 2, ck, reg)
    g2 = lat.gradient_snw(6, 2, ck, reg)
    assert torch.equal(g1, g2)
    for bad in ((5, 2), (6, 3)):
        with pytest.raises(MclbmError):
            lat.gradient_snw(*bad, ck, reg)
    with pytest.raises(MclbmError):
        lat.gradient_snw(6, 2, ck[: ck.numel() // 2], reg)     # smaller than 3 checkpoints
    other = torch.empty_like(ck)
    other.copy_(ck)
    with pytest.raises(MclbmError):
        lat.gradient_snw(6, 2, other, reg)                     # not the buffer that was recorded
    lat.step(1)
    with pytest.raises(MclbmError):
        lat.gradient_snw(6, 2, ck, reg)                        # stepped since the recording
    lat.init_equilibrium(rho_t)
    ck_a = lat.step_checkpointed(6, 2)
    lat.init_equilibrium(rho_t)
    ck_b = lat.step_checkpointed(6, 2)
    with pytest.raises(MclbmError):
        lat.gradient_snw(6, 2, ck_a, reg)                      # superseded by the second recording
    g3 = lat.gradient_snw(6, 2, ck_b, reg)
    assert torch.equal(g1, g3)


@pytest.mark.parametrize("steps,every", [(1, 1), (5, 1), (9, 4), (10, 5), (30, 7)])
def test_level_log_gives_the_same_gradient_bit_for_bit(steps, every):
    """A checkpoint buffer with the level log (every level's pseudopotential
    field and the last segment's states, kept by the forward) lets the reverse
    sweep skip recomputing the densities, the virtual solid densities and the
    last segment.  Both sweeps must give the same gradient bit for bit, for
    both losses, with last segments of one to five steps and with one step
    per segment, and the forward must leave the lattice's state as the plain
    recording does.  A buffer cut below the log it was recorded with is
    refused."""
    import torch
    from paper_2207_01534_amd.lattice import Lattice, LatticeParams, MclbmError
    shape = (20, 14, 12)
    solid = wl.random_mask(shape, 0.3, seed=95)
    xi = wl.uniform_xi(solid, -0.4, 0.4, seed=96)
    rho = wl.tanh_droplet(shape, 4.0)
    rho[:, solid != 0] = 0
    rho_t = torch.as_tensor(rho.astype(np.float32), device="cuda")
    lat = Lattice(LatticeParams(shape=shape, tau=(1.5, 0.6), G=3.5, g=((1e-5, 0, 0), (0, 0, 0))),
                  torch.as_tensor(solid), torch.as_tensor(xi), rho_t)
    reg = torch.zeros(shape[::-1], dtype=torch.uint8, device="cuda")
    reg[:, :, shape[0] // 2:] = 1
    out = {}
    for log in (False, True):
        lat.init_equilibrium(rho_t)
        ck = lat.step_checkpointed(steps, every, level_log=log)
        state = lat.save(torch.zeros(lat.state_bytes(), dtype=torch.uint8, device="cuda"))  # padding zeroed
        out[log] = (lat.gradient_snw(steps, every, ck, reg), lat.gradient_flux(steps, every, ck, reg), state)
        if log:
            with pytest.raises(MclbmError):
                lat.gradient_snw(steps, every, ck[: ck.numel() - 256], reg)
    assert torch.equal(out[True][0], out[False][0])
    assert torch.equal(out[True][1], out[False][1])
    assert torch.equal(out[True][2], out[False][2])
    assert float(out[True][0].abs().max()) > 0 and float(out[True][1].abs().max()) > 0
