"""Failure detection and recovery on the HIP path: a droplet at a cohesion far
beyond the stable range (G = 8) drives densities negative and then
non-finite within a few tens of steps (the FP64 oracle blows up by step 40
too).  The diagnostics count the non-finite nodes and report them as an
error; restoring a saved state recovers the run exactly."""
import numpy as np
import pytest

from oracle.oracle import Oracle, OracleParams
from paper_2207_01534_amd import workloads as wl

from parity_util import gpu_case

pytestmark = pytest.mark.gpu

G_UNSTABLE = 8.0
TAU = (1.0, 1.0)


def test_blow_up_is_detected_and_a_saved_state_restores():
    import torch
    from paper_2207_01534_amd.lattice import MclbmError
    w = wl.workload("droplet32")
    print(f"[case] droplet32 G={G_UNSTABLE} tau={TAU}", flush=True)
    lat = gpu_case(w.shape, w.solid, w.xi, w.rho, TAU, G_UNSTABLE, w.g)
    lat.step(10)
    good = lat.diagnostics()
    assert good["nonfinite"] == 0
    saved = lat.save()
    rho_saved = lat.density().clone()
    detected = None
    for k in range(40):
        lat.step(5)
        d = lat.diagnostics(raise_nonfinite=False)
        if d["nonfinite"] > 0:
            detected = lat.time
            break
    print(f"[failure] non-finite detected at step {detected}", flush=True)
    assert detected is not None and detected <= 210
    with pytest.raises(MclbmError):
        lat.diagnostics()
    # the oracle blows up as well under the same parameters
    o = Oracle(OracleParams(w.shape, tau=TAU, G=G_UNSTABLE, g=w.g), w.solid, w.xi.astype(np.float64))
    o.init_equilibrium(w.rho.astype(np.float32).astype(np.float64))
    o.run(detected)
    r, _, _, _ = o.fields()
    assert not np.isfinite(r).all() or o.diagnostics()[5] > 0
    # recovery from the saved state
    lat.load(saved)
    assert lat.time == 10
    d = lat.diagnostics()
    assert d["nonfinite"] == 0
    assert d["mass1"] == good["mass1"] and d["mass2"] == good["mass2"]
    torch.cuda.synchronize()
    assert torch.equal(lat.density(), rho_saved)


def test_state_of_another_solid_mask_is_refused():
    """Populations are stored per fluid voxel: a state saved under one solid
    mask does not fit another mask of the same shape (nor of the same fluid
    count) and is refused, leaving the lattice's own state untouched."""
    import torch
    from paper_2207_01534_amd.lattice import MclbmError
    shape = (16, 12, 10)
    solid_a = wl.random_mask(shape, 0.25, seed=41)
    solid_b = np.roll(solid_a, 1, axis=2)               # same fluid count, other voxels
    solid_c = wl.random_mask(shape, 0.3, seed=42)
    xi = np.zeros(solid_a.shape, np.float32)
    rho = wl.tanh_droplet(shape, 3.0)
    lat_a = gpu_case(shape, solid_a, xi, np.where(solid_a[None] != 0, 0, rho), TAU, 3.5, ((0, 0, 0), (0, 0, 0)))
    lat_a.step(3)
    saved_a = lat_a.save()
    for solid in (solid_b, solid_c):
        lat = gpu_case(shape, solid, xi, np.where(solid[None] != 0, 0, rho), TAU, 3.5, ((0, 0, 0), (0, 0, 0)))
        lat.step(2)
        before = lat.density()
        with pytest.raises(MclbmError):
            lat.load(saved_a)
        assert lat.time == 2 and torch.equal(lat.density(), before)
    lat_a.step(2)
    lat_a.load(saved_a)                                  # its own mask: accepted
    assert lat_a.time == 3
