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
