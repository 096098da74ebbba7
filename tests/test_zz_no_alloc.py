"""The diagnostics entry point that allocates nothing (its reduction scratch is
the library's own device array) against mclbm_diagnostics, through the C ABI,
on two calls in a row: a lattice of more patches than the array has partial
slots, then a smaller one (whose partials overwrite only part of what the
first call left in the array)."""
import numpy as np
import pytest

from paper_2207_01534_amd import workloads as wl

from parity_util import gpu_case

pytestmark = pytest.mark.gpu

KEYS = ("mass1", "mass2", "S_w", "S_nw", "u_max", "nonfinite", "n_fluid")


def _lattice(shape, seed):
    solid = wl.random_mask(shape, 0.3, seed=seed)
    xi = wl.uniform_xi(solid, -0.4, 0.4, seed=seed + 1)
    rho = wl.tanh_droplet(shape, min(shape) / 4.0)
    rho[:, solid != 0] = 0
    return gpu_case(shape, solid, xi, rho, (1.5, 0.6), 3.5, ((2e-5, 0, 0), (0, 0, 0)))


@pytest.mark.parametrize("shape,patches_beyond_slots", [((256, 128, 64), True), ((40, 24, 20), False)])
def test_noalloc_diagnostics_match_the_workspace_entry_point(shape, patches_beyond_slots):
    print(f"[case] diagnostics_noalloc {shape}", flush=True)
    nx, ny, nz = shape
    assert (((nx + 63) // 64) * ((ny + 3) // 4) * nz > 4096) == patches_beyond_slots
    lat = _lattice(shape, seed=nx + ny + nz)
    lat.step(7)
    ref = lat.diagnostics()
    for _ in range(2):
        got = lat.diagnostics(noalloc=True)
        print(f"[diag] ref={ref} noalloc={got}", flush=True)
        for k in ("S_w", "u_max", "nonfinite", "n_fluid"):
            assert got[k] == ref[k], k                 # counts and the maximum do not depend on grouping
        for k in ("mass1", "mass2", "S_nw"):
            if patches_beyond_slots:
                assert got[k] == pytest.approx(ref[k], rel=1e-13, abs=0), k
            else:
                assert got[k] == ref[k], k             # same partition of the sums: identical bits
    lat.step(1)
    assert lat.diagnostics(noalloc=True)["n_fluid"] == ref["n_fluid"]
