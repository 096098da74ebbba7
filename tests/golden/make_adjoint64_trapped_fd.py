"""Write tests/golden/adjoint64_trapped_fd.json: central finite differences of
the FP64 oracle for the gradient of the trapped non-wetting saturation on the
64^3 adjoint workload.

Workload: the 64^3 sphere pack (r = 6, porosity 0.40, seed 64) with
xi ~ U[-0.4, 0.4] at solid voxels (seed 6401), M = 10, G = 3.5, body force
g1 = 5e-4 along x, and the non-wetting phase (component 1) seeded as twelve
dispersed ganglia of radius 4 at random pore voxels (seed 6403) plus the inlet
buffer.  The trapped region is found on the oracle's own unperturbed run at
T = 500 (component-1-dominated fluid voxels in clusters that do not reach the
inlet buffer, the residual non-wetting phase of Sec. 4.1) and then frozen.
Loss: smooth non-wetting saturation (mean rho1/(rho1+rho2)) over the fluid
voxels of that region after 500 steps.  Derivatives are taken with respect to
xi at 20 solid voxels that touch fluid, drawn with seed 6402, with step
eps = 1e-3; the first three are repeated with eps = 5e-4 as a cross-check of
the finite-difference error.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_adjoint64_trapped_fd.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, OracleParams, lattice_tables  # noqa: E402
from paper_2207_01534_amd import workloads as wl  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint64_trapped_fd.json")
STEPS = 500
EPS = 1e-3
EPS2 = 5e-4
GANGLIA = dict(n_blobs=12, radius=4.0, seed=6403)


def boundary_solid(solid):
    e, _, _ = lattice_tables()
    fluid = solid == 0
    touch = np.zeros_like(fluid)
    for i in range(1, 19):
        touch |= np.roll(fluid, shift=(-e[i][2], -e[i][1], -e[i][0]), axis=(0, 1, 2))
    return (solid != 0) & touch


def run(w, rho, xi64):
    o = Oracle(OracleParams(w.shape, tau=w.tau, G=w.G, g=w.g), w.solid, xi64)
    o.init_equilibrium(rho.astype(np.float32).astype(np.float64))
    o.run(STEPS)
    return o


def main():
    w = wl.workload("adjoint64")
    rho = wl.ganglia_rho(w.solid, GANGLIA["n_blobs"], GANGLIA["radius"], seed=GANGLIA["seed"])
    xi64 = w.xi.astype(np.float64)
    t0 = time.time()
    base = run(w, rho, xi64)
    region = wl.trapped_region(base.fields()[0], w.solid)
    L0 = base.loss_snw(region)
    print(f"trapped region: {int(region.sum())} voxels, L = {L0:.9f} ({time.time() - t0:.0f} s)", flush=True)
    cand = np.argwhere(boundary_solid(w.solid))
    rng = np.random.Generator(np.random.PCG64(6402))
    pick = cand[rng.choice(len(cand), size=20, replace=False)]
    rows = []
    for k, (z, y, x) in enumerate(pick):
        vals = {}
        for eps in ((EPS, EPS2) if k < 3 else (EPS,)):
            xp = xi64.copy()
            xm = xi64.copy()
            xp[z, y, x] += eps
            xm[z, y, x] -= eps
            vals[eps] = (run(w, rho, xp).loss_snw(region) - run(w, rho, xm).loss_snw(region)) / (2 * eps)
        rows.append({"zyx": [int(z), int(y), int(x)], "fd": vals[EPS], "fd_half_eps": vals.get(EPS2)})
        print(f"[{k + 1}/20] {int(z), int(y), int(x)} fd={vals[EPS]:.6e} ({time.time() - t0:.0f} s)", flush=True)
    rec = {"_source": "tests/golden/make_adjoint64_trapped_fd.py (FP64 oracle, central differences)",
           "workload": "adjoint64", "initial": {"ganglia": GANGLIA}, "steps": STEPS, "eps": EPS,
           "eps_check": EPS2, "loss": L0,
           "region": "trapped non-wetting voxels of the unperturbed oracle run at T (workloads.trapped_region)",
           "region_flat_indices": [int(v) for v in np.flatnonzero(region.reshape(-1))],
           "solid_sha256": wl.sha256(w.solid), "xi_sha256": wl.sha256(w.xi),
           "rho_sha256": wl.sha256(rho.astype(np.float32)), "voxels": rows}
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
