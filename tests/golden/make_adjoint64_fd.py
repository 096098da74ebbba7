"""Write tests/golden/adjoint64_fd.json: central finite differences of the FP64
oracle for the wettability gradient on the 64^3 adjoint workload.

Loss: smooth non-wetting saturation (mean rho1/(rho1+rho2)) over the fluid
voxels of the sample region (x in [3, nx-3)) after 500 steps, starting from
the equilibrium of the workload's initial densities.  Derivatives are taken
with respect to xi at 20 solid voxels that touch fluid, drawn with seed 6402,
with step eps = 1e-3; the first five are repeated with eps = 5e-4 as a
cross-check of the finite-difference error.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_adjoint64_fd.py
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint64_fd.json")
STEPS = 500
EPS = 1e-3
EPS2 = 5e-4


def sample_region(shape, buffer=3):
    nx, ny, nz = shape
    region = np.zeros((nz, ny, nx), np.uint8)
    region[:, :, buffer:nx - buffer] = 1
    return region


def boundary_solid(solid):
    e, _, _ = lattice_tables()
    fluid = solid == 0
    touch = np.zeros_like(fluid)
    for i in range(1, 19):
        touch |= np.roll(fluid, shift=(-e[i][2], -e[i][1], -e[i][0]), axis=(0, 1, 2))
    return (solid != 0) & touch


def loss(w, xi64, region):
    o = Oracle(OracleParams(w.shape, tau=w.tau, G=w.G, g=w.g), w.solid, xi64)
    o.init_equilibrium(w.rho.astype(np.float32).astype(np.float64))
    o.run(STEPS)
    return o.loss_snw(region)


def main():
    w = wl.workload("adjoint64")
    region = sample_region(w.shape)
    xi64 = w.xi.astype(np.float64)
    cand = np.argwhere(boundary_solid(w.solid))
    rng = np.random.Generator(np.random.PCG64(6402))
    pick = cand[rng.choice(len(cand), size=20, replace=False)]
    t0 = time.time()
    L0 = loss(w, xi64, region)
    rows = []
    for k, (z, y, x) in enumerate(pick):
        vals = {}
        for eps in ((EPS, EPS2) if k < 5 else (EPS,)):
            xp = xi64.copy()
            xm = xi64.copy()
            xp[z, y, x] += eps
            xm[z, y, x] -= eps
            vals[eps] = (loss(w, xp, region) - loss(w, xm, region)) / (2 * eps)
        rows.append({"zyx": [int(z), int(y), int(x)], "fd": vals[EPS], "fd_half_eps": vals.get(EPS2)})
        print(f"[{k + 1}/20] {int(z), int(y), int(x)} fd={vals[EPS]:.6e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    rec = {"_source": "tests/golden/make_adjoint64_fd.py (FP64 oracle, central differences)",
           "workload": "adjoint64", "steps": STEPS, "eps": EPS, "eps_check": EPS2, "loss": L0,
           "region": "fluid voxels with 3 <= x < nx-3",
           "solid_sha256": wl.sha256(w.solid), "xi_sha256": wl.sha256(w.xi), "voxels": rows}
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
