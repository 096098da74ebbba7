"""Drainage through a pore throat driven by the open inlet/outlet planes
(Sec. 2 inlet/outlet conditions; Sec. 4.1: the non-wetting phase does not
invade until the capillary pressure exceeds a threshold).

A non-wetting reservoir (component 1, xi = -0.2 at the walls, so the wetting
component 2 meets them at theta = 71.96 deg by the paper's cubic) faces a solid
block pierced by a square throat of side w = 8.  Young-Laplace with the
paper's surface tension gamma = 0.071 gives two thresholds:
  entry into the throat   P_entry = 4 gamma cos(theta) / w    (~0.0110)
  exit into open space    P_exit  = 2 gamma / (w / 2)         (~0.0355)
The capillary pressure P_c = P_in - P_out is read with mclbm_open_x_pressure.
Parity unpinned against the paper (its drainage runs use rock data); the
thresholds are the check.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2207_01534_amd import workloads as wl

pytestmark = pytest.mark.gpu

PAPER = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
GAMMA = PAPER["laplace_gamma"]["value"]
W_THROAT = 8
THETA = math.radians(wl.contact_angle_cubic(-0.2))
P_ENTRY = 4.0 * GAMMA * math.cos(THETA) / W_THROAT
P_EXIT = 2.0 * GAMMA / (W_THROAT / 2.0)
HI, LO = 1.05, 0.022          # coexisting bulk densities at G = 3.5


def _run(delta, steps=30000, nxp=80, n=24):
    import torch
    from paper_2207_01534_amd.lattice import Lattice, LatticeParams
    nx = nxp + 2                                         # + ghost planes
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(nx), indexing="ij")
    c = (n - 1) / 2.0
    solid = np.zeros((n, n, nx), np.uint8)
    block = (xx >= 31) & (xx < 51)
    throat = (np.abs(yy - c) < W_THROAT / 2) & (np.abs(zz - c) < W_THROAT / 2)
    solid[block & ~throat] = 1
    phi = 0.5 * (1.0 + np.tanh((27.0 - xx) / 2.5))       # reservoir up to x ~ 27
    rho = np.stack([LO + (HI - LO) * phi, LO + (HI - LO) * (1.0 - phi)]).astype(np.float32)
    xi = np.where(solid != 0, -0.2, 0.0).astype(np.float32)
    lat = Lattice(LatticeParams(shape=(nx, n, n), tau=(1.0, 1.0), G=3.5), torch.as_tensor(solid),
                  torch.as_tensor(xi), torch.as_tensor(rho))
    lat.set_open_x(HI + delta, HI)
    lat.step(steps)
    r = lat.density().cpu().numpy()
    tot = r[0] + r[1]
    oil = np.divide(r[0], tot, out=np.zeros_like(tot), where=tot > 0)   # 0 at solid voxels
    front = max(x for x in range(1, nx - 1) if oil[n // 2, n // 2, x] > 0.5)
    down = float(oil[:, :, 52:nx - 2][solid[:, :, 52:nx - 2] == 0].mean())
    pc = lat.open_x_pressure()["P_c"]
    d = lat.diagnostics()
    print(f"[drainage] delta={delta} P_c={pc:.5f} (entry {P_ENTRY:.5f}, exit {P_EXIT:.5f}) front_x={front} "
          f"downstream_oil={down:.3f} u_max={d['u_max']:.4f}", flush=True)
    return pc, front, down


def test_below_entry_pressure_the_throat_stays_closed():
    pc, front, down = _run(0.015)
    assert pc < 0.75 * P_ENTRY
    assert front <= 33 and down < 0.05


def test_between_entry_and_exit_the_throat_fills_without_breakthrough():
    pc, front, down = _run(0.06)
    assert 1.5 * P_ENTRY < pc < 0.75 * P_EXIT
    assert front >= 48 and down < 0.05


def test_above_exit_pressure_the_nonwetting_phase_breaks_through():
    pc, front, down = _run(0.15)
    assert pc > 1.3 * P_EXIT
    assert down > 0.5
