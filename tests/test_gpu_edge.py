"""Degenerate cases of the step on the HIP path against the FP64 oracle
(Eqs. 1-15): lattices thinner than a tile along every axis (extent 3, where
the periodic neighbours x - 1 and x + 2 coincide), a lattice without fluid,
fluid voxels cut off from every neighbour, zero steps, and all storage forms
on a lattice smaller than one tile."""
import numpy as np
import pytest

from paper_2207_01534_amd import workloads as wl

from parity_util import field_errors, gpu_case, gpu_fields, oracle_case, oracle_fields

pytestmark = pytest.mark.gpu

TAU, G = (1.5, 0.6), 3.5
BODY = ((2e-4, -1e-4, 0.0), (0.0, 0.0, 3e-4))


def _porous(shape, seed):
    solid = wl.random_mask(shape, 0.3, seed=seed)
    xi = wl.uniform_xi(solid, -0.4, 0.4, seed=seed + 1)
    rho = wl.tanh_droplet(shape, max(min(shape) / 3.0, 1.0))
    rho[:, solid != 0] = 0
    return solid, xi, rho


# (64, 4, 3) and (70, 5, 3): lattices just large enough for halos loaded
# straight into LDS (every halo position inside the lattice after one wrap),
# at the tile's x and y extents and ragged; the others take the
# register-staged halos
@pytest.mark.parametrize("shape", [(3, 3, 3), (3, 5, 4), (130, 3, 3), (4, 3, 70), (64, 4, 3), (70, 5, 3)])
def test_thin_extents_against_oracle(shape):
    solid, xi, rho = _porous(shape, seed=sum(shape) * 7 + shape[0])
    print(f"[case] thin {shape} fluid={int((solid == 0).sum())}", flush=True)
    lat = gpu_case(shape, solid, xi, rho, TAU, G, BODY)
    orc = oracle_case(shape, solid, xi, rho, TAU, G, BODY)
    lat.step(25)
    orc.run(25)
    e = field_errors(gpu_fields(lat), oracle_fields(orc), solid)
    print(f"[errors] thin {shape} {e}", flush=True)
    assert e["e_rho"] < 1e-5 and e["e_u"] < 1e-4 and e["e_F"] < 1e-4, e


def test_lattice_without_fluid():
    import torch
    shape = (20, 6, 5)
    solid = np.ones(shape[::-1], np.uint8)
    xi = np.full(shape[::-1], 0.1, np.float32)
    rho = np.zeros((2,) + shape[::-1], np.float32)
    lat = gpu_case(shape, solid, xi, rho, TAU, G, BODY)
    assert lat.fluid_count() == 0 and lat.boundary_count() == 0
    lat.step(3)
    assert lat.time == 3
    d = lat.diagnostics()
    assert d["n_fluid"] == 0 and d["mass1"] == 0 and d["mass2"] == 0 and d["nonfinite"] == 0
    torch.cuda.synchronize()
    assert float(lat.density().abs().max()) == 0.0
    assert float(lat.velocity().abs().max()) == 0.0


def test_isolated_fluid_voxels_keep_their_state():
    """A fluid voxel whose 18 neighbours are all solid only bounces its
    populations back, so its densities never change.  With xi = 0 every
    solid neighbour carries the voxel's own densities as virtual densities
    (Eqs. 14-15 with a single fluid neighbour), the interaction force sums to
    zero by the symmetry of the weights, and with no body force the voxel
    stays at rest."""
    shape = (12, 9, 8)
    nz, ny, nx = shape[::-1]
    solid = np.ones((nz, ny, nx), np.uint8)
    cells = [(2, 2, 2), (5, 6, 9), (7, 4, 5)]
    for z, y, x in cells:
        solid[z, y, x] = 0
    xi = np.zeros((nz, ny, nx), np.float32)
    rho = np.zeros((2, nz, ny, nx), np.float32)
    for k, (z, y, x) in enumerate(cells):
        rho[:, z, y, x] = (0.9 - 0.2 * k, 0.05 + 0.1 * k)
    none = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    lat = gpu_case(shape, solid, xi, rho, TAU, G, none)
    orc = oracle_case(shape, solid, xi, rho, TAU, G, none)
    lat.step(9)
    orc.run(9)
    r, u, F, P = gpu_fields(lat)
    ro, uo, Fo, Po = oracle_fields(orc)
    for z, y, x in cells:
        np.testing.assert_allclose(r[:, z, y, x], rho[:, z, y, x], rtol=2e-6)
        np.testing.assert_allclose(r[:, z, y, x], ro[:, z, y, x], rtol=2e-6)
        assert np.abs(u[:, z, y, x]).max() < 1e-7
    assert lat.boundary_count() == 18 * len(cells)   # the neighbourhoods do not overlap


def test_zero_steps_is_a_no_op():
    import torch
    shape = (19, 13, 11)
    solid, xi, rho = _porous(shape, seed=99)
    lat = gpu_case(shape, solid, xi, rho, TAU, G, BODY)
    lat.step(2)
    a = lat.density().clone()
    lat.step(0)
    assert lat.time == 2
    torch.cuda.synchronize()
    assert torch.equal(a, lat.density())


@pytest.mark.parametrize("storage,bar", [(0, 1e-5), (1, 2e-3), (2, 2e-2)], ids=["f32", "f16", "bf16"])
def test_storage_forms_on_a_lattice_smaller_than_a_tile(storage, bar):
    shape = (5, 3, 4)
    solid, xi, rho = _porous(shape, seed=541)
    lat = gpu_case(shape, solid, xi, rho, TAU, G, BODY, storage=storage)
    orc = oracle_case(shape, solid, xi, rho, TAU, G, BODY)
    lat.step(20)
    orc.run(20)
    e = field_errors(gpu_fields(lat), oracle_fields(orc), solid)
    print(f"[errors] tiny storage={storage} {e}", flush=True)
    assert e["e_rho"] < bar, e
