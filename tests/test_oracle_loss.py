"""Pins of the oracle's smooth non-wetting saturation, the loss whose
gradient the adjoint computes: over the fluid nodes of a region, the mean of
rho1 / (rho1 + rho2) with each component density the sum of all 19 of its
populations (Eq. 3).  The states below have saturations known by
construction, and place each component's mass in chosen directions, so that
a loss that skipped the rest population or a direction, swapped the
components, counted solid nodes or ignored the region would miss them."""
import numpy as np
import pytest

from oracle.oracle import Oracle, OracleParams

SHAPE = (9, 7, 5)          # nx, ny, nz
DIMS = SHAPE[::-1]


def _oracle(solid):
    return Oracle(OracleParams(SHAPE, tau=(1.0, 1.0), G=0.0), solid)


def test_uniform_state_gives_the_component_fraction():
    solid = np.zeros(DIMS, np.uint8)
    o = _oracle(solid)
    a, b = 0.83, 0.07
    rho = np.stack([np.full(DIMS, a), np.full(DIMS, b)])
    o.init_equilibrium(rho)
    region = np.ones(DIMS, np.uint8)
    assert o.loss_snw(region) == pytest.approx(a / (a + b), abs=1e-14)


def test_region_and_solid_nodes_select_the_average():
    """Two kinds of fluid node: component-1 rich (fraction p) and component-2
    rich (fraction q).  Only fluid nodes inside the region count, each with
    the same weight."""
    rng = np.random.default_rng(3)
    solid = (rng.random(DIMS) < 0.3).astype(np.uint8)
    region = (rng.random(DIMS) < 0.6).astype(np.uint8)
    kind = rng.random(DIMS) < 0.5
    r1 = np.where(kind, 0.95, 0.04)
    r2 = np.where(kind, 0.05, 0.96)
    rho = np.stack([r1, r2])
    rho[:, solid != 0] = 0.0
    o = _oracle(solid)
    o.init_equilibrium(rho)
    sel = (solid == 0) & (region != 0)
    n_rich, n_poor = int((sel & kind).sum()), int((sel & ~kind).sum())
    p, q = 0.95 / (0.95 + 0.05), 0.04 / (0.04 + 0.96)
    expect = (n_rich * p + n_poor * q) / (n_rich + n_poor)
    assert n_rich > 10 and n_poor > 10
    assert o.loss_snw(region) == pytest.approx(expect, abs=1e-14)
    assert o.loss_snw(np.zeros(DIMS, np.uint8)) == 0.0          # empty region
    only_solid = (solid != 0).astype(np.uint8)
    assert o.loss_snw(only_solid) == 0.0                         # no fluid node in it


@pytest.mark.parametrize("d1", [0, 1, 6, 18])
def test_every_direction_counts_towards_the_density(d1):
    """Component 1's mass sits in one population (direction d1, the rest
    population included), component 2's is spread over the other eighteen;
    with masses m1 = 1 and m2 = 3 the fraction is 1/4 at every node."""
    solid = np.zeros(DIMS, np.uint8)
    o = _oracle(solid)
    f = np.zeros((2, 19) + DIMS)
    f[0, d1] = 1.0
    others = [i for i in range(19) if i != d1]
    f[1, others] = 3.0 / len(others)
    o.set_state(f)
    region = np.ones(DIMS, np.uint8)
    assert o.loss_snw(region) == pytest.approx(0.25, abs=1e-14)
