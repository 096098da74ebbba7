"""Pins of the oracle's diagnostics on constructed states whose values are
known by construction: the component masses, the water saturation S_w of
Sec. 4.1 (the fraction of fluid nodes occupied by water, component 2, with
ties counted as oil), the smooth non-wetting fraction, the largest fluid
speed and the count of non-finite population values.  With G = 0 and no body
force the velocity of Eq. (8) is the plain barycentric velocity, so a state
built from Eq. (2) equilibria carries exactly the velocities it was built
with.  A diagnostics routine that swapped the components, counted ties as
water, counted solid nodes, took the largest speed over solid nodes or
missed a population in the non-finite count fails one of these."""
import numpy as np
import pytest

from oracle.oracle import Oracle, OracleParams, equilibrium

SHAPE = (9, 7, 5)          # nx, ny, nz
DIMS = SHAPE[::-1]
N = int(np.prod(SHAPE))


def _oracle(solid):
    return Oracle(OracleParams(SHAPE, tau=(1.0, 1.0), G=0.0), solid)


def _state(r1, r2, u=None):
    """Populations (2, 19, nz, ny, nx): Eq. (2) equilibria of the given
    densities at velocity u (3, nz, ny, nx), zero if omitted."""
    f = np.zeros((2, 19) + DIMS)
    if u is None:
        u = np.zeros((3,) + DIMS)
    for z, y, x in np.ndindex(*DIMS):
        uu = u[:, z, y, x]
        f[0, :, z, y, x] = equilibrium(r1[z, y, x], uu)
        f[1, :, z, y, x] = equilibrium(r2[z, y, x], uu)
    return f


def _labelled_nodes(seed):
    """Solid mask and three kinds of fluid node: water (rho2 > rho1), oil
    (rho1 > rho2) and ties (rho1 == rho2 exactly)."""
    rng = np.random.default_rng(seed)
    solid = (rng.random(DIMS) < 0.25).astype(np.uint8)
    kind = rng.integers(0, 3, DIMS)             # 0 water, 1 oil, 2 tie
    r1 = np.where(kind == 0, 0.04, np.where(kind == 1, 0.97, 0.5))
    r2 = np.where(kind == 0, 0.99, np.where(kind == 1, 0.05, 0.5))
    # solid nodes hold component-2-rich populations that must not count
    r1 = np.where(solid != 0, 0.01, r1)
    r2 = np.where(solid != 0, 0.9, r2)
    return solid, kind, r1, r2


def test_masses_and_water_saturation_with_ties():
    solid, kind, r1, r2 = _labelled_nodes(11)
    o = _oracle(solid)
    o.set_state(_state(r1, r2))
    m1, m2, sw, snw, umax, bad = o.diagnostics()
    fl = solid == 0
    n_fluid = int(fl.sum())
    n_water = int((fl & (kind == 0)).sum())
    n_oil = int((fl & (kind == 1)).sum())
    n_tie = int((fl & (kind == 2)).sum())
    assert min(n_water, n_oil, n_tie) >= 20 and int(solid.sum()) >= 20
    assert m1 == pytest.approx(0.04 * n_water + 0.97 * n_oil + 0.5 * n_tie, rel=1e-14)
    assert m2 == pytest.approx(0.99 * n_water + 0.05 * n_oil + 0.5 * n_tie, rel=1e-14)
    # ties count as oil: only the water nodes are occupied by water
    assert sw == n_water / n_fluid
    expect_snw = (n_water * 0.04 / 1.03 + n_oil * 0.97 / 1.02 + n_tie * 0.5) / n_fluid
    assert snw == pytest.approx(expect_snw, abs=1e-14)
    assert umax == pytest.approx(0.0, abs=1e-15)
    assert bad == 0.0


def test_largest_speed_is_over_fluid_nodes_only():
    solid, _, r1, r2 = _labelled_nodes(12)
    rng = np.random.default_rng(13)
    u = rng.uniform(-0.02, 0.02, (3,) + DIMS)
    fl = np.argwhere(solid == 0)
    z, y, x = fl[len(fl) // 2]
    u[:, z, y, x] = (0.03, -0.06, 0.06)         # speed 0.09, the fluid maximum
    sz, sy, sx = np.argwhere(solid != 0)[0]
    u[:, sz, sy, sx] = (0.2, 0.0, 0.0)          # faster, but at a solid node
    o = _oracle(solid)
    o.set_state(_state(r1, r2, u))
    umax = o.diagnostics()[4]
    assert umax == pytest.approx(0.09, rel=1e-13)
    _, _, _, u_o = o.fields()
    assert np.allclose(u_o[:, solid == 0], u[:, solid == 0], atol=1e-15)


def test_non_finite_populations_are_counted_at_fluid_nodes():
    solid, _, r1, r2 = _labelled_nodes(14)
    f = _state(r1, r2)
    fl = np.argwhere(solid == 0)
    planted = 0
    rng = np.random.default_rng(15)
    for k, (z, y, x) in enumerate(fl[rng.choice(len(fl), 6, replace=False)]):
        s, i = k % 2, (7 * k) % 19                # both components, rest population included
        f[s, i, z, y, x] = (np.nan, np.inf, -np.inf)[k % 3]
        planted += 1
    z, y, x = fl[0]
    f[0, 3, z, y, x] = np.nan
    f[1, 3, z, y, x] = np.nan                     # two values at one node count twice
    planted += 2
    for z, y, x in np.argwhere(solid != 0)[:3]:
        f[0, 5, z, y, x] = np.nan                 # solid nodes are not counted
    o = _oracle(solid)
    o.set_state(f)
    assert o.diagnostics()[5] == planted
