"""Cluster measures of the synthetic inputs, pinned on constructed states.
The percolating pore fraction (the share of the sample's pore space joined
to both reservoirs): a straight channel, a closed cavity, channels joined
only across the periodic y or z boundary, and voxels touching along an edge
(D3Q19 neighbours) or only at a corner (not neighbours).  The trapped
non-wetting region (component-1 clusters cut off from the inlet reservoir):
attached and free ganglia, attachment across the periodic boundary, solid
voxels and voxels without a dominant component 1."""
import numpy as np

from paper_2207_01534_amd import workloads as wl

B = 3


def _block(nx=16, ny=8, nz=6):
    s = np.ones((nz, ny, nx), np.uint8)
    s[:, :, :B] = 0
    s[:, :, nx - B:] = 0
    return s


def test_straight_channel_percolates_and_a_cavity_does_not():
    s = _block()
    s[2, 3, :] = 0                       # channel along x
    s[4, 6, 7:9] = 0                     # closed cavity of two voxels
    sample = (s[:, :, B:-B] == 0).sum()
    assert wl.percolating_fraction(s, B) == (sample - 2) / sample


def test_connections_across_the_periodic_y_and_z_boundaries():
    nx, ny, nz = 16, 8, 6
    s = _block(nx, ny, nz)
    s[2, 0, B:8] = 0                     # from the inlet to x = 7 at y = 0
    s[2, ny - 1, 9:nx - B] = 0           # from x = 9 to the outlet at y = ny - 1
    assert wl.percolating_fraction(s, B) == 0.0                 # two apart in x: not joined
    s[2, ny - 1, 8] = 0                  # an edge neighbour of (2, 0, 7) across the y wrap
    assert wl.percolating_fraction(s, B) == 1.0
    s = _block(nx, ny, nz)
    s[0, 3, B:8] = 0
    s[nz - 1, 3, 9:nx - B] = 0
    assert wl.percolating_fraction(s, B) == 0.0
    s[nz - 1, 3, 8] = 0                  # an edge neighbour of (0, 3, 7) across the z wrap
    assert wl.percolating_fraction(s, B) == 1.0


def test_edge_neighbours_connect_and_corner_neighbours_do_not():
    nx = 16
    s = _block(nx)
    s[2, 3, B:8] = 0
    s[3, 4, 8:nx - B] = 0                # (2, 3, 7) -> (3, 4, 8) differs in x, y and z: a corner only
    assert wl.percolating_fraction(s, B) == 0.0
    s[3, 3, 8] = 0                       # (2, 3, 7) -> (3, 3, 8): an edge, and (3, 3, 8) -> (3, 4, 8): a face
    assert wl.percolating_fraction(s, B) == 1.0


def _two_phase(nx=16, ny=8, nz=6):
    """All fluid, component 2 everywhere except the inlet buffer (component 1)."""
    rho = np.zeros((2, nz, ny, nx))
    rho[0], rho[1] = 0.03, 1.0
    rho[0][:, :, :B], rho[1][:, :, :B] = 1.0, 0.03
    return rho


def _oil(rho, z, y, xs):
    rho[0][z, y, xs], rho[1][z, y, xs] = 1.0, 0.03


def test_trapped_region_holds_the_disconnected_non_wetting_clusters():
    nx, ny, nz = 16, 8, 6
    solid = np.zeros((nz, ny, nx), np.uint8)
    rho = _two_phase(nx, ny, nz)
    _oil(rho, 2, 3, slice(B, 6))               # attached to the inlet reservoir
    _oil(rho, 4, 5, slice(9, 11))              # a free ganglion of two voxels
    _oil(rho, 1, 0, slice(B, 8))               # attached, reaching x = 7 at y = 0
    _oil(rho, 1, ny - 1, 8)                    # edge neighbour of (1, 0, 7) across the y wrap: attached
    _oil(rho, 1, ny - 1, slice(11, 13))        # two apart from it in x: free
    region = wl.trapped_region(rho, solid, B)
    expect = np.zeros((nz, ny, nx), np.uint8)
    expect[4, 5, 9:11] = 1
    expect[1, ny - 1, 11:13] = 1
    np.testing.assert_array_equal(region, expect)


def test_trapped_region_excludes_solid_and_follows_the_dominant_component():
    nx, ny, nz = 16, 8, 6
    solid = np.zeros((nz, ny, nx), np.uint8)
    rho = _two_phase(nx, ny, nz)
    _oil(rho, 3, 3, slice(8, 11))
    solid[3, 3, 10] = 1                        # a solid voxel inside the ganglion
    rho[:, 3, 3, 10] = 0.0
    rho[0][3, 3, 9], rho[1][3, 3, 9] = 0.5, 0.5   # equal densities: not non-wetting
    region = wl.trapped_region(rho, solid, B)
    expect = np.zeros((nz, ny, nx), np.uint8)
    expect[3, 3, 8] = 1
    np.testing.assert_array_equal(region, expect)
