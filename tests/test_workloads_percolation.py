"""The percolating pore fraction of the synthetic media (the share of the
sample's pore space joined to both reservoirs), pinned on constructed
geometries: a straight channel, a closed cavity, a channel that connects only
across the periodic y boundary, and channels whose voxels touch along an
edge (D3Q19 neighbours) or only at a corner (not neighbours)."""
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
