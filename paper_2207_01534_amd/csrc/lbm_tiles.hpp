// Tile geometry shared by the tile-sparse kernels of the step and of its
// adjoint: the lattice is cut into tiles of 64 x 4 x 2 nodes; only tiles
// holding fluid are launched, one block of 256 threads each, and a tile's
// fluid nodes are compacted (fluid ids tile base + rank, x fastest inside the
// tile except that the nodes of the three planes at each x end come first).
#pragma once

#include "lbm_device.hpp"

namespace mclbm {

constexpr int TX = 64, TY = 4, TZ = 2;
constexpr int TN = TX * TY * TZ;   // nodes per tile
constexpr int NT = 256;            // threads per block of the tile kernels
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;

// Tile numbering: slabs of SZ tiles in z, one after the other; inside a slab
// z is fastest, then x, then y.  A tile's z neighbours are then the adjacent
// tile numbers, its x neighbours SZ apart and its y neighbours SZ * ntx apart,
// so blocks running at the same time on one XCD share the face cache lines
// that the neighbour gathers of the odd steps and the psi-hat halo touch (with
// x fastest and z slowest the z neighbour, which shares half of a 2-deep
// tile, was ntx * nty tiles away).  The last slab may be shallower.
constexpr int SZ = 4;

__device__ __forceinline__ void tile_origin(int t, const Geo& g, int& x0, int& y0, int& z0) {
    const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + TZ - 1) / TZ;
    const int per_slab = SZ * ntx * nty;
    const int s = t / per_slab, w = t - s * per_slab;
    const int h = min(SZ, ntz - s * SZ);   // depth of this slab in tiles
    const int r = w / h;
    z0 = (s * SZ + (w - r * h)) * TZ;
    x0 = (r % ntx) * TX;
    y0 = (r / ntx) * TY;
}

// Blocks are numbered on a 1D grid (a multiple of 8 blocks) and mapped
// XCD-aware: the hardware deals consecutive block ids round-robin to the 8
// XCDs, so block b takes active tile (b mod 8) * per + b / 8 and each XCD
// works through a contiguous run of neighbouring tiles, whose shared halo
// rows then hit in that XCD's L2.  Returns -1 past the last active tile.
__device__ __forceinline__ int active_of_block(int nactive) {
    const int per = gridDim.x >> 3;
    const int a = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    return a < nactive ? a : -1;
}

// Position of a fluid node inside its tile.
struct TilePos {
    int lx, ly, lz;
    __device__ __forceinline__ explicit TilePos(int p) : lx(p & (TX - 1)), ly((p / TX) & (TY - 1)), lz(p / (TX * TY)) {}
};

inline unsigned xcd_grid(int nblocks) { return (unsigned)(((nblocks + 7) / 8) * 8); }

}  // namespace mclbm
