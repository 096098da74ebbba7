// Host-side launchers of the step kernels (implemented in lbm_kernels.hip).
#pragma once

#include "lbm_tiles.hpp"

namespace mclbm {

// Tile-sparse index structures (built once per geometry).
struct Sparse {
    const int* active;   // ids of the tiles that hold fluid, in tile order
    const int* base;     // per tile: fluid id of its first fluid node
    const int* count;    // per tile: number of fluid nodes
    const uint16_t* loc; // per fluid node: position inside its tile (x + 64 (y + 4 z))
    const uint32_t* nbf; // per fluid node: its neighbourhood word (the F16/BF16 codecs' wall bits)
    const int* fid;      // per lattice node: fluid id, -1 at solid
    int nactive;
};

void launch_store_words(uint64_t* dst, const uint64_t (&w)[4], hipStream_t s);
void launch_neighbour_bits(const uint8_t* solid, uint32_t* nbm, const Geo& g, hipStream_t s);
int boundary_blocks(const Geo& g);
// Boundary solids (solid nodes with a fluid neighbour) in tile order: their
// lattice indices (list), adhesion values (xil) and neighbourhood words (nbl).
void launch_boundary_list(const uint32_t* nbm, const float* xi, int* counts, int* total, int* list,
                          float* xil, uint32_t* nbl, const Geo& g, hipStream_t s);
// Checks a candidate geometry (neighbour words nbm, adhesion xi) without
// changing anything else: out[0] <- boundary solids with |xi| not < 1,
// out[1] <- fluid nodes, out[2] <- order-independent fingerprint of the
// solid mask.  Stream-ordered; out is cleared first.
void launch_geometry_check(const uint32_t* nbm, const float* xi, const Geo& g, unsigned long long* out,
                           hipStream_t s);
int tile_count(const Geo& g);
// Per-tile fluid counts and their scans: totals[0] <- number of fluid nodes,
// totals[1] <- number of tiles holding fluid.
void launch_tile_census(const uint32_t* nbm, const Geo& g, int* cnt, int* base, int* apos, int* totals,
                        hipStream_t s);
// Fluid ids, in-tile positions, neighbourhood words by fluid id and the
// active tile list; loc and nbf must hold totals[0] entries.
void launch_tile_ids(const uint32_t* nbm, const Geo& g, const int* cnt, const int* base, const int* apos, int* fid,
                     uint16_t* loc, uint32_t* nbf, int* active, hipStream_t s);

// Initial state from the densities rho [2][n].  rprev receives the
// pseudopotential field of the level before the first (the initial densities
// at fluid nodes, their virtual densities, Eqs. 14-15, at the boundary solids
// in list/xil), from which the F16/BF16 codec predictors of the stored
// values are taken.  G: the cohesion parameter (codec predictors).
template <class C>
void launch_init(const Pops<C>& P, const uint32_t* nbm, const int* fid, const float* rho, float2* rprev,
                 const int* list, const float* xil, const uint32_t* nbl, int nbound, const Geo& g, float G,
                 hipStream_t s);
template <class C>
void launch_density(const Pops<C>& P, const Sparse& S, const float2* rprev, float2* psi, const Geo& g, float G,
                    int odd, hipStream_t s);
void launch_ivsd(const int* list, const float* xil, const uint32_t* nbl, int count, float2* psi, const Geo& g,
                 hipStream_t s);
template <class C>
void launch_collide_stream(const Pops<C>& P, const Pops<C>& D, const Sparse& S, const float2* rprev,
                           const float2* psi, const Geo& g, const Phys& ph, int odd, hipStream_t s);
int fields_blocks(const Geo& g);
// Readouts and the diagnostics reduction.  max_blocks > 0 caps the grid (each
// block then sums several 64 x 4 patches), which bounds the partials to
// 8 * max_blocks doubles; 0 = one block per patch (fields_blocks).
template <class C>
void launch_fields(const Pops<C>& P, const int* fid, const uint32_t* nbm, const float2* rprev, const float2* psi,
                   const Geo& g, const Phys& ph, int odd, float* o_rho, float* o_u, float* o_F, float* o_P,
                   double* partial, double* out, int skip_ghost_x, hipStream_t s, int max_blocks = 0);

// Device scratch of the library itself (lbm_kernels.hip), for entry points
// that allocate nothing: kScratchBlocks blocks of 8 partials, then 8 result
// words.  scratch_address returns its address on `device`, which must be the
// current device; the first call per device looks the symbol up.
constexpr int kScratchBlocks = 4096;
constexpr int kScratchDoubles = 8 * kScratchBlocks + 8;
constexpr int kMaxDevices = 64;
hipError_t scratch_address(int device, double** out);

}  // namespace mclbm
