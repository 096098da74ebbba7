// HIP kernels of the two-component D3Q19 pseudopotential step (gfx950).
//
// Populations are stored only for fluid nodes, compacted within tiles of
// 64 x 4 x 2 nodes; tiles without fluid are dropped (the paper's sparse
// tiling, Sec. 5, with node compaction inside each tile).  One time
// step is three launches on the caller's stream:
//   k_density        rho^(sigma) at every fluid node from the incoming
//                    populations (Eq. 3), written to the dense psi-hat field.
//   k_ivsd           virtual solid densities at the solid nodes that touch
//                    fluid (Eqs. 14-15), over a compact list; together with
//                    k_density this fills the unified pseudopotential psi-hat.
//   k_collide_stream per fluid node: forces from an LDS-staged psi-hat halo
//                    (Eqs. 10, 11, 13), common velocity and mixture
//                    relaxation time (Eqs. 6-8), forced SRT collision
//                    (Eqs. 1, 2, 9), then in-place AA-pattern streaming with
//                    halfway bounce-back.
// Readouts and diagnostics reuse k_density + k_ivsd and then k_fields.
#include "lbm_kernels.hpp"

#include <mutex>

namespace mclbm {

// ---------------------------------------------------------------------------
// Geometry set-up
// ---------------------------------------------------------------------------
__global__ void k_neighbour_bits(const uint8_t* __restrict__ solid, uint32_t* __restrict__ nbm,
                                 Geo g) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx) return;
    const Nb nb(x, y, z, g);
    uint32_t m = solid[nb.idx] ? SELF_SOLID : 0u;
#pragma unroll
    for (int i = 1; i < Q; ++i)
        if (solid[nb.at(i, +1)]) m |= (1u << i);
    nbm[nb.idx] = m;
}

// A boundary solid node: solid with at least one fluid neighbour.
__device__ __forceinline__ bool is_boundary_solid(uint32_t m) {
    return (m & SELF_SOLID) && ((~m) & NB_BITS);
}

// The list of boundary solids is built tile by tile (one block of 64 x 4 x 2
// threads per tile, every tile of the lattice, in the tiles' numbering), so
// that consecutive list entries are close in all three directions and the
// IVSD gathers of a run of entries hit the same psi-hat lines.
__global__ void k_boundary_count(const uint32_t* __restrict__ nbm, Geo g, int* __restrict__ counts) {
    int x0, y0, z0;
    tile_origin(blockIdx.x, g, x0, y0, z0);
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y, z = z0 + threadIdx.z;
    const bool flag = x < g.nx && y < g.ny && z < g.nz && is_boundary_solid(nbm[x + g.nx * (y + g.ny * z)]);
    const int c = __syncthreads_count(flag);
    if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) counts[blockIdx.x] = c;
}

// Exclusive scan of an int array in place by one block (set-up only); the
// total goes to total[0].
__global__ void k_scan(int* __restrict__ counts, int nblocks, int* __restrict__ total) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int per = (nblocks + 1023) / 1024;
    const int b0 = t * per;
    const int b1 = min(b0 + per, nblocks);
    int s = 0;
    for (int b = b0; b < b1; ++b) s += counts[b];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = t > 0 ? part[t - 1] : 0;
    for (int b = b0; b < b1; ++b) {
        const int c = counts[b];
        counts[b] = run;
        run += c;
    }
    if (t == 1023) total[0] = part[1023];
}

// Rank of this thread's flag among the flagged threads of its block
// (ordered by linear thread id); the block's flagged count goes to *count.
__device__ __forceinline__ int block_rank(bool flag, int* wave_off, int* count) {
    const unsigned long long ball = __ballot(flag);
    const int tid = (threadIdx.z * blockDim.y + threadIdx.y) * blockDim.x + threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int rank = __popcll(ball & ((1ull << lane) - 1ull));
    if (lane == 0) wave_off[wave] = __popcll(ball);
    __syncthreads();
    int base = 0, all = 0;
    const int nw = (int)(blockDim.x * blockDim.y * blockDim.z) >> 6;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) base += wave_off[w];
        all += wave_off[w];
    }
    *count = all;
    return base + rank;
}

__global__ void k_boundary_write(const uint32_t* __restrict__ nbm, const float* __restrict__ xi,
                                 Geo g, const int* __restrict__ offsets, int* __restrict__ list,
                                 float* __restrict__ xil, uint32_t* __restrict__ nbl) {
    __shared__ int wave_off[TN / 64];
    int x0, y0, z0;
    tile_origin(blockIdx.x, g, x0, y0, z0);
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y, z = z0 + threadIdx.z;
    const int idx = x + g.nx * (y + g.ny * z);
    const bool flag = x < g.nx && y < g.ny && z < g.nz && is_boundary_solid(nbm[idx]);
    int cnt;
    const int rank = block_rank(flag, wave_off, &cnt);
    if (flag) {
        const int at = offsets[blockIdx.x] + rank;
        list[at] = idx;
        xil[at] = xi[idx];
        nbl[at] = nbm[idx];
    }
}

// 64-bit finaliser of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): a
// bijective mixing of a node index, summed over the solid nodes to
// fingerprint a solid mask.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Validation of a candidate geometry before anything is committed:
// out[0] += boundary solids whose |xi| is not < 1, out[1] += fluid nodes,
// out[2] += sum of mix64(idx) over solid nodes (integer sums, so the result
// does not depend on the order of the blocks).  One thread per node.
__global__ __launch_bounds__(256) void k_geometry_check(const uint32_t* __restrict__ nbm,
                                                        const float* __restrict__ xi, Geo g,
                                                        unsigned long long* __restrict__ out) {
    __shared__ unsigned long long part[4];
    const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
    bool bad = false, fluid = false;
    unsigned long long h = 0;
    if (idx < (uint32_t)g.n) {
        const uint32_t m = nbm[idx];
        fluid = !(m & SELF_SOLID);
        if (is_boundary_solid(m)) bad = !(fabsf(xi[idx]) < 1.0f);
        if (!fluid) h = mix64(idx);
    }
    const int nbad = __syncthreads_count(bad);
    const int nfluid = __syncthreads_count(fluid);
    for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = h;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (nbad) atomicAdd(out, (unsigned long long)nbad);
        if (nfluid) atomicAdd(out + 1, (unsigned long long)nfluid);
        atomicAdd(out + 2, part[0] + part[1] + part[2] + part[3]);
    }
}

// Per tile: number of fluid nodes (into cnt and, for the scans, into base
// and active_flag).  Block = (64, 4, 2), one thread per tile node.
__global__ void k_tile_count(const uint32_t* __restrict__ nbm, Geo g, int* __restrict__ cnt,
                             int* __restrict__ base, int* __restrict__ active_flag) {
    int x0, y0, z0;
    tile_origin(blockIdx.x, g, x0, y0, z0);
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y, z = z0 + threadIdx.z;
    const bool fluid = x < g.nx && y < g.ny && z < g.nz && !(nbm[x + g.nx * (y + g.ny * z)] & SELF_SOLID);
    const int c = __syncthreads_count(fluid);
    if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) {
        cnt[blockIdx.x] = c;
        base[blockIdx.x] = c;
        active_flag[blockIdx.x] = c > 0 ? 1 : 0;
    }
}

// Fluid ids (tile base + rank inside the tile), the dense id map (-1 at
// solid) and each fluid node's position inside its tile.  Ranks run x
// fastest, except that the nodes on the planes x = 0, 1, 2 and nx-3, nx-2,
// nx-1 (the ghost, boundary and next planes when x is opened) come first, in
// (z, y, x) order: the open-plane rebuild then finds the three nodes of each
// of a tile's rows in consecutive slots, and a tile's rows one after the
// other, instead of one short run per row.
__global__ void k_tile_ids(const uint32_t* __restrict__ nbm, Geo g, const int* __restrict__ base,
                           const int* __restrict__ cnt, const int* __restrict__ active_pos,
                           int* __restrict__ fid, uint16_t* __restrict__ loc, uint32_t* __restrict__ nbf,
                           int* __restrict__ active) {
    __shared__ int wave_off[TN / 64];
    int x0, y0, z0;
    tile_origin(blockIdx.x, g, x0, y0, z0);
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y, z = z0 + threadIdx.z;
    const bool inside = x < g.nx && y < g.ny && z < g.nz;
    const int idx = x + g.nx * (y + g.ny * z);
    const bool fluid = inside && !(nbm[idx] & SELF_SOLID);
    const bool edge = x < 3 || x >= g.nx - 3;
    int c_edge, c;
    const int rank_edge = block_rank(fluid && edge, wave_off, &c_edge);
    __syncthreads();   // wave_off is reused
    const int rank_rest = block_rank(fluid && !edge, wave_off, &c);
    const int rank = edge ? rank_edge : c_edge + rank_rest;
    if (inside) fid[idx] = fluid ? base[blockIdx.x] + rank : -1;
    if (fluid) {
        loc[base[blockIdx.x] + rank] = (uint16_t)(threadIdx.x + TX * (threadIdx.y + TY * threadIdx.z));
        nbf[base[blockIdx.x] + rank] = nbm[idx];
    }
    if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0 && cnt[blockIdx.x] > 0)
        active[active_pos[blockIdx.x]] = blockIdx.x;
}

// ---------------------------------------------------------------------------
// Initial state f_i = w_i rho (fluid at rest), even-parity layout.  The
// values are recorded as written at a level before the first, whose
// pseudopotential field (the codec predictors' field of the F16/BF16 forms)
// is rprev: the initial densities at fluid nodes (k_init_ref, zero at solid
// ones), then the virtual densities at the boundary solids (k_ivsd).
// ---------------------------------------------------------------------------
__global__ void k_init_ref(const uint32_t* __restrict__ nbm, const float* __restrict__ rho_in,
                           float2* __restrict__ rprev, Geo g) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx) return;
    const uint32_t self = (uint32_t)(x + g.nx * (y + g.ny * z));
    rprev[self] = (nbm[self] & SELF_SOLID) ? make_float2(0.f, 0.f)
                                           : make_float2(rho_in[self], rho_in[(size_t)g.n + self]);
}

template <class C>
__global__ void k_init(Pops<C> P, const uint32_t* __restrict__ nbm, const int* __restrict__ fid,
                       const float2* __restrict__ rprev, Geo g, float G) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx) return;
    const Nb nb(x, y, z, g);
    const uint32_t self = nb.idx;
    const uint32_t m = nbm[self];
    if (m & SELF_SOLID) return;
    const uint32_t k = (uint32_t)fid[self];
    const float2 r = rprev[self];
    auto psi_rel = [&](int dx, int dy, int dz) {
        return ld(rprev, self + (uint32_t)(nb.ox[1 + dx] + nb.oy[1 + dy] + nb.oz[1 + dz]));
    };
    float sum0 = 0.f, sum1 = 0.f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const float f0 = weight(i) * r.x, f1 = weight(i) * r.y;
        PredRef q{make_float2(0.f, 0.f), 0.f};
        float inv_t = 0.f;
        if constexpr (C::kRef) {
            // predictor of the node recorded as the writer of slot (i, k):
            // x - e_i if fluid, else x (bounce-back)
            q = pred_read(i, (bool)((m >> opp(i)) & 1u), psi_rel, G);
            inv_t = q.rt > 0.0f ? 1.0f / q.rt : 0.0f;
        }
        const typename C::T h0 = C::enc(f0, q.p.x, inv_t);
        const typename C::T h1 = C::enc(f1, q.p.y, inv_t);
        sum0 += C::dec(h0, q.p.x, q.rt);
        sum1 += C::dec(h1, q.p.y, q.rt);
        st_pop<true>(P.plane(i, g.np), k, typename Pops<C>::P2{{h0, h1}});
    }
    // rest population from the node mass (see store_node)
    st_pop<true>(P.rests(), k, Pair<float>{{r.x - sum0, r.y - sum1}});
}

// ---------------------------------------------------------------------------
// Tile kernels.  One block of 256 threads per active tile (lbm_tiles.hpp);
// thread j handles the tile's fluid nodes j and j + 256 (when they exist).
// ---------------------------------------------------------------------------

// Staging of planes z0-1 .. z0+2 over the tile plus a one-node halo (HZ x HY
// rows of HX values) into LDS.  Wave w copies rows w, w + 4, ...: lane l
// takes column l of each, and lanes 0 .. 2*RPW-1 take the two end columns
// 64-65 of those rows.  Coordinates wrap periodically once; a position one
// wrap cannot bring inside the lattice (extents below the tile size) gets the
// fill value.  HaloSlots holds this thread's share of the positions; gather()
// issues the loads of one field, put() writes them to LDS, and every gather
// of a thread comes before its first put, so all of its loads (and any the
// caller issued before) are in flight together: each put waits for the
// thread's loads in issue order.  direct() loads the same rows straight into
// LDS instead (no registers, no LDS writes by the waves), where every halo
// position lies inside the lattice after one wrap.
struct HaloSlots {
    static constexpr int NW = NT / 64;
    static constexpr int RPW = (HZ * HY + NW - 1) / NW;  // rows per wave (the last ones may run past HZ*HY)
    static_assert(2 * RPW <= 64 && HX == 66, "halo row split");
    int lane, wave, gx, gxt, tp;
    bool inx, has_tail;
    const Geo& g;
    int x0, y0, z0;
    __device__ __forceinline__ HaloSlots(int x0_, int y0_, int z0_, const Geo& g_) : g(g_), x0(x0_), y0(y0_), z0(z0_) {
        lane = threadIdx.x & 63;
        wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        gx = x0 + lane - 1;
        gx = gx < 0 ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
        inx = gx < g.nx;
        has_tail = lane < 2 * RPW;
        tp = lane >> 1;  // row slot of this lane's end-column value
        gxt = x0 + 63 + (lane & 1);
        gxt = gxt >= g.nx ? gxt - g.nx : gxt;
    }
    __device__ __forceinline__ uint32_t row_base(int r, bool& ok) const {
        const int pl = r / HY, hy = r - pl * HY;
        int gy = y0 + hy - 1, gz = z0 - 1 + pl;
        gy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
        gz = gz < 0 ? gz + g.nz : (gz >= g.nz ? gz - g.nz : gz);
        ok = gy < g.ny;
        return (uint32_t)(g.nx * (gy + g.ny * gz));
    }
    template <class T, class Src>
    __device__ __forceinline__ void gather(Src src, T fill, T (&v)[RPW], T& vt) const {
        uint32_t rbt = 0;
        bool okt = false;
#pragma unroll
        for (int p = 0; p < RPW; ++p) {
            bool ok;
            const int r = wave + NW * p;
            const uint32_t rb = row_base(r < HZ * HY ? r : 0, ok);
            ok = ok && r < HZ * HY;
            v[p] = (ok && inx) ? src(rb + (uint32_t)gx) : fill;
            rbt = tp == p ? rb : rbt;
            okt = tp == p ? ok : okt;
        }
        vt = fill;
        if (has_tail && okt && gxt < g.nx) vt = src(rbt + (uint32_t)gxt);
    }
    // every halo position inside the lattice after one wrap: no fill values
    __host__ __device__ static bool direct_ok(const Geo& g) { return g.nx >= TX && g.ny >= TY && g.nz >= TZ; }
    // Rows of 4- or 8-byte elements loaded with global_load_lds: lane l's
    // dword lands at the instruction's LDS address + 4 l, so each instruction
    // fills 64 consecutive dwords of a row (an 8-byte element takes two
    // lanes).  The caller waits for the loads (vmcnt) before the barrier.
    template <class T>
    __device__ __forceinline__ void direct(T (*tile)[HY][HX], const T* src) const {
        constexpr int W = (int)(sizeof(T) / 4);  // dwords per element
        static_assert(HZ * HY == NW * RPW, "whole rows per wave");
#pragma unroll
        for (int p = 0; p < RPW; ++p) {
            const int r = wave + NW * p;
            bool ok;
            const uint32_t rb = row_base(r, ok);
            char* lrow = (char*)&tile[r / HY][r % HY][0];
#pragma unroll
            for (int k = 0; k < (HX * W + 63) / 64; ++k) {
                const int d = 64 * k + lane;  // dword of the row
                const int pos = d / W, c = d - pos * W;
                int x = x0 - 1 + pos;
                x = x < 0 ? x + g.nx : (x >= g.nx ? x - g.nx : x);
                if (d < HX * W)
                    __builtin_amdgcn_global_load_lds(
                        (__attribute__((address_space(1))) void*)((const char*)src +
                                                                  ((size_t)(rb + (uint32_t)x) * W + c) * 4),
                        (__attribute__((address_space(3))) void*)(lrow + 256 * k), 4, 0, 0);
            }
        }
    }
    template <class T>
    __device__ __forceinline__ void put(T (*tile)[HY][HX], const T (&v)[RPW], T vt) const {
#pragma unroll
        for (int p = 0; p < RPW; ++p) {
            const int r = wave + NW * p;
            if (r < HZ * HY) tile[r / HY][r % HY][lane] = v[p];
        }
        const int rt = wave + NW * tp;
        if (has_tail && rt < HZ * HY) tile[rt / HY][rt % HY][64 + (lane & 1)] = vt;
    }
};

// wait for this wave's outstanding vector memory loads (vmcnt(0); the
// expcnt and lgkmcnt fields at their maxima), direct() loads included
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0f70); }

template <class T, class Src>
__device__ __forceinline__ void stage_halo(T (*tile)[HY][HX], int x0, int y0, int z0, const Geo& g, Src src,
                                           T fill) {
    const HaloSlots h(x0, y0, z0, g);
    T v[HaloSlots::RPW], vt;
    h.gather(src, fill, v, vt);
    h.put(tile, v, vt);
}

// Two fields of the same positions staged together (this level's psi-hat and
// the codec's previous-level field in the F16/BF16 collide-stream): one wait
// for both instead of one each.
template <class T, class SrcA, class SrcB>
__device__ __forceinline__ void stage_halo2(T (*ta)[HY][HX], SrcA srca, T (*tb)[HY][HX], SrcB srcb, int x0, int y0,
                                            int z0, const Geo& g, T fill) {
    const HaloSlots h(x0, y0, z0, g);
    T va[HaloSlots::RPW], vb[HaloSlots::RPW], vta, vtb;
    h.gather(srca, fill, va, vta);
    h.gather(srcb, fill, vb, vtb);
    h.put(ta, va, vta);
    h.put(tb, vb, vtb);
}

// Fluid ids of the staged halo around one tile node: fid of x + s e_i, -1
// at solid nodes.
struct HaloFid {
    const int (*t)[HY][HX];
    int tx, ty, tz;
    __device__ __forceinline__ int operator()(int i, int s) const {
        return t[tz + s * DZ[i]][ty + s * DY[i]][tx + s * DX[i]];
    }
};

// K1: densities.  psi[x] = (rho1, rho2) at fluid nodes.  In odd steps the
// fluid-id halo is staged first (the gathers need it); with the F16/BF16
// codecs the previous level's pseudopotential field, which gives the codec
// predictors, is staged as an LDS halo as well, while the thread's first
// node is loaded.  At least 8 waves per SIMD in even steps (7 with a
// decoding halo) and 6 in odd steps; the compiler's default schedule would
// hold ~105 VGPRs.
template <class C, bool ODD, bool WIDE, bool DIRECT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(ODD ? 6 : (C::kRef ? 7 : 8))))
void k_density(Pops<C> P, Sparse S, const float2* __restrict__ rprev, float2* __restrict__ psi, Geo g, float G) {
    const int a = active_of_block(S.nactive);
    if (a < 0) return;
    const int t = S.active[a];
    int x0, y0, z0;
    tile_origin(t, g, x0, y0, z0);
    const int base = S.base[t], count = S.count[t];
    __shared__ int fidt[ODD ? HZ : 1][HY][HX];
    __shared__ float2 reft[C::kRef ? HZ : 1][HY][HX];
    // with the F16/BF16 codecs the first node's in-tile position is requested
    // before the fluid-id halo is staged, so that the odd level's gathers wait
    // for one round trip after the halo, not two (measured neutral to slightly
    // slower for FP32, whose kernels load it in fetch)
    const int j0 = threadIdx.x;
    const uint16_t loc0 = (C::kRef && j0 < count) ? S.loc[base + j0] : (uint16_t)0;
    if constexpr (ODD) {
        // odd levels: the codec's previous-level halo (F16/BF16) is staged with
        // the fluid-id halo the gathers need, under one wait and one barrier
        const HaloSlots hs(x0, y0, z0, g);
        if constexpr (DIRECT) {
            hs.direct(fidt, S.fid);
            if constexpr (C::kRef) hs.direct(reft, rprev);
            wait_vm();
        } else {
            int vf[HaloSlots::RPW], vft;
            float2 vr[HaloSlots::RPW], vrt;
            hs.gather([&](uint32_t i) { return S.fid[i]; }, -1, vf, vft);
            if constexpr (C::kRef) hs.gather([&](uint32_t i) { return ld(rprev, i); }, make_float2(0.f, 0.f), vr, vrt);
            hs.put(fidt, vf, vft);
            if constexpr (C::kRef) hs.put(reft, vr, vrt);
        }
        __syncthreads();
    }
    // the F16/BF16 decoders also need the node's neighbourhood word (by fluid
    // id, so coalesced and with no lookup before it); it is requested with the
    // populations, not after the wait for them
    auto fetch = [&](int j, uint16_t lc, RawNode<C>& r, TilePos& q, uint32_t& m) {
        const uint32_t k = (uint32_t)(base + j);
        q = TilePos(C::kRef ? lc : S.loc[k]);
        load_raw<C, ODD, WIDE>(r, P, k, HaloFid{fidt, q.lx + 1, q.ly + 1, q.lz + 1}, g.np);
        m = C::kRef ? S.nbf[k] : 0u;
    };
    auto finish = [&](const RawNode<C>& r, const TilePos& q, uint32_t m) {
        const uint32_t idx = (uint32_t)(x0 + q.lx + g.nx * (y0 + q.ly + g.ny * (z0 + q.lz)));
        const int tx = q.lx + 1, ty = q.ly + 1, tz = q.lz + 1;
        float f[2][Q];
        if constexpr (C::kRef) {
            auto psi_rel = [&](int dx, int dy, int dz) { return reft[tz + dz][ty + dy][tx + dx]; };
            decode_node<C>(f, r, m, [&](int i, bool wall) { return pred_read(i, wall, psi_rel, G); });
        } else {
            decode_node<C>(f, r, m, [&](int, bool) { return PredRef{make_float2(0.f, 0.f), 0.f}; });
        }
        st(psi, idx, make_float2(sum19(f[0]), sum19(f[1])));
    };
    RawNode<C> r;
    TilePos q(0);
    uint32_t m = 0u;
    if (j0 < count) fetch(j0, loc0, r, q, m);
    if constexpr (C::kRef && !ODD) {
        if constexpr (DIRECT) {
            HaloSlots(x0, y0, z0, g).direct(reft, rprev);
            wait_vm();
        } else {
            stage_halo(reft, x0, y0, z0, g, [&](uint32_t i) { return ld(rprev, i); }, make_float2(0.f, 0.f));
        }
        __syncthreads();
    }
    if (j0 < count) finish(r, q, m);
    for (int j = j0 + NT; j < count; j += NT) {
        fetch(j, C::kRef ? S.loc[base + j] : (uint16_t)0, r, q, m);
        finish(r, q, m);
    }
}


// K1b: IVSD virtual solid density at boundary solid nodes (Eqs. 14-15):
// rho~^(s) = chi^(s) sum_i w_i rho^(s)(x+e_i) [fluid] / sum_i w_i [fluid],
// chi^(1) = 1 + xi, chi^(2) = 1 - xi.
// The node's neighbourhood word comes from the list-ordered copy nbl, so it
// is requested together with the node's index instead of after it: the
// neighbour loads, whose addresses depend on both, then wait for one round
// trip instead of two.
__global__ __launch_bounds__(256) void k_ivsd(const int* __restrict__ list, const float* __restrict__ xil,
                                              int count, const uint32_t* __restrict__ nbl,
                                              float2* __restrict__ psi, Geo g) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int idx = list[k];
    const uint32_t m = nbl[k];
    const int x = idx % g.nx;
    const int y = (idx / g.nx) % g.ny;
    const int z = idx / (g.nx * g.ny);
    const Nb nb(x, y, z, g);
    // all 18 neighbour loads issued together: a solid neighbour reads the
    // node's own entry instead (a value only this thread writes, after the
    // loads) and its term is dropped by a select
    float2 r[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) r[i] = ld((const float2*)psi, ((m >> i) & 1u) ? (uint32_t)idx : nb.at(i, +1));
    float den = 0.f, n0 = 0.f, n1 = 0.f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const bool fluid = !((m >> i) & 1u);
        den += fluid ? weight(i) : 0.0f;
        n0 += fluid ? weight(i) * r[i].x : 0.0f;
        n1 += fluid ? weight(i) * r[i].y : 0.0f;
    }
    const float v = xil[k];
    const float inv = 1.0f / den;  // den > 0: the list holds only nodes with a fluid neighbour
    psi[idx] = make_float2((1.0f + v) * n0 * inv, (1.0f - v) * n1 * inv);
}

// K2: fused force + collision + streaming for the fluid nodes of one tile.
// The psi-hat values (and, in odd steps, the fluid ids) of planes z0-1 ..
// z0+2 over the tile and a one-node halo are staged in LDS; each node then
// reads its 18 neighbours from LDS.  The populations of a thread's first
// node are requested before the psi-hat staging so that the two overlap:
// in even steps straight away (they sit in the node's own slots), in odd
// steps right after the fluid-id halo is in LDS (they are gathered from the
// neighbours' slots).  P is the state read, D the state written: the same
// buffer for the in-place step, two buffers when a step is recomputed into
// a separate slot.
// Register budgets: the compiler's default schedule holds up to ~140 VGPRs
// (3 waves per SIMD), too few waves to hide the memory latency of the
// population traffic.  FP32 runs 4 waves per SIMD (up to 128 VGPRs; no
// spill with 32-bit slot offsets); the FP16/BF16 codecs, whose populations
// take half the registers, run 5 (odd steps spill a few dwords, which costs
// less than the lost wave).
template <class C, bool ODD, bool WIDE, bool DIRECT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(C::kRef ? 5 : 4))) void k_collide_stream(Pops<C> P, Pops<C> D, Sparse S,
                                                       const float2* __restrict__ rprev,
                                                       const float2* __restrict__ psi, Geo g, Phys ph) {
    const int a = active_of_block(S.nactive);
    if (a < 0) return;
    const int t = S.active[a];
    int x0, y0, z0;
    tile_origin(t, g, x0, y0, z0);
    const int base = S.base[t], count = S.count[t];
    __shared__ float2 psit[HZ][HY][HX];
    __shared__ int fidt[ODD ? HZ : 1][HY][HX];
    // with the F16/BF16 codecs the first node's in-tile position is requested
    // before the fluid-id halo is staged, so that the odd level's gathers wait
    // for one round trip after the halo, not two (measured neutral to slightly
    // slower for FP32, whose kernels load it in fetch)
    const int j0 = threadIdx.x;
    const uint16_t loc0 = (C::kRef && j0 < count) ? S.loc[base + j0] : (uint16_t)0;
    __shared__ float2 reft[C::kRef ? HZ : 1][HY][HX];
    if constexpr (ODD) {
        // odd levels: the psi-hat halos are staged with the fluid-id halo the
        // gathers need, under one wait and one barrier
        const HaloSlots hs(x0, y0, z0, g);
        if constexpr (DIRECT) {
            hs.direct(fidt, S.fid);
            hs.direct(psit, psi);
            if constexpr (C::kRef) hs.direct(reft, rprev);
            wait_vm();
        } else {
            int vf[HaloSlots::RPW], vft;
            float2 vp[HaloSlots::RPW], vpt, vr[HaloSlots::RPW], vrt;
            hs.gather([&](uint32_t i) { return S.fid[i]; }, -1, vf, vft);
            hs.gather([&](uint32_t i) { return ld(psi, i); }, make_float2(0.f, 0.f), vp, vpt);
            if constexpr (C::kRef) hs.gather([&](uint32_t i) { return ld(rprev, i); }, make_float2(0.f, 0.f), vr, vrt);
            hs.put(fidt, vf, vft);
            hs.put(psit, vp, vpt);
            if constexpr (C::kRef) hs.put(reft, vr, vrt);
        }
        __syncthreads();
    }
    // the F16/BF16 codecs also need the node's neighbourhood word (by fluid
    // id, so coalesced and with no lookup before it); it is requested with the
    // populations, not after the wait for them
    auto fetch = [&](int j, uint16_t lc, RawNode<C>& r, HaloFid& h, uint32_t& m) {
        const uint32_t k = (uint32_t)(base + j);
        const TilePos q(C::kRef ? lc : S.loc[k]);
        h = HaloFid{fidt, q.lx + 1, q.ly + 1, q.lz + 1};
        load_raw<C, ODD, WIDE>(r, P, k, h, g.np);
        m = C::kRef ? S.nbf[k] : 0u;
    };
    auto finish = [&](int j, const RawNode<C>& r, const HaloFid& h, uint32_t m) {
        const uint32_t k = (uint32_t)(base + j);
        float f[2][Q];
        if constexpr (C::kRef) {
            auto prev_rel = [&](int dx, int dy, int dz) { return reft[h.tz + dz][h.ty + dy][h.tx + dx]; };
            decode_node<C>(f, r, m, [&](int i, bool wall) { return pred_read(i, wall, prev_rel, ph.G); });
        } else {
            decode_node<C>(f, r, m, [&](int, bool) { return PredRef{make_float2(0.f, 0.f), 0.f}; });
        }
        const float rho[2] = {sum19(f[0]), sum19(f[1])};
        float acc[2][3];
        psi_sum([&](int i) { return psit[h.tz + DZ[i]][h.ty + DY[i]][h.tx + DX[i]]; }, acc);
        float F[2][3];
        total_force(rho, acc, ph, F);
        float u[3];
        collide(f, rho, F, ph, u);
        // codec predictors of the values written (F16/BF16) come from this
        // level's psi-hat, the readers' previous level
        // (a laundered zero offset keeps the compiler from reading them all
        // before the collision and holding them across it)
        int zero = 0;
        asm volatile("" : "+v"(zero));
        auto cur_rel = [&](int dx, int dy, int dz) { return psit[h.tz + dz][h.ty + dy][h.tx + dx + zero]; };
        const float2 own = psit[h.tz][h.ty][h.tx];
        store_node<C, ODD, WIDE>(
            f, D, rho, [&](int i) { return pred_write(i, (bool)((m >> i) & 1u), cur_rel, ph.G); },
            own.x + own.y, C::kRef ? inv_total(own) : 0.0f, k, h, g.np);
    };
    RawNode<C> r;
    HaloFid h;
    uint32_t m = 0u;
    if (j0 < count) fetch(j0, loc0, r, h, m);
    if constexpr (!ODD) {
        if constexpr (DIRECT) {
            const HaloSlots hs(x0, y0, z0, g);
            hs.direct(psit, psi);
            if constexpr (C::kRef) hs.direct(reft, rprev);
            wait_vm();
        } else if constexpr (C::kRef) {
            stage_halo2(psit, [&](uint32_t i) { return ld(psi, i); }, reft, [&](uint32_t i) { return ld(rprev, i); },
                        x0, y0, z0, g, make_float2(0.f, 0.f));
        } else {
            stage_halo(psit, x0, y0, z0, g, [&](uint32_t i) { return ld(psi, i); }, make_float2(0.f, 0.f));
        }
        __syncthreads();
    }
    if (j0 < count) finish(j0, r, h, m);
    for (int j = j0 + NT; j < count; j += NT) {
        fetch(j, C::kRef ? S.loc[base + j] : (uint16_t)0, r, h, m);
        finish(j, r, h, m);
    }
}

// ---------------------------------------------------------------------------
// Readouts and diagnostics at the current time level (psi already filled by
// k_density + k_ivsd for this level).  Dense over all nodes, in patches of
// 64 x 4 nodes of one z plane numbered x fastest; block b handles patches
// b, b + gridDim.x, ... (one patch each when the grid covers them all), so
// the per-block FP64 partials hold a fixed set of patches summed in a fixed
// order.
// ---------------------------------------------------------------------------
template <class C, bool ODD>
__global__ __launch_bounds__(256) void k_fields(Pops<C> P, const int* __restrict__ fid,
                                                    const uint32_t* __restrict__ nbm,
                                                    const float2* __restrict__ rprev,
                                                    const float2* __restrict__ psi, Geo g, Phys ph,
                                                    float* __restrict__ o_rho, float* __restrict__ o_u,
                                                    float* __restrict__ o_F, float* __restrict__ o_P,
                                                    double* __restrict__ partial, int skip_ghost_x) {
    const int gx = (g.nx + 63) / 64, gy = (g.ny + 3) / 4;
    const int npatch = gx * gy * g.nz;
    double d[7] = {0, 0, 0, 0, 0, 0, 0};  // m1, m2, water, snw, |u|max, bad, nfluid
    for (int b = blockIdx.x; b < npatch; b += gridDim.x) {
        const int bx = b % gx, r = b / gx;
        const int x = bx * 64 + threadIdx.x;
        const int y = (r % gy) * 4 + threadIdx.y;
        const int z = r / gy;
        if (!(x < g.nx && y < g.ny)) continue;
        const Nb nb(x, y, z, g);
        const uint32_t self = nb.idx;
        const size_t n = (size_t)g.n;
        const uint32_t m = nbm[self];
        float rho[2] = {0.f, 0.f}, u[3] = {0.f, 0.f, 0.f}, F[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
        float pr = 0.f;
        if (!(m & SELF_SOLID)) {
            float f[2][Q];
            load_node<C, ODD>(f, P, rprev, m, nb, (uint32_t)fid[self],
                              [&](int i, int s) { return fid[nb.at(i, s)]; }, g.np, ph.G);
            rho[0] = sum19(f[0]);
            rho[1] = sum19(f[1]);
            float acc[2][3];
            psi_sum([&](int i) { return ld(psi, nb.at(i, +1)); }, acc);
            total_force(rho, acc, ph, F);
            collide(f, rho, F, ph, u);  // computes u; the collided f is discarded
            // Eq. (12), ordered pairs: P = c_s^2 (rho1 + rho2) + c_s^2 G rho1 rho2
            pr = (rho[0] + rho[1]) * (1.0f / 3.0f) + (ph.G / 3.0f) * rho[0] * rho[1];
            const double r0 = rho[0], r1 = rho[1];
            const double um = sqrt((double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2]);
            // with open x planes the ghost planes stay out of the diagnostics
            if (!(skip_ghost_x && (x == 0 || x == g.nx - 1))) {
                d[0] += r0;
                d[1] += r1;
                d[2] += r1 > r0 ? 1.0 : 0.0;
                d[3] += r0 / (r0 + r1);
                d[4] = fmax(d[4], um);
                d[5] += (isfinite(rho[0]) && isfinite(rho[1]) && isfinite(um)) ? 0.0 : 1.0;
                d[6] += 1.0;
            }
        }
        if (o_rho) { o_rho[self] = rho[0]; o_rho[n + self] = rho[1]; }
        if (o_u) { o_u[self] = u[0]; o_u[n + self] = u[1]; o_u[2 * n + self] = u[2]; }
        if (o_F)
            for (int s = 0; s < 2; ++s)
                for (int a = 0; a < 3; ++a) o_F[(size_t)(s * 3 + a) * n + self] = F[s][a];
        if (o_P) o_P[self] = pr;
    }
    if (!partial) return;
    // block reduction in FP64 (wave shuffles, then LDS across waves)
    __shared__ double red[4][7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        double v = d[k];
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off);
            v = (k == 4) ? fmax(v, o) : v + o;
        }
        d[k] = v;
    }
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if ((tid & 63) == 0)
        for (int k = 0; k < 7; ++k) red[tid >> 6][k] = d[k];
    __syncthreads();
    if (tid < 7) {
        double v = red[0][tid];
        for (int w = 1; w < 4; ++w) v = (tid == 4) ? fmax(v, red[w][tid]) : v + red[w][tid];
        partial[(size_t)blockIdx.x * 8 + tid] = v;
    }
}

// Final deterministic reduction of the per-block partials by one block.
__global__ void k_reduce_partials(const double* __restrict__ partial, int nblocks,
                                  double* __restrict__ out) {
    __shared__ double red[1024];
    const int t = threadIdx.x;
    for (int k = 0; k < 7; ++k) {
        double v = 0.0;
        for (int b = t; b < nblocks; b += 1024) {
            const double p = partial[(size_t)b * 8 + k];
            v = (k == 4) ? fmax(v, p) : v + p;
        }
        red[t] = v;
        __syncthreads();
        for (int off = 512; off > 0; off >>= 1) {
            if (t < off) red[t] = (k == 4) ? fmax(red[t], red[t + off]) : red[t] + red[t + off];
            __syncthreads();
        }
        if (t == 0) out[k] = red[0];
        __syncthreads();
    }
}

// Writes a few 64-bit words (checkpoint headers) in stream order.
__global__ void k_store_words(uint64_t* __restrict__ dst, uint64_t w0, uint64_t w1, uint64_t w2,
                              uint64_t w3) {
    const int t = threadIdx.x;
    const uint64_t v = t == 0 ? w0 : (t == 1 ? w1 : (t == 2 ? w2 : w3));
    if (t < 4) dst[t] = v;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
void launch_store_words(uint64_t* dst, const uint64_t (&w)[4], hipStream_t s) {
    hipLaunchKernelGGL(k_store_words, dim3(1), dim3(64), 0, s, dst, w[0], w[1], w[2], w[3]);
}

static dim3 row_grid(const Geo& g) { return dim3((g.nx + 63) / 64, g.ny, g.nz); }
// readout blocks: 64 x 4 nodes of one z plane
static dim3 tile_grid3(const Geo& g) { return dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz); }

int tile_count(const Geo& g) {
    return ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + TZ - 1) / TZ);
}

void launch_neighbour_bits(const uint8_t* solid, uint32_t* nbm, const Geo& g, hipStream_t s) {
    hipLaunchKernelGGL(k_neighbour_bits, row_grid(g), dim3(64), 0, s, solid, nbm, g);
}

int boundary_blocks(const Geo& g) { return tile_count(g); }

void launch_boundary_list(const uint32_t* nbm, const float* xi, int* counts, int* total, int* list,
                          float* xil, uint32_t* nbl, const Geo& g, hipStream_t s) {
    const int nb = boundary_blocks(g);
    hipLaunchKernelGGL(k_boundary_count, dim3(nb), dim3(TX, TY, TZ), 0, s, nbm, g, counts);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, nb, total);
    hipLaunchKernelGGL(k_boundary_write, dim3(nb), dim3(TX, TY, TZ), 0, s, nbm, xi, g,
                       (const int*)counts, list, xil, nbl);
}

void launch_geometry_check(const uint32_t* nbm, const float* xi, const Geo& g, unsigned long long* out,
                           hipStream_t s) {
    const uint64_t zero[4] = {0, 0, 0, 0};
    launch_store_words((uint64_t*)out, zero, s);
    hipLaunchKernelGGL(k_geometry_check, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, s, nbm, xi, g, out);
}

void launch_tile_census(const uint32_t* nbm, const Geo& g, int* cnt, int* base, int* apos, int* totals,
                        hipStream_t s) {
    const int nt = tile_count(g);
    hipLaunchKernelGGL(k_tile_count, dim3(nt), dim3(TX, TY, TZ), 0, s, nbm, g, cnt, base, apos);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, base, nt, totals);      // fluid ids
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, apos, nt, totals + 1);  // active tiles
}

void launch_tile_ids(const uint32_t* nbm, const Geo& g, const int* cnt, const int* base, const int* apos, int* fid,
                     uint16_t* loc, uint32_t* nbf, int* active, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_ids, dim3(tile_count(g)), dim3(TX, TY, TZ), 0, s, nbm, g, base, cnt, apos, fid, loc,
                       nbf, active);
}


template <class C>
void launch_init(const Pops<C>& P, const uint32_t* nbm, const int* fid, const float* rho, float2* rprev,
                 const int* list, const float* xil, const uint32_t* nbl, int nbound, const Geo& g, float G,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_init_ref, row_grid(g), dim3(64), 0, s, nbm, rho, rprev, g);
    launch_ivsd(list, xil, nbl, nbound, rprev, g, s);
    hipLaunchKernelGGL(k_init<C>, row_grid(g), dim3(64), 0, s, P, nbm, fid, (const float2*)rprev, g, G);
}

// halos loaded straight into LDS wherever no halo position needs a fill value
template <class C, bool ODD, bool WIDE>
static void launch_density_as(const Pops<C>& P, const Sparse& S, const float2* rprev, float2* psi, const Geo& g,
                              float G, hipStream_t s) {
    if (HaloSlots::direct_ok(g))
        hipLaunchKernelGGL((k_density<C, ODD, WIDE, true>), dim3(xcd_grid(S.nactive)), dim3(NT), 0, s, P, S, rprev,
                           psi, g, G);
    else
        hipLaunchKernelGGL((k_density<C, ODD, WIDE, false>), dim3(xcd_grid(S.nactive)), dim3(NT), 0, s, P, S, rprev,
                           psi, g, G);
}

template <class C>
void launch_density(const Pops<C>& P, const Sparse& S, const float2* rprev, float2* psi, const Geo& g, float G,
                    int odd, hipStream_t s) {
    if (S.nactive <= 0) return;
    const bool wide = pops_wide(g.np);
    if (odd)
        wide ? launch_density_as<C, true, true>(P, S, rprev, psi, g, G, s)
             : launch_density_as<C, true, false>(P, S, rprev, psi, g, G, s);
    else
        wide ? launch_density_as<C, false, true>(P, S, rprev, psi, g, G, s)
             : launch_density_as<C, false, false>(P, S, rprev, psi, g, G, s);
}

void launch_ivsd(const int* list, const float* xil, const uint32_t* nbl, int count, float2* psi, const Geo& g,
                 hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_ivsd, dim3((count + 255) / 256), dim3(256), 0, s, list, xil, count, nbl, psi, g);
}

template <class C, bool ODD, bool WIDE>
static void launch_collide_as(const Pops<C>& P, const Pops<C>& D, const Sparse& S, const float2* rprev,
                              const float2* psi, const Geo& g, const Phys& ph, hipStream_t s) {
    if (HaloSlots::direct_ok(g))
        hipLaunchKernelGGL((k_collide_stream<C, ODD, WIDE, true>), dim3(xcd_grid(S.nactive)), dim3(NT), 0, s, P, D, S,
                           rprev, psi, g, ph);
    else
        hipLaunchKernelGGL((k_collide_stream<C, ODD, WIDE, false>), dim3(xcd_grid(S.nactive)), dim3(NT), 0, s, P, D,
                           S, rprev, psi, g, ph);
}

template <class C>
void launch_collide_stream(const Pops<C>& P, const Pops<C>& D, const Sparse& S, const float2* rprev,
                           const float2* psi, const Geo& g, const Phys& ph, int odd, hipStream_t s) {
    if (S.nactive <= 0) return;
    const bool wide = pops_wide(g.np);
    if (odd)
        wide ? launch_collide_as<C, true, true>(P, D, S, rprev, psi, g, ph, s)
             : launch_collide_as<C, true, false>(P, D, S, rprev, psi, g, ph, s);
    else
        wide ? launch_collide_as<C, false, true>(P, D, S, rprev, psi, g, ph, s)
             : launch_collide_as<C, false, false>(P, D, S, rprev, psi, g, ph, s);
}

int fields_blocks(const Geo& g) {
    const dim3 gr = tile_grid3(g);
    return (int)(gr.x * gr.y * gr.z);
}

template <class C>
void launch_fields(const Pops<C>& P, const int* fid, const uint32_t* nbm, const float2* rprev, const float2* psi,
                   const Geo& g, const Phys& ph, int odd, float* o_rho, float* o_u, float* o_F, float* o_P,
                   double* partial, double* out, int skip_ghost_x, hipStream_t s, int max_blocks) {
    const int all = fields_blocks(g);
    const int nb = max_blocks > 0 && max_blocks < all ? max_blocks : all;
    if (odd)
        hipLaunchKernelGGL((k_fields<C, true>), dim3(nb), dim3(64, 4), 0, s, P, fid, nbm, rprev, psi, g,
                           ph, o_rho, o_u, o_F, o_P, partial, skip_ghost_x);
    else
        hipLaunchKernelGGL((k_fields<C, false>), dim3(nb), dim3(64, 4), 0, s, P, fid, nbm, rprev, psi, g,
                           ph, o_rho, o_u, o_F, o_P, partial, skip_ghost_x);
    if (partial)
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, s, (const double*)partial, nb, out);
}

// The library's own device scratch for callers that cannot allocate (FP64
// partials and results of the diagnostics reduction): one copy per GPU,
// kept until the process ends.  Host code never passes the array's name to
// a kernel; it uses the address hipGetSymbolAddress returns for the device.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = (double*)g_scratch_ptr[device];
    return hipSuccess;
}

#define MCLBM_INSTANTIATE(C)                                                                              \
    template void launch_init<C>(const Pops<C>&, const uint32_t*, const int*, const float*, float2*,      \
                                 const int*, const float*, const uint32_t*, int, const Geo&, float,      \
                                 hipStream_t);                                                          \
    template void launch_density<C>(const Pops<C>&, const Sparse&, const float2*, float2*, const Geo&,    \
                                    float, int, hipStream_t);                                             \
    template void launch_collide_stream<C>(const Pops<C>&, const Pops<C>&, const Sparse&, const float2*,   \
                                           const float2*, const Geo&, const Phys&, int, hipStream_t);    \
    template void launch_fields<C>(const Pops<C>&, const int*, const uint32_t*, const float2*,            \
                                   const float2*, const Geo&, const Phys&, int, float*, float*, float*,   \
                                   float*, double*, double*, int, hipStream_t, int);

MCLBM_INSTANTIATE(CodecF32)
MCLBM_INSTANTIATE(CodecF16)
MCLBM_INSTANTIATE(CodecBF16)

}  // namespace mclbm
