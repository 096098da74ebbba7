// HIP kernels of the two-component D3Q19 pseudopotential step (gfx950).
//
// One time step is three launches on the caller's stream:
//   k_density        rho^(sigma) at every fluid node from the incoming
//                    populations (Eq. 3); 0 at solid nodes.
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

constexpr int kListBlock = 256;

__global__ void k_boundary_count(const uint32_t* __restrict__ nbm, int n, int* __restrict__ counts) {
    const int idx = blockIdx.x * kListBlock + threadIdx.x;
    const bool flag = idx < n && is_boundary_solid(nbm[idx]);
    const int c = __syncthreads_count(flag);
    if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

// Exclusive scan of the per-block counts by one block (set-up only).
__global__ void k_boundary_scan(int* __restrict__ counts, int nblocks, int* __restrict__ total) {
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

__global__ void k_boundary_write(const uint32_t* __restrict__ nbm, const float* __restrict__ xi,
                                 int n, const int* __restrict__ offsets, int* __restrict__ list,
                                 float* __restrict__ xil, int* __restrict__ bad) {
    __shared__ int wave_off[kListBlock / 64];
    const int idx = blockIdx.x * kListBlock + threadIdx.x;
    const bool flag = idx < n && is_boundary_solid(nbm[idx]);
    const unsigned long long ball = __ballot(flag);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int rank = __popcll(ball & ((1ull << lane) - 1ull));
    if (lane == 0) wave_off[wave] = __popcll(ball);
    __syncthreads();
    int base = offsets[blockIdx.x];
    for (int w = 0; w < wave; ++w) base += wave_off[w];
    bool invalid = false;
    if (flag) {
        const float v = xi[idx];
        list[base + rank] = idx;
        xil[base + rank] = v;
        invalid = !(fabsf(v) < 1.0f);
    }
    const int any_bad = __syncthreads_or(invalid);
    if (threadIdx.x == 0) bad[blockIdx.x] = any_bad;
}

// ---------------------------------------------------------------------------
// Initial state f_i = w_i rho (fluid at rest), even-parity layout.
// ---------------------------------------------------------------------------
template <class C>
__global__ void k_init(Pops<C> P, const uint32_t* __restrict__ nbm, const float* __restrict__ rho_in,
                       float2* __restrict__ rprev, Geo g) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx) return;
    const Nb nb(x, y, z, g);
    const uint32_t self = nb.idx;
    const uint32_t m = nbm[self];
    if (m & SELF_SOLID) {
        rprev[self] = make_float2(0.f, 0.f);
        return;
    }
    const float r0 = rho_in[self], r1 = rho_in[(size_t)g.n + self];
    rprev[self] = make_float2(r0, r1);
    float sum0 = 0.f, sum1 = 0.f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const float f0 = weight(i) * r0, f1 = weight(i) * r1;
        typename C::T h0, h1;
        if constexpr (C::kRef) {
            // reference densities of the node recorded as the writer of
            // slot (i, x): x - e_i if fluid, else x
            const bool src_solid = (m >> opp(i)) & 1u;
            const uint32_t w = src_solid ? self : nb.at(i, -1);
            const float2 rw = src_solid ? make_float2(r0, r1) : make_float2(rho_in[w], rho_in[(size_t)g.n + w]);
            const float inv_t = inv_total(rw);
            const float rt = rw.x + rw.y;
            h0 = C::enc(f0, weight(i), rw.x, inv_t);
            h1 = C::enc(f1, weight(i), rw.y, inv_t);
            sum0 += C::dec(h0, weight(i), rw.x, rt);
            sum1 += C::dec(h1, weight(i), rw.y, rt);
        } else {
            h0 = C::enc(f0, weight(i), 0.f, 0.f);
            h1 = C::enc(f1, weight(i), 0.f, 0.f);
            sum0 += C::dec(h0, weight(i), 0.f, 0.f);
            sum1 += C::dec(h1, weight(i), 0.f, 0.f);
        }
        st(P.plane(0, i, g.np), self, h0);
        st(P.plane(1, i, g.np), self, h1);
    }
    // rest population from the node mass (see store_node)
    st(P.rest, self, r0 - sum0);
    st(P.rest + g.np, self, r1 - sum1);
}

// ---------------------------------------------------------------------------
// Tiles of 64 x 4 nodes in one z plane.  Blocks are numbered on a 1D grid and
// mapped XCD-aware: the hardware deals consecutive block ids round-robin to
// the 8 XCDs, so block b takes tile (b mod 8) * per + b / 8 and every XCD
// works through a contiguous run of neighbouring tiles, whose shared halo
// rows then hit in that XCD's L2.
// ---------------------------------------------------------------------------
constexpr int TX = 64, TY = 4;
constexpr int HX = TX + 2, HY = TY + 2;

struct TileGrid {
    int ntx, nty, ntiles, grid;
};

__device__ __forceinline__ bool tile_of_block(const TileGrid& T, int& bx, int& by, int& bz) {
    const int per = gridDim.x >> 3;
    const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (tile >= T.ntiles) return false;
    bx = tile % T.ntx;
    by = (tile / T.ntx) % T.nty;
    bz = tile / (T.ntx * T.nty);
    return true;
}

// ---------------------------------------------------------------------------
// K1: densities.  psi[x] = (rho1, rho2) at fluid nodes, (0, 0) at solid.
// ---------------------------------------------------------------------------
template <class C, bool ODD>
__global__ __launch_bounds__(TX * TY) void k_density(Pops<C> P, const uint32_t* __restrict__ nbm,
                                                     const float2* __restrict__ rprev,
                                                     float2* __restrict__ psi, Geo g, TileGrid T) {
    int bx, by, z;
    if (!tile_of_block(T, bx, by, z)) return;
    const int x = bx * TX + threadIdx.x, y = by * TY + threadIdx.y;
    if (x >= g.nx || y >= g.ny) return;
    const Nb nb(x, y, z, g);
    const uint32_t m = ld(nbm, nb.idx);
    if (m & SELF_SOLID) {
        st(psi, nb.idx, make_float2(0.f, 0.f));
        return;
    }
    float f[2][Q];
    load_node<C>(f, P, rprev, ODD, m, nb, g.np);
    st(psi, nb.idx, make_float2(sum19(f[0]), sum19(f[1])));
}

// ---------------------------------------------------------------------------
// K1b: IVSD virtual solid density at boundary solid nodes (Eqs. 14-15):
// rho~^(s) = chi^(s) sum_i w_i rho^(s)(x+e_i) [fluid] / sum_i w_i [fluid],
// chi^(1) = 1 + xi, chi^(2) = 1 - xi.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ivsd(const int* __restrict__ list, const float* __restrict__ xil,
                                              int count, const uint32_t* __restrict__ nbm,
                                              float2* __restrict__ psi, Geo g) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int idx = list[k];
    const int x = idx % g.nx;
    const int y = (idx / g.nx) % g.ny;
    const int z = idx / (g.nx * g.ny);
    const Nb nb(x, y, z, g);
    const uint32_t m = nbm[idx];
    float den = 0.f, n0 = 0.f, n1 = 0.f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (!((m >> i) & 1u)) {
            const float2 r = ld((const float2*)psi, nb.at(i, +1));
            den += weight(i);
            n0 += weight(i) * r.x;
            n1 += weight(i) * r.y;
        }
    }
    const float v = xil[k];
    const float inv = 1.0f / den;  // den > 0: the list holds only nodes with a fluid neighbour
    psi[idx] = make_float2((1.0f + v) * n0 * inv, (1.0f - v) * n1 * inv);
}

// ---------------------------------------------------------------------------
// K2: fused force + collision + streaming, one 64 x 4 tile of one z plane per
// block.  The psi-hat values of planes z-1, z, z+1 over the tile and a
// one-node halo are staged in LDS once (one barrier); each fluid node then
// reads its 18 neighbours from LDS.  P is the state read, D the state
// written: the same buffer for the in-place step, two buffers when a step is
// recomputed into a separate slot (the AA addressing writes every slot the
// next step reads, so an out-of-place step produces a complete state).
// ---------------------------------------------------------------------------
template <class C, bool ODD>
__global__ __launch_bounds__(TX * TY) void k_collide_stream(
    Pops<C> P, Pops<C> D, const uint32_t* __restrict__ nbm, const float2* __restrict__ rprev,
    const float2* __restrict__ psi, Geo g, Phys ph, TileGrid T) {
    int bx, by, z;
    if (!tile_of_block(T, bx, by, z)) return;
    const int x0 = bx * TX, y0 = by * TY;

    __shared__ float2 tile[3][HY][HX];
    {
        const int nxy = g.nx * g.ny;
        const int zs[3] = {(z == 0 ? g.nz - 1 : z - 1) * nxy, z * nxy, (z == g.nz - 1 ? 0 : z + 1) * nxy};
        for (int k = threadIdx.y * TX + threadIdx.x; k < 3 * HX * HY; k += TX * TY) {
            const int pl = k / (HX * HY);
            const int r = k - pl * (HX * HY);
            const int hy = r / HX, hx = r - hy * HX;
            int gx = x0 + hx - 1, gy = y0 + hy - 1;
            gx = gx < 0 ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
            gy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
            float2 v = make_float2(0.f, 0.f);
            if (gx < g.nx && gy < g.ny) v = ld(psi, (uint32_t)(gx + g.nx * gy + zs[pl]));
            tile[pl][hy][hx] = v;
        }
    }
    __syncthreads();

    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    if (x >= g.nx || y >= g.ny) return;
    const Nb nb(x, y, z, g);
    const uint32_t m = ld(nbm, nb.idx);
    if (m & SELF_SOLID) return;

    float f[2][Q];
    load_node<C>(f, P, rprev, ODD, m, nb, g.np);
    const float rho[2] = {sum19(f[0]), sum19(f[1])};
    const int tx = threadIdx.x + 1, ty = threadIdx.y + 1;
    float acc[2][3];
    psi_sum([&](int i) { return tile[1 + DZ[i]][ty + DY[i]][tx + DX[i]]; }, acc);
    float F[2][3];
    total_force(rho, acc, ph, F);
    float u[3];
    collide(f, rho, F, ph, u);
    store_node<C>(f, D, rho, tile[1][ty][tx], ODD, m, nb, g.np);
}

// ---------------------------------------------------------------------------
// Readouts and diagnostics at the current time level (psi already filled by
// k_density + k_ivsd for this level).
// ---------------------------------------------------------------------------
template <class C, bool ODD>
__global__ __launch_bounds__(TX * TY) void k_fields(Pops<C> P, const uint32_t* __restrict__ nbm,
                                                    const float2* __restrict__ rprev,
                                                    const float2* __restrict__ psi, Geo g, Phys ph,
                                                    float* __restrict__ o_rho, float* __restrict__ o_u,
                                                    float* __restrict__ o_F, float* __restrict__ o_P,
                                                    double* __restrict__ partial) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    const bool inside = x < g.nx && y < g.ny;
    double d[7] = {0, 0, 0, 0, 0, 0, 0};  // m1, m2, water, snw, |u|max, bad, nfluid
    if (inside) {
        const Nb nb(x, y, z, g);
        const uint32_t self = nb.idx;
        const size_t n = (size_t)g.n;
        const uint32_t m = nbm[self];
        float rho[2] = {0.f, 0.f}, u[3] = {0.f, 0.f, 0.f}, F[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
        float pr = 0.f;
        if (!(m & SELF_SOLID)) {
            float f[2][Q];
            load_node<C>(f, P, rprev, ODD, m, nb, g.np);
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
            d[0] = r0;
            d[1] = r1;
            d[2] = r1 > r0 ? 1.0 : 0.0;
            d[3] = r0 / (r0 + r1);
            d[4] = um;
            d[5] = (isfinite(rho[0]) && isfinite(rho[1]) && isfinite(um)) ? 0.0 : 1.0;
            d[6] = 1.0;
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
        const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        partial[(size_t)b * 8 + tid] = v;
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
static dim3 tile_grid3(const Geo& g) { return dim3((g.nx + TX - 1) / TX, (g.ny + TY - 1) / TY, g.nz); }

static TileGrid tiles(const Geo& g) {
    TileGrid T;
    T.ntx = (g.nx + TX - 1) / TX;
    T.nty = (g.ny + TY - 1) / TY;
    T.ntiles = T.ntx * T.nty * g.nz;
    T.grid = ((T.ntiles + 7) / 8) * 8;
    return T;
}

void launch_neighbour_bits(const uint8_t* solid, uint32_t* nbm, const Geo& g, hipStream_t s) {
    hipLaunchKernelGGL(k_neighbour_bits, row_grid(g), dim3(64), 0, s, solid, nbm, g);
}

int boundary_blocks(const Geo& g) { return (g.n + kListBlock - 1) / kListBlock; }

void launch_boundary_list(const uint32_t* nbm, const float* xi, int* counts, int* total, int* list,
                          float* xil, int* bad, const Geo& g, hipStream_t s) {
    const int nb = boundary_blocks(g);
    hipLaunchKernelGGL(k_boundary_count, dim3(nb), dim3(kListBlock), 0, s, nbm, g.n, counts);
    hipLaunchKernelGGL(k_boundary_scan, dim3(1), dim3(1024), 0, s, counts, nb, total);
    hipLaunchKernelGGL(k_boundary_write, dim3(nb), dim3(kListBlock), 0, s, nbm, xi, g.n,
                       (const int*)counts, list, xil, bad);
}

template <class C>
void launch_init(const Pops<C>& P, const uint32_t* nbm, const float* rho, float2* rprev, const Geo& g,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_init<C>, row_grid(g), dim3(64), 0, s, P, nbm, rho, rprev, g);
}

template <class C>
void launch_density(const Pops<C>& P, const uint32_t* nbm, const float2* rprev, float2* psi,
                    const Geo& g, int odd, hipStream_t s) {
    const TileGrid T = tiles(g);
    if (odd)
        hipLaunchKernelGGL((k_density<C, true>), dim3(T.grid), dim3(TX, TY), 0, s, P, nbm, rprev, psi, g, T);
    else
        hipLaunchKernelGGL((k_density<C, false>), dim3(T.grid), dim3(TX, TY), 0, s, P, nbm, rprev, psi, g, T);
}

void launch_ivsd(const int* list, const float* xil, int count, const uint32_t* nbm, float2* psi,
                 const Geo& g, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_ivsd, dim3((count + 255) / 256), dim3(256), 0, s, list, xil, count, nbm, psi,
                       g);
}

template <class C>
void launch_collide_stream(const Pops<C>& P, const Pops<C>& D, const uint32_t* nbm, const float2* rprev,
                           const float2* psi, const Geo& g, const Phys& ph, int odd, hipStream_t s) {
    const TileGrid T = tiles(g);
    if (odd)
        hipLaunchKernelGGL((k_collide_stream<C, true>), dim3(T.grid), dim3(TX, TY), 0, s, P, D, nbm, rprev,
                           psi, g, ph, T);
    else
        hipLaunchKernelGGL((k_collide_stream<C, false>), dim3(T.grid), dim3(TX, TY), 0, s, P, D, nbm, rprev,
                           psi, g, ph, T);
}

int fields_blocks(const Geo& g) {
    const dim3 gr = tile_grid3(g);
    return (int)(gr.x * gr.y * gr.z);
}

template <class C>
void launch_fields(const Pops<C>& P, const uint32_t* nbm, const float2* rprev, const float2* psi,
                   const Geo& g, const Phys& ph, int odd, float* o_rho, float* o_u, float* o_F,
                   float* o_P, double* partial, double* out, hipStream_t s) {
    if (odd)
        hipLaunchKernelGGL((k_fields<C, true>), tile_grid3(g), dim3(TX, TY), 0, s, P, nbm, rprev, psi, g, ph,
                           o_rho, o_u, o_F, o_P, partial);
    else
        hipLaunchKernelGGL((k_fields<C, false>), tile_grid3(g), dim3(TX, TY), 0, s, P, nbm, rprev, psi, g, ph,
                           o_rho, o_u, o_F, o_P, partial);
    if (partial)
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(1024), 0, s, (const double*)partial,
                           fields_blocks(g), out);
}

#define MCLBM_INSTANTIATE(C)                                                                           \
    template void launch_init<C>(const Pops<C>&, const uint32_t*, const float*, float2*, const Geo&,   \
                                 hipStream_t);                                                         \
    template void launch_density<C>(const Pops<C>&, const uint32_t*, const float2*, float2*,           \
                                    const Geo&, int, hipStream_t);                                     \
    template void launch_collide_stream<C>(const Pops<C>&, const Pops<C>&, const uint32_t*,            \
                                           const float2*, const float2*, const Geo&, const Phys&, int, \
                                           hipStream_t);                                               \
    template void launch_fields<C>(const Pops<C>&, const uint32_t*, const float2*, const float2*,      \
                                   const Geo&, const Phys&, int, float*, float*, float*, float*,       \
                                   double*, double*, hipStream_t);

MCLBM_INSTANTIATE(CodecF32)
MCLBM_INSTANTIATE(CodecF16)
MCLBM_INSTANTIATE(CodecBF16)

}  // namespace mclbm
