// Open inlet/outlet planes along x (Sec. 2, the inlet and outlet conditions;
// Sec. 4.1, the drainage drive).
//
// The lattice keeps its x extent; planes x = 0 and x = nx-1 become ghost
// planes outside the physical domain, the physical inlet is x = 1 and the
// outlet x = nx-2.  The step kernels run unchanged (periodic in x) and two
// thin-plane kernels make the planes open:
//   k_open_mirror   after the pseudopotential field is complete: the ghost
//                   planes take psi-hat of the mirror image of the boundary
//                   plane's missing neighbours, psi(0) = psi(2) and
//                   psi(nx-1) = psi(nx-3), so the force sums at x = 1 and
//                   x = nx-2 see the pairing printed after Eq. (11);
//   k_open_rebuild  after collision and streaming, per boundary node x_b:
//                   non-equilibrium extrapolation (NEEM) of the imposed
//                   component from x_f = x_b +- 1 (component 1 to rho_in at
//                   the inlet, component 2 to rho_out at the outlet),
//                     f_i(x_b) = f_i(x_f) + feq_i(rho_b, u_f) - feq_i(rho_f, u_f),
//                   u_f the bare barycentric velocity at x_f; the other
//                   component's entering populations (e_x = +1 at the inlet,
//                   -1 at the outlet) take their held values.  Whatever the
//                   ghost planes streamed into the boundary planes is thereby
//                   replaced; the ghost nodes themselves are reset to rest
//                   equilibrium at their mirrored densities so they stay finite.
// Planes 0, 1, 2, nx-3, nx-2 and nx-1 must be fluid (checked on the host).
#include "lbm_open.hpp"
#include "lbm_tiles.hpp"

namespace mclbm {

// Slot of f_i(x) at a time level of the given parity (AA pattern, see
// lbm_device.hpp): the plane's direction index and the fluid id.  Also
// returns the node whose density normalised the stored value (F16/BF16).
struct OpenSlot {
    int dir;
    uint32_t id;
    uint32_t writer;
};

__device__ __forceinline__ OpenSlot slot_of(int i, bool odd, uint32_t k, uint32_t m, const Nb& nb,
                                            const int* __restrict__ fid) {
    const bool up_solid = (m >> opp(i)) & 1u;  // x - e_i solid
    OpenSlot s;
    s.writer = up_solid ? nb.idx : nb.at(i, -1);
    if (!odd || up_solid) {
        s.dir = i;
        s.id = k;
    } else {
        s.dir = opp(i);
        s.id = (uint32_t)fid[nb.at(i, -1)];
    }
    return s;
}

// Value of f_i(x) of component s stored in slot q, decoded with the codec
// predictor of the value as read at x (pred_read) from the previous level's
// pseudopotential field psi (F16/BF16 only).
template <class C>
__device__ __forceinline__ float read_pop(const Pops<C>& P, int s, const OpenSlot& q, int i, uint32_t m,
                                          const Nb& nb, const float2* psi, float G, int np) {
    const typename C::T h = *P.at(s, q.dir, q.id, np);
    if constexpr (C::kRef) {
        auto psi_rel = [&](int dx, int dy, int dz) {
            return ld(psi, nb.idx + (uint32_t)(nb.ox[1 + dx] + nb.oy[1 + dy] + nb.oz[1 + dz]));
        };
        const PredRef r = pred_read(i, (bool)((m >> opp(i)) & 1u), psi_rel, G);
        return C::dec(h, s ? r.p.y : r.p.x, r.rt);
    } else {
        return C::dec(h, 0.0f, 0.0f);
    }
}

// Eq. (2) at one direction.
__device__ __forceinline__ float feq(int i, float rho, const float (&u)[3], float usq) {
    const float eu = DX[i] * u[0] + DY[i] * u[1] + DZ[i] * u[2];
    return weight(i) * rho * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * usq);
}

__global__ void k_open_mirror(float2* __restrict__ psi, Geo g) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= g.ny * g.nz) return;
    const uint32_t row = (uint32_t)a * (uint32_t)g.nx;
    psi[row] = psi[row + 2];
    psi[row + g.nx - 1] = psi[row + g.nx - 3];
}

// Rebuild launch shape: one thread per (y, z) row and side, a block of
// 256 threads per 16 x 16 patch of rows of one side, patches dealt to the
// XCDs in contiguous runs (active_of_block).  A row's three nodes (ghost,
// boundary, next inwards) sit in consecutive slots of every direction plane,
// and at odd levels their slots are addressed through the fluid ids of the
// rows next to it; the block stages those ids once in LDS (five x positions
// over the patch and a one-row halo in y and z), with the F16/BF16 codecs
// also the previous-level densities that decode and encode each slot, and
// every slot moves both components in one access where both are read or
// written.
constexpr int OPEN_PATCH = 16;
constexpr int OPEN_XS = 5, OPEN_H = OPEN_PATCH + 2;

__host__ __device__ inline int open_patches(const Geo& g) {
    return ((g.ny + OPEN_PATCH - 1) / OPEN_PATCH) * ((g.nz + OPEN_PATCH - 1) / OPEN_PATCH);
}

// Slot of f_i at staged x position k of the thread's row (AA pattern): the
// direction plane, the fluid id, and whether x - e_i is solid (fluid id -1).
struct StagedSlot {
    int dir;
    uint32_t id;
    bool up_solid;
};

__device__ __forceinline__ StagedSlot staged_slot(int i, bool odd, int k, int ly, int lz,
                                                  const int (&sf)[OPEN_XS][OPEN_H][OPEN_H]) {
    const int own = sf[k][lz + 1][ly + 1];
    const int up = sf[k - DX[i]][lz + 1 - DZ[i]][ly + 1 - DY[i]];
    StagedSlot q;
    q.up_solid = up < 0;
    q.dir = (!odd || q.up_solid) ? i : opp(i);
    q.id = (uint32_t)((!odd || q.up_solid) ? own : up);
    return q;
}

// Codec predictor and scale of f_i as read at staged x position k of the
// thread's row (pred_read over the block's staged copy of the previous
// level's pseudopotential field; F16/BF16 only).
struct CodecRef {
    float p[2], rt, inv;
};

template <class C, class Staged>
__device__ __forceinline__ CodecRef codec_ref(const Staged& sr, int k, int ly, int lz, int i, bool up_solid,
                                              float G) {
    CodecRef c{{0.f, 0.f}, 0.f, 0.f};
    if constexpr (C::kRef) {
        auto psi_rel = [&](int dx, int dy, int dz) { return sr[k + dx][lz + 1 + dz][ly + 1 + dy]; };
        const PredRef r = pred_read(i, up_solid, psi_rel, G);
        c.p[0] = r.p.x;
        c.p[1] = r.p.y;
        c.rt = r.rt;
        c.inv = r.rt > 0.0f ? 1.0f / r.rt : 0.0f;
    }
    return c;
}

// odd: parity of the time level the populations are at (the one just
// reached); psi: densities of the level before, the codec reference of every
// value written in the last step.
template <class C>
__global__ void __launch_bounds__(OPEN_PATCH * OPEN_PATCH)
k_open_rebuild(Pops<C> P, const int* __restrict__ fid, const float2* __restrict__ psi,
               const float* __restrict__ held, Geo g, int odd, float rho_in, float rho_out, float G) {
    using T = typename C::T;
    using P2 = Pair<T>;
    __shared__ int sf[OPEN_XS][OPEN_H][OPEN_H];   // [x position][z][y]
    __shared__ float2 sr[C::kRef ? OPEN_XS : 1][OPEN_H][OPEN_H];   // codec references, same positions
    const int npatch = open_patches(g);
    const int b = active_of_block(2 * npatch);
    if (b < 0) return;                             // uniform over the block
    const int side = b >= npatch ? 1 : 0;
    const int p = b - side * npatch, pyn = (g.ny + OPEN_PATCH - 1) / OPEN_PATCH;
    const int y0 = (p % pyn) * OPEN_PATCH, z0 = (p / pyn) * OPEN_PATCH;
    // staged x positions k = 0..4: x = -1..3 (inlet) or nx-4..nx (outlet), periodic
    const int xbase = side ? g.nx - 4 : g.nx - 1;
    for (int e = threadIdx.x; e < OPEN_XS * OPEN_H * OPEN_H; e += blockDim.x) {
        const int k = e % OPEN_XS, r = e / OPEN_XS;
        const int hy = r % OPEN_H, hz = r / OPEN_H;
        const int x = (xbase + k) % g.nx;
        const int y = (y0 - 1 + hy + g.ny) % g.ny, z = (z0 - 1 + hz + g.nz) % g.nz;
        const uint32_t idx = (uint32_t)x + (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
        sf[k][hz][hy] = fid[idx];
        if constexpr (C::kRef) sr[k][hz][hy] = ld(psi, idx);
    }
    __syncthreads();
    const int ly = (int)(threadIdx.x % OPEN_PATCH), lz = (int)(threadIdx.x / OPEN_PATCH);
    const int y = y0 + ly, z = z0 + lz;
    if (y >= g.ny || z >= g.nz) return;
    const int A = g.ny * g.nz;
    const int yz = y + g.ny * z;
    const int kf = side ? 1 : 3, kb = 2, kg = side ? 3 : 1;   // staged positions of x_f, x_b, x_g
    const int imposed = side, other = 1 - side, dir_in = side ? -1 : 1;
    const float rho_b = side ? rho_out : rho_in;
    const int np = g.np;
    const Nb ng(side ? g.nx - 1 : 0, y, z, g);

    // populations of x_f at the new level
    float ff[2][Q];
    {
        const Pair<float> r = ld(P.rests(), (uint32_t)sf[kf][lz + 1][ly + 1]);
        ff[0][0] = r.v[0];
        ff[1][0] = r.v[1];
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const StagedSlot q = staged_slot(i, odd, kf, ly, lz, sf);
        const CodecRef c = codec_ref<C>(sr, kf, ly, lz, i, q.up_solid, G);
        const P2 h = ld(P.plane(q.dir, np), q.id);
        ff[0][i] = C::dec(h.v[0], c.p[0], c.rt);
        ff[1][i] = C::dec(h.v[1], c.p[1], c.rt);
    }
    float rf[2] = {0.f, 0.f}, j[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            rf[s] += ff[s][i];
            j[0] += DX[i] * ff[s][i];
            j[1] += DY[i] * ff[s][i];
            j[2] += DZ[i] * ff[s][i];
        }
    const float inv = 1.0f / (rf[0] + rf[1]);
    const float u[3] = {j[0] * inv, j[1] * inv, j[2] * inv};
    const float usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

    // boundary node: the imposed component by NEEM; the other component's
    // entering populations from the held values (both components of those
    // slots in one store)
    const uint32_t idb = (uint32_t)sf[kb][lz + 1][ly + 1];
    float moving = 0.f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const StagedSlot q = staged_slot(i, odd, kb, ly, lz, sf);
        const CodecRef c = codec_ref<C>(sr, kb, ly, lz, i, q.up_solid, G);
        const float v = ff[imposed][i] + feq(i, rho_b, u, usq) - feq(i, rf[imposed], u, usq);
        const T hi = C::enc(v, c.p[imposed], c.inv);
        moving += C::dec(hi, c.p[imposed], c.rt);
        if (DX[i] == dir_in) {
            const float vo = held[((size_t)side * Q + i) * A + yz];
            const T ho = C::enc(vo, c.p[other], c.inv);
            P2 pr;
            pr.v[imposed] = hi;
            pr.v[other] = ho;
            st(P.plane(q.dir, np), q.id, pr);
        } else {
            *P.at(imposed, q.dir, q.id, np) = hi;
        }
    }
    *P.rest_at(imposed, idb) = rho_b - moving;   // exact imposed density

    // ghost node: rest equilibrium at its (mirrored) densities
    const float2 rg = psi[ng.idx];
    float sum[2] = {0.f, 0.f};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const StagedSlot q = staged_slot(i, odd, kg, ly, lz, sf);
        const CodecRef c = codec_ref<C>(sr, kg, ly, lz, i, q.up_solid, G);
        P2 pr;
        pr.v[0] = C::enc(weight(i) * rg.x, c.p[0], c.inv);
        pr.v[1] = C::enc(weight(i) * rg.y, c.p[1], c.inv);
        sum[0] += C::dec(pr.v[0], c.p[0], c.rt);
        sum[1] += C::dec(pr.v[1], c.p[1], c.rt);
        st(P.plane(q.dir, np), q.id, pr);
    }
    st(P.rests(), (uint32_t)sf[kg][lz + 1][ly + 1], Pair<float>{{rg.x - sum[0], rg.y - sum[1]}});
}

// Mean pressure (Eq. 12) over the fluid nodes of the inlet (x = 1) and outlet
// (x = nx-2) planes from the densities in psi; one block per side, FP64.
__global__ void k_open_pressure(const float2* __restrict__ psi, const uint32_t* __restrict__ nbm, Geo g,
                                float G, double* __restrict__ out) {
    const int side = blockIdx.x;
    const int x = side ? g.nx - 2 : 1;
    double acc = 0.0, cnt = 0.0;
    for (int a = threadIdx.x; a < g.ny * g.nz; a += blockDim.x) {
        const uint32_t idx = (uint32_t)x + (uint32_t)a * (uint32_t)g.nx;
        if (nbm[idx] & SELF_SOLID) continue;
        const float2 r = psi[idx];
        acc += (double)(r.x + r.y) / 3.0 + (double)G / 3.0 * (double)r.x * (double)r.y;
        cnt += 1.0;
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = acc;
    red[1][threadIdx.x] = cnt;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[side] = red[1][0] > 0.0 ? red[0][0] / red[1][0] : 0.0;
}

// Held populations: the current values of the entering directions at the
// boundary planes (inlet: component 2, e_x = +1; outlet: component 1, e_x = -1).
template <class C>
__global__ void k_open_capture(Pops<C> P, const int* __restrict__ fid, const uint32_t* __restrict__ nbm,
                               const float2* __restrict__ rprev, float* __restrict__ held, Geo g, int odd,
                               float G) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int A = g.ny * g.nz;
    if (a >= 2 * A) return;
    const int side = a >= A ? 1 : 0;
    const int yz = a - side * A;
    const int y = yz % g.ny, z = yz / g.ny;
    const int other = 1 - side, dir_in = side ? -1 : 1;
    const Nb nb(side ? g.nx - 2 : 1, y, z, g);
    const uint32_t kb = (uint32_t)fid[nb.idx];
    const uint32_t mb = nbm[nb.idx];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        float v = 0.f;
        if (i > 0 && DX[i] == dir_in)
            v = read_pop<C>(P, other, slot_of(i, odd, kb, mb, nb, fid), i, mb, nb, rprev, G, g.np);
        held[((size_t)side * Q + i) * A + yz] = v;
    }
}

// Number of solid nodes on planes 0, 1, 2, nx-3, nx-2, nx-1 (must be zero);
// one block of 1024 threads.
__global__ void k_open_check(const uint32_t* __restrict__ nbm, Geo g, int* __restrict__ count) {
    const int A = g.ny * g.nz;
    int total = 0;
    for (int base = 0; base < 6 * A; base += blockDim.x) {
        const int a = base + threadIdx.x;
        bool solid = false;
        if (a < 6 * A) {
            const int p = a / A, yz = a - p * A;
            const int x = p < 3 ? p : g.nx - 6 + p;
            solid = nbm[(uint32_t)x + (uint32_t)yz * (uint32_t)g.nx] & SELF_SOLID;
        }
        total += __syncthreads_count(solid);
    }
    if (threadIdx.x == 0) *count = total;
}

// ---------------------------------------------------------------------------
static unsigned blocks_for(int n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_open_mirror(float2* psi, const Geo& g, hipStream_t s) {
    hipLaunchKernelGGL(k_open_mirror, dim3(blocks_for(g.ny * g.nz, 256)), dim3(256), 0, s, psi, g);
}

template <class C>
void launch_open_rebuild(const Pops<C>& P, const int* fid, const float2* psi, const float* held, const Geo& g,
                         int odd, float rho_in, float rho_out, float G, hipStream_t s) {
    hipLaunchKernelGGL(k_open_rebuild<C>, dim3(xcd_grid(2 * open_patches(g))), dim3(OPEN_PATCH * OPEN_PATCH), 0, s,
                       P, fid, psi, held, g, odd, rho_in, rho_out, G);
}

template <class C>
void launch_open_capture(const Pops<C>& P, const int* fid, const uint32_t* nbm, const float2* rprev, float* held,
                         const Geo& g, int odd, float G, hipStream_t s) {
    hipLaunchKernelGGL(k_open_capture<C>, dim3(blocks_for(2 * g.ny * g.nz, 64)), dim3(64), 0, s, P, fid, nbm,
                       rprev, held, g, odd, G);
}

void launch_open_pressure(const float2* psi, const uint32_t* nbm, const Geo& g, float G, double* out,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_open_pressure, dim3(2), dim3(256), 0, s, psi, nbm, g, G, out);
}

void launch_open_check(const uint32_t* nbm, const Geo& g, int* count, hipStream_t s) {
    hipLaunchKernelGGL(k_open_check, dim3(1), dim3(1024), 0, s, nbm, g, count);
}

#define MCLBM_OPEN_INSTANTIATE(C)                                                                              \
    template void launch_open_rebuild<C>(const Pops<C>&, const int*, const float2*, const float*, const Geo&, \
                                         int, float, float, float, hipStream_t);                             \
    template void launch_open_capture<C>(const Pops<C>&, const int*, const uint32_t*, const float2*, float*, \
                                         const Geo&, int, float, hipStream_t);
MCLBM_OPEN_INSTANTIATE(CodecF32)
MCLBM_OPEN_INSTANTIATE(CodecF16)
MCLBM_OPEN_INSTANTIATE(CodecBF16)

}  // namespace mclbm
