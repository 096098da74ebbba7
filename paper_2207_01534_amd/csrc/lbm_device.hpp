// Device-side building blocks of the two-component D3Q19 step for gfx950:
// the velocity set, the population storage codecs, and the single-buffer
// (AA-pattern) addressing with halfway bounce-back.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mclbm {

constexpr int Q = 19;

// D3Q19 (Sec. 2, the velocity set listed under Eq. 2), numbered so that each
// moving direction sits next to its opposite: 2k-1 and 2k are opposite for
// k = 1..9.  Directions 1..6 are the axis links (weight 1/18), 7..18 the
// edge diagonals (weight 1/36), 0 is the rest population (weight 1/3).
constexpr int DX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int DY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int DZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__host__ __device__ constexpr float weight(int i) {
    return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Bit layout of the per-node neighbourhood word: bit 0 = the node itself is
// solid, bit i (1..18) = the neighbour x + e_i is solid.
constexpr uint32_t SELF_SOLID = 1u;
constexpr uint32_t NB_BITS = ((1u << Q) - 1u) & ~1u;

struct Geo {
    int nx, ny, nz;
    int n;        // nx * ny * nz (< 2^31)
    int np;       // population plane stride in elements (>= n)
};

__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// Storage codecs.  Moving populations (i = 1..18) are stored in type T; the
// rest population of each component always stays FP32.
//   F32:  stored value = f.
//   F16 / BF16: stored value q = f / rho_w - w_i, where rho_w is the density
//         (at the previous time level) of the node that wrote the value; the
//         decoder multiplies back with the same FP32 rho_w.
// ---------------------------------------------------------------------------
struct CodecF32 {
    using T = float;
    static constexpr bool kRef = false;
    __device__ static __forceinline__ float dec(T h, float, float) { return h; }
    __device__ static __forceinline__ T enc(float f, float, float) { return f; }
};

struct CodecF16 {
    using T = __half;
    static constexpr bool kRef = true;
    __device__ static __forceinline__ float dec(T h, float w, float rho_w) {
        return (__half2float(h) + w) * rho_w;
    }
    __device__ static __forceinline__ T enc(float f, float w, float inv_rho) {
        return __float2half_rn(f * inv_rho - w);
    }
};

struct CodecBF16 {
    using T = __hip_bfloat16;
    static constexpr bool kRef = true;
    __device__ static __forceinline__ float dec(T h, float w, float rho_w) {
        return (__bfloat162float(h) + w) * rho_w;
    }
    __device__ static __forceinline__ T enc(float f, float w, float inv_rho) {
        return __float2bfloat16(f * inv_rho - w);
    }
};

// Population storage: 36 moving planes of T (component-major, direction
// 1..18) followed, elsewhere in the workspace, by 2 FP32 rest planes.
template <class C>
struct Pops {
    typename C::T* mv;
    float* rest;
    __device__ __forceinline__ typename C::T* plane(int s, int i, int np) const {
        return mv + (size_t)(s * (Q - 1) + (i - 1)) * (size_t)np;
    }
};

// Wrapped coordinates of a node and its 26 neighbours' linear indices are
// assembled from three wrapped x, y and z coordinates.
struct Nbr {
    int xs[3], ys[3], zs[3];  // index 0: -1, 1: 0, 2: +1
    int nx, nxy;
    __device__ __forceinline__ Nbr(int x, int y, int z, const Geo& g) {
        xs[0] = wrap1(x - 1, g.nx); xs[1] = x; xs[2] = wrap1(x + 1, g.nx);
        ys[0] = wrap1(y - 1, g.ny); ys[1] = y; ys[2] = wrap1(y + 1, g.ny);
        zs[0] = wrap1(z - 1, g.nz); zs[1] = z; zs[2] = wrap1(z + 1, g.nz);
        nx = g.nx;
        nxy = g.nx * g.ny;
    }
    // index of x + s * e_i  (s = +1 or -1)
    __device__ __forceinline__ int at(int i, int s) const {
        return xs[1 + s * DX[i]] + nx * ys[1 + s * DY[i]] + nxy * zs[1 + s * DZ[i]];
    }
    __device__ __forceinline__ int self() const { return xs[1] + nx * ys[1] + nxy * zs[1]; }
};

// ---------------------------------------------------------------------------
// AA-pattern single-buffer addressing.  The state at an even time level keeps
// f_i(x) in slot (i, x).  An even step reads slots (i, x) and writes the
// post-collision f*_i(x) into slot (opp i, x); an odd step reads f_i(x) from
// slot (opp i, x - e_i) -- or from slot (i, x) when x - e_i is solid
// (bounce-back) -- and writes f*_i(x) into slot (i, x + e_i) -- or into slot
// (opp i, x) when x + e_i is solid.  Each thread reads exactly the slots it
// later writes, so the update is race-free in place.
// The node that wrote the value read as f_i(x) is x - e_i if that node is
// fluid and x itself otherwise, in both parities.
// ---------------------------------------------------------------------------
struct ReadSlot {
    int dir;     // direction plane to read
    int idx;     // node index of the slot
    int writer;  // node whose density normalised the stored value
};

__device__ __forceinline__ ReadSlot read_slot(int i, bool odd, uint32_t nbm, const Nbr& nb) {
    const int self = nb.self();
    const bool src_solid = (nbm >> opp(i)) & 1u;
    const int src = nb.at(i, -1);
    ReadSlot r;
    r.writer = src_solid ? self : src;
    if (!odd) {
        r.dir = i;
        r.idx = self;
    } else if (src_solid) {
        r.dir = i;
        r.idx = self;
    } else {
        r.dir = opp(i);
        r.idx = src;
    }
    return r;
}

struct WriteSlot {
    int dir;
    int idx;
};

__device__ __forceinline__ WriteSlot write_slot(int i, bool odd, uint32_t nbm, const Nbr& nb) {
    const int self = nb.self();
    WriteSlot w;
    if (!odd) {
        w.dir = opp(i);
        w.idx = self;
    } else if ((nbm >> i) & 1u) {
        w.dir = opp(i);
        w.idx = self;
    } else {
        w.dir = i;
        w.idx = nb.at(i, +1);
    }
    return w;
}

// Load and decode the 19 incoming populations of both components at a fluid
// node.  rprev: densities of the previous time level (used by F16/BF16 only).
template <class C>
__device__ __forceinline__ void load_node(float (&f)[2][Q], const Pops<C>& P, const float2* rprev,
                                          bool odd, uint32_t nbm, const Nbr& nb, int np) {
    const int self = nb.self();
    f[0][0] = P.rest[self];
    f[1][0] = P.rest[(size_t)np + self];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const ReadSlot r = read_slot(i, odd, nbm, nb);
        const typename C::T h0 = P.plane(0, r.dir, np)[r.idx];
        const typename C::T h1 = P.plane(1, r.dir, np)[r.idx];
        if constexpr (C::kRef) {
            const float2 rw = rprev[r.writer];
            f[0][i] = C::dec(h0, weight(i), rw.x);
            f[1][i] = C::dec(h1, weight(i), rw.y);
        } else {
            f[0][i] = C::dec(h0, weight(i), 1.0f);
            f[1][i] = C::dec(h1, weight(i), 1.0f);
        }
    }
}

// Sum of populations in a fixed order (shared by every kernel that needs the
// density, so all of them produce the same bits).
__device__ __forceinline__ float sum19(const float (&f)[Q]) {
    float a = f[0];
#pragma unroll
    for (int i = 1; i < Q; ++i) a += f[i];
    return a;
}

// Encode and store the post-collision moving populations of one fluid node;
// the rest population is set from the node's mass balance,
//   f*_0 = rho - sum_{i>=1} decode(encode(f*_i)),
// which equals the collided rest population in exact arithmetic (the
// collision conserves rho^(sigma) and the weights sum to 1) and keeps the
// stored mass equal to rho to FP32 round-off: no bias from the FP32 weights
// not summing exactly to 1, and the FP16/BF16 rounding of the moving
// populations is absorbed by the FP32 rest population.
// mass: incoming component densities; rho_ref: this node's density as the
// decoder will read it next step (used by the F16/BF16 codecs only).
template <class C>
__device__ __forceinline__ void store_node(const float (&fs)[2][Q], const Pops<C>& P, const float (&mass)[2],
                                           float2 rho_ref, bool odd, uint32_t nbm, const Nbr& nb,
                                           int np) {
    const int self = nb.self();
    float sum0 = 0.0f, sum1 = 0.0f;
    float inv0 = 1.0f, inv1 = 1.0f;
    if constexpr (C::kRef) {
        inv0 = rho_ref.x > 0.0f ? 1.0f / rho_ref.x : 0.0f;
        inv1 = rho_ref.y > 0.0f ? 1.0f / rho_ref.y : 0.0f;
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const WriteSlot w = write_slot(i, odd, nbm, nb);
        const typename C::T h0 = C::enc(fs[0][i], weight(i), inv0);
        const typename C::T h1 = C::enc(fs[1][i], weight(i), inv1);
        P.plane(0, w.dir, np)[w.idx] = h0;
        P.plane(1, w.dir, np)[w.idx] = h1;
        sum0 += C::dec(h0, weight(i), rho_ref.x);
        sum1 += C::dec(h1, weight(i), rho_ref.y);
    }
    P.rest[self] = mass[0] - sum0;
    P.rest[(size_t)np + self] = mass[1] - sum1;
}

// Physical parameters in FP32.
struct Phys {
    float a[2];     // tau^(sigma) - 1/2
    float G;        // G_coh
    float g[2][3];  // body acceleration per component
};

// Forced SRT collision at one node (Eqs. 1, 2, 6-9), in place on the moving
// populations f[s][1..18]; the rest population follows from mass balance in
// store_node.  F: total force per component (Eq. 10).  Returns u through uo.
__device__ __forceinline__ void collide(float (&f)[2][Q], const float (&rho)[2], const float (&F)[2][3],
                                        const Phys& ph, float (&uo)[3]) {
    float j[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (DX[i]) j[0] += DX[i] * f[s][i];
            if (DY[i]) j[1] += DY[i] * f[s][i];
            if (DZ[i]) j[2] += DZ[i] * f[s][i];
        }
    const float rt = rho[0] + rho[1];
    const float inv_rt = 1.0f / rt;
    // common velocity with the half-force shift (Eq. 8, Guo forcing)
    const float ux = (j[0] + 0.5f * (F[0][0] + F[1][0])) * inv_rt;
    const float uy = (j[1] + 0.5f * (F[0][1] + F[1][1])) * inv_rt;
    const float uz = (j[2] + 0.5f * (F[0][2] + F[1][2])) * inv_rt;
    uo[0] = ux; uo[1] = uy; uo[2] = uz;
    // mixture relaxation time (Eqs. 6-7 with nu = c_s^2 (tau - 1/2))
    const float tau_s = (rho[0] * ph.a[0] + rho[1] * ph.a[1]) * inv_rt + 0.5f;
    const float om = 1.0f / tau_s;
    const float cf = 1.0f - 0.5f * om;
    const float usq15 = 1.5f * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const float uF = ux * F[s][0] + uy * F[s][1] + uz * F[s][2];
        const float r = rho[s];
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const float eu = DX[i] * ux + DY[i] * uy + DZ[i] * uz;
            const float eF = DX[i] * F[s][0] + DY[i] * F[s][1] + DZ[i] * F[s][2];
            const float feq = weight(i) * r * (1.0f + 3.0f * eu + 4.5f * eu * eu - usq15);
            const float S = weight(i) * (3.0f * (eF - uF) + 9.0f * eu * eF);
            f[s][i] = f[s][i] - om * (f[s][i] - feq) + cf * S;
        }
    }
}

// Pseudopotential force sum sum_{i>=1} w_i psi(x + e_i) e_i for both
// components, with psi supplied by a functor psi_at(i) -> float2.
template <class PsiAt>
__device__ __forceinline__ void psi_sum(PsiAt psi_at, float (&acc)[2][3]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) acc[s][0] = acc[s][1] = acc[s][2] = 0.0f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const float2 p = psi_at(i);
        const float w = weight(i);
        if (DX[i]) { acc[0][0] += (w * DX[i]) * p.x; acc[1][0] += (w * DX[i]) * p.y; }
        if (DY[i]) { acc[0][1] += (w * DY[i]) * p.x; acc[1][1] += (w * DY[i]) * p.y; }
        if (DZ[i]) { acc[0][2] += (w * DZ[i]) * p.x; acc[1][2] += (w * DZ[i]) * p.y; }
    }
}

// Total force per component (Eqs. 10, 11, 13): the other component's psi
// acts on this one; F^b = rho g.
__device__ __forceinline__ void total_force(const float (&rho)[2], const float (&acc)[2][3],
                                            const Phys& ph, float (&F)[2][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        F[0][a] = -ph.G * rho[0] * acc[1][a] + rho[0] * ph.g[0][a];
        F[1][a] = -ph.G * rho[1] * acc[0][a] + rho[1] * ph.g[1][a];
    }
}

}  // namespace mclbm
