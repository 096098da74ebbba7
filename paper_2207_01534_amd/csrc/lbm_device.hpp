// Device-side building blocks of the two-component D3Q19 step for gfx950:
// the velocity set, the population storage codecs, the single-buffer
// (AA-pattern) addressing with halfway bounce-back, and the per-node
// physics (forces, forced SRT collision).
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

// Per-node neighbourhood word: bit 0 = the node itself is solid, bit i
// (1..18) = the neighbour x + e_i is solid.
constexpr uint32_t SELF_SOLID = 1u;
constexpr uint32_t NB_BITS = ((1u << Q) - 1u) & ~1u;

struct Geo {
    int nx, ny, nz;
    int n;   // nx * ny * nz (< 2^30, so byte offsets of a plane fit in 32 bits)
    int np;  // population plane stride in elements (>= the fluid capacity)
};

// Loads and stores at a 32-bit element offset from a wave-uniform base, so
// that the compiler can address with a scalar base plus a 32-bit vector
// offset instead of a 64-bit address per lane.  That holds for elements of
// at most 4 bytes (offsets < 2^30 elements: lattice indices, fluid ids);
// wider elements (the float2 psi-hat and density fields, indexed by lattice
// node) scale in 64 bits, since 8 * idx passes 2^32 beyond 2^29 nodes.
template <class T>
__device__ __forceinline__ T ld(const T* base, uint32_t i) {
    if constexpr (sizeof(T) > 4)
        return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint64_t)i * sizeof(T));
    else
        return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st(T* base, uint32_t i, T v) {
    if constexpr (sizeof(T) > 4)
        *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint64_t)i * sizeof(T)) = v;
    else
        *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T)) = v;
}

// Population slots at an element offset scaled in 32 bits (NARROW: the
// caller guarantees offset * sizeof(T) < 2^32) or in 64 bits (WIDE).
template <bool WIDE, class T>
__device__ __forceinline__ T ld_pop(const T* base, uint32_t i) {
    if constexpr (WIDE)
        return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint64_t)i * sizeof(T));
    else
        return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}
template <bool WIDE, class T>
__device__ __forceinline__ void st_pop(T* base, uint32_t i, T v) {
    if constexpr (WIDE)
        *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint64_t)i * sizeof(T)) = v;
    else
        *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T)) = v;
}

// Node index and periodic neighbour offsets of one node.
struct Nb {
    uint32_t idx;
    int ox[3], oy[3], oz[3];  // offsets of the -1 / 0 / +1 neighbour along each axis
    __device__ __forceinline__ Nb(int x, int y, int z, const Geo& g) {
        const int nxy = g.nx * g.ny;
        idx = (uint32_t)(x + g.nx * y + nxy * z);
        ox[0] = x == 0 ? g.nx - 1 : -1;
        ox[1] = 0;
        ox[2] = x == g.nx - 1 ? 1 - g.nx : 1;
        oy[0] = (y == 0 ? g.ny - 1 : -1) * g.nx;
        oy[1] = 0;
        oy[2] = (y == g.ny - 1 ? 1 - g.ny : 1) * g.nx;
        oz[0] = (z == 0 ? g.nz - 1 : -1) * nxy;
        oz[1] = 0;
        oz[2] = (z == g.nz - 1 ? 1 - g.nz : 1) * nxy;
    }
    // index of x + s e_i (s = +1 or -1)
    __device__ __forceinline__ uint32_t at(int i, int s) const {
        return idx + (uint32_t)(ox[1 + s * DX[i]] + oy[1 + s * DY[i]] + oz[1 + s * DZ[i]]);
    }
};

// ---------------------------------------------------------------------------
// Storage codecs.  Moving populations (i = 1..18) are stored in type T; the
// rest population of each component always stays FP32.
//   F32:  stored value = f.
//   F16 / BF16: stored value q = (f - p) / rhot_w, the deviation of the
//         population from a predictor p of it, scaled by the total density
//         rhot_w = rho1 + rho2 of the node that wrote it.  The predictor and
//         the scale come from the writer's state at the previous time level
//         as both the writing and the reading kernels see it (the
//         pseudopotential field of that level, below), so they are the same
//         numbers on both sides; the decoder evaluates f = q rhot_w + p with
//         one explicit FMA and the encoder's mass balance uses the same
//         expression, so encoder and decoder agree bit for bit.  Scaling by
//         the total density keeps q bounded where one component's density
//         vanishes.
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
    __device__ static __forceinline__ float dec(T h, float pred, float rhot_w) {
        return fmaf(__half2float(h), rhot_w, pred);
    }
    __device__ static __forceinline__ T enc(float f, float pred, float inv_rhot_w) {
        return __float2half_rn((f - pred) * inv_rhot_w);
    }
};

struct CodecBF16 {
    using T = __hip_bfloat16;
    static constexpr bool kRef = true;
    __device__ static __forceinline__ float dec(T h, float pred, float rhot_w) {
        return fmaf(__bfloat162float(h), rhot_w, pred);
    }
    __device__ static __forceinline__ T enc(float f, float pred, float inv_rhot_w) {
        return __float2bfloat16((f - pred) * inv_rhot_w);
    }
};

// ---------------------------------------------------------------------------
// Codec predictors (F16/BF16).  The post-collision population f*_j^(s) of a
// node departs from its lattice-weight share w_j rho^(s) mostly through its
// first moment, and at interfaces and walls that moment is dominated by the
// component's own force: the cohesion and adhesion of Eqs. (11) and (13)
// push component s down the gradient of the other component's
// pseudopotential psi^(s'), and the Guo source of Eq. (9) with the half-force
// shift puts about 3/2 w_j e_j.F^(s) into direction j.  Storing the deviation
// from a predictor that follows this gradient leaves a much smaller number to
// round.  Only the previous level's pseudopotential field psi-hat (rho at
// fluid nodes, the virtual density of Eq. 15 at solid ones) is common to the
// writer and all its readers, so the predictor uses nothing else:
//   p^(s) = w_j rho^(s)(x) (1 - (G/4) D_j^(s')),
// x the writing node, j the direction it writes, and D_j the difference of
// psi^(s') along e_j:
//   D_j = psi(x + e_j) - psi(x)        when x + e_j is fluid (the value
//                                      streams there; both ends are within
//                                      one link of the reader),
//   D_j = psi(x + e_j) - psi(x - e_j)  when x + e_j is solid (the value comes
//                                      back to x by bounce-back and only x
//                                      reads it, so the central difference
//                                      across the wall is available).
// The factor 1/4 was chosen by measuring the stored error against the FP64
// reference on porous and droplet cases.  Contraction is off here so every
// kernel evaluates the predictor with the same roundings.
// ---------------------------------------------------------------------------
struct PredRef {
    float2 p;   // predictor of both components
    float rt;   // writer's total density (the scale)
};

// Predictor of a value written by x along direction j: rw = psi-hat(x), d =
// the difference D_j of psi-hat (both components; component s uses the
// other one's).
__device__ __forceinline__ float2 pred_value(int j, float2 rw, float2 d, float G) {
#pragma clang fp contract(off)
    const float kG = 0.25f * G;
    const float m0 = fmaf(-kG, d.y, 1.0f);
    const float m1 = fmaf(-kG, d.x, 1.0f);
    return make_float2(weight(j) * rw.x * m0, weight(j) * rw.y * m1);
}

__device__ __forceinline__ float2 psi_diff(float2 a, float2 b) {
#pragma clang fp contract(off)
    return make_float2(a.x - b.x, a.y - b.y);
}

// Predictor and scale of f_i as read at x: the value was written by x - e_i
// along i, or, when x - e_i is solid (wall), by x itself along opp(i) (same
// weight) and bounced back.  psi_rel(dx, dy, dz) = previous-level psi-hat at
// x + (dx, dy, dz).  Both neighbours are read and the cases selected without
// branches.
template <class PsiRel>
__device__ __forceinline__ PredRef pred_read(int i, bool wall, PsiRel psi_rel, float G) {
    const float2 own = psi_rel(0, 0, 0);
    const float2 up = psi_rel(-DX[i], -DY[i], -DZ[i]);
    const float2 dn = psi_rel(DX[i], DY[i], DZ[i]);
    const float2 rw = make_float2(wall ? own.x : up.x, wall ? own.y : up.y);
    const float2 a = make_float2(wall ? up.x : own.x, wall ? up.y : own.y);
    const float2 b = make_float2(wall ? dn.x : up.x, wall ? dn.y : up.y);
    return PredRef{pred_value(i, rw, psi_diff(a, b), G), rw.x + rw.y};
}

// Predictor of f*_i written by x (direction i); wall: x + e_i is solid.  The
// same expressions as pred_read at the reader.
template <class PsiRel>
__device__ __forceinline__ float2 pred_write(int i, bool wall, PsiRel psi_rel, float G) {
    const float2 own = psi_rel(0, 0, 0);
    const float2 dn = psi_rel(DX[i], DY[i], DZ[i]);
    const float2 up = psi_rel(-DX[i], -DY[i], -DZ[i]);
    const float2 other = make_float2(wall ? up.x : own.x, wall ? up.y : own.y);
    return pred_value(i, own, psi_diff(dn, other), G);
}

__device__ __forceinline__ float inv_total(float2 r) {
    const float t = r.x + r.y;
    return t > 0.0f ? 1.0f / t : 0.0f;
}

// One population of both components (same direction, same slot), stored
// next to each other so that one load or store moves both.
template <class T>
struct alignas(2 * sizeof(T)) Pair {
    T v[2];
};

// Population storage: 18 moving planes (directions 1..18) of component pairs
// in the codec's type, and one plane of FP32 rest-population pairs; each plane
// is np slots long and indexed by fluid id.
template <class C>
struct Pops {
    typename C::T* mv;
    float* rest;
    using P2 = Pair<typename C::T>;
    __device__ __forceinline__ P2* plane(int i, int np) const {
        return reinterpret_cast<P2*>(mv) + (size_t)(i - 1) * (size_t)np;
    }
    __device__ __forceinline__ Pair<float>* rests() const { return reinterpret_cast<Pair<float>*>(rest); }
    // component s of direction i at slot k
    __device__ __forceinline__ typename C::T* at(int s, int i, uint32_t k, int np) const {
        return plane(i, np)[k].v + s;
    }
    __device__ __forceinline__ float* rest_at(int s, uint32_t k) const { return rests()[k].v + s; }
};

// Slot offsets reach 2 np pairs (odd steps address a pair of planes from the
// lower one) of at most 8 bytes: 32-bit byte offsets hold while 16 np < 2^32.
inline bool pops_wide(int np) { return (uint64_t)16 * (uint64_t)np >= (1ull << 32); }

// ---------------------------------------------------------------------------
// Tile-sparse AA-pattern streaming with halfway bounce-back.
// Only fluid nodes own populations: fluid node k (its fluid id) owns slot
// (i, k) of each direction plane, which holds f_i of both components side by
// side, so every slot access moves the two components in one load or store.
// The state at an even time level keeps f_i(x) in
// slot (i, k(x)); at an odd level f_i(x) sits in slot (opp i, k(x - e_i)) if
// x - e_i is fluid and in (i, k(x)) otherwise (the bounced population).
//   even step at fluid x: read slots (i, k); write f*_i(x) to (opp i, k);
//   odd step at fluid x:  read (opp i, k(x - e_i)) or, across a wall, (i, k);
//     write f*_i(x) to (i, k(x + e_i)) or, across a wall, to (opp i, k).
// Each thread reads exactly the slots it later writes, so the update is
// race-free in place, and an even step touches no other node's slots.  The
// same code runs out of place (separate source and destination buffers).
// The node whose density normalised the value read as f_i(x) (F16/BF16) is
// x - e_i if that node is fluid and x itself otherwise, in both parities.
// FidAt(i, s) returns the fluid id of x + s e_i, or -1 if it is solid.
// ---------------------------------------------------------------------------

// Stored values of the 19 incoming populations of both components at one
// fluid node: the moving ones in the codec's type, the rest ones in FP32.
template <class C>
struct RawNode {
    typename C::T h[2][Q];  // h[.][0] unused
    float rest[2];
};

// Issue the loads of fluid node k's incoming populations (no decoding).
template <class C, bool ODD, bool WIDE, class FidAt>
__device__ __forceinline__ void load_raw(RawNode<C>& r, const Pops<C>& P, uint32_t k, FidAt fid_at, int np) {
    const Pair<float> rp = ld_pop<WIDE>(P.rests(), k);
    r.rest[0] = rp.v[0];
    r.rest[1] = rp.v[1];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if constexpr (!ODD) {
            const typename Pops<C>::P2 p = ld_pop<WIDE>(P.plane(i, np), k);
            r.h[0][i] = p.v[0];
            r.h[1][i] = p.v[1];
        } else {
            // slot (opp i, src) or, across a wall, (i, k); directions 2k-1, 2k
            // have adjacent planes, so both are one offset from the lower one
            const int src = fid_at(i, -1);
            const bool wall = src < 0;
            const int lo = (i & 1) ? i : i - 1;
            const uint32_t e = wall ? k + ((i & 1) ? 0u : (uint32_t)np) : (uint32_t)src + ((i & 1) ? (uint32_t)np : 0u);
            const typename Pops<C>::P2 p = ld_pop<WIDE>(P.plane(lo, np), e);
            r.h[0][i] = p.v[0];
            r.h[1][i] = p.v[1];
        }
    }
}

// Decode a loaded node.  PredAt(i, wall) returns the codec predictor and
// scale of f_i(x) (pred_read; wall: x - e_i is solid), F16/BF16 only; nbm is
// the node's neighbourhood word.
template <class C, class PredAt>
__device__ __forceinline__ void decode_node(float (&f)[2][Q], const RawNode<C>& r, uint32_t nbm, PredAt pred_at) {
    f[0][0] = r.rest[0];
    f[1][0] = r.rest[1];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if constexpr (C::kRef) {
            const PredRef q = pred_at(i, (bool)((nbm >> opp(i)) & 1u));
            f[0][i] = C::dec(r.h[0][i], q.p.x, q.rt);
            f[1][i] = C::dec(r.h[1][i], q.p.y, q.rt);
        } else {
            f[0][i] = C::dec(r.h[0][i], 0.0f, 0.0f);
            f[1][i] = C::dec(r.h[1][i], 0.0f, 0.0f);
        }
    }
}

// Load and decode the 19 incoming populations of both components at fluid
// node k, with the previous-level pseudopotential read from the dense field
// rprev (F16/BF16 only).
template <class C, bool ODD, class FidAt>
__device__ __forceinline__ void load_node(float (&f)[2][Q], const Pops<C>& P, const float2* rprev,
                                          uint32_t nbm, const Nb& nb, uint32_t k, FidAt fid_at, int np, float G) {
    RawNode<C> r;
    load_raw<C, ODD, true>(r, P, k, fid_at, np);
    if constexpr (C::kRef) {
        auto psi_rel = [&](int dx, int dy, int dz) {
            return ld(rprev, nb.idx + (uint32_t)(nb.ox[1 + dx] + nb.oy[1 + dy] + nb.oz[1 + dz]));
        };
        decode_node<C>(f, r, nbm, [&](int i, bool wall) { return pred_read(i, wall, psi_rel, G); });
    } else {
        decode_node<C>(f, r, nbm, [&](int, bool) { return PredRef{make_float2(0.f, 0.f), 0.f}; });
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

// Encode and store the post-collision moving populations of fluid node k;
// the rest population is set from the node's mass balance,
//   f*_0 = rho - sum_{i>=1} decode(encode(f*_i)),
// which equals the collided rest population in exact arithmetic (the
// collision conserves rho^(sigma) and the weights sum to 1) and keeps the
// stored mass equal to rho to FP32 round-off: no bias from the FP32 weights
// not summing exactly to 1, and the FP16/BF16 rounding of the moving
// populations is absorbed by the FP32 rest population.
// mass: incoming component densities; PredW(i) returns the codec predictor
// of f*_i (pred_write), rt and inv_rt this node's previous-level total
// density and its inverse (F16/BF16 codecs only).
template <class C, bool ODD, bool WIDE, class FidAt, class PredW>
__device__ __forceinline__ void store_node(const float (&fs)[2][Q], const Pops<C>& D, const float (&mass)[2],
                                           PredW pred_w, float rt, float inv_rt, uint32_t k, FidAt fid_at, int np) {
    float sum0 = 0.0f, sum1 = 0.0f;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const float2 pr = C::kRef ? pred_w(i) : make_float2(0.f, 0.f);
        const typename C::T h0 = C::enc(fs[0][i], pr.x, inv_rt);
        const typename C::T h1 = C::enc(fs[1][i], pr.y, inv_rt);
        const typename Pops<C>::P2 hp{{h0, h1}};
        if constexpr (!ODD) {
            st_pop<WIDE>(D.plane(opp(i), np), k, hp);
        } else {
            // slot (i, dst) or, across a wall, (opp i, k), from the pair's lower plane
            const int dst = fid_at(i, +1);
            const bool wall = dst < 0;
            const int lo = (i & 1) ? i : i - 1;
            const uint32_t e = wall ? k + ((i & 1) ? (uint32_t)np : 0u) : (uint32_t)dst + ((i & 1) ? 0u : (uint32_t)np);
            st_pop<WIDE>(D.plane(lo, np), e, hp);
        }
        sum0 += C::dec(h0, pr.x, rt);
        sum1 += C::dec(h1, pr.y, rt);
    }
    st_pop<WIDE>(D.rests(), k, Pair<float>{{mass[0] - sum0, mass[1] - sum1}});
}

// Physical parameters in FP32.
struct Phys {
    float a[2];     // tau^(sigma) - 1/2
    float G;        // G_coh
    float g[2][3];  // body acceleration per component
};

// Forced SRT collision at one node (Eqs. 1, 2, 6-9), in place on the moving
// populations f[s][1..18]; the rest population follows from mass balance in
// store_node.  F: total force per component (Eq. 10).  Returns u in uo.
// Opposite directions (2k-1, 2k) share e.u and e.F up to sign, so the
// equilibrium and source are split into their even and odd parts per pair.
__device__ __forceinline__ void collide(float (&f)[2][Q], const float (&rho)[2], const float (&F)[2][3],
                                        const Phys& ph, float (&uo)[3]) {
    float j[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const float d = f[s][i] - f[s][i + 1];
            if (DX[i]) j[0] += DX[i] * d;
            if (DY[i]) j[1] += DY[i] * d;
            if (DZ[i]) j[2] += DZ[i] * d;
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
    const float keep = 1.0f - om;
    // Per pair and component, with X = 1 + 4.5 (e.u)^2 - 1.5 u^2 and
    // t = 3 (e.u)(e.F) - u.F:
    //   om f^eq + cf S = A X + B t   (even part),  A 3 e.u + B e.F  (odd part),
    // A = om w rho^(sigma), B = 3 cf w; the odd part flips sign between the
    // two directions of a pair.
    const float c1 = 1.0f - 1.5f * (ux * ux + uy * uy + uz * uz);
    float A[2][2], uF[2];
    const float B[2] = {3.0f * cf * weight(1), 3.0f * cf * weight(7)};   // axis, diagonal pairs
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        A[s][0] = om * weight(1) * rho[s];
        A[s][1] = om * weight(7) * rho[s];
        uF[s] = ux * F[s][0] + uy * F[s][1] + uz * F[s][2];
    }
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const int c = i < 7 ? 0 : 1;
        const float eu = DX[i] * ux + DY[i] * uy + DZ[i] * uz;
        const float eu3 = 3.0f * eu;
        const float X = fmaf(1.5f * eu, eu3, c1);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float eF = DX[i] * F[s][0] + DY[i] * F[s][1] + DZ[i] * F[s][2];
            const float t = fmaf(eu3, eF, -uF[s]);
            const float ge = fmaf(A[s][c], X, B[c] * t);
            const float go = fmaf(A[s][c], eu3, B[c] * eF);
            f[s][i] = fmaf(keep, f[s][i], ge + go);
            f[s][i + 1] = fmaf(keep, f[s][i + 1], ge - go);
        }
    }
}

// Pseudopotential force sum sum_{i>=1} w_i psi(x + e_i) e_i for both
// components, with psi supplied by a functor psi_at(i) -> float2; opposite
// pairs enter as differences.
template <class PsiAt>
__device__ __forceinline__ void psi_sum(PsiAt psi_at, float (&acc)[2][3]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) acc[s][0] = acc[s][1] = acc[s][2] = 0.0f;
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const float2 p = psi_at(i), q = psi_at(i + 1);
        const float w = weight(i);
        const float d0 = w * (p.x - q.x), d1 = w * (p.y - q.y);
        if (DX[i]) { acc[0][0] += DX[i] * d0; acc[1][0] += DX[i] * d1; }
        if (DY[i]) { acc[0][1] += DY[i] * d0; acc[1][1] += DY[i] * d1; }
        if (DZ[i]) { acc[0][2] += DZ[i] * d0; acc[1][2] += DZ[i] * d1; }
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
