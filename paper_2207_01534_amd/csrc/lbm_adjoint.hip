// Reverse mode of the two-component D3Q19 step with respect to the per-voxel
// adhesion parameter xi (Eqs. 13-15), for FP32 population storage.
//
// One forward step maps f(t) -> f(t+1) through
//   rho = sum_i f_i,  psi-hat = rho (fluid) | chi N / D (boundary solid),
//   A^s = sum_i w_i e_i psi-hat^s(x+e_i),  F^s = -G rho^s A^(other s) + rho^s g^s,
//   u, tau_s, f* = (1-om) f + om f^eq + (1 - om/2) S,  then streaming.
// Its adjoint runs as three kernels per step, with lambda = dL/df(t+1):
//   k_adj_collide  per fluid x: lambda*_i(x) = lambda_i(x+e_i) (or the
//                  bounced lambda at home), the vector-Jacobian product of
//                  the local collision, giving the local part of dL/df(t)
//                  and the adjoint Abar of the pseudopotential sums;
//   k_adj_ivsd     per boundary solid y: psibar(y) = -sum_k w_k e_k .
//                  Abar(y+e_k), which yields dL/dxi(y) and the adjoint Nbar
//                  of the virtual-density numerator;
//   k_adj_rho      per fluid z: the non-local density adjoint
//                  rhobar(z) = -sum_k w_k e_k . Abar(z+e_k)
//                              + sum_{solid z+e_m} w_m Nbar(z+e_m).
// dL/df_i(t) at a fluid node is lambda_loc_i + rhobar, kept as the two parts
// and added where the next reverse step gathers them.  Both are indexed by
// fluid id (plane stride np, like the populations), so their gathers touch
// no solid slots; lambda holds the two components of a direction side by
// side (one 8-byte access per direction, as the populations do).  Abar and
// Nbar stay indexed by lattice node, since solid neighbours read them.
#include "lbm_adjoint.hpp"

namespace mclbm {

using CF = CodecF32;

// Work item of this thread for kernels over a 1D range of n items launched
// on an XCD-aware grid (xcd_grid(blocks of 256)): the hardware deals
// consecutive blocks round-robin to the 8 XCDs, so block b takes chunk
// (b mod 8) * per + b / 8 and each XCD walks a contiguous run of chunks,
// whose neighbour gathers then share that XCD's L2.  Returns -1 past n.
__device__ __forceinline__ int xcd_item(int n) {
    const int per = gridDim.x >> 3;
    const int chunk = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    const int k = chunk * (int)blockDim.x + (int)threadIdx.x;
    return k < n ? k : -1;
}

// ---------------------------------------------------------------------------
// Loss L = (1/|R|) sum_{fluid x in R} rho1 / (rho1 + rho2), FP64 partials.
// ---------------------------------------------------------------------------
template <bool ODD>
__global__ __launch_bounds__(256) void k_loss_partial(Pops<CF> P, const int* __restrict__ fid,
                                                      const uint32_t* __restrict__ nbm,
                                                      const uint8_t* __restrict__ region, Geo g,
                                                      double* __restrict__ partial) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double v = 0.0, c = 0.0;
    if (x < g.nx && y < g.ny) {
        const Nb nb(x, y, z, g);
        const uint32_t m = nbm[nb.idx];
        if (!(m & SELF_SOLID) && region[nb.idx]) {
            float f[2][Q];
            load_node<CF, ODD>(f, P, nullptr, m, nb, (uint32_t)fid[nb.idx],
                               [&](int i, int s) { return fid[nb.at(i, s)]; }, g.np, 0.0f);
            const double r0 = sum19(f[0]), r1 = sum19(f[1]);
            v = r0 / (r0 + r1);
            c = 1.0;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        v += __shfl_xor(v, off);
        c += __shfl_xor(c, off);
    }
    __shared__ double red[4][2];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if ((tid & 63) == 0) {
        red[tid >> 6][0] = v;
        red[tid >> 6][1] = c;
    }
    __syncthreads();
    if (tid < 2) {
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += red[w][tid];
        const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        partial[(size_t)b * 2 + tid] = s;
    }
}

__global__ void k_loss_final(const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
    __shared__ double red[2][1024];
    const int t = threadIdx.x;
    double v = 0.0, c = 0.0;
    for (int b = t; b < nblocks; b += 1024) {
        v += partial[(size_t)b * 2];
        c += partial[(size_t)b * 2 + 1];
    }
    red[0][t] = v;
    red[1][t] = c;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (t < off) {
            red[0][t] += red[0][t + off];
            red[1][t] += red[1][t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = red[1][0] > 0 ? red[0][0] / red[1][0] : 0.0;
        out[1] = red[1][0];
    }
}

// ---------------------------------------------------------------------------
// Outlet flux L = sum_{fluid x in R} rho1 u_x with the common velocity of
// Eq. 8 (half-force shift included): FP64 partials of (L, |R|).  psi holds
// psi-hat of the same time level (its forces enter u).
// ---------------------------------------------------------------------------
// Local quantities of the flux loss at one fluid node.
struct FluxNode {
    float rho[2], A[2][3], u[3], rt;
};

template <bool ODD>
__device__ __forceinline__ FluxNode flux_node(const Pops<CF>& P, const int* fid, const float2* psi, uint32_t m,
                                              const Nb& nb, const Geo& g, const Phys& ph) {
    FluxNode q;
    float f[2][Q];
    load_node<CF, ODD>(f, P, nullptr, m, nb, (uint32_t)fid[nb.idx], [&](int i, int s) { return fid[nb.at(i, s)]; },
                       g.np, 0.0f);
    q.rho[0] = sum19(f[0]);
    q.rho[1] = sum19(f[1]);
    psi_sum([&](int i) { return ld(psi, nb.at(i, +1)); }, q.A);
    float F[2][3];
    total_force(q.rho, q.A, ph, F);
    float j[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            j[0] += DX[i] * f[s][i];
            j[1] += DY[i] * f[s][i];
            j[2] += DZ[i] * f[s][i];
        }
    q.rt = q.rho[0] + q.rho[1];
#pragma unroll
    for (int a = 0; a < 3; ++a) q.u[a] = (j[a] + 0.5f * (F[0][a] + F[1][a])) / q.rt;
    return q;
}

template <bool ODD>
__global__ __launch_bounds__(256) void k_loss_flux_partial(Pops<CF> P, const int* __restrict__ fid,
                                                           const uint32_t* __restrict__ nbm,
                                                           const uint8_t* __restrict__ region,
                                                           const float2* __restrict__ psi, Geo g, Phys ph,
                                                           double* __restrict__ partial) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double v = 0.0, c = 0.0;
    if (x < g.nx && y < g.ny) {
        const Nb nb(x, y, z, g);
        const uint32_t m = nbm[nb.idx];
        if (!(m & SELF_SOLID) && region[nb.idx]) {
            const FluxNode q = flux_node<ODD>(P, fid, psi, m, nb, g, ph);
            v = (double)q.rho[0] * (double)q.u[0];
            c = 1.0;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        v += __shfl_xor(v, off);
        c += __shfl_xor(c, off);
    }
    __shared__ double red[4][2];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if ((tid & 63) == 0) {
        red[tid >> 6][0] = v;
        red[tid >> 6][1] = c;
    }
    __syncthreads();
    if (tid < 2) {
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += red[w][tid];
        const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        partial[(size_t)b * 2 + tid] = s;
    }
}

// Seed of the flux loss at the final time.  With u_x = (j_x + (F1_x + F2_x)/2)
// / rho and F^s = -G rho^s A^(other) + rho^s g^s, holding A fixed:
//   dL/drho1 = u_x + rho1 ((g1_x - G A2_x)/2 - u_x) / rho,
//   dL/drho2 = rho1 ((g2_x - G A1_x)/2 - u_x) / rho,   dL/dj_x = rho1 / rho,
//   dL/dA1_x = -G rho1 rho2 / (2 rho),               dL/dA2_x = -G rho1^2 / (2 rho);
// so lambda_loc_i^s = dL/drho^s + e_ix rho1/rho, and Abar carries the A terms
// (per axis a pair: A of component 1, A of component 2) to the IVSD and
// density adjoints, which return the neighbours' share and the direct xi term.
template <bool ODD>
__global__ __launch_bounds__(256) void k_adj_seed_flux(Pops<CF> P, const int* __restrict__ fid,
                                                       const uint32_t* __restrict__ nbm,
                                                       const uint8_t* __restrict__ region,
                                                       const float2* __restrict__ psi, Geo g, Phys ph,
                                                       float* __restrict__ lam, float* __restrict__ abar) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const Nb nb(x, y, z, g);
    const size_t n = (size_t)g.n;
    const uint32_t m = nbm[nb.idx];
    float l0 = 0.f, l1 = 0.f, lj = 0.f, a1 = 0.f, a2 = 0.f;
    if (!(m & SELF_SOLID) && region[nb.idx]) {
        const FluxNode q = flux_node<ODD>(P, fid, psi, m, nb, g, ph);
        const float inv = 1.0f / q.rt;
        l0 = q.u[0] + q.rho[0] * (0.5f * (ph.g[0][0] - ph.G * q.A[1][0]) - q.u[0]) * inv;
        l1 = q.rho[0] * (0.5f * (ph.g[1][0] - ph.G * q.A[0][0]) - q.u[0]) * inv;
        lj = q.rho[0] * inv;
        a1 = -0.5f * ph.G * q.rho[0] * q.rho[1] * inv;
        a2 = -0.5f * ph.G * q.rho[0] * q.rho[0] * inv;
    }
    if (m & SELF_SOLID) return;
    const uint32_t kf = (uint32_t)fid[nb.idx];
    const size_t np = (size_t)g.np;
    float2* lam2 = reinterpret_cast<float2*>(lam);
#pragma unroll
    for (int i = 0; i < Q; ++i) lam2[(size_t)i * np + kf] = make_float2(l0 + DX[i] * lj, l1 + DX[i] * lj);
    {
        float2* ab = reinterpret_cast<float2*>(abar);
        ab[nb.idx] = make_float2(a1, a2);
        ab[n + nb.idx] = make_float2(0.f, 0.f);
        ab[2 * n + nb.idx] = make_float2(0.f, 0.f);
    }
}

// ---------------------------------------------------------------------------
// Seed at the final time: dL/df_i = dL/drho, identical over i; it is stored
// as lambda_loc = 0 plus rhobar = (rho2, -rho1) / (rho1+rho2)^2 / |R|.
// ---------------------------------------------------------------------------
template <bool ODD>
__global__ __launch_bounds__(256) void k_adj_seed(Pops<CF> P, const int* __restrict__ fid,
                                                  const uint32_t* __restrict__ nbm,
                                                  const uint8_t* __restrict__ region, Geo g,
                                                  const double* __restrict__ loss, float* __restrict__ lam,
                                                  float2* __restrict__ rbar) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const Nb nb(x, y, z, g);
    const uint32_t m = nbm[nb.idx];
    if (m & SELF_SOLID) return;
    const uint32_t kf = (uint32_t)fid[nb.idx];
    const size_t np = (size_t)g.np;
    float2* lam2 = reinterpret_cast<float2*>(lam);
    for (int i = 0; i < Q; ++i) lam2[(size_t)i * np + kf] = make_float2(0.0f, 0.0f);
    float2 r = make_float2(0.f, 0.f);
    if (region[nb.idx] && loss[1] > 0) {
        float f[2][Q];
        load_node<CF, ODD>(f, P, nullptr, m, nb, kf,
                           [&](int i, int s) { return fid[nb.at(i, s)]; }, g.np, 0.0f);
        const double r0 = sum19(f[0]), r1 = sum19(f[1]);
        const double rt = r0 + r1;
        const double s = 1.0 / (rt * rt * loss[1]);
        r = make_float2((float)(r1 * s), (float)(-r0 * s));
    }
    rbar[kf] = r;
}

// Neighbour fluid ids of every fluid node, by fluid id: nfid[(i-1) np + k] =
// fluid id of x(k) + e_i, -1 where that node is solid.  Built once per
// gradient call, so that the reverse collide reads a node's neighbour ids as
// 18 coalesced loads that depend on nothing, instead of gathering them from
// the lattice map after its own lattice index has arrived.
__global__ __launch_bounds__(256) void k_adj_neighbours(const int* __restrict__ node_of, int nfluid,
                                                        const int* __restrict__ fid, Geo g, int* __restrict__ nfid) {
    const int kf = xcd_item(nfluid);
    if (kf < 0) return;
    const int idx = node_of[kf];
    const Nb nb(idx % g.nx, (idx / g.nx) % g.ny, idx / (g.nx * g.ny), g);
    const size_t np = (size_t)g.np;
#pragma unroll
    for (int i = 1; i < Q; ++i) nfid[(size_t)(i - 1) * np + kf] = fid[nb.at(i, +1)];
}

// ---------------------------------------------------------------------------
// A1: adjoint of streaming and of the local collision at fluid nodes.
// ---------------------------------------------------------------------------
// One thread per fluid node, in fluid-id order (node_of: fluid id -> lattice
// index); Abar stays zero at solid nodes (cleared once per gradient call).
template <bool ODD>
__global__ __launch_bounds__(256) void k_adj_collide(Pops<CF> P, const int* __restrict__ nfid,
                                                     const int* __restrict__ node_of, int nfluid,
                                                     const float2* __restrict__ psi,
                                                     const float* __restrict__ lam_next,
                                                     const float2* __restrict__ rbar_next,
                                                     float* __restrict__ lam_cur, float* __restrict__ abar,
                                                     Geo g, Phys ph) {
    const int kf = xcd_item(nfluid);
    if (kf < 0) return;
    const int idx = node_of[kf];
    const int x = idx % g.nx, y = (idx / g.nx) % g.ny, z = idx / (g.nx * g.ny);
    const Nb nb(x, y, z, g);
    const size_t n = (size_t)g.n, np = (size_t)g.np;
    // fluid id of x + s e_i (-1 at solid): x - e_i is x + e_opp(i)
    auto nf = [&](int i, int s) { return nfid[(size_t)((s > 0 ? i : opp(i)) - 1) * np + kf]; };
    // forward quantities of this node at time t
    float f[2][Q];
    load_node<CF, ODD>(f, P, nullptr, 0u, nb, (uint32_t)kf, nf, g.np, 0.0f);
    const float rho[2] = {sum19(f[0]), sum19(f[1])};
    float A[2][3];
    psi_sum([&](int i) { return ld(psi, nb.at(i, +1)); }, A);
    float F[2][3];
    total_force(rho, A, ph, F);
    float j[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            j[0] += DX[i] * f[s][i];
            j[1] += DY[i] * f[s][i];
            j[2] += DZ[i] * f[s][i];
        }
    const float rt = rho[0] + rho[1];
    const float inv_rt = 1.0f / rt;
    const float u[3] = {(j[0] + 0.5f * (F[0][0] + F[1][0])) * inv_rt, (j[1] + 0.5f * (F[0][1] + F[1][1])) * inv_rt,
                        (j[2] + 0.5f * (F[0][2] + F[1][2])) * inv_rt};
    const float tau_s = (rho[0] * ph.a[0] + rho[1] * ph.a[1]) * inv_rt + 0.5f;
    const float om = 1.0f / tau_s;
    const float cf = 1.0f - 0.5f * om;
    const float usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

    // lambda* = dL/df*: the adjoint of streaming gathers from downstream
    float ls[2][Q];
    {
        const float2* ln = reinterpret_cast<const float2*>(lam_next);
        const float2 rb0 = rbar_next[kf];
        const float2 l0 = ln[kf];
        ls[0][0] = l0.x + rb0.x;
        ls[1][0] = l0.y + rb0.y;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int nbf = nf(i, +1);
            const bool wall = nbf < 0;
            const uint32_t at = wall ? (uint32_t)kf : (uint32_t)nbf;
            const int dir = wall ? opp(i) : i;
            const float2 rb = rbar_next[at];
            const float2 lv = ln[(size_t)dir * np + at];
            ls[0][i] = lv.x + rb.x;
            ls[1][i] = lv.y + rb.y;
        }
    }

    // vector-Jacobian product of f* = (1-om) f + om f^eq(rho, u) + (1 - om/2) S(u, F)
    float om_bar = 0.f;
    float rb[2] = {0.f, 0.f};
    float M0[2] = {0.f, 0.f};
    float V[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    float Wv[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const float uF = u[0] * F[s][0] + u[1] * F[s][1] + u[2] * F[s][2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float w = weight(i);
            const float eu = DX[i] * u[0] + DY[i] * u[1] + DZ[i] * u[2];
            const float eF = DX[i] * F[s][0] + DY[i] * F[s][1] + DZ[i] * F[s][2];
            const float B = 1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * usq;
            const float feq = w * rho[s] * B;
            const float S = w * (3.0f * (eF - uF) + 9.0f * eu * eF);
            const float l = ls[s][i];
            om_bar += l * (feq - f[s][i] - 0.5f * S);
            const float lw = l * w;
            rb[s] += om * lw * B;
            M0[s] += lw;
            const float c1 = lw * (3.0f + 9.0f * eu);
            const float c2 = lw * eF;
            if (DX[i]) { V[s][0] += c1 * DX[i]; Wv[s][0] += c2 * DX[i]; }
            if (DY[i]) { V[s][1] += c1 * DY[i]; Wv[s][1] += c2 * DY[i]; }
            if (DZ[i]) { V[s][2] += c1 * DZ[i]; Wv[s][2] += c2 * DZ[i]; }
        }
    }
    float ubar[3], Fbar[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ubar[a] = 0.f;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float t0 = V[s][a] - 3.0f * u[a] * M0[s];
            ubar[a] += om * rho[s] * t0 + cf * (9.0f * Wv[s][a] - 3.0f * F[s][a] * M0[s]);
            Fbar[s][a] = cf * t0;
        }
    }
    // om = 1/tau_s, tau_s = (rho1 a1 + rho2 a2)/rho + 1/2
    const float tau_bar = -om * om * om_bar;
#pragma unroll
    for (int s = 0; s < 2; ++s) rb[s] += tau_bar * (ph.a[s] - (tau_s - 0.5f)) * inv_rt;
    // u = (j + (F1 + F2)/2) / rho
    const float Pbar[3] = {ubar[0] * inv_rt, ubar[1] * inv_rt, ubar[2] * inv_rt};
    const float uu = (ubar[0] * u[0] + ubar[1] * u[1] + ubar[2] * u[2]) * inv_rt;
    rb[0] -= uu;
    rb[1] -= uu;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) Fbar[s][a] += 0.5f * Pbar[a];
    // F^s = -G rho^s A^(other) + rho^s g^s
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int o = 1 - s;
#pragma unroll
        for (int a = 0; a < 3; ++a) rb[s] += Fbar[s][a] * (-ph.G * A[o][a] + ph.g[s][a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        reinterpret_cast<float2*>(abar)[(size_t)a * n + nb.idx] =
            make_float2(-ph.G * rho[1] * Fbar[1][a], -ph.G * rho[0] * Fbar[0][a]);  // adjoints of A^(1), A^(2)
    }
    // local part of dL/df_i(t): direct term, momentum term, density term
    const float keep = 1.0f - om;
    float2* lc = reinterpret_cast<float2*>(lam_cur);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float ej = DX[i] * Pbar[0] + DY[i] * Pbar[1] + DZ[i] * Pbar[2];
        lc[(size_t)i * np + kf] = make_float2(keep * ls[0][i] + ej + rb[0], keep * ls[1][i] + ej + rb[1]);
    }
}

// psibar(y) = -sum_k w_k e_k . Abar(y + e_k), both components.
__device__ __forceinline__ float2 psi_adjoint(const float* __restrict__ abar, const Nb& nb, size_t n) {
    float p0 = 0.f, p1 = 0.f;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
        const uint32_t at = nb.at(k, +1);
        const float w = weight(k);
        float d0 = 0.f, d1 = 0.f;
        const float2* ab = reinterpret_cast<const float2*>(abar);
        if (DX[k]) { const float2 v = ab[at]; d0 += DX[k] * v.x; d1 += DX[k] * v.y; }
        if (DY[k]) { const float2 v = ab[n + at]; d0 += DY[k] * v.x; d1 += DY[k] * v.y; }
        if (DZ[k]) { const float2 v = ab[2 * n + at]; d0 += DZ[k] * v.x; d1 += DZ[k] * v.y; }
        p0 -= w * d0;
        p1 -= w * d1;
    }
    return make_float2(p0, p1);
}

// ---------------------------------------------------------------------------
// A2: boundary solid nodes.  rho~^s = chi^s N^s / D with chi = 1 +- xi gives
// dL/dxi = psibar^1 N^1/D - psibar^2 N^2/D and Nbar^s = psibar^s chi^s / D.
// N^s/D is read back from the forward's psi-hat at y (rho~^s / chi^s) and D
// follows from the neighbourhood word, so no neighbour densities are loaded.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_ivsd(const int* __restrict__ list, const float* __restrict__ xil,
                                                  int count, const uint32_t* __restrict__ nbm,
                                                  const float2* __restrict__ psi, const float* __restrict__ abar,
                                                  Geo g, double* __restrict__ grad_acc,
                                                  float2* __restrict__ nbar) {
    const int k = xcd_item(count);
    if (k < 0) return;
    const int idx = list[k];
    const int x = idx % g.nx;
    const int y = (idx / g.nx) % g.ny;
    const int z = idx / (g.nx * g.ny);
    const Nb nb(x, y, z, g);
    const uint32_t m = nbm[idx];
    const float2 vd = psi[idx];
    const float v = xil[k];
    const float2 pb = psi_adjoint(abar, nb, (size_t)g.n);
    float den = 0.f;
#pragma unroll
    for (int i = 1; i < Q; ++i) den += ((m >> i) & 1u) ? 0.0f : weight(i);
    const float inv = 1.0f / den;  // den > 0: the list holds only nodes with a fluid neighbour
    const float c0 = 1.0f + v, c1 = 1.0f - v;  // > 0: |xi| < 1 at listed nodes
    grad_acc[k] += (double)(pb.x * (vd.x / c0)) - (double)(pb.y * (vd.y / c1));
    nbar[idx] = make_float2(pb.x * c0 * inv, pb.y * c1 * inv);
}

// ---------------------------------------------------------------------------
// A3: non-local density adjoint at fluid nodes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_rho(const int* __restrict__ node_of, int nfluid,
                                                 const uint32_t* __restrict__ nbm, const float* __restrict__ abar,
                                                 const float2* __restrict__ nbar, Geo g,
                                                 float2* __restrict__ rbar) {
    const int kf = xcd_item(nfluid);
    if (kf < 0) return;
    const int idx = node_of[kf];
    const Nb nb(idx % g.nx, (idx / g.nx) % g.ny, idx / (g.nx * g.ny), g);
    const uint32_t m = nbm[nb.idx];
    float2 r = psi_adjoint(abar, nb, (size_t)g.n);
    // all neighbour loads issued together (nbar is read-only here); fluid
    // neighbours are dropped by a select
    float2 nv[Q];
#pragma unroll
    for (int i = 1; i < Q; ++i) nv[i] = nbar[nb.at(i, +1)];
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const bool solid = (m >> i) & 1u;
        r.x += solid ? weight(i) * nv[i].x : 0.0f;
        r.y += solid ? weight(i) * nv[i].y : 0.0f;
    }
    rbar[kf] = r;
}

// node_of[fid[idx]] = idx for every fluid node.
__global__ void k_node_of(const int* __restrict__ fid, int n, int* __restrict__ node_of) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int k = fid[idx];
    if (k >= 0) node_of[k] = idx;
}

__global__ void k_zero_words(uint32_t* __restrict__ p, size_t nwords) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_grad_scatter(const int* __restrict__ list, int count, const double* __restrict__ acc,
                               double* __restrict__ grad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) grad[list[k]] = acc[k];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// 64 x 4 blocks over (x, y), one z plane per grid row
static dim3 rows(const Geo& g) { return dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz); }
static const dim3 kBlock(64, 4);

int loss_blocks(const Geo& g) {
    const dim3 r = rows(g);
    return (int)(r.x * r.y * r.z);
}

void launch_loss(const Pops<CF>& P, const int* fid, const uint32_t* nbm, const uint8_t* region, const Geo& g,
                 int odd, double* partial, double* out, hipStream_t s) {
    if (odd)
        hipLaunchKernelGGL(k_loss_partial<true>, rows(g), kBlock, 0, s, P, fid, nbm, region, g, partial);
    else
        hipLaunchKernelGGL(k_loss_partial<false>, rows(g), kBlock, 0, s, P, fid, nbm, region, g, partial);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, s, (const double*)partial, loss_blocks(g), out);
}

void launch_adj_seed(const Pops<CF>& P, const int* fid, const uint32_t* nbm, const uint8_t* region, const Geo& g,
                     int odd, const double* loss, float* lam, float2* rbar, hipStream_t s) {
    if (odd)
        hipLaunchKernelGGL(k_adj_seed<true>, rows(g), kBlock, 0, s, P, fid, nbm, region, g, loss, lam, rbar);
    else
        hipLaunchKernelGGL(k_adj_seed<false>, rows(g), kBlock, 0, s, P, fid, nbm, region, g, loss, lam, rbar);
}

void launch_loss_flux(const Pops<CF>& P, const int* fid, const uint32_t* nbm, const uint8_t* region,
                      const float2* psi, const Geo& g, const Phys& ph, int odd, double* partial, double* out,
                      hipStream_t s) {
    if (odd)
        hipLaunchKernelGGL(k_loss_flux_partial<true>, rows(g), kBlock, 0, s, P, fid, nbm, region, psi, g, ph, partial);
    else
        hipLaunchKernelGGL(k_loss_flux_partial<false>, rows(g), kBlock, 0, s, P, fid, nbm, region, psi, g, ph,
                           partial);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, s, (const double*)partial, loss_blocks(g), out);
}

void launch_adj_seed_flux(const Pops<CF>& P, const int* fid, const uint32_t* nbm, const uint8_t* region,
                          const float2* psi, const Geo& g, const Phys& ph, int odd, float* lam, float* abar,
                          hipStream_t s) {
    if (odd)
        hipLaunchKernelGGL(k_adj_seed_flux<true>, rows(g), kBlock, 0, s, P, fid, nbm, region, psi, g, ph, lam, abar);
    else
        hipLaunchKernelGGL(k_adj_seed_flux<false>, rows(g), kBlock, 0, s, P, fid, nbm, region, psi, g, ph, lam,
                           abar);
}

void launch_node_of(const int* fid, const Geo& g, int* node_of, hipStream_t s) {
    hipLaunchKernelGGL(k_node_of, dim3((g.n + 255) / 256), dim3(256), 0, s, fid, g.n, node_of);
}

void launch_adj_neighbours(const int* node_of, int nfluid, const int* fid, const Geo& g, int* nfid, hipStream_t s) {
    if (nfluid <= 0) return;
    hipLaunchKernelGGL(k_adj_neighbours, dim3(xcd_grid((nfluid + 255) / 256)), dim3(256), 0, s, node_of, nfluid, fid,
                       g, nfid);
}

void launch_adj_collide(const Pops<CF>& P, const int* nfid, const int* node_of, int nfluid, const float2* psi,
                        const float* lam_next, const float2* rbar_next, float* lam_cur, float* abar, const Geo& g,
                        const Phys& ph, int odd, hipStream_t s) {
    if (nfluid <= 0) return;
    const dim3 grid(xcd_grid((nfluid + 255) / 256));
    if (odd)
        hipLaunchKernelGGL(k_adj_collide<true>, grid, dim3(256), 0, s, P, nfid, node_of, nfluid, psi, lam_next,
                           rbar_next, lam_cur, abar, g, ph);
    else
        hipLaunchKernelGGL(k_adj_collide<false>, grid, dim3(256), 0, s, P, nfid, node_of, nfluid, psi, lam_next,
                           rbar_next, lam_cur, abar, g, ph);
}

void launch_adj_ivsd(const int* list, const float* xil, int count, const uint32_t* nbm, const float2* psi,
                     const float* abar, const Geo& g, double* grad_acc, float2* nbar, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_adj_ivsd, dim3(xcd_grid((count + 255) / 256)), dim3(256), 0, s, list, xil, count, nbm, psi,
                       abar, g, grad_acc, nbar);
}

void launch_adj_rho(const int* node_of, int nfluid, const uint32_t* nbm, const float* abar, const float2* nbar,
                    const Geo& g, float2* rbar, hipStream_t s) {
    if (nfluid <= 0) return;
    hipLaunchKernelGGL(k_adj_rho, dim3(xcd_grid((nfluid + 255) / 256)), dim3(256), 0, s, node_of, nfluid, nbm, abar,
                       nbar, g, rbar);
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t words = bytes / 4;
    if (!words) return;
    const size_t blocks = (words + 255) / 256;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s,
                       (uint32_t*)p, words);
}

void launch_grad_scatter(const int* list, int count, const double* acc, double* grad, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_grad_scatter, dim3((count + 255) / 256), dim3(256), 0, s, list, count, acc, grad);
}

}  // namespace mclbm
