// Host-side launchers of the adjoint kernels (implemented in lbm_adjoint.hip).
#pragma once

#include "lbm_kernels.hpp"

namespace mclbm {

int loss_blocks(const Geo& g);
void launch_loss(const Pops<CodecF32>& P, const int* fid, const uint32_t* nbm, const uint8_t* region,
                 const Geo& g, int odd, double* partial, double* out, hipStream_t s);
void launch_adj_seed(const Pops<CodecF32>& P, const int* fid, const uint32_t* nbm, const uint8_t* region,
                     const Geo& g, int odd, const double* loss, float* lam, float2* rbar, hipStream_t s);
// outlet flux: out[0] = mean of rho1 u_x over the region's fluid nodes, out[1] = their count
void launch_loss_flux(const Pops<CodecF32>& P, const int* fid, const uint32_t* nbm, const uint8_t* region,
                      const float2* psi, const Geo& g, const Phys& ph, int odd, double* partial, double* out,
                      hipStream_t s);
void launch_adj_seed_flux(const Pops<CodecF32>& P, const int* fid, const uint32_t* nbm, const uint8_t* region,
                          const float2* psi, const Geo& g, const Phys& ph, int odd, float* lam, float* abar,
                          hipStream_t s);
// node_of[k] = lattice index of fluid id k
void launch_node_of(const int* fid, const Geo& g, int* node_of, hipStream_t s);
// nfid[(i-1) np + k] = fluid id of the neighbour x(k) + e_i (-1 at solid)
void launch_adj_neighbours(const int* node_of, int nfluid, const int* fid, const Geo& g, int* nfid, hipStream_t s);
void launch_adj_collide(const Pops<CodecF32>& P, const int* nfid, const int* node_of, int nfluid, const float2* psi,
                        const float* lam_next, const float2* rbar_next, float* lam_cur, float* abar, const Geo& g,
                        const Phys& ph, int odd, hipStream_t s);
void launch_adj_ivsd(const int* list, const float* xil, int count, const uint32_t* nbm, const float2* psi,
                     const float* abar, const Geo& g, double* grad_acc, float2* nbar, hipStream_t s);
void launch_adj_rho(const int* node_of, int nfluid, const uint32_t* nbm, const float* abar, const float2* nbar,
                    const Geo& g, float2* rbar, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);
void launch_grad_scatter(const int* list, int count, const double* acc, double* grad, hipStream_t s);

}  // namespace mclbm
