// Host-side launchers of the open inlet/outlet plane kernels (lbm_open.hip).
#pragma once

#include "lbm_device.hpp"

namespace mclbm {

// psi-hat of the ghost planes from the mirror images: psi(0) = psi(2),
// psi(nx-1) = psi(nx-3).
void launch_open_mirror(float2* psi, const Geo& g, hipStream_t s);
// Boundary rebuild at the level of parity odd; psi holds the densities of the
// level before (the codec predictors' field); held: [2][19][ny*nz] FP32;
// G: the cohesion parameter (codec predictors).
template <class C>
void launch_open_rebuild(const Pops<C>& P, const int* fid, const float2* psi, const float* held, const Geo& g,
                         int odd, float rho_in, float rho_out, float G, hipStream_t s);
// Capture the held populations from the state at the level of parity odd
// (rprev: the pseudopotential field of the level before, the codec
// predictors' field).
template <class C>
void launch_open_capture(const Pops<C>& P, const int* fid, const uint32_t* nbm, const float2* rprev, float* held,
                         const Geo& g, int odd, float G, hipStream_t s);
// out[0], out[1]: mean Eq. (12) pressure over the fluid nodes of x = 1 and x = nx-2.
void launch_open_pressure(const float2* psi, const uint32_t* nbm, const Geo& g, float G, double* out,
                          hipStream_t s);
// *count <- number of solid nodes on planes 0, 1, 2, nx-3, nx-2, nx-1.
void launch_open_check(const uint32_t* nbm, const Geo& g, int* count, hipStream_t s);

}  // namespace mclbm
