/*
 * mclbm.h -- C ABI of the two-component D3Q19 pseudopotential lattice
 * Boltzmann step for MI355X (gfx950).
 *
 * The method is the improved multi-component pseudopotential LBM of
 * Sedahmed et al., Phys. Fluids 34 (2022), arXiv 2207.01534, Sec. 2:
 *   forced SRT lattice Boltzmann equation            Eq. (1)
 *   second-order equilibrium on the common velocity  Eq. (2)
 *   densities, velocities, mixture density           Eqs. (3)-(5)
 *   mixture relaxation time from viscosities         Eqs. (6)-(7)
 *   common equilibrium velocity                      Eq. (8)
 *   forcing source                                   Eq. (9)
 *   total, inter-component and fluid-solid forces    Eqs. (10), (11), (13)
 *   IVSD solid pseudopotential and virtual density   Eqs. (14)-(15)
 *   pressure                                         Eq. (12)
 *   halfway bounce-back at fluid-solid interfaces    Secs. 3.2, 4.1
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: nx * ny * nz nodes, node index idx = x + nx*(y + ny*z) (x fastest),
 * periodic in all three directions; walls are made of solid voxels.
 * Component 1 is sigma = 0 in arrays, component 2 is sigma = 1.
 * Lattice units throughout (dx = dt = 1).
 *
 * Memory ownership: the caller allocates and owns ALL device memory -- the
 * workspace handed to mclbm_create, every input, output, saved state,
 * adjoint buffer and gradient.  The library never allocates or frees device
 * memory.  It owns only the small host-side handle, released by
 * mclbm_destroy.  "Device pointer" below means memory of the device that was
 * current when mclbm_create was called.
 *
 * Streams: all device work is enqueued, in order, on the stream given to
 * mclbm_create (a hipStream_t passed as void*; NULL = the default stream).
 * Only mclbm_set_geometry, mclbm_diagnostics and mclbm_loss synchronise that
 * stream, because they return host values.  Calls on one handle must not
 * overlap from several threads.
 *
 * Errors: every call returns an mclbm_status.  MCLBM_EINVAL leaves the
 * handle, its geometry and its state unchanged.  HIP failures return MCLBM_EHIP; mclbm_last_error()
 * gives a thread-local description of the most recent failure.
 */
#ifndef MCLBM_H
#define MCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCLBM_ABI_VERSION 2u

typedef enum {
    MCLBM_OK = 0,
    MCLBM_EINVAL = -1,      /* bad argument; nothing was changed            */
    MCLBM_EHIP = -2,        /* a HIP runtime call failed                      */
    MCLBM_ENONFINITE = -3,  /* diagnostics found a non-finite population      */
    MCLBM_ESTATE = -4,      /* call out of order (e.g. step before geometry)  */
    MCLBM_EVERSION = -5     /* params.abi_version != MCLBM_ABI_VERSION        */
} mclbm_status;

/* Storage of the populations between steps.  Arithmetic is FP32 in all
 * three; FP64 is used only in the mass / saturation / loss reductions.
 *   MCLBM_F32   38 FP32 values per node.
 *   MCLBM_F16   the 36 moving populations stored in FP16 as offsets from
 *               their lattice-weight share, q_i = (f_i - w_i rho_src) /
 *               (rho1_src + rho2_src), where rho_src are the densities of
 *               the node that wrote the value one step earlier; the two rest
 *               populations stay FP32 and absorb the rounding residual of the
 *               node's moving populations, so component mass is conserved to
 *               FP32 round-off.
 *   MCLBM_BF16  as MCLBM_F16 with BF16 rounding. */
typedef enum { MCLBM_F32 = 0, MCLBM_F16 = 1, MCLBM_BF16 = 2 } mclbm_storage;

typedef struct {
    uint32_t abi_version; /* must equal MCLBM_ABI_VERSION                         */
    int32_t nx, ny, nz;   /* lattice extents, each >= 3, nx*ny*nz < 2^30          */
    int32_t storage;      /* mclbm_storage                                        */
    int32_t fluid_capacity; /* populations are stored for fluid voxels only; the
                               workspace holds this many (0 = nx*ny*nz).
                               set_geometry fails with EINVAL on more.            */
    double tau[2];        /* relaxation times tau^(1), tau^(2) > 0.5 (Eqs. 6-7)   */
    double G;             /* cohesion / adhesion strength G_coh (Eqs. 11, 13)     */
    double g[2][3];       /* body acceleration per component: F^b = rho g (Eq. 10) */
} mclbm_params;

typedef struct mclbm_lattice mclbm_lattice; /* opaque host-side handle */

/* Version of the library binary (compare with MCLBM_ABI_VERSION). */
uint32_t mclbm_abi_version(void);

/* Bytes of device workspace mclbm_create needs for these parameters.
 * EINVAL on invalid parameters. */
mclbm_status mclbm_workspace_bytes(const mclbm_params* params, size_t* bytes);

/* Create a lattice in the caller's device workspace (>= workspace_bytes,
 * 256-byte aligned, kept alive and untouched until mclbm_destroy).
 * stream: hipStream_t for all later work.  *out receives the handle. */
mclbm_status mclbm_create(const mclbm_params* params, void* d_workspace, size_t bytes,
                          void* stream, mclbm_lattice** out);

/* Geometry and wettability (Eqs. 13-15).
 * d_solid: uint8[N], nonzero = solid voxel (phi = 1).
 * d_xi:    float[N], adhesion parameter xi per voxel, read only at solid
 *          voxels that have a fluid neighbour; chi^(1) = 1 + xi,
 *          chi^(2) = 1 - xi.  |xi| < 1 required there (EINVAL otherwise).
 * Both are copied into the workspace; the caller may free them afterwards.
 * Builds the sparse storage: populations live only at fluid voxels,
 * compacted within tiles of 64 x 4 x 2 voxels; tiles without fluid are
 * dropped.  Synchronises the stream.
 * The candidate geometry is checked before anything is replaced: on EINVAL
 * (|xi| >= 1 where it is read, or more fluid voxels than fluid_capacity) the
 * lattice keeps its previous geometry, state, step counter and open planes,
 * and can go on stepping.  On success the step counter is reset to 0, the
 * state must be initialised again (init_equilibrium or load_state) and x is
 * periodic again (open planes off). */
mclbm_status mclbm_set_geometry(mclbm_lattice* lat, const uint8_t* d_solid, const float* d_xi);

/* Number of fluid voxels.  Valid after set_geometry. */
mclbm_status mclbm_fluid_count(const mclbm_lattice* lat, int64_t* count);

/* Number of solid voxels with at least one fluid neighbour (the voxels whose
 * xi matters and where gradients are non-zero).  Valid after set_geometry. */
mclbm_status mclbm_boundary_count(const mclbm_lattice* lat, int64_t* count);

/* Initial state f_i^(sigma) = w_i rho^(sigma) (fluid at rest).
 * d_rho: float[2][N] (component-major); values at solid voxels are ignored.
 * Resets the step counter to 0 and makes x periodic again (open planes
 * capture their held populations from the state they are opened on). */
mclbm_status mclbm_init_equilibrium(mclbm_lattice* lat, const float* d_rho);

/* Advance nsteps >= 0 time steps (Eq. 1: collide with Eqs. 2, 6-11, 13-15,
 * then stream with halfway bounce-back).  Asynchronous on the stream. */
mclbm_status mclbm_step(mclbm_lattice* lat, int32_t nsteps);

/* Completed steps since the last init / set_geometry / load_state. */
mclbm_status mclbm_get_time(const mclbm_lattice* lat, int64_t* t);

/* Open inlet/outlet planes along x, the drive of the paper's drainage
 * simulations (Sec. 2, the inlet and outlet boundary conditions; Sec. 4.1).
 * Planes x = 0 and x = nx-1 become ghost planes outside the physical domain;
 * the physical inlet is x = 1, the outlet x = nx-2.  Every step then:
 *   - force sums at the inlet/outlet planes see, for each missing neighbour,
 *     the pseudopotential of its mirror image across the plane (the pairing
 *     printed after Eq. 11);
 *   - after streaming, component 1 at the inlet and component 2 at the
 *     outlet are rebuilt by non-equilibrium extrapolation to the imposed
 *     densities rho1_in and rho2_out from the next plane inwards (bare
 *     barycentric velocity of that plane), so their densities equal the
 *     imposed values; the other component's five entering populations keep
 *     the values they had when the planes were first opened.
 * enable = 1: the first call (from periodic x) checks that planes 0, 1, 2,
 *   nx-3, nx-2, nx-1 are fluid (MCLBM_EINVAL otherwise; synchronises the
 *   stream) and captures the held populations from the current state; later
 *   calls only change rho1_in / rho2_out (e.g. an inlet-density ramp between
 *   step calls).  Needs an initialised state and nx >= 6; densities must be
 *   finite and > 0.
 * enable = 0: periodic x again (the held values are dropped).  set_geometry,
 *   init_equilibrium and load_state also return x to periodic.
 * Readouts still cover the whole lattice (values on the ghost planes carry
 * no physical meaning); the diagnostics' sums and maxima then leave the ghost
 * planes out.  The adjoint entry points refuse a lattice with open planes. */
mclbm_status mclbm_set_open_x(mclbm_lattice* lat, int32_t enable, double rho1_in, double rho2_out);

/* Mean Eq. (12) pressure over the fluid voxels of the inlet plane x = 1 and
 * the outlet plane x = nx-2 at the current time level, copied to the host
 * (synchronises the stream): h_out[0] = P_in, h_out[1] = P_out,
 * h_out[2] = P_c = P_in - P_out (Sec. 4.1). */
mclbm_status mclbm_open_x_pressure(mclbm_lattice* lat, double h_out[3]);

/* Readouts of the state at the current time level (pre-collision).
 * Each output is a caller device buffer; 0 is written at solid voxels.
 *   density  float[2][N]     rho^(sigma), Eq. (3)
 *   velocity float[3][N]     common velocity u = u^eq including the
 *                            half-force shift, Eq. (8)
 *   force    float[2][3][N]  F^(sigma),tot, Eq. (10)
 *   pressure float[N]        Eq. (12) */
mclbm_status mclbm_read_density(mclbm_lattice* lat, float* d_rho);
mclbm_status mclbm_read_velocity(mclbm_lattice* lat, float* d_u);
mclbm_status mclbm_read_force(mclbm_lattice* lat, float* d_F);
mclbm_status mclbm_read_pressure(mclbm_lattice* lat, float* d_P);

/* Diagnostics of the current state, reduced in FP64, copied to the host
 * (synchronises the stream):
 *   h_out[0], h_out[1]  component masses over fluid voxels
 *   h_out[2]            water saturation S_w (Sec. 4.1): fraction of fluid
 *                       voxels with rho^(2) > rho^(1)
 *   h_out[3]            smooth non-wetting fraction, mean rho1/(rho1+rho2)
 *   h_out[4]            max |u| over fluid voxels
 *   h_out[5]            number of non-finite values among rho, u at fluid voxels
 *   h_out[6]            number of fluid voxels
 * Returns MCLBM_ENONFINITE (after filling h_out) if h_out[5] > 0. */
mclbm_status mclbm_diagnostics(mclbm_lattice* lat, double h_out[7]);

/* mclbm_diagnostics for callers that cannot allocate device memory (code
 * that must not call hipMalloc, tight serving loops): the same outputs and
 * errors, with the FP64 partials and results of the reduction kept in a
 * device array of the library itself instead of the lattice's workspace --
 * 4096 blocks of 8 partials plus 8 result words (256 KiB per GPU, held until
 * the process ends).  Any lattice size fits: beyond 4096 patches of 64 x 4
 * nodes each block sums several patches (the sums then group differently
 * from mclbm_diagnostics, up to FP64 rounding; counts and the maximum are
 * identical).  Allocates nothing.  The device that was current at
 * mclbm_create must be current (EINVAL otherwise); the first call on a
 * device looks the array up.  Every call on one GPU shares that array, so
 * calls that overlap on one GPU (several threads or streams at once) race;
 * calls in sequence do not. */
mclbm_status mclbm_diagnostics_noalloc(mclbm_lattice* lat, double h_out[7]);

/* Checkpoint / restore of the full state (populations, the density field
 * the FP16/BF16 codecs decode against, and the step counter).
 * d_dst / d_src: device buffers of mclbm_state_bytes bytes, 256-byte
 * aligned.  Restoring reproduces later steps bit for bit.  Populations are
 * stored per fluid voxel, so load_state refuses (EINVAL, nothing changed) a
 * state saved for another shape, storage form or solid mask (the header
 * keeps the fluid count and a fingerprint of the mask).  load_state makes x
 * periodic again. */
mclbm_status mclbm_state_bytes(const mclbm_lattice* lat, size_t* bytes);
mclbm_status mclbm_save_state(mclbm_lattice* lat, void* d_dst);
mclbm_status mclbm_load_state(mclbm_lattice* lat, const void* d_src);

/* ---- Differentiation with respect to the adhesion parameter xi ---------
 * Loss: the smooth non-wetting saturation over a region (the water
 * saturation of Sec. 4.1 with the node count replaced by the component-1
 * fraction), L = (1/|R|) sum over fluid voxels x in R of
 * rho1(x) / (rho1(x) + rho2(x)), reduced in FP64.  d_region: uint8[N],
 * nonzero = in R.  These entry points need MCLBM_F32 storage (EINVAL
 * otherwise). */

/* L at the current time level; synchronises the stream. */
mclbm_status mclbm_loss_snw(mclbm_lattice* lat, const uint8_t* d_region, double* h_L);

/* Outlet flux of component 1 through a region (the alternative loss of the
 * adjoint): L = sum over the fluid voxels x of d_region of rho1(x) u_x(x),
 * with rho1 from Eq. 3 and u the common velocity of Eq. 8 including the
 * half-force shift (Eqs. 10-15 at the current time level).  d_region:
 * uint8[N] (nonzero = in the region).  FP64 sum; synchronises the stream. */
mclbm_status mclbm_loss_flux(mclbm_lattice* lat, const uint8_t* d_region, double* h_L);

/* Bytes of the checkpoint buffer for nsteps steps saved every `every`
 * steps: ceil(nsteps/every) population states. */
mclbm_status mclbm_checkpoint_bytes(const mclbm_lattice* lat, int32_t nsteps, int32_t every, size_t* bytes);

/* Bytes of a checkpoint buffer that also holds the level log: after the
 * mclbm_checkpoint_bytes of checkpoints (rounded up to 256 bytes), the
 * pseudopotential field psi-hat (Eqs. 3, 14-15: N component pairs, each
 * field rounded up to 256 bytes) of each of the nsteps levels, then the
 * states of the last segment's levels after its first.  Given a buffer at
 * least this large, mclbm_step_checkpointed writes each level's psi-hat
 * into the log as it computes it and steps the last segment out of place
 * through its slots (the same kernels and bytes as mclbm_step), and the
 * reverse sweep then recomputes the other segments' states with the
 * collide-stream kernel alone and the last segment not at all. */
mclbm_status mclbm_checkpoint_bytes_log(const mclbm_lattice* lat, int32_t nsteps, int32_t every, size_t* bytes);

/* Bytes of the work buffer mclbm_gradient_snw needs: two buffers of
 * `every` - 1 recomputed states (a segment's first state is read from its
 * checkpoint) and `every` psi-hat fields (one segment is recomputed while the
 * next is reversed) plus the adjoint fields. */
mclbm_status mclbm_adjoint_work_bytes(const mclbm_lattice* lat, int32_t every, size_t* bytes);

/* mclbm_step(nsteps) that also copies the state into slot k of d_ckpt
 * before step k*every (k = 0, 1, ...).  d_ckpt: device, 256-byte aligned,
 * >= mclbm_checkpoint_bytes.  With bytes >= mclbm_checkpoint_bytes_log it
 * also keeps the level log there; the lattice's state and fields are left
 * as mclbm_step leaves them either way. */
mclbm_status mclbm_step_checkpointed(mclbm_lattice* lat, int32_t nsteps, int32_t every, void* d_ckpt,
                                     size_t bytes);

/* Reverse sweep: dL/dxi for the loss at the current time level, through the
 * nsteps steps recorded by the last mclbm_step_checkpointed on this lattice:
 * d_ckpt, nsteps and every must be that call's (EINVAL otherwise), ckpt_bytes
 * the size of d_ckpt (EINVAL below mclbm_checkpoint_bytes, or below
 * mclbm_checkpoint_bytes_log when the recording kept the level log), and
 * nothing may have changed the state since -- a step, init_equilibrium, load_state,
 * set_geometry or set_open_x (ESTATE otherwise).  Each segment of `every`
 * steps is recomputed from its checkpoint into d_work (its states only with
 * the level log, which also holds the last segment), then the adjoint
 * steps run backwards through it (adjoint of streaming with bounce-back,
 * of the forced collision, Eqs. 1-2, 6-9, and of the forces and virtual
 * solid densities, Eqs. 10-15).  d_grad_xi: double[N] (output; written in
 * full, non-zero only at solid voxels with a fluid neighbour).  The
 * lattice's state is left unchanged.  Asynchronous on the stream: the
 * segment recomputes run on a second, non-blocking stream that the library
 * creates on first use (kept until mclbm_destroy), ordered against the
 * lattice's stream by events; the gradient is complete when the lattice's
 * stream reaches the end of the call's work. */
mclbm_status mclbm_gradient_snw(mclbm_lattice* lat, int32_t nsteps, int32_t every, const void* d_ckpt,
                                size_t ckpt_bytes, const uint8_t* d_region, void* d_work, size_t work_bytes,
                                double* d_grad_xi);

/* The same reverse sweep for the outlet flux of mclbm_loss_flux (same
 * arguments, work buffer and output).  The flux depends on the forces at
 * the final time, so its seed includes the adjoint of the pseudopotential
 * sums there: xi receives a direct term through the final virtual solid
 * densities (Eqs. 14-15) besides the one carried back through the steps. */
mclbm_status mclbm_gradient_flux(mclbm_lattice* lat, int32_t nsteps, int32_t every, const void* d_ckpt,
                                 size_t ckpt_bytes, const uint8_t* d_region, void* d_work, size_t work_bytes,
                                 double* d_grad_xi);

/* Per-kernel timing of mclbm_step with HIP events recorded on the lattice's
 * stream around each launch (measurement support; two event records per
 * launch while enabled, no device memory).
 *   mclbm_profile(lat, 1) clears earlier records and starts collecting;
 *   mclbm_profile(lat, 0) stops.
 *   mclbm_profile_read synchronises the stream and returns, for the three
 *   kernels of a step {0: densities (Eq. 3), 1: virtual solid densities
 *   (Eqs. 14-15), 2: forces + collision + streaming (Eqs. 1-2, 6-11, 13)},
 *   the summed durations in milliseconds and the number of launches timed. */
mclbm_status mclbm_profile(mclbm_lattice* lat, int32_t enable);
mclbm_status mclbm_profile_read(mclbm_lattice* lat, double h_ms[3], int64_t h_launches[3]);

/* Destroy the handle (the workspace is the caller's to free afterwards). */
void mclbm_destroy(mclbm_lattice* lat);

const char* mclbm_status_string(mclbm_status s);
const char* mclbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCLBM_H */
