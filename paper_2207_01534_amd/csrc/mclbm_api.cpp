// C ABI of the two-component D3Q19 step (declared in include/mclbm.h):
// parameter validation, workspace carving and launch sequencing on the
// caller's stream.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mclbm.h"
#include "lbm_adjoint.hpp"
#include "lbm_open.hpp"
#include "lbm_kernels.hpp"

using namespace mclbm;

namespace {

thread_local std::string g_last_error;

mclbm_status fail(mclbm_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(MCLBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(int storage) { return storage == MCLBM_F32 ? 4 : 2; }

struct Layout {
    size_t mv, rest, R0, R1, nbm, list, xil, nbl, counts, partial, misc, total;
    size_t fid, loc, nbf, tcnt, tbase, tapos, tact, held;
    size_t mv_bytes, rest_bytes, r_bytes;
    int np, cap;
};

int capacity_of(const mclbm_params& p) {
    const int n = p.nx * p.ny * p.nz;
    return p.fluid_capacity > 0 && p.fluid_capacity < n ? p.fluid_capacity : n;
}

Layout make_layout(const mclbm_params& p) {
    Layout L{};
    const size_t n = (size_t)p.nx * p.ny * p.nz;
    L.cap = capacity_of(p);
    // population planes hold the fluid nodes only; the stride is padded and
    // skewed by 256 elements so that the 38 streams do not start on the same
    // HBM channel when the capacity is a power of two
    L.np = (int)align_up((size_t)L.cap + 256, 256);
    const Geo g{p.nx, p.ny, p.nz, (int)n, L.np};
    const size_t nt = (size_t)tile_count(g);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, kAlign);
        return at;
    };
    L.mv_bytes = (size_t)(2 * (Q - 1)) * L.np * elem_bytes(p.storage);
    L.rest_bytes = (size_t)2 * L.np * sizeof(float);
    L.r_bytes = n * sizeof(float2);
    L.mv = take(L.mv_bytes);
    L.rest = take(L.rest_bytes);
    L.R0 = take(L.r_bytes);
    L.R1 = take(L.r_bytes);
    L.nbm = take(n * sizeof(uint32_t));
    L.list = take(n * sizeof(int));
    L.xil = take(n * sizeof(float));
    L.nbl = take(n * sizeof(uint32_t));
    L.counts = take((size_t)boundary_blocks(g) * sizeof(int));
    L.partial = take((size_t)fields_blocks(g) * 8 * sizeof(double));
    L.fid = take(n * sizeof(int));
    L.loc = take((size_t)L.cap * sizeof(uint16_t));
    L.nbf = take((size_t)L.cap * sizeof(uint32_t));
    L.tcnt = take(nt * sizeof(int));
    L.tbase = take(nt * sizeof(int));
    L.tapos = take(nt * sizeof(int));
    L.tact = take(nt * sizeof(int));
    L.held = take((size_t)2 * Q * p.ny * p.nz * sizeof(float));
    L.misc = take(256);
    L.total = off;
    return L;
}

mclbm_status check_params(const mclbm_params* p) {
    if (!p) return fail(MCLBM_EINVAL, "params is NULL");
    if (p->abi_version != MCLBM_ABI_VERSION) return fail(MCLBM_EVERSION, "abi_version mismatch");
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return fail(MCLBM_EINVAL, "extents must be >= 3");
    const double n = (double)p->nx * p->ny * p->nz;
    if (n + 512 >= 1073741824.0) return fail(MCLBM_EINVAL, "nx*ny*nz must be < 2^30");
    if (p->storage < MCLBM_F32 || p->storage > MCLBM_BF16) return fail(MCLBM_EINVAL, "bad storage");
    if (p->fluid_capacity < 0) return fail(MCLBM_EINVAL, "fluid_capacity must be >= 0");
    for (int s = 0; s < 2; ++s) {
        if (!(p->tau[s] > 0.5) || !std::isfinite(p->tau[s]))
            return fail(MCLBM_EINVAL, "tau must be finite and > 0.5");
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(p->g[s][a])) return fail(MCLBM_EINVAL, "g must be finite");
    }
    if (!std::isfinite(p->G)) return fail(MCLBM_EINVAL, "G must be finite");
    return MCLBM_OK;
}

}  // namespace

struct mclbm_lattice {
    mclbm_params p;
    Geo g;
    Phys ph;
    Layout L;
    hipStream_t stream;
    int device = -1;  // current device at mclbm_create
    char* ws;
    int64_t t;
    int nbound;
    int nfluid;
    int nactive;
    bool geometry;
    bool initialized;
    uint64_t geo_hash = 0;   // fingerprint of the solid mask (k_geometry_check)
    // Bumped by every call that changes the geometry or the state, so that a
    // reverse sweep can tell whether the state is still the one its
    // checkpoints led to.
    uint64_t generation = 0;
    struct {
        uint64_t generation;  // lattice generation right after the recording
        const void* ckpt;
        size_t bytes;
        int32_t nsteps, every;
        bool level_log;       // the level log kept after the checkpoints
        bool valid;
    } record{};
    // open inlet/outlet planes along x (lbm_open.hip)
    bool open = false;
    float rho_in = 0.f, rho_out = 0.f;
    // per-kernel event pairs recorded by mclbm_step while profiling
    bool profiling = false;
    std::vector<hipEvent_t> ev[3];
    // reverse sweep: a second stream (non-blocking, default priority) that
    // recomputes the next segment while the current one is reversed
    hipStream_t aux = nullptr;
    hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};

    float2* R(int k) const { return (float2*)(ws + (k ? L.R1 : L.R0)); }
    uint32_t* nbm() const { return (uint32_t*)(ws + L.nbm); }
    int* list() const { return (int*)(ws + L.list); }
    float* xil() const { return (float*)(ws + L.xil); }
    uint32_t* nbl() const { return (uint32_t*)(ws + L.nbl); }
    double* partial() const { return (double*)(ws + L.partial); }
    int* misc_int() const { return (int*)(ws + L.misc); }
    double* diag_out() const { return (double*)(ws + L.misc + 64); }     // 8 doubles
    double* open_out() const { return (double*)(ws + L.misc + 128); }    // 2 doubles
    int* open_count() const { return (int*)(ws + L.misc + 160); }
    unsigned long long* check_out() const { return (unsigned long long*)(ws + L.misc + 192); }  // 3 words
    float* held() const { return (float*)(ws + L.held); }
    int* fid() const { return (int*)(ws + L.fid); }
    Sparse sparse() const {
        return Sparse{(const int*)(ws + L.tact), (const int*)(ws + L.tbase), (const int*)(ws + L.tcnt),
                      (const uint16_t*)(ws + L.loc), (const uint32_t*)(ws + L.nbf), fid(), nactive};
    }

    template <class C>
    Pops<C> pops() const {
        return Pops<C>{(typename C::T*)(ws + L.mv), (float*)(ws + L.rest)};
    }
    template <class F>
    void with_codec(F&& fn) const {
        if (p.storage == MCLBM_F16)
            fn(CodecF16{});
        else if (p.storage == MCLBM_BF16)
            fn(CodecBF16{});
        else
            fn(CodecF32{});
    }
    // psi-hat of the current time level in R[t & 1]
    void fill_psi() {
        const int odd = (int)(t & 1);
        float2* psi = R((int)(t & 1));
        const float2* rprev = R((int)((t + 1) & 1));
        with_codec([&](auto c) {
            using C = decltype(c);
            launch_density<C>(pops<C>(), sparse(), rprev, psi, g, ph.G, odd, stream);
        });
        launch_ivsd(list(), xil(), nbl(), nbound, psi, g, stream);
        if (open) launch_open_mirror(psi, g, stream);
    }
    void fields(float* o_rho, float* o_u, float* o_F, float* o_P, double* partial, double* out,
                int max_blocks = 0) {
        fill_psi();
        const int odd = (int)(t & 1);
        const float2* psi = R((int)(t & 1));
        const float2* rprev = R((int)((t + 1) & 1));
        with_codec([&](auto c) {
            using C = decltype(c);
            launch_fields<C>(pops<C>(), fid(), nbm(), rprev, psi, g, ph, odd, o_rho, o_u, o_F, o_P, partial,
                             out, open ? 1 : 0, stream, max_blocks);
        });
    }
};

extern "C" {

uint32_t mclbm_abi_version(void) { return MCLBM_ABI_VERSION; }

mclbm_status mclbm_workspace_bytes(const mclbm_params* params, size_t* bytes) {
    mclbm_status st = check_params(params);
    if (st != MCLBM_OK) return st;
    if (!bytes) return fail(MCLBM_EINVAL, "bytes is NULL");
    *bytes = make_layout(*params).total;
    return MCLBM_OK;
}

mclbm_status mclbm_create(const mclbm_params* params, void* d_workspace, size_t bytes, void* stream,
                          mclbm_lattice** out) {
    mclbm_status st = check_params(params);
    if (st != MCLBM_OK) return st;
    if (!out) return fail(MCLBM_EINVAL, "out is NULL");
    if (!d_workspace) return fail(MCLBM_EINVAL, "workspace is NULL");
    if (((uintptr_t)d_workspace) % kAlign) return fail(MCLBM_EINVAL, "workspace must be 256-byte aligned");
    const Layout L = make_layout(*params);
    if (bytes < L.total) return fail(MCLBM_EINVAL, "workspace too small");
    mclbm_lattice* lat = new (std::nothrow) mclbm_lattice();
    if (!lat) return fail(MCLBM_EINVAL, "out of host memory");
    lat->p = *params;
    lat->L = L;
    lat->g = Geo{params->nx, params->ny, params->nz, params->nx * params->ny * params->nz, L.np};
    for (int s = 0; s < 2; ++s) {
        lat->ph.a[s] = (float)(params->tau[s] - 0.5);
        for (int a = 0; a < 3; ++a) lat->ph.g[s][a] = (float)params->g[s][a];
    }
    lat->ph.G = (float)params->G;
    lat->stream = (hipStream_t)stream;
    // creation itself does no device work (and succeeds without a device);
    // the device only matters to the entry points that use the library's
    // own per-device scratch
    if (hipGetDevice(&lat->device) != hipSuccess) {
        lat->device = -1;
        (void)hipGetLastError();
    }
    lat->ws = (char*)d_workspace;
    lat->t = 0;
    lat->nbound = 0;
    lat->nfluid = 0;
    lat->nactive = 0;
    lat->geometry = false;
    lat->initialized = false;
    *out = lat;
    return MCLBM_OK;
}

mclbm_status mclbm_set_geometry(mclbm_lattice* lat, const uint8_t* d_solid, const float* d_xi) {
    if (!lat || !d_solid || !d_xi) return fail(MCLBM_EINVAL, "NULL argument");
    const Geo& g = lat->g;
    const Layout& L = lat->L;
    hipStream_t s = lat->stream;
    // Validate first, committing nothing: the candidate neighbour words go to
    // the psi-hat field of the current level, which every step and readout
    // rewrites before reading it, so a refused geometry leaves the lattice's
    // geometry and state as they were.
    uint32_t* cand = (uint32_t*)lat->R((int)(lat->t & 1));
    launch_neighbour_bits(d_solid, cand, g, s);
    launch_geometry_check(cand, d_xi, g, lat->check_out(), s);
    HIP_TRY(hipGetLastError());
    unsigned long long chk[3] = {0, 0, 0};  // bad xi, fluid nodes, mask fingerprint
    HIP_TRY(hipMemcpyAsync(chk, lat->check_out(), sizeof(chk), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (chk[0]) return fail(MCLBM_EINVAL, "|xi| must be < 1 at solid voxels with a fluid neighbour");
    if (chk[1] > (unsigned long long)L.cap) return fail(MCLBM_EINVAL, "more fluid voxels than params.fluid_capacity");
    // commit
    lat->geometry = false;
    lat->initialized = false;
    lat->open = false;
    lat->record.valid = false;
    lat->generation += 1;
    HIP_TRY(hipMemcpyAsync(lat->nbm(), cand, (size_t)g.n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    int* counts = (int*)(lat->ws + L.counts);
    launch_boundary_list(lat->nbm(), d_xi, counts, lat->misc_int(), lat->list(), lat->xil(), lat->nbl(), g, s);
    int* tcnt = (int*)(lat->ws + L.tcnt);
    int* tbase = (int*)(lat->ws + L.tbase);
    int* tapos = (int*)(lat->ws + L.tapos);
    launch_tile_census(lat->nbm(), g, tcnt, tbase, tapos, lat->misc_int() + 1, s);
    launch_tile_ids(lat->nbm(), g, tcnt, tbase, tapos, lat->fid(), (uint16_t*)(lat->ws + L.loc),
                    (uint32_t*)(lat->ws + L.nbf), (int*)(lat->ws + L.tact), s);
    HIP_TRY(hipGetLastError());
    int totals[3] = {0, 0, 0};  // boundary solids, fluid nodes, active tiles
    HIP_TRY(hipMemcpyAsync(totals, lat->misc_int(), sizeof(totals), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    lat->nbound = totals[0];
    lat->nfluid = totals[1];
    lat->nactive = totals[2];
    lat->geo_hash = chk[2];
    lat->geometry = true;
    lat->t = 0;
    return MCLBM_OK;
}

mclbm_status mclbm_fluid_count(const mclbm_lattice* lat, int64_t* count) {
    if (!lat || !count) return fail(MCLBM_EINVAL, "NULL argument");
    if (!lat->geometry) return fail(MCLBM_ESTATE, "geometry not set");
    *count = lat->nfluid;
    return MCLBM_OK;
}

mclbm_status mclbm_boundary_count(const mclbm_lattice* lat, int64_t* count) {
    if (!lat || !count) return fail(MCLBM_EINVAL, "NULL argument");
    if (!lat->geometry) return fail(MCLBM_ESTATE, "geometry not set");
    *count = lat->nbound;
    return MCLBM_OK;
}

mclbm_status mclbm_init_equilibrium(mclbm_lattice* lat, const float* d_rho) {
    if (!lat || !d_rho) return fail(MCLBM_EINVAL, "NULL argument");
    if (!lat->geometry) return fail(MCLBM_ESTATE, "set_geometry must come first");
    // state at t = 0; the codecs' reference density of the previous level is R[1]
    lat->with_codec([&](auto c) {
        using C = decltype(c);
        launch_init<C>(lat->pops<C>(), lat->nbm(), lat->fid(), d_rho, lat->R(1), lat->list(), lat->xil(), lat->nbl(),
                       lat->nbound, lat->g, lat->ph.G, lat->stream);
    });
    HIP_TRY(hipGetLastError());
    lat->t = 0;
    lat->initialized = true;
    lat->open = false;  // held entering populations belong to the state they were captured from
    lat->record.valid = false;
    lat->generation += 1;
    return MCLBM_OK;
}

mclbm_status mclbm_step(mclbm_lattice* lat, int32_t nsteps) {
    if (!lat) return fail(MCLBM_EINVAL, "NULL handle");
    if (nsteps < 0) return fail(MCLBM_EINVAL, "nsteps must be >= 0");
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    hipError_t mark_err = hipSuccess;  // first failure of the profiling events
    auto mark = [&](int k) {
        if (!lat->profiling || mark_err != hipSuccess) return;
        hipEvent_t e;
        mark_err = hipEventCreate(&e);
        if (mark_err != hipSuccess) return;
        lat->ev[k].push_back(e);
        mark_err = hipEventRecord(e, lat->stream);
    };
    for (int32_t k = 0; k < nsteps; ++k) {
        const int odd = (int)(lat->t & 1);
        float2* psi = lat->R((int)(lat->t & 1));
        const float2* rprev = lat->R((int)((lat->t + 1) & 1));
        lat->with_codec([&](auto c) {
            using C = decltype(c);
            mark(0);
            launch_density<C>(lat->pops<C>(), lat->sparse(), rprev, psi, lat->g, lat->ph.G, odd, lat->stream);
            mark(0);
            mark(1);
            launch_ivsd(lat->list(), lat->xil(), lat->nbl(), lat->nbound, psi, lat->g, lat->stream);
            mark(1);
            if (lat->open) launch_open_mirror(psi, lat->g, lat->stream);
            mark(2);
            launch_collide_stream<C>(lat->pops<C>(), lat->pops<C>(), lat->sparse(), rprev, psi, lat->g, lat->ph, odd,
                                     lat->stream);
            mark(2);
            if (lat->open)
                launch_open_rebuild<C>(lat->pops<C>(), lat->fid(), psi, lat->held(), lat->g, 1 - odd,
                                       lat->rho_in, lat->rho_out, lat->ph.G, lat->stream);
        });
        lat->t += 1;
    }
    if (nsteps > 0) lat->generation += 1;
    HIP_TRY(hipGetLastError());
    HIP_TRY(mark_err);
    return MCLBM_OK;
}

mclbm_status mclbm_set_open_x(mclbm_lattice* lat, int32_t enable, double rho1_in, double rho2_out) {
    if (!lat) return fail(MCLBM_EINVAL, "NULL handle");
    if (!enable) {
        if (lat->open) lat->generation += 1;
        lat->open = false;
        return MCLBM_OK;
    }
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    if (!(rho1_in > 0.0) || !(rho2_out > 0.0) || !std::isfinite(rho1_in) || !std::isfinite(rho2_out))
        return fail(MCLBM_EINVAL, "imposed densities must be finite and > 0");
    if (lat->g.nx < 6) return fail(MCLBM_EINVAL, "open x planes need nx >= 6");
    if (!lat->open) {
        int solid = 0;
        launch_open_check(lat->nbm(), lat->g, lat->open_count(), lat->stream);
        HIP_TRY(hipMemcpyAsync(&solid, lat->open_count(), sizeof(int), hipMemcpyDeviceToHost, lat->stream));
        HIP_TRY(hipStreamSynchronize(lat->stream));
        if (solid) return fail(MCLBM_EINVAL, "planes x = 0, 1, 2, nx-3, nx-2, nx-1 must be fluid");
        const int odd = (int)(lat->t & 1);
        lat->with_codec([&](auto c) {
            using C = decltype(c);
            launch_open_capture<C>(lat->pops<C>(), lat->fid(), lat->nbm(), lat->R(1 - odd), lat->held(), lat->g,
                                   odd, lat->ph.G, lat->stream);
        });
        HIP_TRY(hipGetLastError());
    }
    lat->rho_in = (float)rho1_in;
    lat->rho_out = (float)rho2_out;
    lat->open = true;
    lat->generation += 1;
    return MCLBM_OK;
}

mclbm_status mclbm_open_x_pressure(mclbm_lattice* lat, double h_out[3]) {
    if (!lat || !h_out) return fail(MCLBM_EINVAL, "NULL argument");
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    if (lat->g.nx < 6) return fail(MCLBM_EINVAL, "open x planes need nx >= 6");
    lat->fill_psi();
    launch_open_pressure(lat->R((int)(lat->t & 1)), lat->nbm(), lat->g, lat->ph.G, lat->open_out(), lat->stream);
    double out[2];
    HIP_TRY(hipMemcpyAsync(out, lat->open_out(), sizeof(out), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    h_out[0] = out[0];
    h_out[1] = out[1];
    h_out[2] = out[0] - out[1];
    return MCLBM_OK;
}

mclbm_status mclbm_get_time(const mclbm_lattice* lat, int64_t* t) {
    if (!lat || !t) return fail(MCLBM_EINVAL, "NULL argument");
    *t = lat->t;
    return MCLBM_OK;
}

static mclbm_status readout(mclbm_lattice* lat, float* r, float* u, float* F, float* P) {
    if (!lat || !(r || u || F || P)) return fail(MCLBM_EINVAL, "NULL argument");
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    lat->fields(r, u, F, P, nullptr, nullptr);
    HIP_TRY(hipGetLastError());
    return MCLBM_OK;
}

mclbm_status mclbm_read_density(mclbm_lattice* lat, float* d_rho) {
    return readout(lat, d_rho, nullptr, nullptr, nullptr);
}
mclbm_status mclbm_read_velocity(mclbm_lattice* lat, float* d_u) {
    return readout(lat, nullptr, d_u, nullptr, nullptr);
}
mclbm_status mclbm_read_force(mclbm_lattice* lat, float* d_F) {
    return readout(lat, nullptr, nullptr, d_F, nullptr);
}
mclbm_status mclbm_read_pressure(mclbm_lattice* lat, float* d_P) {
    return readout(lat, nullptr, nullptr, nullptr, d_P);
}

// Copies the reduced diagnostics to the host and turns counts into fractions.
static mclbm_status finish_diagnostics(mclbm_lattice* lat, const double* d_out, double h_out[7]) {
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h_out, d_out, 7 * sizeof(double), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    // the kernels return counts and sums; saturations are fractions of the fluid voxels
    if (h_out[6] > 0) {
        h_out[2] /= h_out[6];
        h_out[3] /= h_out[6];
    }
    if (h_out[5] > 0) return fail(MCLBM_ENONFINITE, "non-finite density or velocity");
    return MCLBM_OK;
}

mclbm_status mclbm_diagnostics(mclbm_lattice* lat, double h_out[7]) {
    if (!lat || !h_out) return fail(MCLBM_EINVAL, "NULL argument");
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    lat->fields(nullptr, nullptr, nullptr, nullptr, lat->partial(), lat->diag_out());
    return finish_diagnostics(lat, lat->diag_out(), h_out);
}

mclbm_status mclbm_diagnostics_noalloc(mclbm_lattice* lat, double h_out[7]) {
    if (!lat || !h_out) return fail(MCLBM_EINVAL, "NULL argument");
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (lat->device < 0 || dev != lat->device)
        return fail(MCLBM_EINVAL, "the device current at mclbm_create must be the current device");
    double* scr = nullptr;
    HIP_TRY(scratch_address(dev, &scr));
    // at most kScratchBlocks partials whatever the lattice size: a larger
    // lattice gives each block several patches to sum
    double* out = scr + 8 * (size_t)kScratchBlocks;
    lat->fields(nullptr, nullptr, nullptr, nullptr, scr, out, kScratchBlocks);
    return finish_diagnostics(lat, out, h_out);
}

// Saved state: [header 256 B][moving planes][rest planes][previous-level densities]
// Populations are indexed by fluid id, so a state fits only a lattice with
// the same solid mask: the header keeps the fluid count and the mask's
// fingerprint.
struct StateHeader {
    uint64_t magic;
    int64_t t;
    int32_t nx, ny, nz, storage;
    int64_t nfluid;
    uint64_t geo_hash;
    uint64_t pad[2];
};
static constexpr uint64_t kMagic = 0x4d434c424d535432ull;  // "MCLBMST2"

mclbm_status mclbm_state_bytes(const mclbm_lattice* lat, size_t* bytes) {
    if (!lat || !bytes) return fail(MCLBM_EINVAL, "NULL argument");
    *bytes = kAlign + align_up(lat->L.mv_bytes, kAlign) + align_up(lat->L.rest_bytes, kAlign) +
             align_up(lat->L.r_bytes, kAlign);
    return MCLBM_OK;
}

mclbm_status mclbm_save_state(mclbm_lattice* lat, void* d_dst) {
    if (!lat || !d_dst) return fail(MCLBM_EINVAL, "NULL argument");
    if (((uintptr_t)d_dst) % kAlign) return fail(MCLBM_EINVAL, "state buffer must be 256-byte aligned");
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    const Layout& L = lat->L;
    char* dst = (char*)d_dst;
    StateHeader h{kMagic, lat->t, lat->p.nx, lat->p.ny, lat->p.nz, lat->p.storage, lat->nfluid, lat->geo_hash, {0, 0}};
    uint64_t words[8];
    static_assert(sizeof(h) == sizeof(words), "header is eight 64-bit words");
    std::memcpy(words, &h, sizeof(h));
    launch_store_words((uint64_t*)dst, {words[0], words[1], words[2], words[3]}, lat->stream);
    launch_store_words((uint64_t*)dst + 4, {words[4], words[5], words[6], words[7]}, lat->stream);
    size_t off = kAlign;
    HIP_TRY(hipMemcpyAsync(dst + off, lat->ws + L.mv, L.mv_bytes, hipMemcpyDeviceToDevice, lat->stream));
    off += align_up(L.mv_bytes, kAlign);
    HIP_TRY(hipMemcpyAsync(dst + off, lat->ws + L.rest, L.rest_bytes, hipMemcpyDeviceToDevice, lat->stream));
    off += align_up(L.rest_bytes, kAlign);
    HIP_TRY(hipMemcpyAsync(dst + off, lat->R((int)((lat->t + 1) & 1)), L.r_bytes, hipMemcpyDeviceToDevice,
                           lat->stream));
    return MCLBM_OK;
}

mclbm_status mclbm_load_state(mclbm_lattice* lat, const void* d_src) {
    if (!lat || !d_src) return fail(MCLBM_EINVAL, "NULL argument");
    if (((uintptr_t)d_src) % kAlign) return fail(MCLBM_EINVAL, "state buffer must be 256-byte aligned");
    if (!lat->geometry) return fail(MCLBM_ESTATE, "set_geometry must come first");
    const Layout& L = lat->L;
    const char* src = (const char*)d_src;
    StateHeader h{};
    HIP_TRY(hipMemcpyAsync(&h, src, sizeof(h), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    if (h.magic != kMagic || h.nx != lat->p.nx || h.ny != lat->p.ny || h.nz != lat->p.nz ||
        h.storage != lat->p.storage || h.t < 0)
        return fail(MCLBM_EINVAL, "state buffer does not match this lattice");
    if (h.nfluid != lat->nfluid || h.geo_hash != lat->geo_hash)
        return fail(MCLBM_EINVAL, "state buffer was saved under another solid mask");
    size_t off = kAlign;
    HIP_TRY(hipMemcpyAsync(lat->ws + L.mv, src + off, L.mv_bytes, hipMemcpyDeviceToDevice, lat->stream));
    off += align_up(L.mv_bytes, kAlign);
    HIP_TRY(hipMemcpyAsync(lat->ws + L.rest, src + off, L.rest_bytes, hipMemcpyDeviceToDevice, lat->stream));
    off += align_up(L.rest_bytes, kAlign);
    HIP_TRY(hipMemcpyAsync(lat->R((int)((h.t + 1) & 1)), src + off, L.r_bytes, hipMemcpyDeviceToDevice,
                           lat->stream));
    lat->t = h.t;
    lat->initialized = true;
    lat->open = false;  // held entering populations belong to the state they were captured from
    lat->record.valid = false;
    lat->generation += 1;
    return MCLBM_OK;
}

// ---------------------------------------------------------------------------
// Loss and adjoint (FP32 population storage)
// ---------------------------------------------------------------------------
static size_t state_slot_bytes(const Layout& L) {
    return align_up(L.mv_bytes, kAlign) + align_up(L.rest_bytes, kAlign);
}
static Pops<CodecF32> slot_pops(char* base, const Layout& L) {
    return Pops<CodecF32>{(float*)base, (float*)(base + align_up(L.mv_bytes, kAlign))};
}

mclbm_status mclbm_loss_snw(mclbm_lattice* lat, const uint8_t* d_region, double* h_L) {
    if (!lat || !d_region || !h_L) return fail(MCLBM_EINVAL, "NULL argument");
    if (lat->p.storage != MCLBM_F32) return fail(MCLBM_EINVAL, "loss and adjoint need FP32 storage");
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    double out[2];
    launch_loss(lat->pops<CodecF32>(), lat->fid(), lat->nbm(), d_region, lat->g, (int)(lat->t & 1), lat->partial(),
                lat->diag_out(), lat->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, lat->diag_out(), sizeof(out), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    *h_L = out[0];
    return MCLBM_OK;
}

mclbm_status mclbm_loss_flux(mclbm_lattice* lat, const uint8_t* d_region, double* h_L) {
    if (!lat || !d_region || !h_L) return fail(MCLBM_EINVAL, "NULL argument");
    if (lat->p.storage != MCLBM_F32) return fail(MCLBM_EINVAL, "loss and adjoint need FP32 storage");
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    lat->fill_psi();
    launch_loss_flux(lat->pops<CodecF32>(), lat->fid(), lat->nbm(), d_region, lat->R((int)(lat->t & 1)), lat->g,
                     lat->ph, (int)(lat->t & 1), lat->partial(), lat->diag_out(), lat->stream);
    HIP_TRY(hipGetLastError());
    double out[2];
    HIP_TRY(hipMemcpyAsync(out, lat->diag_out(), sizeof(out), hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    *h_L = out[0] * out[1];  // mean times count: the sum over the region
    return MCLBM_OK;
}

mclbm_status mclbm_checkpoint_bytes(const mclbm_lattice* lat, int32_t nsteps, int32_t every, size_t* bytes) {
    if (!lat || !bytes || nsteps < 1 || every < 1) return fail(MCLBM_EINVAL, "bad argument");
    *bytes = (size_t)((nsteps + every - 1) / every) * state_slot_bytes(lat->L);
    return MCLBM_OK;
}

// One psi-hat field (N component pairs) of the checkpoint buffer's level log.
static size_t psi_field_bytes(const Geo& g) { return align_up((size_t)g.n * sizeof(float2), kAlign); }

// A checkpoint buffer with the level log: the checkpoints, then the psi-hat
// field of every level (offset psi), then the states of the last segment
// after its first, which is its checkpoint (offset tail, tail_slots slots).
struct LevelLog {
    size_t psi, tail, total;
    int tail_slots;
};

static LevelLog level_log_layout(const mclbm_lattice* lat, int32_t nsteps, int32_t every) {
    size_t states = 0;
    mclbm_checkpoint_bytes(lat, nsteps, every, &states);
    LevelLog o;
    o.psi = align_up(states, kAlign);
    o.tail = o.psi + (size_t)nsteps * psi_field_bytes(lat->g);
    o.tail_slots = nsteps - (nsteps - 1) / every * every - 1;  // the last segment's length - 1
    o.total = o.tail + (size_t)o.tail_slots * state_slot_bytes(lat->L);
    return o;
}

mclbm_status mclbm_checkpoint_bytes_log(const mclbm_lattice* lat, int32_t nsteps, int32_t every, size_t* bytes) {
    if (!lat || !bytes || nsteps < 1 || every < 1) return fail(MCLBM_EINVAL, "bad argument");
    *bytes = level_log_layout(lat, nsteps, every).total;
    return MCLBM_OK;
}

struct AdjointWork {
    char* seg[2];   // two segment buffers of `every` - 1 state slots (a segment's first state is its checkpoint)
    char* psi[2];   // and of `every` psi-hat fields (n float2 each)
    float* lam[2];   // [19][np] component pairs, by fluid id
    float* abar;     // [3][n] pairs (component 1, component 2), by lattice node (read at solid neighbours)
    float2* rbar[2]; // [np], by fluid id
    float2* nbar;
    double* gacc;   // per boundary-list entry
    int* node_of;   // lattice index of each fluid id
    int* nfid;      // [18][np] neighbour fluid ids of each fluid id (-1 at solid)
    size_t total;
};

static AdjointWork adjoint_layout(const mclbm_lattice* lat, int32_t every, char* base) {
    const size_t n = (size_t)lat->g.n;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t at = off;
        off = align_up(off + b, kAlign);
        return base + at;
    };
    AdjointWork w;
    for (int b = 0; b < 2; ++b) {
        w.seg[b] = take((size_t)(every - 1) * state_slot_bytes(lat->L));
        w.psi[b] = take((size_t)every * align_up(n * sizeof(float2), kAlign));
    }
    const size_t np = (size_t)lat->L.np;  // the adjoint of the populations is indexed by fluid id
    w.lam[0] = (float*)take(2 * Q * np * sizeof(float));
    w.lam[1] = (float*)take(2 * Q * np * sizeof(float));
    w.abar = (float*)take(6 * n * sizeof(float));
    w.rbar[0] = (float2*)take(np * sizeof(float2));
    w.rbar[1] = (float2*)take(np * sizeof(float2));
    w.nbar = (float2*)take(n * sizeof(float2));
    w.gacc = (double*)take(n * sizeof(double));
    w.node_of = (int*)take((size_t)lat->L.cap * sizeof(int));
    w.nfid = (int*)take((size_t)(Q - 1) * np * sizeof(int));
    w.total = off;
    return w;
}

mclbm_status mclbm_adjoint_work_bytes(const mclbm_lattice* lat, int32_t every, size_t* bytes) {
    if (!lat || !bytes || every < 1) return fail(MCLBM_EINVAL, "bad argument");
    *bytes = adjoint_layout(lat, every, nullptr).total;
    return MCLBM_OK;
}

mclbm_status mclbm_step_checkpointed(mclbm_lattice* lat, int32_t nsteps, int32_t every, void* d_ckpt,
                                     size_t bytes) {
    if (!lat || !d_ckpt || nsteps < 1 || every < 1) return fail(MCLBM_EINVAL, "bad argument");
    if (lat->p.storage != MCLBM_F32) return fail(MCLBM_EINVAL, "loss and adjoint need FP32 storage");
    if (((uintptr_t)d_ckpt) % kAlign) return fail(MCLBM_EINVAL, "checkpoint buffer must be 256-byte aligned");
    if (!lat->initialized) return fail(MCLBM_ESTATE, "state not initialised");
    if (lat->open) return fail(MCLBM_EINVAL, "the adjoint covers periodic x only (open planes are enabled)");
    size_t need = 0;
    mclbm_checkpoint_bytes(lat, nsteps, every, &need);
    if (bytes < need) return fail(MCLBM_EINVAL, "checkpoint buffer too small");
    const Layout& L = lat->L;
    const Geo& g = lat->g;
    hipStream_t s = lat->stream;
    // With room for the level log, each level's psi-hat is written there (the
    // same kernels and bytes as mclbm_step), and the levels of the last
    // segment run out of place through its slots, so that the reverse sweep
    // recomputes neither.  The last two levels' psi-hat still goes through
    // the lattice's own fields, which are left as mclbm_step leaves them, as
    // is the state.  Solid nodes without a fluid neighbour keep whatever the
    // log held: no kernel reads psi-hat there.
    const LevelLog LL = level_log_layout(lat, nsteps, every);
    const bool level_log = bytes >= LL.total;
    const int k_last = (nsteps - 1) / every * every;  // first level of the last segment
    const Pops<CodecF32> P = lat->pops<CodecF32>();
    auto tail = [&](int j) { return slot_pops((char*)d_ckpt + LL.tail + (size_t)j * state_slot_bytes(L), L); };
    for (int32_t k = 0; k < nsteps; ++k) {
        if (k % every == 0) {
            char* slot = (char*)d_ckpt + (size_t)(k / every) * state_slot_bytes(L);
            const Pops<CodecF32> d = slot_pops(slot, L);
            HIP_TRY(hipMemcpyAsync(d.mv, lat->ws + L.mv, L.mv_bytes, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(d.rest, lat->ws + L.rest, L.rest_bytes, hipMemcpyDeviceToDevice, s));
        }
        if (!level_log) {
            mclbm_status st = mclbm_step(lat, 1);
            if (st != MCLBM_OK) return st;
            continue;
        }
        const int odd = (int)(lat->t & 1);
        float2* logged = (float2*)((char*)d_ckpt + LL.psi + (size_t)k * psi_field_bytes(g));
        float2* psi = k + 2 >= nsteps ? lat->R(odd) : logged;
        const Pops<CodecF32> src = k <= k_last ? P : tail(k - k_last - 1);
        const Pops<CodecF32> dst = (k < k_last || k + 1 == nsteps) ? P : tail(k - k_last);
        launch_density<CodecF32>(src, lat->sparse(), lat->R(0) /* not read for FP32 */, psi, g, lat->ph.G, odd, s);
        launch_ivsd(lat->list(), lat->xil(), lat->nbl(), lat->nbound, psi, g, s);
        launch_collide_stream<CodecF32>(src, dst, lat->sparse(), psi, psi, g, lat->ph, odd, s);
        HIP_TRY(hipGetLastError());
        if (psi != logged)
            HIP_TRY(hipMemcpyAsync(logged, psi, (size_t)g.n * sizeof(float2), hipMemcpyDeviceToDevice, s));
        lat->t += 1;
        lat->generation += 1;
    }
    lat->record.generation = lat->generation;
    lat->record.ckpt = d_ckpt;
    lat->record.bytes = bytes;
    lat->record.nsteps = nsteps;
    lat->record.every = every;
    lat->record.level_log = level_log;
    lat->record.valid = true;
    return MCLBM_OK;
}

// The reverse sweep's auxiliary stream and events, created on first use on
// the lattice's device and kept until mclbm_destroy.
// All or nothing: on a failure the lattice keeps no partial set.
static hipError_t ensure_aux(mclbm_lattice* lat) {
    if (lat->aux) return hipSuccess;
    hipStream_t st = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    for (int k = 0; k < 5 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        if (st) (void)hipStreamDestroy(st);
        return e;
    }
    lat->aux = st;
    lat->ev_start = ev[0];
    lat->ev_rec[0] = ev[1];
    lat->ev_rec[1] = ev[2];
    lat->ev_rev[0] = ev[3];
    lat->ev_rev[1] = ev[4];
    return hipSuccess;
}

enum class LossKind { Snw, Flux };

static mclbm_status gradient(mclbm_lattice* lat, LossKind kind, int32_t nsteps, int32_t every, const void* d_ckpt,
                             size_t ckpt_bytes, const uint8_t* d_region, void* d_work, size_t work_bytes,
                             double* d_grad_xi) {
    if (!lat || !d_ckpt || !d_region || !d_work || !d_grad_xi || nsteps < 1 || every < 1)
        return fail(MCLBM_EINVAL, "bad argument");
    if (lat->p.storage != MCLBM_F32) return fail(MCLBM_EINVAL, "loss and adjoint need FP32 storage");
    if (((uintptr_t)d_work) % kAlign || ((uintptr_t)d_ckpt) % kAlign)
        return fail(MCLBM_EINVAL, "work and checkpoint buffers must be 256-byte aligned");
    if (lat->open) return fail(MCLBM_EINVAL, "the adjoint covers periodic x only (open planes are enabled)");
    size_t need = 0;
    mclbm_checkpoint_bytes(lat, nsteps, every, &need);
    if (ckpt_bytes < need) return fail(MCLBM_EINVAL, "checkpoint buffer smaller than nsteps / every need");
    if (!lat->initialized || !lat->record.valid || lat->record.generation != lat->generation)
        return fail(MCLBM_ESTATE, "the state is not the one left by the last step_checkpointed "
                                  "(the lattice was stepped, re-initialised or reloaded since)");
    if (lat->record.ckpt != d_ckpt || lat->record.nsteps != nsteps || lat->record.every != every)
        return fail(MCLBM_EINVAL, "checkpoints, nsteps or every differ from the last step_checkpointed");
    const bool level_log = lat->record.level_log;
    const LevelLog LL = level_log_layout(lat, nsteps, every);
    if (level_log && ckpt_bytes < LL.total)
        return fail(MCLBM_EINVAL, "checkpoint buffer smaller than the level log it was recorded with");
    const AdjointWork W = adjoint_layout(lat, every, (char*)d_work);
    if (work_bytes < W.total) return fail(MCLBM_EINVAL, "work buffer too small");
    const Layout& L = lat->L;
    const Geo& g = lat->g;
    const size_t n = (size_t)g.n;
    const size_t slot = state_slot_bytes(L);
    const size_t psi_stride = psi_field_bytes(g);
    hipStream_t s = lat->stream;
    const int64_t t_end = lat->t, t0 = t_end - nsteps;
    const int nseg = (nsteps + every - 1) / every;
    // state of level k of segment seg: the first is the checkpoint itself
    // (which every kernel here only reads), the others are recomputed into
    // buffer b or, for the last segment, kept by the level log
    auto level_pops = [&](int seg, int b, int k) {
        if (k == 0) return slot_pops((char*)d_ckpt + (size_t)seg * slot, L);
        if (level_log && seg == nseg - 1) return slot_pops((char*)d_ckpt + LL.tail + (size_t)(k - 1) * slot, L);
        return slot_pops(W.seg[b] + (size_t)(k - 1) * slot, L);
    };
    // psi-hat of level k of segment seg: from the level log, or recomputed
    // into buffer b
    auto level_psi = [&](int seg, int b, int k) {
        return level_log ? (float2*)((char*)d_ckpt + LL.psi + (size_t)(seg * every + k) * psi_stride)
                         : (float2*)(W.psi[b] + (size_t)k * psi_stride);
    };

    launch_zero(W.gacc, (size_t)lat->nbound * sizeof(double), s);
    launch_zero(W.abar, 6 * n * sizeof(float), s);  // solid entries are never written by the reverse steps
    launch_node_of(lat->fid(), g, W.node_of, s);
    launch_adj_neighbours(W.node_of, lat->nfluid, lat->fid(), g, W.nfid, s);
    launch_zero(d_grad_xi, n * sizeof(double), s);
    // seed from the final state (the lattice's current populations)
    int cur = 0;  // lam[cur], rbar[cur] hold dL/df at the time level being processed
    if (kind == LossKind::Snw) {
        launch_loss(lat->pops<CodecF32>(), lat->fid(), lat->nbm(), d_region, g, (int)(t_end & 1), lat->partial(),
                    lat->diag_out(), s);
        launch_adj_seed(lat->pops<CodecF32>(), lat->fid(), lat->nbm(), d_region, g, (int)(t_end & 1),
                        lat->diag_out(), W.lam[cur], W.rbar[cur], s);
    } else {
        // the flux depends on the forces at the final time: its seed holds a
        // local part and the adjoint of the pseudopotential sums, which the
        // IVSD and density adjoints turn into the direct xi term and the
        // neighbours' density adjoint
        lat->fill_psi();
        const float2* psi_end = lat->R((int)(t_end & 1));
        launch_adj_seed_flux(lat->pops<CodecF32>(), lat->fid(), lat->nbm(), d_region, psi_end, g, lat->ph,
                             (int)(t_end & 1), W.lam[cur], W.abar, s);
        launch_adj_ivsd(lat->list(), lat->xil(), lat->nbound, lat->nbm(), psi_end, W.abar, g, W.gacc, W.nbar, s);
        launch_adj_rho(W.node_of, lat->nfluid, lat->nbm(), W.abar, W.nbar, g, W.rbar[cur], s);
    }
    // Segment seg is recomputed into buffer seg & 1 on the auxiliary stream
    // and reversed from it on the lattice's stream; the recompute of segment
    // seg - 1 runs while segment seg is reversed (the two touch disjoint
    // memory; the lattice's geometry and the checkpoints are only read), and
    // waits for the reverse of segment seg + 1, the last user of its buffer.
    HIP_TRY(ensure_aux(lat));
    hipStream_t s2 = lat->aux;
    HIP_TRY(hipEventRecord(lat->ev_start, s));
    HIP_TRY(hipStreamWaitEvent(s2, lat->ev_start, 0));
    // on every way out, later work on the lattice's stream also waits for
    // whatever was queued on the auxiliary stream (already implied on success)
    struct JoinAux {
        hipStream_t s, s2;
        hipEvent_t e;
        ~JoinAux() {
            if (hipEventRecord(e, s2) == hipSuccess) (void)hipStreamWaitEvent(s, e, 0);
        }
    } join{s, s2, lat->ev_start};
    auto recompute = [&](int seg) -> mclbm_status {
        const int b = seg & 1;
        const int64_t ta = t0 + (int64_t)seg * every;
        const int len = (int)((ta + every <= t_end ? ta + every : t_end) - ta);
        // the segment's states (and their psi-hat fields when there is no
        // level log, which also holds the last segment's states)
        for (int k = 0; k < len && !(level_log && seg == nseg - 1); ++k) {
            const int odd = (int)((ta + k) & 1);
            const Pops<CodecF32> sk = level_pops(seg, b, k);
            float2* psi = level_psi(seg, b, k);
            if (!level_log) {
                launch_density<CodecF32>(sk, lat->sparse(), lat->R(0) /* not read for FP32 */, psi, g, lat->ph.G,
                                         odd, s2);
                launch_ivsd(lat->list(), lat->xil(), lat->nbl(), lat->nbound, psi, g, s2);
            }
            if (k + 1 < len)
                launch_collide_stream<CodecF32>(sk, level_pops(seg, b, k + 1), lat->sparse(), psi, psi, g, lat->ph,
                                                odd, s2);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(lat->ev_rec[b], s2));
        return MCLBM_OK;
    };
    mclbm_status st = recompute(nseg - 1);
    if (st != MCLBM_OK) return st;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int b = seg & 1;
        if (seg > 0) {
            if (seg + 1 < nseg) HIP_TRY(hipStreamWaitEvent(s2, lat->ev_rev[1 - b], 0));
            st = recompute(seg - 1);
            if (st != MCLBM_OK) return st;
        }
        HIP_TRY(hipStreamWaitEvent(s, lat->ev_rec[b], 0));
        const int64_t ta = t0 + (int64_t)seg * every;
        const int len = (int)((ta + every <= t_end ? ta + every : t_end) - ta);
        // reverse steps
        for (int k = len - 1; k >= 0; --k) {
            const int odd = (int)((ta + k) & 1);
            const Pops<CodecF32> sk = level_pops(seg, b, k);
            const float2* psi = level_psi(seg, b, k);
            const int nxt = cur, now = 1 - cur;
            launch_adj_collide(sk, W.nfid, W.node_of, lat->nfluid, psi, W.lam[nxt], W.rbar[nxt], W.lam[now], W.abar, g,
                               lat->ph, odd, s);
            launch_adj_ivsd(lat->list(), lat->xil(), lat->nbound, lat->nbm(), psi, W.abar, g, W.gacc, W.nbar, s);
            launch_adj_rho(W.node_of, lat->nfluid, lat->nbm(), W.abar, W.nbar, g, W.rbar[now], s);
            cur = now;
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(lat->ev_rev[b], s));
    }
    launch_grad_scatter(lat->list(), lat->nbound, W.gacc, d_grad_xi, s);
    HIP_TRY(hipGetLastError());
    return MCLBM_OK;
}

mclbm_status mclbm_gradient_snw(mclbm_lattice* lat, int32_t nsteps, int32_t every, const void* d_ckpt,
                                size_t ckpt_bytes, const uint8_t* d_region, void* d_work, size_t work_bytes,
                                double* d_grad_xi) {
    return gradient(lat, LossKind::Snw, nsteps, every, d_ckpt, ckpt_bytes, d_region, d_work, work_bytes, d_grad_xi);
}

mclbm_status mclbm_gradient_flux(mclbm_lattice* lat, int32_t nsteps, int32_t every, const void* d_ckpt,
                                 size_t ckpt_bytes, const uint8_t* d_region, void* d_work, size_t work_bytes,
                                 double* d_grad_xi) {
    return gradient(lat, LossKind::Flux, nsteps, every, d_ckpt, ckpt_bytes, d_region, d_work, work_bytes, d_grad_xi);
}

static void drop_events(mclbm_lattice* lat) {
    for (auto& v : lat->ev) {
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
        v.clear();
    }
}

mclbm_status mclbm_profile(mclbm_lattice* lat, int32_t enable) {
    if (!lat) return fail(MCLBM_EINVAL, "NULL handle");
    if (enable) drop_events(lat);
    lat->profiling = enable != 0;
    return MCLBM_OK;
}

mclbm_status mclbm_profile_read(mclbm_lattice* lat, double h_ms[3], int64_t h_launches[3]) {
    if (!lat || !h_ms || !h_launches) return fail(MCLBM_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(lat->stream));
    for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        const size_t pairs = lat->ev[k].size() / 2;
        for (size_t j = 0; j < pairs; ++j) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, lat->ev[k][2 * j], lat->ev[k][2 * j + 1]));
            acc += ms;
        }
        h_ms[k] = acc;
        h_launches[k] = (int64_t)pairs;
    }
    return MCLBM_OK;
}

void mclbm_destroy(mclbm_lattice* lat) {
    if (!lat) return;
    drop_events(lat);
    if (lat->aux) {
        (void)hipStreamSynchronize(lat->aux);
        for (hipEvent_t e : {lat->ev_start, lat->ev_rec[0], lat->ev_rec[1], lat->ev_rev[0], lat->ev_rev[1]})
            if (e) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(lat->aux);
    }
    delete lat;
}

const char* mclbm_status_string(mclbm_status s) {
    switch (s) {
        case MCLBM_OK: return "ok";
        case MCLBM_EINVAL: return "invalid argument";
        case MCLBM_EHIP: return "HIP runtime error";
        case MCLBM_ENONFINITE: return "non-finite values in the state";
        case MCLBM_ESTATE: return "call out of order";
        case MCLBM_EVERSION: return "ABI version mismatch";
    }
    return "unknown status";
}

const char* mclbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
