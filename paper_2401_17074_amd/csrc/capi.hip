// C-ABI layer of the TSLB library: argument checks, buffer ownership,
// the time-step loop and the checkpointed gradient driver.  All numerical
// work happens in the kernels launched from here.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/tslb.h"

#include "tslb_internal.h"

using namespace tslb;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(TSLB_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

inline hipStream_t S(void* s) { return (hipStream_t)s; }

inline bool ghost_kind(int k) { return k == TSLB_INLET || k == TSLB_OUTLET; }

// The update proper (without the wall fix-up pass of the tiled kernel).
hipError_t run_main_update(tslb_ctx* h, const void* in, void* out, hipStream_t s) {
    if (h->lattice == TSLB_D2Q9) return launch_update_d2q9(h->storage, in, out, h->p, s);
    switch (h->kernel) {
    case 0: return launch_update_tiled(h->storage, in, out, h->p, s);
    case 1: return launch_update_direct(h->storage, in, out, h->p, s);
    case 2: return launch_update_poplayout(h->storage, in, out, h->pop, h->p, s);
    }
    return hipErrorInvalidValue;
}

hipError_t run_update(tslb_ctx* h, const void* in, void* out, hipStream_t s) {
    hipError_t e = run_main_update(h, in, out, s);
    if (e != hipSuccess || h->kernel != 0 || h->lattice == TSLB_D2Q9) return e;
    return launch_wall_fixup(h->storage, in, out, h->p, s);
}

// Make `dev` current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int ensure_staging(tslb_ctx* h) {
    if (h->staging) return TSLB_OK;
    if (hipMalloc((void**)&h->staging, sizeof(float) * 10 * (size_t)h->p.geo.N) != hipSuccess)
        return fail(TSLB_E_NOMEM, "staging allocation of %zu bytes failed", sizeof(float) * 10 * (size_t)h->p.geo.N);
    return TSLB_OK;
}

// after_update: st was just written by run_update / run_main_update, so the
// tiled D3 update may already have refilled the plain x-face ghost nodes
int fill_ghosts(tslb_ctx* h, void* st, hipStream_t s, bool after_update = false) {
    if (!h->has_ghosts) return TSLB_OK;
    const int x_done = after_update && h->kernel == 0 && h->lattice != TSLB_D2Q9 &&
                       tslb::tiled_writes_x_ghosts(h->storage, h->p);
    HIP_TRY(launch_ghost_fill(h->storage, st, h->p, h->inlet, h->t, x_done, s));
    return TSLB_OK;
}

}  // namespace

extern "C" {

const char* tslb_last_error(void) { return g_err; }

int tslb_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src) return fail(TSLB_E_INVALID, "NULL buffer");
    if (bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
        return fail(TSLB_E_INVALID, "bytes and both addresses must be multiples of 16");
    const uintptr_t d = (uintptr_t)dst, a = (uintptr_t)src;
    if (d < a + bytes && a < d + bytes) return fail(TSLB_E_INVALID, "source and destination overlap");
    HIP_TRY(launch_stream_copy(src, dst, (long long)(bytes / 16), S(stream)));
    return TSLB_OK;
}

int tslb_create(int nx, int ny, int nz, int lattice, float tau, const float force[3], const tslb_bc* bc,
                tslb_handle* out) {
    if (!out) return fail(TSLB_E_INVALID, "out handle pointer is NULL");
    *out = nullptr;
    if (lattice != TSLB_D3Q27 && lattice != TSLB_D3Q19 && lattice != TSLB_D2Q9)
        return fail(TSLB_E_UNSUPPORTED, "lattice %d: D3Q27 (27), D3Q19 (19) and D2Q9 (9) are provided", lattice);
    if (nx < 1 || ny < 1 || nz < 1) return fail(TSLB_E_INVALID, "grid dimensions must be >= 1");
    if ((long long)nx * ny * nz >= TSLB_MAX_NODES)
        return fail(TSLB_E_INVALID, "grid of %lld nodes: at most %lld nodes (32-bit byte offsets per field)",
                    (long long)nx * ny * nz, (long long)TSLB_MAX_NODES - 1);
    if (!(tau > 0.5f) || !isfinite(tau)) return fail(TSLB_E_INVALID, "tau must exceed 1/2 (got %g)", (double)tau);
    tslb_bc b;
    memset(&b, 0, sizeof b);
    if (bc) b = *bc;
    const int dims[3] = {nx, ny, nz};
    for (int d = 0; d < 3; ++d) {
        const int lo = b.face[2 * d], hi = b.face[2 * d + 1];
        if (lo < 0 || lo > 3 || hi < 0 || hi > 3) return fail(TSLB_E_INVALID, "face kind out of range on axis %d", d);
        if ((lo == TSLB_PERIODIC) != (hi == TSLB_PERIODIC))
            return fail(TSLB_E_INVALID, "periodic faces must be paired (axis %d)", d);
        if (lo != TSLB_PERIODIC && dims[d] < 3)
            return fail(TSLB_E_INVALID, "a non-periodic axis needs at least 3 nodes (axis %d)", d);
    }
    if (b.storage < 0 || b.storage > 2) return fail(TSLB_E_INVALID, "storage kind %d out of range", b.storage);
    const float def16[3] = {4096.0f, 4096.0f, 65536.0f};
    for (int k = 0; k < 3; ++k) {
        float s = b.scale[k];
        if (b.storage == TSLB_FP32) s = 1.0f;
        if (s == 0.0f) s = b.storage == TSLB_FP16 ? def16[k] : 1.0f;
        int e;
        if (!(s > 0.0f) || frexpf(s, &e) != 0.5f)
            return fail(TSLB_E_INVALID, "scale[%d] = %g is not a positive power of two", k, (double)s);
        b.scale[k] = s;
    }
    if (!(b.inlet_radius >= 0.0f) || !(b.inlet_noise >= 0.0f))
        return fail(TSLB_E_INVALID, "inlet radius and noise must be >= 0");
    if (b.order == 0) b.order = 3;
    if (b.order != 2 && b.order != 3) return fail(TSLB_E_INVALID, "Hermite order %d is not 2 or 3", b.order);
    if (b.inlet_noise_kind != 0 && b.inlet_noise_kind != 1)
        return fail(TSLB_E_INVALID, "inlet noise kind %d is not 0 or 1", b.inlet_noise_kind);
    if (lattice == TSLB_D2Q9 && (nz != 1 || b.face[4] != TSLB_PERIODIC || b.face[5] != TSLB_PERIODIC ||
                                 b.inlet_u[2] != 0.0f || (force && force[2] != 0.0f)))
        return fail(TSLB_E_INVALID, "D2Q9 needs nz = 1, periodic z faces and no z velocity or force");

    tslb_ctx* h = new (std::nothrow) tslb_ctx;
    if (!h) return fail(TSLB_E_NOMEM, "host allocation failed");
    memset(h, 0, sizeof *h);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(TSLB_E_HIP, "no HIP device");
    }
    Geometry& g = h->p.geo;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = dims[d];
        if (b.face[2 * d] == TSLB_PERIODIC) g.periodic |= 1 << d;
        if (b.face[2 * d] == TSLB_WALL) g.lo_solid |= 1 << d;
        if (b.face[2 * d + 1] == TSLB_WALL) g.hi_solid |= 1 << d;
        if (ghost_kind(b.face[2 * d])) g.lo_ghost |= 1 << d;
        if (ghost_kind(b.face[2 * d + 1])) g.hi_ghost |= 1 << d;
    }
    g.N = (long long)nx * ny * nz;
    h->p.one_minus_omega = (float)(1.0 - 1.0 / (double)tau);
    h->p.order = b.order;
    h->buf_owned = true;
    h->p.dims = lattice == TSLB_D2Q9 ? 2 : 3;
    h->p.lattice = lattice;
    h->lattice = lattice;
    h->stats_prof_axis = -1;
    for (int a = 0; a < 3; ++a) h->p.force[a] = force ? force[a] : 0.0f;
    h->p.gfield = nullptr;
    for (int k = 0; k < 3; ++k) {
        h->p.scale[k] = b.scale[k];
        h->p.inv_scale[k] = 1.0f / b.scale[k];
    }
    for (int f = 0; f < 6; ++f) h->inlet.face_kind[f] = b.face[f];
    const double umag = sqrt((double)b.inlet_u[0] * b.inlet_u[0] + (double)b.inlet_u[1] * b.inlet_u[1] +
                             (double)b.inlet_u[2] * b.inlet_u[2]);
    for (int a = 0; a < 3; ++a) h->inlet.u[a] = b.inlet_u[a];
    h->inlet.center[0] = b.inlet_center[0];
    h->inlet.center[1] = b.inlet_center[1];
    h->inlet.radius2 = b.inlet_radius * b.inlet_radius;
    h->inlet.amp = (float)((double)b.inlet_noise * umag);
    h->inlet.seed = b.seed;
    h->inlet.noise_kind = b.inlet_noise_kind;
    h->has_ghosts = (g.lo_ghost | g.hi_ghost) != 0;
    // layers next to wall faces (raw sums of the tiled update, fix-up pass)
    h->p.wall_nodes = 0;
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
        const bool wall = (f & 1) ? ((g.hi_solid >> d) & 1) : ((g.lo_solid >> d) & 1);
        h->p.wall_off[f] = wall ? h->p.wall_nodes : -1;
        if (wall) h->p.wall_nodes += (long long)dims[d1] * dims[d2];
    }
    h->p.wall_side = nullptr;
    h->storage = b.storage;
    h->elem_bytes = b.storage == TSLB_FP32 ? 4 : 2;
    h->kernel = 0;
    h->red_blocks = 1024;
    const size_t bytes = h->elem_bytes * 10 * (size_t)g.N;
    if (hipMalloc(&h->buf[0], bytes) != hipSuccess || hipMalloc(&h->buf[1], bytes) != hipSuccess ||
        hipMalloc((void**)&h->red_partials, sizeof(double) * kRedSums * h->red_blocks) != hipSuccess ||
        hipMalloc((void**)&h->red_out, sizeof(double) * kRedSums) != hipSuccess ||
        (h->p.wall_nodes > 0 && tiled_uses_wall_side() &&
         hipMalloc((void**)&h->p.wall_side, sizeof(float) * 10 * (size_t)h->p.wall_nodes) != hipSuccess)) {
        tslb_destroy(h);
        return fail(TSLB_E_NOMEM, "device allocation of 2 x %zu bytes failed", bytes);
    }
    if (lattice != TSLB_D2Q9) {
        // work list of the tiled update for this grid and this GPU
        std::vector<int4> seg;
        int grid = 0, nseg = 0;
        if (tiled_schedule(g, seg, grid, nseg) != hipSuccess) {
            tslb_destroy(h);
            return fail(TSLB_E_INVALID, "no work list for the tiled update of this grid");
        }
        if (hipMalloc((void**)&h->sched, sizeof(int4) * seg.size()) != hipSuccess) {
            tslb_destroy(h);
            return fail(TSLB_E_NOMEM, "device allocation of the tile work list failed");
        }
        if (hipMemcpy(h->sched, seg.data(), sizeof(int4) * seg.size(), hipMemcpyHostToDevice) != hipSuccess) {
            tslb_destroy(h);
            return fail(TSLB_E_HIP, "uploading the tile work list failed");
        }
        h->p.sched = h->sched;
        h->p.sched_grid = grid;
        h->p.sched_nseg = nseg;
    }
    // rest state: drho = 0, u = 0, Pi = 0 in every format is all-zero bits
    if (hipMemset(h->buf[0], 0, bytes) != hipSuccess || hipMemset(h->buf[1], 0, bytes) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        tslb_destroy(h);
        return fail(TSLB_E_HIP, "initialising the state failed");
    }
    *out = h;
    return TSLB_OK;
}

int tslb_destroy(tslb_handle h) {
    if (!h) return TSLB_OK;
    DeviceGuard dg(h->device);
    (void)hipDeviceSynchronize();
    if (h->buf_owned) {
        (void)hipFree(h->buf[0]);
        (void)hipFree(h->buf[1]);
    }
    (void)hipFree(h->gfield);
    (void)hipFree(h->staging);
    (void)hipFree(h->red_partials);
    (void)hipFree(h->red_out);
    (void)hipFree(h->p.wall_side);
    (void)hipFree(h->pop);
    (void)hipFree(h->omo_z);
    (void)hipFree(h->stats_prof);
    (void)hipFree(h->stats_part);
    (void)hipFree(h->stats_field);
    (void)hipFree(h->sched);
    delete h;
    return TSLB_OK;
}

int tslb_set_kernel(tslb_handle h, int variant) {
    if (!h) return fail(TSLB_E_INVALID, "NULL handle");
    if (variant < 0 || variant > 2) return fail(TSLB_E_INVALID, "kernel variant %d out of range", variant);
    if (h->lattice != TSLB_D3Q27 && variant != 0)
        return fail(TSLB_E_UNSUPPORTED, "D3Q19 and D2Q9 have one update kernel (variant 0)");
    if (variant == 2 && !h->pop) {
        DeviceGuard dg(h->device);
        const size_t bytes = sizeof(float) * 27 * (size_t)h->p.geo.N;
        if (hipMalloc((void**)&h->pop, bytes) != hipSuccess) {
            h->pop = nullptr;
            return fail(TSLB_E_NOMEM, "population array of %zu bytes", bytes);
        }
    }
    h->kernel = variant;
    return TSLB_OK;
}

int tslb_set_moments(tslb_handle h, const float* rho, const float* u, const float* pineq, int flags, void* stream) {
    if (!h || !rho || !u) return fail(TSLB_E_INVALID, "NULL handle or rho/u pointer");
    DeviceGuard dg(h->device);
    const size_t N = (size_t)h->p.geo.N;
    hipStream_t s = S(stream);
    const float *r = rho, *v = u, *pi = pineq;
    if (!(flags & TSLB_DEVICE)) {
        int rc = ensure_staging(h);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(h->staging, rho, sizeof(float) * N, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(h->staging + N, u, sizeof(float) * 3 * N, hipMemcpyHostToDevice, s));
        if (pineq) HIP_TRY(hipMemcpyAsync(h->staging + 4 * N, pineq, sizeof(float) * 6 * N, hipMemcpyHostToDevice, s));
        r = h->staging;
        v = h->staging + N;
        pi = pineq ? h->staging + 4 * N : nullptr;
    }
    void* cur = h->buf[h->cur];
    HIP_TRY(launch_pack(h->storage, r, v, pi, (flags & TSLB_RHO_DEVIATION) ? 1 : 0, cur, h->p, s));
    int rc = fill_ghosts(h, cur, s);
    if (rc) return rc;
    // keep solid nodes identical in both buffers (the update never writes them)
    HIP_TRY(hipMemcpyAsync(h->buf[1 - h->cur], cur, h->elem_bytes * 10 * N, hipMemcpyDeviceToDevice, s));
    if (!(flags & TSLB_DEVICE)) HIP_TRY(hipStreamSynchronize(s));
    return TSLB_OK;
}

int tslb_get_moments(tslb_handle h, float* rho, float* u, float* pineq, int flags, void* stream) {
    if (!h) return fail(TSLB_E_INVALID, "NULL handle");
    DeviceGuard dg(h->device);
    const size_t N = (size_t)h->p.geo.N;
    hipStream_t s = S(stream);
    const int rd = (flags & TSLB_RHO_DEVIATION) ? 1 : 0;
    if (flags & TSLB_DEVICE) {
        HIP_TRY(launch_unpack(h->storage, h->buf[h->cur], rho, u, pineq, rd, h->p, s));
        return TSLB_OK;
    }
    int rc = ensure_staging(h);
    if (rc) return rc;
    HIP_TRY(launch_unpack(h->storage, h->buf[h->cur], h->staging, h->staging + N, h->staging + 4 * N, rd, h->p, s));
    if (rho) HIP_TRY(hipMemcpyAsync(rho, h->staging, sizeof(float) * N, hipMemcpyDeviceToHost, s));
    if (u) HIP_TRY(hipMemcpyAsync(u, h->staging + N, sizeof(float) * 3 * N, hipMemcpyDeviceToHost, s));
    if (pineq) HIP_TRY(hipMemcpyAsync(pineq, h->staging + 4 * N, sizeof(float) * 6 * N, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return TSLB_OK;
}

int tslb_set_force_field(tslb_handle h, const float* g, void* stream) {
    if (!h) return fail(TSLB_E_INVALID, "NULL handle");
    DeviceGuard dg(h->device);
    const size_t N = (size_t)h->p.geo.N;
    if (!g) {
        h->p.gfield = nullptr;
        return TSLB_OK;
    }
    if (!h->gfield && hipMalloc((void**)&h->gfield, sizeof(float) * 3 * N) != hipSuccess)
        return fail(TSLB_E_NOMEM, "force-field allocation failed");
    HIP_TRY(hipMemcpyAsync(h->gfield, g, sizeof(float) * 3 * N, hipMemcpyDeviceToDevice, S(stream)));
    h->p.gfield = h->gfield;
    return TSLB_OK;
}

int tslb_set_relaxation_profile(tslb_handle h, const float* tau_z, void* stream) {
    if (!h) return fail(TSLB_E_INVALID, "NULL handle");
    if (!tau_z) {
        h->p.omo_z = nullptr;
        return TSLB_OK;
    }
    const int nz = h->p.geo.n[2];
    std::vector<float> omo((size_t)nz);
    for (int z = 0; z < nz; ++z) {
        const float t = tau_z[z];
        if (!(t > 0.5f) || !isfinite(t))
            return fail(TSLB_E_INVALID, "tau_z[%d] = %g must be finite and exceed 1/2", z, (double)t);
        omo[(size_t)z] = (float)(1.0 - 1.0 / (double)t);
    }
    DeviceGuard dg(h->device);
    if (!h->omo_z && hipMalloc((void**)&h->omo_z, sizeof(float) * (size_t)nz) != hipSuccess) {
        h->omo_z = nullptr;
        return fail(TSLB_E_NOMEM, "relaxation profile allocation failed");
    }
    HIP_TRY(hipMemcpyAsync(h->omo_z, omo.data(), sizeof(float) * (size_t)nz, hipMemcpyHostToDevice, S(stream)));
    HIP_TRY(hipStreamSynchronize(S(stream)));
    h->p.omo_z = h->omo_z;
    return TSLB_OK;
}

int tslb_bind_state(tslb_handle h, void* buf0, void* buf1, void* stream) {
    if (!h || !buf0 || !buf1 || buf0 == buf1) return fail(TSLB_E_INVALID, "NULL or aliasing state buffers");
    if (((uintptr_t)buf0 & 255) || ((uintptr_t)buf1 & 255))
        return fail(TSLB_E_INVALID, "state buffers must be 256-byte aligned");
    const size_t bytes = tslb_state_bytes(h);
    const char *b0 = (const char*)buf0, *b1 = (const char*)buf1;
    if (b0 < b1 + bytes && b1 < b0 + bytes) return fail(TSLB_E_INVALID, "state buffers overlap");
    DeviceGuard dg(h->device);
    hipStream_t s = S(stream);
    HIP_TRY(hipMemcpyAsync(buf0, h->buf[h->cur], bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(buf1, h->buf[1 - h->cur], bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h->buf_owned) {
        (void)hipFree(h->buf[0]);
        (void)hipFree(h->buf[1]);
    }
    h->buf[0] = buf0;
    h->buf[1] = buf1;
    h->cur = 0;
    h->buf_owned = false;
    return TSLB_OK;
}

int tslb_stats_begin(tslb_handle h, int kinds, int axis, void* stream) {
    if (!h) return fail(TSLB_E_INVALID, "NULL handle");
    if (kinds <= 0 || (kinds & ~(TSLB_STATS_PROFILE | TSLB_STATS_FIELD)))
        return fail(TSLB_E_INVALID, "statistics kinds %d", kinds);
    if ((kinds & TSLB_STATS_PROFILE) && (axis < 0 || axis > 2)) return fail(TSLB_E_INVALID, "axis %d", axis);
    DeviceGuard dg(h->device);
    hipStream_t s = S(stream);
    const Geometry& g = h->p.geo;
    if (kinds & TSLB_STATS_PROFILE) {
        if (h->stats_prof_axis != axis) {
            (void)hipFree(h->stats_prof);
            (void)hipFree(h->stats_part);
            h->stats_prof = nullptr;
            h->stats_part = nullptr;
            h->stats_prof_axis = -1;
            const size_t n_axis = (size_t)g.n[axis];
            const size_t bpp = (size_t)stats_blocks_per_plane(g, axis);
            if (hipMalloc((void**)&h->stats_prof, sizeof(double) * 13 * n_axis) != hipSuccess ||
                hipMalloc((void**)&h->stats_part, sizeof(double) * 13 * n_axis * bpp) != hipSuccess) {
                (void)hipFree(h->stats_prof);
                h->stats_prof = nullptr;
                h->stats_part = nullptr;
                return fail(TSLB_E_NOMEM, "profile statistics allocation failed");
            }
            h->stats_prof_axis = axis;
        }
        HIP_TRY(hipMemsetAsync(h->stats_prof, 0, sizeof(double) * 13 * (size_t)g.n[axis], s));
    }
    if (kinds & TSLB_STATS_FIELD) {
        if (!h->stats_field && hipMalloc((void**)&h->stats_field, sizeof(double) * 9 * (size_t)g.N) != hipSuccess) {
            h->stats_field = nullptr;
            return fail(TSLB_E_NOMEM, "field statistics allocation of %zu bytes failed",
                        sizeof(double) * 9 * (size_t)g.N);
        }
        HIP_TRY(hipMemsetAsync(h->stats_field, 0, sizeof(double) * 9 * (size_t)g.N, s));
    }
    h->stats_kinds = kinds;
    h->stats_axis = axis;
    h->stats_samples = 0;
    return TSLB_OK;
}

int tslb_stats_sample(tslb_handle h, void* stream) {
    if (!h) return fail(TSLB_E_INVALID, "NULL handle");
    if (!h->stats_kinds) return fail(TSLB_E_INVALID, "tslb_stats_begin was not called");
    DeviceGuard dg(h->device);
    hipStream_t s = S(stream);
    if (h->stats_kinds & TSLB_STATS_PROFILE)
        HIP_TRY(launch_stats_profile(h->storage, h->buf[h->cur], h->stats_part, h->stats_prof, h->p, h->stats_axis, s));
    if (h->stats_kinds & TSLB_STATS_FIELD)
        HIP_TRY(launch_stats_field(h->storage, h->buf[h->cur], h->stats_field, h->p, s));
    h->stats_samples += 1;
    return TSLB_OK;
}

int tslb_stats_profile(tslb_handle h, double* sums, int64_t* nsamples, void* stream) {
    if (!h || !sums) return fail(TSLB_E_INVALID, "NULL handle or output");
    if (!(h->stats_kinds & TSLB_STATS_PROFILE)) return fail(TSLB_E_INVALID, "profile statistics are not enabled");
    DeviceGuard dg(h->device);
    hipStream_t s = S(stream);
    HIP_TRY(hipMemcpyAsync(sums, h->stats_prof, sizeof(double) * 13 * (size_t)h->p.geo.n[h->stats_axis],
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (nsamples) *nsamples = h->stats_samples;
    return TSLB_OK;
}

int tslb_stats_field(tslb_handle h, float* mean_u, float* cov, void* stream) {
    if (!h) return fail(TSLB_E_INVALID, "NULL handle");
    if (!(h->stats_kinds & TSLB_STATS_FIELD) || h->stats_samples < 1)
        return fail(TSLB_E_INVALID, "no field statistics sampled");
    DeviceGuard dg(h->device);
    HIP_TRY(launch_stats_field_moments(h->stats_field, h->p.geo.N, 1.0 / (double)h->stats_samples, mean_u, cov,
                                       S(stream)));
    return TSLB_OK;
}

int tslb_stats_jet(tslb_handle h, int axis, const float center[2], float* uc, float* rhalf, void* stream) {
    if (!h || !center || !uc || !rhalf) return fail(TSLB_E_INVALID, "NULL argument");
    if (axis < 0 || axis > 2) return fail(TSLB_E_INVALID, "axis %d", axis);
    if (!(h->stats_kinds & TSLB_STATS_FIELD) || h->stats_samples < 1)
        return fail(TSLB_E_INVALID, "no field statistics sampled");
    const Geometry& g = h->p.geo;
    const int d1 = axis == 0 ? 1 : 0, d2 = axis == 2 ? 1 : 2;
    if (!(center[0] >= 0.0f && center[0] <= (float)(g.n[d1] - 1) && center[1] >= 0.0f &&
          center[1] <= (float)(g.n[d2] - 1)))
        return fail(TSLB_E_INVALID, "jet centre (%g, %g) outside the cross-section", (double)center[0],
                    (double)center[1]);
    if ((size_t)stats_jet_bins(g, axis, center[0], center[1]) * 3 * sizeof(double) > 65536)
        return fail(TSLB_E_INVALID, "cross-section too wide for the radial bins");
    DeviceGuard dg(h->device);
    HIP_TRY(launch_stats_jet(h->stats_field, g, axis, center[0], center[1], 1.0 / (double)h->stats_samples, uc,
                             rhalf, S(stream)));
    return TSLB_OK;
}

int tslb_step(tslb_handle h, int nsteps, void* stream) {
    if (!h) return fail(TSLB_E_INVALID, "NULL handle");
    if (nsteps < 0) return fail(TSLB_E_INVALID, "nsteps must be >= 0");
    DeviceGuard dg(h->device);
    hipStream_t s = S(stream);
    for (int k = 0; k < nsteps; ++k) {
        void* in = h->buf[h->cur];
        void* out = h->buf[1 - h->cur];
        HIP_TRY(run_update(h, in, out, s));
        h->cur = 1 - h->cur;
        h->t += 1;
        int rc = fill_ghosts(h, out, s, true);
        if (rc) return rc;
    }
    return TSLB_OK;
}

int tslb_step_timed(tslb_handle h, int nsteps, double ms[2], void* stream) {
    if (!h || !ms) return fail(TSLB_E_INVALID, "NULL handle or output");
    if (nsteps < 1 || nsteps > 100000) return fail(TSLB_E_INVALID, "nsteps must be in [1, 100000]");
    DeviceGuard dg(h->device);
    hipStream_t s = S(stream);
    std::vector<hipEvent_t> ev(3 * (size_t)nsteps, nullptr);
    int rc = TSLB_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            rc = fail(TSLB_E_HIP, "hipEventCreate failed");
            break;
        }
    for (int k = 0; rc == TSLB_OK && k < nsteps; ++k) {
        void* in = h->buf[h->cur];
        void* out = h->buf[1 - h->cur];
        hipError_t e = hipEventRecord(ev[3 * k], s);
        if (e == hipSuccess) e = run_main_update(h, in, out, s);
        if (e == hipSuccess) e = hipEventRecord(ev[3 * k + 1], s);
        if (e == hipSuccess && h->kernel == 0 && h->lattice != TSLB_D2Q9)
            e = launch_wall_fixup(h->storage, in, out, h->p, s);
        if (e != hipSuccess) {
            rc = fail(TSLB_E_HIP, "timed step: %s", hipGetErrorString(e));
            break;
        }
        h->cur = 1 - h->cur;
        h->t += 1;
        rc = fill_ghosts(h, out, s, true);
        if (rc == TSLB_OK && hipEventRecord(ev[3 * k + 2], s) != hipSuccess) rc = fail(TSLB_E_HIP, "hipEventRecord failed");
    }
    if (rc == TSLB_OK) {
        if (hipStreamSynchronize(s) != hipSuccess) rc = fail(TSLB_E_HIP, "hipStreamSynchronize failed");
    }
    double main_ms = 0.0, aux_ms = 0.0;
    for (int k = 0; rc == TSLB_OK && k < nsteps; ++k) {
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, ev[3 * k], ev[3 * k + 1]) != hipSuccess ||
            hipEventElapsedTime(&b, ev[3 * k + 1], ev[3 * k + 2]) != hipSuccess)
            rc = fail(TSLB_E_HIP, "hipEventElapsedTime failed");
        main_ms += a;
        aux_ms += b;
    }
    for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc == TSLB_OK) {
        ms[0] = main_ms;
        ms[1] = aux_ms;
    }
    return rc;
}

int64_t tslb_get_time(tslb_handle h) { return h ? h->t : -1; }

int tslb_set_time(tslb_handle h, int64_t t) {
    if (!h || t < 0) return fail(TSLB_E_INVALID, "NULL handle or negative level");
    h->t = t;
    return TSLB_OK;
}

int tslb_reduce(tslb_handle h, double out[5], void* stream) {
    if (!h || !out) return fail(TSLB_E_INVALID, "NULL handle or output");
    DeviceGuard dg(h->device);
    hipStream_t s = S(stream);
    double host[kRedSums];
    HIP_TRY(launch_reduce(h->storage, h->buf[h->cur], h->red_partials, h->red_blocks, h->red_out, h->p, s));
    HIP_TRY(hipMemcpyAsync(host, h->red_out, sizeof host, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < 5; ++k) out[k] = host[k];
    if (host[5] != 0.0) return fail(TSLB_E_UNSTABLE, "%.0f fluid nodes hold NaN or Inf moments", host[5]);
    return TSLB_OK;
}

// ------------------------------------------------ allocation-free reduction
// The per-block partials of tslb_reduce_noalloc live in this fixed device
// array: one copy per GPU, held until the process ends.  Its name is a
// host-side stand-in in host code, never a device address: the address of
// each GPU's copy is looked up once per device, with that device current,
// and kept in g_noalloc_scratch.
static __device__ __align__(256) double scratch[kRedSums * TSLB_NOALLOC_REDUCE_BLOCKS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_scratch[kMaxDevices] = {};

// Device address of this GPU's scratch array (the caller has made `dev`
// current).
int noalloc_scratch(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(TSLB_E_INVALID, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(TSLB_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_noalloc_scratch[dev] = (double*)ptr;
    }
    *out = g_noalloc_scratch[dev];
    return TSLB_OK;
}
}  // namespace

int tslb_reduce_noalloc(tslb_handle h, double* out_dev, void* stream) {
    if (!h || !out_dev) return fail(TSLB_E_INVALID, "NULL handle or output");
    if (h->red_blocks < 1 || h->red_blocks > TSLB_NOALLOC_REDUCE_BLOCKS)
        return fail(TSLB_E_INVALID, "reduction over %d blocks exceeds the fixed scratch of %d blocks", h->red_blocks,
                    TSLB_NOALLOC_REDUCE_BLOCKS);
    DeviceGuard dg(h->device);
    double* part = nullptr;
    const int rc = noalloc_scratch(h->device, &part);
    if (rc != TSLB_OK) return rc;
    // every partial is written before it is read: nothing to clear
    HIP_TRY(launch_reduce(h->storage, h->buf[h->cur], part, h->red_blocks, out_dev, h->p, S(stream)));
    return TSLB_OK;
}

int tslb_objective(tslb_handle h, int objective, double* out, void* stream) {
    if (!h || !out) return fail(TSLB_E_INVALID, "NULL handle or output");
    if (objective != TSLB_OBJ_KINETIC_ENERGY && objective != TSLB_OBJ_WALL_SHEAR)
        return fail(TSLB_E_UNSUPPORTED, "objective %d", objective);
    DeviceGuard dg(h->device);
    hipStream_t s = S(stream);
    double host[kRedSums];
    HIP_TRY(launch_reduce(h->storage, h->buf[h->cur], h->red_partials, h->red_blocks, h->red_out, h->p, s));
    HIP_TRY(hipMemcpyAsync(host, h->red_out, sizeof host, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = objective == TSLB_OBJ_WALL_SHEAR ? host[6] : host[4];
    if (host[5] != 0.0) return fail(TSLB_E_UNSTABLE, "%.0f fluid nodes hold NaN or Inf moments", host[5]);
    return TSLB_OK;
}

size_t tslb_state_bytes(tslb_handle h) { return h ? h->elem_bytes * 10 * (size_t)h->p.geo.N : 0; }

int tslb_save_state(tslb_handle h, void* dst, void* stream) {
    if (!h || !dst) return fail(TSLB_E_INVALID, "NULL handle or destination");
    DeviceGuard dg(h->device);
    HIP_TRY(hipMemcpyAsync(dst, h->buf[h->cur], tslb_state_bytes(h), hipMemcpyDeviceToDevice, S(stream)));
    return TSLB_OK;
}

int tslb_load_state(tslb_handle h, const void* src, void* stream) {
    if (!h || !src) return fail(TSLB_E_INVALID, "NULL handle or source");
    DeviceGuard dg(h->device);
    HIP_TRY(hipMemcpyAsync(h->buf[h->cur], src, tslb_state_bytes(h), hipMemcpyDeviceToDevice, S(stream)));
    HIP_TRY(hipMemcpyAsync(h->buf[1 - h->cur], src, tslb_state_bytes(h), hipMemcpyDeviceToDevice, S(stream)));
    return TSLB_OK;
}

int tslb_adjoint_seed(tslb_handle h, const void* state, int objective, float* lam, void* stream) {
    if (!h || !state || !lam) return fail(TSLB_E_INVALID, "NULL argument");
    if (objective != TSLB_OBJ_KINETIC_ENERGY && objective != TSLB_OBJ_WALL_SHEAR)
        return fail(TSLB_E_UNSUPPORTED, "objective %d", objective);
    if (h->storage != TSLB_FP32) return fail(TSLB_E_UNSUPPORTED, "the adjoint needs FP32 storage");
    DeviceGuard dg(h->device);
    HIP_TRY(launch_adjoint_seed((const float*)state, lam, h->p, objective, S(stream)));
    return TSLB_OK;
}

int tslb_adjoint_step(tslb_handle h, const void* state_t, const void* state_t1, float* lam_t1, float* lam_t,
                      float* dg_accum, void* stream) {
    if (!h || !state_t || !state_t1 || !lam_t1 || !lam_t) return fail(TSLB_E_INVALID, "NULL argument");
    if (lam_t == lam_t1) return fail(TSLB_E_INVALID, "lam_t may not alias lam_t1");
    if (h->storage != TSLB_FP32) return fail(TSLB_E_UNSUPPORTED, "the adjoint needs FP32 storage");
    if (h->p.order != 3) return fail(TSLB_E_UNSUPPORTED, "the adjoint differentiates the third-order update only");
    if (h->lattice != TSLB_D3Q27) return fail(TSLB_E_UNSUPPORTED, "the adjoint is provided for D3Q27 only");
    DeviceGuard dg(h->device);
    // the ghost refill of level t+1 first (its transpose, in place)
    if (h->has_ghosts) HIP_TRY(launch_ghost_fold(lam_t1, h->p, h->inlet, S(stream)));
    if (h->kernel != 1)
        HIP_TRY(launch_adjoint_tiled((const float*)state_t, (const float*)state_t1, lam_t1, lam_t, dg_accum, h->p,
                                     S(stream)));
    else
        HIP_TRY(launch_adjoint_step((const float*)state_t, (const float*)state_t1, lam_t1, lam_t, dg_accum, h->p,
                                    S(stream)));
    return TSLB_OK;
}

size_t tslb_rollout_workspace_bytes(tslb_handle h, int nsteps, int every) {
    if (!h || nsteps < 1 || every < 1) return 0;
    const size_t nseg = (size_t)((nsteps + every - 1) / every);
    const size_t sb = tslb_state_bytes(h);
    return (nseg + (size_t)every + 1) * sb + sizeof(float) * 10 * (size_t)h->p.geo.N;
}

int tslb_rollout_forward(tslb_handle h, int nsteps, int every, void* ws, size_t ws_bytes, void* stream) {
    if (!h || !ws || nsteps < 1 || every < 1) return fail(TSLB_E_INVALID, "bad rollout arguments");
    if (ws_bytes < tslb_rollout_workspace_bytes(h, nsteps, every)) return fail(TSLB_E_INVALID, "workspace too small");
    if (h->p.order != 3 || h->lattice != TSLB_D3Q27)
        return fail(TSLB_E_UNSUPPORTED, "the adjoint differentiates the third-order D3Q27 update only");
    const size_t sb = tslb_state_bytes(h);
    char* ck = (char*)ws;
    for (int s0 = 0, seg = 0; s0 < nsteps; s0 += every, ++seg) {
        int rc = tslb_save_state(h, ck + (size_t)seg * sb, stream);
        if (rc) return rc;
        rc = tslb_step(h, (nsteps - s0 < every) ? nsteps - s0 : every, stream);
        if (rc) return rc;
    }
    return TSLB_OK;
}

int tslb_rollout_backward(tslb_handle h, int nsteps, int every, void* ws, size_t ws_bytes, float* lam,
                          float* dg_accum, void* stream) {
    if (!h || !ws || !lam || nsteps < 1 || every < 1) return fail(TSLB_E_INVALID, "bad rollout arguments");
    if (ws_bytes < tslb_rollout_workspace_bytes(h, nsteps, every)) return fail(TSLB_E_INVALID, "workspace too small");
    if (h->p.order != 3 || h->lattice != TSLB_D3Q27)
        return fail(TSLB_E_UNSUPPORTED, "the adjoint differentiates the third-order D3Q27 update only");
    if (h->storage != TSLB_FP32) return fail(TSLB_E_UNSUPPORTED, "the adjoint needs FP32 storage");
    DeviceGuard dg(h->device);
    hipStream_t s = S(stream);
    const size_t sb = tslb_state_bytes(h);
    const int nseg = (nsteps + every - 1) / every;
    char* ck = (char*)ws;
    char* seg_states = ck + (size_t)nseg * sb;
    float* lam_tmp = (float*)(seg_states + (size_t)(every + 1) * sb);
    float* a = lam;      // holds lambda at the current level
    float* b = lam_tmp;
    const int64_t t_end = h->t;
    // The update writes fluid nodes only and relies on wall nodes holding the
    // rest state, so before the first recomputation every slot gets a
    // checkpoint's copy; afterwards the slots hold earlier levels, whose wall
    // nodes are at rest as well.
    if ((h->p.geo.lo_solid | h->p.geo.hi_solid) != 0)
        for (int k = 1; k <= every; ++k)
            HIP_TRY(hipMemcpyAsync(seg_states + (size_t)k * sb, ck, sb, hipMemcpyDeviceToDevice, s));
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int s0 = seg * every;
        const int len = (nsteps - s0 < every) ? nsteps - s0 : every;
        // recompute the segment once from its checkpoint, each level straight
        // into its slot (the handle's own buffers are not touched)
        HIP_TRY(hipMemcpyAsync(seg_states, ck + (size_t)seg * sb, sb, hipMemcpyDeviceToDevice, s));
        for (int k = 1; k <= len; ++k) {
            h->t = t_end - nsteps + s0 + k - 1;
            HIP_TRY(run_update(h, seg_states + (size_t)(k - 1) * sb, seg_states + (size_t)k * sb, s));
            h->t += 1;
            const int rc = fill_ghosts(h, seg_states + (size_t)k * sb, s, true);
            if (rc) {
                h->t = t_end;
                return rc;
            }
        }
        h->t = t_end;
        for (int k = len - 1; k >= 0; --k) {
            const int rc = tslb_adjoint_step(h, seg_states + (size_t)k * sb, seg_states + (size_t)(k + 1) * sb, a, b,
                                   dg_accum, stream);
            if (rc) return rc;
            float* tmp = a;
            a = b;
            b = tmp;
        }
    }
    // the initial level's ghosts were refilled from its interior as well
    if (h->has_ghosts) HIP_TRY(launch_ghost_fold(a, h->p, h->inlet, s));
    if (a != lam) HIP_TRY(hipMemcpyAsync(lam, a, sizeof(float) * 10 * (size_t)h->p.geo.N, hipMemcpyDeviceToDevice, s));
    return TSLB_OK;
}

}  // extern "C"
