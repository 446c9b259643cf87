// sw2d_api.hip - C ABI of the 2DSW step library: validation, handles, launch sequencing.
//
// The library never allocates device memory: the caller passes the state buffers and a
// workspace sized by sw2d_workspace_bytes(). Data stay on the device for the whole run
// (the paper's compiler likewise keeps buffers on the accelerator and copies once per
// run, Sect. 4.3); sw2d_step copies nothing, and only sw2d_reduce reads a few bytes back.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "sw2d_handle.h"
#include "sw2d_internal.h"

using namespace sw2d;

struct sw2d_ctx {
    sw2d_params p;
    hipStream_t stream;
    float* state[2][3];  // [buffer][eta, u, v]
    int cur;             // buffer holding the current state
    float* hp;           // packed depth: H on water, 0 on land
    PrepFlags* flags;
    sw2d_red* ring;
    FoldPartial* part;
    int part_capacity;  // partial slots per step
    StepGeometry geo;   // one step per pass
    StepGeometry geok[kMaxStepsPerPass + 1];  // K steps per pass (K >= 2)
    int steps_per_pass; // 1 .. kMaxStepsPerPass
    StepCoef coef;
    int64_t step;             // steps done
    int64_t ring_first;       // first step whose fold is valid in the ring
    double h_max;
    double h_sum;  // sum over water cells of H
};

namespace {

thread_local char g_hip_msg[256] = "";

int hip_fail(hipError_t e, const char* what) {
    std::snprintf(g_hip_msg, sizeof g_hip_msg, "%s: %s", what, hipGetErrorString(e));
    return SW2D_EHIP;
}

#define SW2D_HIP(call)                                  \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

bool params_ok(const sw2d_params* p) {
    if (!p) return false;
    if (p->nx < 3 || p->ny < 3) return false;
    if ((int64_t)p->nx * p->ny > ((int64_t)1 << 31)) return false;
    if (p->nx > (1 << 28)) return false;  // row byte offsets stay below the kernels' no-lane offset
    if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->dt)) return false;
    if (!std::isfinite(p->g) || p->g < 0.0) return false;
    if (!std::isfinite(p->eps) || p->eps < 0.0 || p->eps > 1.0) return false;
    if (p->flags & ~(uint32_t)(SW2D_FRICTION | SW2D_FILTER_UV | SW2D_ADVECTION | SW2D_WETDRY)) return false;
    if ((p->flags & SW2D_WETDRY) && p->flags != SW2D_WETDRY) return false;
    if (!std::isfinite(p->cd) || p->cd < 0.0) return false;
    if (!std::isfinite(p->hmin) || p->hmin < 0.0) return false;
    return true;
}

struct Layout {
    size_t hp, flags, ring, part, total;
    int part_capacity;
};

Layout layout(const sw2d_params* p) {
    Layout L;
    const size_t cells = (size_t)p->nx * p->ny;
    int cap = 0;
    for (int K = 1; K <= kMaxStepsPerPass; ++K) {
        const int out = K == 1 ? single_strip_out(p->flags) : kstep_strip_out(K, p->flags);
        const int nb = make_geometry(p->nx, p->ny, kMinRows, out).nblocks;
        if (nb > cap) cap = nb;
    }
    L.part_capacity = cap;
    size_t off = 0;
    L.hp = off;
    off = align_up(off + cells * sizeof(float));
    L.flags = off;
    off = align_up(off + sizeof(PrepFlags));
    L.ring = off;
    off = align_up(off + (size_t)kRingCap * sizeof(sw2d_red));
    L.part = off;
    size_t part_bytes = (size_t)kFoldChunk * L.part_capacity * sizeof(FoldPartial);
    if (part_bytes < kHsumBlocks * sizeof(double)) part_bytes = kHsumBlocks * sizeof(double);
    off = align_up(off + part_bytes);
    L.total = off;
    return L;
}

int default_rows(int ny) {
    // Measured: the single-step pass is fastest on the shortest bands, on the 8192^2 basin
    // (396 us per step against 409 at 16 rows: the rows in flight stay close together in
    // HBM, which outweighs the 4 halo rows each band re-reads) as on a 1024^2 grid (9.7 us
    // per step against 11.8 at 16 rows, where short bands also give more workgroups).
    return ny < kMinRows ? ny : kMinRows;
}

StepCoef make_coef(const sw2d_params* p) {
    StepCoef k;
    k.cx = (float)(p->g * p->dt / p->dx);
    k.cy = (float)(p->g * p->dt / p->dy);
    k.rx = (float)(p->dt / p->dx);
    k.ry = (float)(p->dt / p->dy);
    k.e4 = (float)(p->eps / 4.0);
    k.kf = (p->flags & SW2D_FRICTION) ? (float)(p->dt * p->cd) : 0.f;
    k.hmin = (p->flags & SW2D_WETDRY) ? (float)p->hmin : 0.f;
    return k;
}

int flush_folds(sw2d_ctx* h, int pending, int nparts) {
    if (pending <= 0) return SW2D_OK;
    SW2D_HIP(launch_fold(h->part, nparts, h->part_capacity, pending, h->step - pending + 1, h->ring,
                         kRingCap, h->p.dx * h->p.dy, h->h_sum, h->stream));
    return SW2D_OK;
}

// Enqueue nsteps steps: passes of steps_per_pass steps, a single step for an odd remainder;
// the fold partials of up to kFoldChunk steps are buffered, then added by one fold launch.
// With events (2 per pass, at most kFoldChunk passes per chunk) the step kernels are timed.
int enqueue_steps(sw2d_ctx* h, int32_t nsteps, hipEvent_t* ev, double* total_ms) {
    int pending = 0, nparts = 0, passes = 0;
    int32_t done = 0;
    while (done < nsteps) {
        const int k = (nsteps - done < h->steps_per_pass) ? nsteps - done : h->steps_per_pass;
        const StepGeometry& g = (k >= 2) ? h->geok[k] : h->geo;
        if (pending + k > kFoldChunk || (pending > 0 && g.nblocks != nparts)) {
            int rc = flush_folds(h, pending, nparts);
            if (rc) return rc;
            if (ev) {
                SW2D_HIP(hipEventSynchronize(ev[2 * passes - 1]));
                for (int i = 0; i < passes; ++i) {
                    float ms = 0.f;
                    SW2D_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
                    *total_ms += ms;
                }
            }
            pending = 0;
            passes = 0;
        }
        float* const* src = h->state[h->cur];
        float* const* dst = h->state[h->cur ^ 1];
        FoldPartial* part = h->part + (size_t)pending * h->part_capacity;
        if (ev) SW2D_HIP(hipEventRecord(ev[2 * passes], h->stream));
        if (k >= 2)
            SW2D_HIP(launch_stepk(k, (int)h->p.flags, src[0], src[1], src[2], h->hp, dst[0], dst[1], dst[2], part,
                                  h->part_capacity, g, h->coef, h->stream));
        else
            SW2D_HIP(launch_step((int)h->p.flags, src[0], src[1], src[2], h->hp, dst[0], dst[1], dst[2], part, g, h->coef,
                                 h->stream));
        if (ev) SW2D_HIP(hipEventRecord(ev[2 * passes + 1], h->stream));
        h->cur ^= 1;
        h->step += k;
        pending += k;
        nparts = g.nblocks;
        ++passes;
        done += k;
    }
    int rc = flush_folds(h, pending, nparts);
    if (rc) return rc;
    if (ev && passes > 0) {
        SW2D_HIP(hipEventSynchronize(ev[2 * passes - 1]));
        for (int i = 0; i < passes; ++i) {
            float ms = 0.f;
            SW2D_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
            *total_ms += ms;
        }
    }
    return SW2D_OK;
}

}  // namespace

namespace sw2d {
namespace detail {
bool params_valid(const sw2d_params* p) { return params_ok(p); }
StepCoef make_coef(const sw2d_params* p) { return ::make_coef(p); }
void set_hip_message(const char* msg) { std::snprintf(g_hip_msg, sizeof g_hip_msg, "%s", msg); }
bool handle_info(sw2d_t h, hipStream_t* stream, int* nx, int* ny) {
    if (!h) return false;
    *stream = h->stream;
    *nx = h->p.nx;
    *ny = h->p.ny;
    return true;
}
}  // namespace detail
}  // namespace sw2d

extern "C" {

size_t sw2d_workspace_bytes(const sw2d_params* p) {
    if (!params_ok(p)) return 0;
    return layout(p).total;
}

int32_t sw2d_ring_capacity(void) { return kRingCap; }

int sw2d_create(const sw2d_params* p, const float* d_H, const uint8_t* d_mask, float* d_state,
                void* d_work, size_t work_bytes, void* hip_stream, sw2d_t* out) {
    if (!out) return SW2D_ESTATE;
    *out = nullptr;
    if (!params_ok(p) || !d_H || !d_mask || !d_state || !d_work) return SW2D_EINVAL;
    const Layout L = layout(p);
    if (work_bytes < L.total) return SW2D_ENOSPC;
    if (reinterpret_cast<uintptr_t>(d_work) % kAlign != 0) return SW2D_EINVAL;

    sw2d_ctx* h = new (std::nothrow) sw2d_ctx();
    if (!h) return SW2D_ESTATE;
    h->p = *p;
    h->stream = static_cast<hipStream_t>(hip_stream);
    const size_t cells = (size_t)p->nx * p->ny;
    for (int b = 0; b < 2; ++b)
        for (int f = 0; f < 3; ++f) h->state[b][f] = d_state + (size_t)(3 * b + f) * cells;
    h->cur = 0;
    char* w = static_cast<char*>(d_work);
    h->hp = reinterpret_cast<float*>(w + L.hp);
    h->flags = reinterpret_cast<PrepFlags*>(w + L.flags);
    h->ring = reinterpret_cast<sw2d_red*>(w + L.ring);
    h->part = reinterpret_cast<FoldPartial*>(w + L.part);
    h->part_capacity = L.part_capacity;
    h->geo = make_geometry(p->nx, p->ny, default_rows(p->ny), single_strip_out(p->flags));
    for (int K = 2; K <= kMaxStepsPerPass; ++K)
        h->geok[K] = make_geometry(p->nx, p->ny, default_rows(p->ny), kstep_strip_out(K, p->flags));
    h->steps_per_pass = 1;
    h->coef = make_coef(p);
    h->step = 0;
    h->ring_first = 1;

    PrepFlags host_flags{0u, 0u, 0.0};
    hipError_t e = hipMemcpyAsync(h->flags, &host_flags, sizeof host_flags, hipMemcpyHostToDevice,
                                  h->stream);
    if (e == hipSuccess)
        e = launch_prep(d_H, d_mask, h->state[0][0], h->state[0][1], h->state[0][2], p->nx, p->ny,
                        h->hp, h->flags, reinterpret_cast<double*>(h->part), h->stream,
                        (p->flags & SW2D_WETDRY) != 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&host_flags, h->flags, sizeof host_flags, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "sw2d_create");
    }
    if (host_flags.bad != 0 || host_flags.hmax_bits == 0) {
        delete h;
        return SW2D_EINVAL;
    }
    float hmax;
    std::memcpy(&hmax, &host_flags.hmax_bits, sizeof hmax);
    h->h_max = hmax;
    h->h_sum = host_flags.h_sum;
    const double courant =
        p->dt * std::sqrt(p->g * h->h_max) * std::sqrt(1.0 / (p->dx * p->dx) + 1.0 / (p->dy * p->dy));
    if (!(courant <= 1.0)) {
        delete h;
        return SW2D_EINVAL;
    }
    *out = h;
    return SW2D_OK;
}

int sw2d_step(sw2d_t h, int32_t nsteps) {
    if (!h || nsteps < 0) return SW2D_ESTATE;
    return enqueue_steps(h, nsteps, nullptr, nullptr);
}

int sw2d_step_timed(sw2d_t h, int32_t nsteps, double* mean_step_ms) {
    if (!h || nsteps < 1 || !mean_step_ms) return SW2D_ESTATE;
    hipEvent_t ev[2 * kFoldChunk];
    for (int i = 0; i < 2 * kFoldChunk; ++i) {
        hipError_t e = hipEventCreate(&ev[i]);
        if (e != hipSuccess) {
            for (int k = 0; k < i; ++k) (void)hipEventDestroy(ev[k]);
            return hip_fail(e, "hipEventCreate");
        }
    }
    double total_ms = 0.0;
    int rc = enqueue_steps(h, nsteps, ev, &total_ms);
    for (int i = 0; i < 2 * kFoldChunk; ++i) (void)hipEventDestroy(ev[i]);
    if (rc == SW2D_OK) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        *mean_step_ms = total_ms / nsteps;
    }
    return rc;
}

size_t sw2d_unfused_scratch_bytes(const sw2d_params* p) {
    if (!params_ok(p)) return 0;
    return 3 * (size_t)p->nx * p->ny * sizeof(float);
}

int sw2d_step_unfused(sw2d_t h, int32_t nsteps, float* d_scratch, size_t scratch_bytes) {
    if (!h || nsteps < 0 || !d_scratch) return SW2D_ESTATE;
    if (h->p.flags != 0) return SW2D_EINVAL;  // the comparison path has no model variants
    if (scratch_bytes < sw2d_unfused_scratch_bytes(&h->p)) return SW2D_ENOSPC;
    const int nparts = h->part_capacity < 1024 ? h->part_capacity : 1024;
    int pending = 0;
    for (int32_t s = 0; s < nsteps; ++s) {
        float* const* src = h->state[h->cur];
        float* const* dst = h->state[h->cur ^ 1];
        SW2D_HIP(launch_unfused_step(src[0], src[1], src[2], h->hp, dst[0], dst[1], dst[2], d_scratch, h->p.nx,
                                     h->p.ny, h->coef, h->part + (size_t)pending * h->part_capacity, nparts,
                                     h->stream));
        h->cur ^= 1;
        h->step += 1;
        if (++pending == kFoldChunk) {
            int rc = flush_folds(h, pending, nparts);
            if (rc) return rc;
            pending = 0;
        }
    }
    return flush_folds(h, pending, nparts);
}

int sw2d_set_band_rows(sw2d_t h, int32_t rows) {
    if (!h) return SW2D_ESTATE;
    if (rows < kMinRows || rows > h->p.ny) return SW2D_EINVAL;
    h->geo = make_geometry(h->p.nx, h->p.ny, rows, single_strip_out(h->p.flags));
    return SW2D_OK;
}

int sw2d_set_time_blocking(sw2d_t h, int32_t steps_per_pass, int32_t rows) {
    if (!h) return SW2D_ESTATE;
    if (steps_per_pass < 1 || steps_per_pass > kMaxStepsPerPass) return SW2D_EINVAL;
    // filter_uv and advection reach further per step: they step one at a time
    if (steps_per_pass >= 2 && !kstep_variant_ok(h->p.flags)) return SW2D_EINVAL;
    if (steps_per_pass >= 2) {
        if (rows < kMinRows || rows > h->p.ny) return SW2D_EINVAL;
        // the same band height for the shorter passes that finish a step count
        for (int K = 2; K <= kMaxStepsPerPass; ++K)
            h->geok[K] = make_geometry(h->p.nx, h->p.ny, rows, kstep_strip_out(K, h->p.flags));
    }
    h->steps_per_pass = steps_per_pass;
    return SW2D_OK;
}

int32_t sw2d_time_blocking(sw2d_t h) { return h ? h->steps_per_pass : -1; }

int32_t sw2d_band_rows(sw2d_t h) { return h ? h->geo.rows : -1; }

int sw2d_reduce(sw2d_t h, sw2d_red* host_out, int32_t k) {
    if (!h || !host_out) return SW2D_ESTATE;
    const int64_t avail = h->step - h->ring_first + 1;
    if (k < 1 || k > avail || k > kRingCap) return SW2D_ESTATE;
    const int64_t first = h->step - k + 1;  // 1-based step of the oldest entry requested
    const int64_t s0 = (first - 1) % kRingCap;
    const int64_t n0 = (s0 + k <= kRingCap) ? k : kRingCap - s0;
    SW2D_HIP(hipMemcpyAsync(host_out, h->ring + s0, (size_t)n0 * sizeof(sw2d_red),
                            hipMemcpyDeviceToHost, h->stream));
    if (n0 < k)
        SW2D_HIP(hipMemcpyAsync(host_out + n0, h->ring, (size_t)(k - n0) * sizeof(sw2d_red),
                                hipMemcpyDeviceToHost, h->stream));
    SW2D_HIP(hipStreamSynchronize(h->stream));
    for (int32_t i = 0; i < k; ++i) {
        const sw2d_red& r = host_out[i];
        if (!std::isfinite(r.vol_total) || !std::isfinite(r.vol_disp) ||
            !std::isfinite(r.max_abs_u) || !std::isfinite(r.max_abs_v))
            return SW2D_EUNSTABLE;
    }
    return SW2D_OK;
}

int sw2d_state(sw2d_t h, float** d_eta, float** d_u, float** d_v) {
    if (!h) return SW2D_ESTATE;
    if (d_eta) *d_eta = h->state[h->cur][0];
    if (d_u) *d_u = h->state[h->cur][1];
    if (d_v) *d_v = h->state[h->cur][2];
    return SW2D_OK;
}

int64_t sw2d_steps_done(sw2d_t h) { return h ? h->step : -1; }

int sw2d_set_state(sw2d_t h, const float* d_eta, const float* d_u, const float* d_v, int64_t step) {
    if (!h || !d_eta || !d_u || !d_v || step < 0) return SW2D_ESTATE;
    const size_t bytes = (size_t)h->p.nx * h->p.ny * sizeof(float);
    const float* src[3] = {d_eta, d_u, d_v};
    for (int f = 0; f < 3; ++f) {
        if (src[f] != h->state[h->cur][f])
            SW2D_HIP(hipMemcpyAsync(h->state[h->cur][f], src[f], bytes, hipMemcpyDeviceToDevice,
                                    h->stream));
    }
    h->step = step;
    h->ring_first = step + 1;
    return SW2D_OK;
}

int sw2d_destroy(sw2d_t h) {
    delete h;
    return SW2D_OK;
}

const char* sw2d_strerror(int code) {
    switch (code) {
        case SW2D_OK: return "ok";
        case SW2D_EINVAL: return "invalid argument (sizes, constants, mask, depth or CFL)";
        case SW2D_EHIP: return "HIP runtime error";
        case SW2D_EUNSTABLE: return "non-finite folds: the run is unstable";
        case SW2D_ESTATE: return "invalid handle use";
        case SW2D_ENOSPC: return "workspace too small (or a grid larger than a fixed library array holds)";
        default: return "unknown status";
    }
}

const char* sw2d_last_hip_error(void) { return g_hip_msg; }

}  // extern "C"
