// sw2d_batch.hip - ensembles of independent 2DSW basins of uneven sizes, advanced by one
// persistent launch per chunk of steps, with a grid barrier between steps.
//
// Work list: every (instance, band, strip) is one item for one wave; items are ordered
// instance by instance, in blocks of two vertically adjacent bands, so the waves that
// run together cover a compact region and the zig-zag march shares band-boundary rows
// through L2 (as in the single-grid kernel). Every item runs the same tile routine as
// sw2d_step_kernel, so each instance is bitwise equal to the same basin stepped alone.
//
// Per step: waves process their items (round robin over the work list), write one fold
// partial per item, then the whole grid meets at a barrier. After the barrier, workgroup
// b adds the partials of instances b, b+G, ... in a fixed order and writes their folds
// to the ring, then goes on with the next step. The barrier spin has a wall-clock
// deadline: on expiry it raises an error flag and the kernel returns, so no wave can
// wait forever even if the grid were not co-resident.
//
// The steps done so far live in device memory and are advanced by the kernel itself, so
// a captured graph of launches can be replayed without host-side parameters.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "sw2d_internal.h"
#include "sw2d_tile.h"

namespace sw2d {

struct BatchInst {
    const float* hp;
    float* state[2][3];
    int nx, ny;
    StepCoef k;
    double cell_area;
    double h_sum;
    int item_begin, item_end;  // items of this instance in the work list
};

struct BatchItem {
    int inst, j0, j1;
    int strip2;  // 2 * strip + 1 if the band marches south
};

struct BatchControl {
    unsigned barrier;      // arrivals in the current launch (reset before every launch)
    unsigned error;        // 1: a barrier wait ran past its deadline
    long long steps_done;  // advanced by the kernel at the end of every launch
};

constexpr int kBatchThreads = 256;
constexpr int kBatchWaves = kBatchThreads / kWave;
constexpr int kBatchRing = 64;  // steps of per-instance folds kept

struct BatchArgs {
    const BatchInst* inst;
    const BatchItem* items;
    FoldPartial* part;  // [2][n_items]
    sw2d_red* ring;     // [kBatchRing][n_inst]
    BatchControl* ctl;
    int n_inst, n_items, steps;
    unsigned long long timeout_ticks;
};

__global__ void sw2d_batch_reset_kernel(BatchControl* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->barrier = 0u;
    }
}

__device__ __forceinline__ bool grid_barrier(BatchControl* ctl, unsigned target,
                                             unsigned long long timeout_ticks) {
    __shared__ int s_ok;
    __threadfence();  // every wave: its stores of this step are visible device-wide
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(&ctl->barrier, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        const unsigned long long deadline = wall_clock64() + timeout_ticks;
        while (__hip_atomic_load(&ctl->barrier, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (wall_clock64() > deadline) {
                __hip_atomic_fetch_or(&ctl->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        s_ok = ok;
    }
    __syncthreads();
    __threadfence();  // acquire: see the other workgroups' stores
    return s_ok != 0;
}

// Adds the item partials of instance i (fixed order) and writes its fold entry for `step`.
__device__ void fold_instance(const BatchArgs& a, int i, int slot, long long step) {
    __shared__ double s_disp[kBatchThreads];
    __shared__ float s_mu[kBatchThreads], s_mv[kBatchThreads];
    const BatchInst& in = a.inst[i];
    const FoldPartial* p = a.part + (size_t)slot * a.n_items;
    double disp = 0.0;
    float mu = 0.f, mv = 0.f;
    for (int it = in.item_begin + threadIdx.x; it < in.item_end; it += kBatchThreads) {
        disp += p[it].disp;
        mu = fmaxf(mu, p[it].mu);
        mv = fmaxf(mv, p[it].mv);
    }
    const int t = threadIdx.x;
    s_disp[t] = disp;
    s_mu[t] = mu;
    s_mv[t] = mv;
    __syncthreads();
    for (int half = kBatchThreads / 2; half > 0; half >>= 1) {
        if (t < half) {
            s_disp[t] += s_disp[t + half];
            s_mu[t] = fmaxf(s_mu[t], s_mu[t + half]);
            s_mv[t] = fmaxf(s_mv[t], s_mv[t + half]);
        }
        __syncthreads();
    }
    if (t == 0) {
        sw2d_red* o = a.ring + (size_t)((step - 1) % kBatchRing) * a.n_inst + i;
        o->step = step;
        o->vol_total = in.cell_area * (in.h_sum + s_disp[0]);
        o->vol_disp = in.cell_area * s_disp[0];
        o->max_abs_u = s_mu[0];
        o->max_abs_v = s_mv[0];
    }
    __syncthreads();
}

__device__ __forceinline__ void fold_step(const BatchArgs& a, int logical_wg, int nwg, int slot,
                                          long long step) {
    for (int i = logical_wg; i < a.n_inst; i += nwg) fold_instance(a, i, slot, step);
}

__device__ __forceinline__ int logical_block(int b, int n) {
    const int q = n / kXcds, r = n % kXcds;
    const int x = b % kXcds, k = b / kXcds;
    return x * q + min(x, r) + k;
}

__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) void sw2d_batch_kernel(BatchArgs a) {
    const int nwg = gridDim.x;
    const int lwg = logical_block(blockIdx.x, nwg);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nwaves = nwg * kBatchWaves;
    const int lwave = lwg * kBatchWaves + wave;
    const long long base = a.ctl->steps_done;

    for (int s = 0; s < a.steps; ++s) {
        const long long step_idx = base + s;  // 0-based index of the step being made
        const int cur = (int)(step_idx & 1);
        if (s > 0) fold_step(a, lwg, nwg, (s - 1) & 1, step_idx);
        FoldPartial* part = a.part + (size_t)(s & 1) * a.n_items;
        for (int it = lwave; it < a.n_items; it += nwaves) {
            const BatchItem item = a.items[it];
            const BatchInst& in = a.inst[item.inst];
            const int c = (item.strip2 >> 1) * kStripOut - kHalo + lane;
            const bool col_in = c >= 0 && c < in.nx;
            const bool out_lane = col_in && lane >= kHalo && lane < kWave - kHalo;
            const float* const* src = in.state[cur];
            float* const* dst = in.state[cur ^ 1];
            double f_disp = 0.0;
            float f_mu = 0.f, f_mv = 0.f;
            if (item.strip2 & 1)
                march<false>(src[0], src[1], src[2], in.hp, dst[0], dst[1], dst[2], in.nx, in.ny, c,
                             col_in, out_lane, item.j0, item.j1, in.k, f_disp, f_mu, f_mv);
            else
                march<true>(src[0], src[1], src[2], in.hp, dst[0], dst[1], dst[2], in.nx, in.ny, c,
                            col_in, out_lane, item.j0, item.j1, in.k, f_disp, f_mu, f_mv);
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) {
                f_disp += __shfl_xor(f_disp, off, kWave);
                f_mu = fmaxf(f_mu, __shfl_xor(f_mu, off, kWave));
                f_mv = fmaxf(f_mv, __shfl_xor(f_mv, off, kWave));
            }
            if (lane == 0) {
                part[it].disp = f_disp;
                part[it].mu = f_mu;
                part[it].mv = f_mv;
            }
        }
        if (!grid_barrier(a.ctl, (unsigned)nwg * (unsigned)(s + 1), a.timeout_ticks)) return;
    }
    fold_step(a, lwg, nwg, (a.steps - 1) & 1, base + a.steps);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->steps_done = base + a.steps;
}

}  // namespace sw2d

// ---------------------------------------------------------------------------------------
// C ABI of the batched form

using namespace sw2d;

struct sw2d_bctx {
    int n;
    std::vector<sw2d_params> p;
    std::vector<float*> state;  // [n][6]
    hipStream_t stream;         // the caller's
    hipStream_t capture;        // private stream used only to record graphs
    BatchInst* d_inst;
    BatchItem* d_items;
    FoldPartial* d_part;
    sw2d_red* d_ring;
    BatchControl* d_ctl;
    int n_items;
    int grid;
    int steps_per_launch;
    bool use_graph;
    int64_t steps_done;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int graph_n;
    unsigned long long timeout_ticks;
};

namespace {

thread_local char g_batch_msg[256] = "";

int batch_hip_fail(hipError_t e, const char* what) {
    std::snprintf(g_batch_msg, sizeof g_batch_msg, "%s: %s", what, hipGetErrorString(e));
    sw2d::detail::set_hip_message(g_batch_msg);
    return SW2D_EHIP;
}

#define SW2D_BHIP(call)                                          \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return batch_hip_fail(e_, #call);  \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct BatchLayout {
    std::vector<size_t> hp;  // per instance
    size_t flags, scratch, inst, items, part, ring, ctl, total;
    int n_items;
    std::vector<int> items_of;  // per instance
};

int rows_for(const sw2d_params& p, const int32_t* band_rows, int i) {
    int r = band_rows ? band_rows[i] : 16;
    if (r > p.ny) r = p.ny;
    return r;
}

bool batch_layout(int n, const sw2d_params* p, const int32_t* band_rows, BatchLayout& L) {
    if (n < 1) return false;
    size_t off = 0;
    L.hp.resize(n);
    L.items_of.resize(n);
    L.n_items = 0;
    for (int i = 0; i < n; ++i) {
        if (!sw2d::detail::params_valid(&p[i])) return false;
        const int rows = rows_for(p[i], band_rows, i);
        if (rows < 1 || (band_rows && band_rows[i] < kMinRows)) return false;
        L.hp[i] = off;
        off = align_up(off + (size_t)p[i].nx * p[i].ny * sizeof(float));
        const int strips = (p[i].nx + kStripOut - 1) / kStripOut;
        const int bands = (p[i].ny + rows - 1) / rows;
        L.items_of[i] = strips * bands;
        if ((int64_t)L.n_items + L.items_of[i] > (1 << 30)) return false;
        L.n_items += L.items_of[i];
    }
    L.flags = off;
    off = align_up(off + (size_t)n * sizeof(PrepFlags));
    L.scratch = off;
    off = align_up(off + kHsumBlocks * sizeof(double));
    L.inst = off;
    off = align_up(off + (size_t)n * sizeof(BatchInst));
    L.items = off;
    off = align_up(off + (size_t)L.n_items * sizeof(BatchItem));
    L.part = off;
    off = align_up(off + 2 * (size_t)L.n_items * sizeof(FoldPartial));
    L.ring = off;
    off = align_up(off + (size_t)kBatchRing * n * sizeof(sw2d_red));
    L.ctl = off;
    off = align_up(off + sizeof(BatchControl));
    L.total = off;
    return true;
}

int enqueue_chunks(sw2d_bctx* b, int32_t nsteps, hipStream_t s) {
    BatchArgs a;
    a.inst = b->d_inst;
    a.items = b->d_items;
    a.part = b->d_part;
    a.ring = b->d_ring;
    a.ctl = b->d_ctl;
    a.n_inst = b->n;
    a.n_items = b->n_items;
    a.timeout_ticks = b->timeout_ticks;
    for (int32_t done = 0; done < nsteps;) {
        a.steps = (nsteps - done < b->steps_per_launch) ? nsteps - done : b->steps_per_launch;
        hipLaunchKernelGGL(sw2d_batch_reset_kernel, dim3(1), dim3(64), 0, s, b->d_ctl);
        SW2D_BHIP(hipGetLastError());
        hipLaunchKernelGGL(sw2d_batch_kernel, dim3(b->grid), dim3(kBatchThreads), 0, s, a);
        SW2D_BHIP(hipGetLastError());
        done += a.steps;
    }
    return SW2D_OK;
}

void drop_graph(sw2d_bctx* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_n = -1;
}

}  // namespace

extern "C" {

size_t sw2d_batch_workspace_bytes(int32_t n, const sw2d_params* p, const int32_t* band_rows) {
    BatchLayout L;
    if (!p || !batch_layout(n, p, band_rows, L)) return 0;
    return L.total;
}

int sw2d_batch_create(int32_t n, const sw2d_params* p, const float* const* d_H,
                      const uint8_t* const* d_mask, float* const* d_state, const int32_t* band_rows,
                      void* d_work, size_t work_bytes, void* hip_stream, sw2d_batch_t* out) {
    if (!out) return SW2D_ESTATE;
    *out = nullptr;
    BatchLayout L;
    if (!p || !d_H || !d_mask || !d_state || !d_work || !batch_layout(n, p, band_rows, L))
        return SW2D_EINVAL;
    if (work_bytes < L.total) return SW2D_ENOSPC;
    if (reinterpret_cast<uintptr_t>(d_work) % kAlign != 0) return SW2D_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!d_H[i] || !d_mask[i] || !d_state[i]) return SW2D_EINVAL;

    sw2d_bctx* b = new (std::nothrow) sw2d_bctx();
    if (!b) return SW2D_ESTATE;
    b->n = n;
    b->p.assign(p, p + n);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->capture = nullptr;
    b->graph = nullptr;
    b->exec = nullptr;
    b->graph_n = -1;
    b->steps_per_launch = 50;
    b->use_graph = true;
    b->steps_done = 0;
    b->n_items = L.n_items;
    char* w = static_cast<char*>(d_work);
    b->d_inst = reinterpret_cast<BatchInst*>(w + L.inst);
    b->d_items = reinterpret_cast<BatchItem*>(w + L.items);
    b->d_part = reinterpret_cast<FoldPartial*>(w + L.part);
    b->d_ring = reinterpret_cast<sw2d_red*>(w + L.ring);
    b->d_ctl = reinterpret_cast<BatchControl*>(w + L.ctl);
    PrepFlags* d_flags = reinterpret_cast<PrepFlags*>(w + L.flags);
    double* d_scratch = reinterpret_cast<double*>(w + L.scratch);

    auto fail = [&](int rc) {
        if (b->capture) (void)hipStreamDestroy(b->capture);
        delete b;
        return rc;
    };

    std::vector<PrepFlags> flags(n, PrepFlags{0u, 0u, 0.0});
    hipError_t e = hipMemcpyAsync(d_flags, flags.data(), n * sizeof(PrepFlags), hipMemcpyHostToDevice,
                                  b->stream);
    b->state.resize((size_t)n * 6);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        const size_t cells = (size_t)p[i].nx * p[i].ny;
        for (int f = 0; f < 6; ++f) b->state[(size_t)i * 6 + f] = d_state[i] + f * cells;
        e = launch_prep(d_H[i], d_mask[i], d_state[i], d_state[i] + cells, d_state[i] + 2 * cells,
                        p[i].nx, p[i].ny, reinterpret_cast<float*>(w + L.hp[i]), d_flags + i, d_scratch,
                        b->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(flags.data(), d_flags, n * sizeof(PrepFlags), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail(batch_hip_fail(e, "sw2d_batch_create"));

    std::vector<BatchInst> inst(n);
    std::vector<BatchItem> items;
    items.reserve(L.n_items);
    for (int i = 0; i < n; ++i) {
        if (flags[i].bad != 0 || flags[i].hmax_bits == 0) return fail(SW2D_EINVAL);
        float hmax;
        std::memcpy(&hmax, &flags[i].hmax_bits, sizeof hmax);
        const sw2d_params& q = p[i];
        const double courant =
            q.dt * std::sqrt(q.g * (double)hmax) * std::sqrt(1.0 / (q.dx * q.dx) + 1.0 / (q.dy * q.dy));
        if (!(courant <= 1.0)) return fail(SW2D_EINVAL);
        BatchInst& in = inst[i];
        in.hp = reinterpret_cast<const float*>(w + L.hp[i]);
        const size_t cells = (size_t)q.nx * q.ny;
        for (int buf = 0; buf < 2; ++buf)
            for (int f = 0; f < 3; ++f) in.state[buf][f] = d_state[i] + (size_t)(3 * buf + f) * cells;
        in.nx = q.nx;
        in.ny = q.ny;
        in.k = sw2d::detail::make_coef(&q);
        in.cell_area = q.dx * q.dy;
        in.h_sum = flags[i].h_sum;
        in.item_begin = (int)items.size();
        const int rows = rows_for(q, band_rows, i);
        const int strips = (q.nx + kStripOut - 1) / kStripOut;
        const int bands = (q.ny + rows - 1) / rows;
        for (int blk = 0; blk < bands; blk += 2)
            for (int st = 0; st < strips; ++st)
                for (int bd = blk; bd < blk + 2 && bd < bands; ++bd) {
                    const int j0 = bd * rows;
                    const int j1 = (j0 + rows < q.ny) ? j0 + rows : q.ny;
                    items.push_back(BatchItem{i, j0, j1, 2 * st + (bd & 1)});
                }
        in.item_end = (int)items.size();
    }
    BatchControl ctl{0u, 0u, 0};
    e = hipMemcpyAsync(b->d_inst, inst.data(), n * sizeof(BatchInst), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(BatchItem),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail(batch_hip_fail(e, "sw2d_batch_create upload"));

    // persistent grid: no more workgroups than the device can hold at once
    int dev = 0, cus = 0, per_cu = 0, clock_khz = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sw2d_batch_kernel, kBatchThreads, 0);
    if (e != hipSuccess) return fail(batch_hip_fail(e, "occupancy query"));
    if (per_cu < 1 || cus < 1) return fail(SW2D_EINVAL);
    if (per_cu > 8) per_cu = 8;
    b->grid = cus * per_cu;
    if (clock_khz <= 0) clock_khz = 100000;
    b->timeout_ticks = (unsigned long long)clock_khz * 1000ull * 2ull;  // 2 s per barrier
    e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(batch_hip_fail(e, "hipStreamCreateWithFlags"));
    *out = b;
    return SW2D_OK;
}

int sw2d_batch_set_launch(sw2d_batch_t b, int32_t steps_per_launch, int32_t use_graph, int32_t grid) {
    if (!b) return SW2D_ESTATE;
    if (steps_per_launch < 1 || grid < 0) return SW2D_EINVAL;
    if (grid > 0) {
        int dev = 0, cus = 0, per_cu = 0;
        SW2D_BHIP(hipGetDevice(&dev));
        SW2D_BHIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        SW2D_BHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sw2d_batch_kernel,
                                                               kBatchThreads, 0));
        if (grid > cus * per_cu) return SW2D_EINVAL;  // must stay co-resident
        b->grid = grid;
    }
    b->steps_per_launch = steps_per_launch;
    b->use_graph = use_graph != 0;
    drop_graph(b);
    return SW2D_OK;
}

int sw2d_batch_step(sw2d_batch_t b, int32_t nsteps) {
    if (!b || nsteps < 0) return SW2D_ESTATE;
    if (nsteps == 0) return SW2D_OK;
    if (!b->use_graph) {
        int rc = enqueue_chunks(b, nsteps, b->stream);
        if (rc) return rc;
    } else {
        if (b->graph_n != nsteps) {
            drop_graph(b);
            SW2D_BHIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_chunks(b, nsteps, b->capture);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->capture, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return batch_hip_fail(e, "hipStreamEndCapture");
            b->graph = g;
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                drop_graph(b);
                return batch_hip_fail(e, "hipGraphInstantiate");
            }
            b->graph_n = nsteps;
        }
        SW2D_BHIP(hipGraphLaunch(b->exec, b->stream));
    }
    b->steps_done += nsteps;
    return SW2D_OK;
}

int sw2d_batch_step_timed(sw2d_batch_t b, int32_t nsteps, double* ms_per_step) {
    if (!b || nsteps < 1 || !ms_per_step) return SW2D_ESTATE;
    hipEvent_t e0, e1;
    SW2D_BHIP(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return batch_hip_fail(e, "hipEventCreate");
    }
    int rc = SW2D_OK;
    e = hipEventRecord(e0, b->stream);
    if (e == hipSuccess) rc = sw2d_batch_step(b, nsteps);
    if (e == hipSuccess && rc == SW2D_OK) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess && rc == SW2D_OK) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess && rc == SW2D_OK) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (e != hipSuccess) return batch_hip_fail(e, "sw2d_batch_step_timed");
    *ms_per_step = (double)ms / nsteps;
    return SW2D_OK;
}

int sw2d_batch_reduce(sw2d_batch_t b, sw2d_red* host_out) {
    if (!b || !host_out) return SW2D_ESTATE;
    if (b->steps_done < 1) return SW2D_ESTATE;
    BatchControl ctl;
    SW2D_BHIP(hipMemcpyAsync(&ctl, b->d_ctl, sizeof ctl, hipMemcpyDeviceToHost, b->stream));
    const size_t slot = (size_t)((b->steps_done - 1) % kBatchRing);
    SW2D_BHIP(hipMemcpyAsync(host_out, b->d_ring + slot * b->n, (size_t)b->n * sizeof(sw2d_red),
                             hipMemcpyDeviceToHost, b->stream));
    SW2D_BHIP(hipStreamSynchronize(b->stream));
    if (ctl.error != 0) {
        std::snprintf(g_batch_msg, sizeof g_batch_msg, "grid barrier wait ran past its deadline");
        sw2d::detail::set_hip_message(g_batch_msg);
        return SW2D_EHIP;
    }
    if (ctl.steps_done != b->steps_done) return SW2D_ESTATE;
    for (int i = 0; i < b->n; ++i) {
        const sw2d_red& r = host_out[i];
        if (!std::isfinite(r.vol_total) || !std::isfinite(r.vol_disp) || !std::isfinite(r.max_abs_u) ||
            !std::isfinite(r.max_abs_v))
            return SW2D_EUNSTABLE;
    }
    return SW2D_OK;
}

int sw2d_batch_state(sw2d_batch_t b, int32_t k, float** d_eta, float** d_u, float** d_v) {
    if (!b || k < 0 || k >= b->n) return SW2D_ESTATE;
    const int cur = (int)(b->steps_done & 1);
    float* const* s = &b->state[(size_t)k * 6 + 3 * cur];
    if (d_eta) *d_eta = s[0];
    if (d_u) *d_u = s[1];
    if (d_v) *d_v = s[2];
    return SW2D_OK;
}

int64_t sw2d_batch_steps_done(sw2d_batch_t b) { return b ? b->steps_done : -1; }

int sw2d_batch_set_barrier_timeout(sw2d_batch_t b, double seconds) {
    if (!b || !(seconds >= 0.0) || seconds > 60.0) return SW2D_EINVAL;
    int dev = 0, clock_khz = 0;
    SW2D_BHIP(hipGetDevice(&dev));
    SW2D_BHIP(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev));
    if (clock_khz <= 0) clock_khz = 100000;
    b->timeout_ticks = (unsigned long long)(seconds * clock_khz * 1000.0);
    drop_graph(b);
    return SW2D_OK;
}

int32_t sw2d_batch_grid(sw2d_batch_t b) { return b ? b->grid : -1; }

int sw2d_batch_destroy(sw2d_batch_t b) {
    if (!b) return SW2D_OK;
    drop_graph(b);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
    return SW2D_OK;
}

}  // extern "C"
