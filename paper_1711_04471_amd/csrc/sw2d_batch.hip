// sw2d_batch.hip - ensembles of independent 2DSW basins of uneven sizes, advanced by one
// persistent launch per chunk of steps, with a grid barrier between steps.
//
// Work list: every (instance, band, group of 4 strips) is one tile for one workgroup, as
// in the single-grid kernel (same tile routine, so each instance is bitwise equal to the
// same basin stepped alone). Tiles are listed instance by instance in blocks of two
// vertically adjacent bands and handed out costliest first: each workgroup takes the next
// tile from a work ticket (one atomic per tile) until the pass's tiles run out, so a
// workgroup that finishes early takes more and the grid reaches the barrier together.
//
// Per pass: workgroups process tiles and write one fold partial per tile and step, then the
// grid meets at a barrier, where workgroup 0 also rewinds the ticket of the next pass. After the barrier, workgroup b adds the partials of instances
// b, b+G, ... in a fixed order and writes their folds to the ring, then goes on with the
// next step.
//
// The barrier uses no contended atomics: every workgroup publishes the epoch it has
// reached in its own flag (after an agent-scope release), workgroup 0 waits for all
// flags in parallel and publishes the epoch in one "go" word, which the others poll.
// Epochs are the global step counts, so they only grow and no flag is ever reset. Every
// wait has a wall-clock deadline: on expiry it raises an error flag and the kernel
// returns, so no wave can wait forever even if the grid were not co-resident.
//
// The steps done so far live in device memory and are advanced by the kernel itself, so
// a captured graph of launches can be replayed without host-side parameters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "sw2d_internal.h"
#include "sw2d_tile.h"

namespace sw2d {

struct BatchInst {
    const float* hp;
    float* state[2][3];
    int nx, ny, strips;
    StepCoef k;
    double cell_area;
    double h_sum;
    int tile_begin, tile_end;  // tiles of this instance in the work list
};

// A self-contained tile descriptor (128 B): everything one workgroup needs for one tile,
// so a tile starts without dependent loads. Copied to LDS once per launch.
struct alignas(16) BatchTile {
    const float* hp;
    float* state[2][3];
    int nx, ny, strips, j0, j1;
    int group2;  // 2 * group + 1 if the band marches south
    int inst;
    int pad0;
    StepCoef k;
    int pad1[3];
};
static_assert(sizeof(BatchTile) == 128, "tile descriptor size");

constexpr int kFlagStride = 16;  // 64-bit words between flags: one 128 B line each

struct BatchControl {
    unsigned error;         // 1: a barrier wait ran past its deadline
    unsigned pad0;
    long long steps_done;   // advanced by the kernel at the end of every launch
    long long passes_done;  // passes over the state so far: its parity picks the current buffer
    unsigned next_tile[2];  // work tickets of the passes of each parity (position in the order)
    long long pad1[kFlagStride - 4];
    unsigned long long go;  // last epoch every workgroup has reached (own line)
    unsigned long long pad2[kFlagStride - 1];
    // followed by one flag line per workgroup
};

constexpr int kBatchThreads = kGroupThreads;
constexpr int kMaxBatchK = 3;  // steps per pass of the batched kernel: 1..3
// Owned columns of a strip for K steps per pass: one column per lane. (Two columns per lane,
// as the single-grid K-step kernel, measured slower on the ensemble: the members are small,
// odd widths need 4-byte accesses, and the persistent grid drops from 4 to 3 resident
// workgroups per CU.)
constexpr int batch_strip_out(int K) { return K == 1 ? kStripOut : kWave - 4 * K; }
constexpr int kBatchRing = 64;  // steps of per-instance folds kept

struct BatchArgs {
    const BatchInst* inst;
    const BatchTile* tiles;
    const int* order;      // tile ids, costliest first: the order in which tiles are handed out
    FoldPartial* part;  // [2][K][n_tiles]
    sw2d_red* ring;     // [kBatchRing][n_inst]
    BatchControl* ctl;
    unsigned long long* flags;  // [grid][kFlagStride]
    int n_inst, n_tiles, steps;
    unsigned long long timeout_ticks;
};

__device__ __forceinline__ bool spin_until(const unsigned long long* word, unsigned long long epoch,
                                           unsigned long long deadline, BatchControl* ctl) {
    while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        __builtin_amdgcn_s_sleep(2);
        if (wall_clock64() > deadline) {
            __hip_atomic_fetch_or(&ctl->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// Returns false (for the whole workgroup) if a wait ran past the deadline. Workgroup 0 also
// rewinds the work ticket of the next pass (`rewind`): its last use, two passes back, is over
// once every workgroup has arrived.
__device__ bool grid_barrier(const BatchArgs& a, unsigned long long epoch, unsigned* rewind) {
    __shared__ int s_ok;
    const unsigned long long deadline = wall_clock64() + a.timeout_ticks;
    if (threadIdx.x == 0) s_ok = 1;
    __syncthreads();  // every wave's stores of this step precede thread 0's release
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(a.flags + (size_t)blockIdx.x * kFlagStride, epoch, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0) {
        for (int w = threadIdx.x; w < (int)gridDim.x; w += kBatchThreads)
            if (!spin_until(a.flags + (size_t)w * kFlagStride, epoch, deadline, a.ctl)) s_ok = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        if (threadIdx.x == 0 && s_ok) {
            __hip_atomic_store(rewind, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&a.ctl->go, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (threadIdx.x == 0 && s_ok) {
        if (!spin_until(&a.ctl->go, epoch, deadline, a.ctl)) s_ok = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return s_ok != 0;
}

// Adds the tile partials of instance i (fixed order) and writes its fold entry for `step`.
__device__ void fold_instance(const BatchArgs& a, int i, int slot, long long step) {
    __shared__ double s_disp[kBatchThreads];
    __shared__ float s_mu[kBatchThreads], s_mv[kBatchThreads];
    const BatchInst& in = a.inst[i];
    const FoldPartial* p = a.part + (size_t)slot * a.n_tiles;
    double disp = 0.0;
    float mu = 0.f, mv = 0.f;
    for (int it = in.tile_begin + threadIdx.x; it < in.tile_end; it += kBatchThreads) {
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

// the K steps of one pass: partial slots slot0 .. slot0 + K - 1, steps first .. first + K - 1
__device__ __forceinline__ void fold_pass(const BatchArgs& a, int logical_wg, int nwg, int slot0,
                                          long long first, int K) {
    for (int s = 0; s < K; ++s) fold_step(a, logical_wg, nwg, slot0 + s, first + s);
}

__device__ __forceinline__ int logical_block(int b, int n) {
    const int q = n / kXcds, r = n % kXcds;
    const int x = b % kXcds, k = b / kXcds;
    return x * q + min(x, r) + k;
}

__device__ __forceinline__ void batch_wave_sums(double& disp, float& mu, float& mv) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        disp += __shfl_xor(disp, off, kWave);
        mu = fmaxf(mu, __shfl_xor(mu, off, kWave));
        mv = fmaxf(mv, __shfl_xor(mv, off, kWave));
    }
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uintptr_t v = reinterpret_cast<uintptr_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T*>(((uintptr_t)hi << 32) | lo);
}

__device__ __forceinline__ float uniform_f(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// K steps per pass over each member (temporal blocking as in the single-grid K-step
// kernel: bands read a 2K-row halo, strips lose 2K columns on each side); the grid meets once
// per pass.
template <int K>
__global__ __launch_bounds__(kBatchThreads) void sw2d_batch_kernel(BatchArgs a) {
    __shared__ BatchTile s_tile;
    __shared__ int s_pos, s_id;
    __shared__ double s_disp[kWavesPerGroup];
    __shared__ float s_mu[kWavesPerGroup], s_mv[kWavesPerGroup];
    constexpr int kOut = batch_strip_out(K);
    constexpr int kEdge = (K == 1) ? kHalo : 2 * K;  // unowned columns on each side of a strip
    const int nwg = gridDim.x;
    const int lwg = logical_block(blockIdx.x, nwg);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const long long base = a.ctl->steps_done;
    const long long pbase = a.ctl->passes_done;
    const int passes = a.steps / K;

    for (int ps = 0; ps < passes; ++ps) {
        const long long step0 = base + (long long)ps * K;  // steps made before this pass
        const long long gpass = pbase + ps;                // passes made before this one
        const int cur = (int)(gpass & 1);
        if (ps > 0) fold_pass(a, lwg, nwg, ((ps - 1) & 1) * K, step0 - K + 1, K);
        FoldPartial* part = a.part + (size_t)(ps & 1) * K * a.n_tiles;
        unsigned* ticket = &a.ctl->next_tile[gpass & 1];
        // Tiles are handed out costliest first, one per request, so a workgroup that finishes
        // early takes more of them and every workgroup reaches the barrier at about the same
        // time. Which workgroup steps a tile changes no bit of any result.
        for (;;) {
            if (threadIdx.x == 0)
                s_pos = (int)__hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const int pos = s_pos;
            if (pos >= a.n_tiles) break;  // the same value in every thread of the workgroup
            constexpr int kChunks = sizeof(BatchTile) / 16;
            if (threadIdx.x < kChunks) {
                const int id = a.order[pos];
                reinterpret_cast<uint4*>(&s_tile)[threadIdx.x] = reinterpret_cast<const uint4*>(a.tiles + id)[threadIdx.x];
                if (threadIdx.x == 0) s_id = id;
            }
            __syncthreads();
            const BatchTile& t = s_tile;
            const int nx = uniform(t.nx), ny = uniform(t.ny);
            const int group2 = uniform(t.group2);
            const int strip = (group2 >> 1) * kWavesPerGroup + wave;
            const int c = strip * kOut - kEdge + lane;  // this lane's column
            const bool col_in = c >= 0 && c < nx;
            const bool out_lane = col_in && lane >= kEdge && lane < kWave - kEdge;
            LaneFolds F[K];
            if (strip < uniform(t.strips)) {
                StepCoef kc;
                kc.cx = uniform_f(t.k.cx);
                kc.cy = uniform_f(t.k.cy);
                kc.rx = uniform_f(t.k.rx);
                kc.ry = uniform_f(t.k.ry);
                kc.e4 = uniform_f(t.k.e4);
                kc.kf = 0.f;
                const float* hp = uniform_ptr(t.hp);
                const float* e0 = uniform_ptr(t.state[cur][0]);
                const float* u0 = uniform_ptr(t.state[cur][1]);
                const float* v0 = uniform_ptr(t.state[cur][2]);
                float* e1 = uniform_ptr(t.state[cur ^ 1][0]);
                float* u1 = uniform_ptr(t.state[cur ^ 1][1]);
                float* v1 = uniform_ptr(t.state[cur ^ 1][2]);
                const int j0 = uniform(t.j0), j1 = uniform(t.j1);
                if constexpr (K == 1) {
                    double f_disp = 0.0;
                    float f_mu = 0.f, f_mv = 0.f;
                    if (group2 & 1)
                        march<false>(e0, u0, v0, hp, e1, u1, v1, nx, ny, c, col_in, out_lane, j0, j1, kc, f_disp,
                                     f_mu, f_mv);
                    else
                        march<true>(e0, u0, v0, hp, e1, u1, v1, nx, ny, c, col_in, out_lane, j0, j1, kc, f_disp,
                                    f_mu, f_mv);
                    F[0].disp = f_disp;
                    F[0].max_u = f_mu;
                    F[0].max_v = f_mv;
                } else {
                    if (group2 & 1)
                        marchK<K, false>(e0, u0, v0, hp, e1, u1, v1, nx, ny, c, col_in, out_lane, j0, j1, kc, F);
                    else
                        marchK<K, true>(e0, u0, v0, hp, e1, u1, v1, nx, ny, c, col_in, out_lane, j0, j1, kc, F);
                }
            }
            const int it = s_id;
#pragma unroll
            for (int s = 0; s < K; ++s) {
                double f_disp = F[s].disp;
                float f_mu = F[s].mu(), f_mv = F[s].mv();
                batch_wave_sums(f_disp, f_mu, f_mv);
                if (lane == 0) {
                    s_disp[wave] = f_disp;
                    s_mu[wave] = f_mu;
                    s_mv[wave] = f_mv;
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    double d = 0.0;
                    float m1 = 0.f, m2 = 0.f;
#pragma unroll
                    for (int w = 0; w < kWavesPerGroup; ++w) {
                        d += s_disp[w];
                        m1 = fmaxf(m1, s_mu[w]);
                        m2 = fmaxf(m2, s_mv[w]);
                    }
                    FoldPartial* q = part + (size_t)s * a.n_tiles + it;
                    q->disp = d;
                    q->mu = m1;
                    q->mv = m2;
                }
                __syncthreads();
            }
        }
        if (!grid_barrier(a, (unsigned long long)(step0 + K), &a.ctl->next_tile[(gpass + 1) & 1])) return;
    }
    fold_pass(a, lwg, nwg, ((passes - 1) & 1) * K, base + (long long)(passes - 1) * K + 1, K);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctl->steps_done = base + a.steps;
        a.ctl->passes_done = pbase + passes;
    }
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
    BatchTile* d_tiles;
    int* d_order;         // tile ids, costliest first
    FoldPartial* d_part;
    sw2d_red* d_ring;
    BatchControl* d_ctl;
    unsigned long long* d_flags;
    int max_grid;
    int n_tiles;
    int grid;
    int steps_per_launch;
    int steps_per_pass;            // K of the batched kernel, 1..kMaxBatchK
    bool use_graph;
    int64_t steps_done;
    int64_t passes_done;
    std::vector<BatchInst> inst;   // host copy (tile ranges for the current K)
    std::vector<int> rows;         // band height per member
    size_t tile_capacity;          // descriptors the workspace holds
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
    size_t flags, scratch, inst, tiles, order, part, ring, ctl, gflags, total;
    int n_tiles;
    std::vector<int> tiles_of;  // per instance
};

constexpr int kMaxBatchGrid = 256 * 8;  // flag lines reserved: 8 workgroups on each of 256 CUs
// Resident workgroups per CU that the grid may count on. The occupancy query counts vector
// registers and LDS, but a SIMD of this family also holds at most 800 scalar registers, so a
// kernel near 100 SGPRs fits 7 waves per SIMD even when its vector registers would allow 8;
// a grid barrier that waits for a workgroup that never became resident would only end at
// its deadline. 6 keeps a margin below that bound.
constexpr int kBatchWgPerCu = 6;


int rows_for(const sw2d_params& p, const int32_t* band_rows, int i) {
    int r = band_rows ? band_rows[i] : 16;
    if (r > p.ny) r = p.ny;
    return r;
}

bool batch_layout(int n, const sw2d_params* p, const int32_t* band_rows, BatchLayout& L) {
    if (n < 1) return false;
    size_t off = 0;
    L.hp.resize(n);
    L.tiles_of.resize(n);
    L.n_tiles = 0;
    for (int i = 0; i < n; ++i) {
        if (!sw2d::detail::params_valid(&p[i]) || p[i].flags != 0) return false;  // plain model only
        const int rows = rows_for(p[i], band_rows, i);
        if (rows < 1 || (band_rows && band_rows[i] < kMinRows)) return false;
        L.hp[i] = off;
        off = align_up(off + (size_t)p[i].nx * p[i].ny * sizeof(float));
        // the narrowest strips of any K give the most tiles
        int narrow = batch_strip_out(1);
        for (int K = 2; K <= kMaxBatchK; ++K) narrow = std::min(narrow, batch_strip_out(K));
        const int strips = (p[i].nx + narrow - 1) / narrow;
        const int groups = (strips + kWavesPerGroup - 1) / kWavesPerGroup;
        const int bands = (p[i].ny + rows - 1) / rows;
        L.tiles_of[i] = groups * bands;
        if ((int64_t)L.n_tiles + L.tiles_of[i] > (1 << 30)) return false;
        L.n_tiles += L.tiles_of[i];
    }
    L.flags = off;
    off = align_up(off + (size_t)n * sizeof(PrepFlags));
    L.scratch = off;
    off = align_up(off + kHsumBlocks * sizeof(double));
    L.inst = off;
    off = align_up(off + (size_t)n * sizeof(BatchInst));
    L.tiles = off;
    off = align_up(off + (size_t)L.n_tiles * sizeof(BatchTile));
    L.order = off;
    off = align_up(off + (size_t)L.n_tiles * sizeof(int));
    L.part = off;
    off = align_up(off + 2 * (size_t)kMaxBatchK * L.n_tiles * sizeof(FoldPartial));
    L.ring = off;
    off = align_up(off + (size_t)kBatchRing * n * sizeof(sw2d_red));
    L.ctl = off;
    off = align_up(off + sizeof(BatchControl));
    L.gflags = off;
    off = align_up(off + (size_t)kMaxBatchGrid * kFlagStride * sizeof(unsigned long long));
    L.total = off;
    return true;
}

int enqueue_chunks(sw2d_bctx* b, int32_t nsteps, hipStream_t s) {
    BatchArgs a;
    a.inst = b->d_inst;
    a.tiles = b->d_tiles;
    a.order = b->d_order;
    a.part = b->d_part;
    a.ring = b->d_ring;
    a.ctl = b->d_ctl;
    a.flags = b->d_flags;
    a.n_inst = b->n;
    a.n_tiles = b->n_tiles;
    a.timeout_ticks = b->timeout_ticks;
    const int K = b->steps_per_pass;
    const int per_launch = b->steps_per_launch >= K ? b->steps_per_launch / K * K : K;
    for (int32_t done = 0; done < nsteps;) {
        a.steps = (nsteps - done < per_launch) ? nsteps - done : per_launch;  // a multiple of K
        switch (K) {
            case 1:
                hipLaunchKernelGGL(sw2d_batch_kernel<1>, dim3(b->grid), dim3(kBatchThreads), 0, s, a);
                break;
            case 2:
                hipLaunchKernelGGL(sw2d_batch_kernel<2>, dim3(b->grid), dim3(kBatchThreads), 0, s, a);
                break;
            case 3:
                hipLaunchKernelGGL(sw2d_batch_kernel<3>, dim3(b->grid), dim3(kBatchThreads), 0, s, a);
                break;
            default:
                return SW2D_EINVAL;
        }
        SW2D_BHIP(hipGetLastError());
        done += a.steps;
    }
    return SW2D_OK;
}

// Tile list of every member for K steps per pass (strips of batch_strip_out(K) columns),
// written to the device with the members' tile ranges.
int upload_tiles(sw2d_bctx* b, int K) {
    std::vector<BatchTile> tiles;
    std::vector<int> cost;
    const int out = batch_strip_out(K);
    for (int i = 0; i < b->n; ++i) {
        BatchInst& in = b->inst[i];
        in.strips = (in.nx + out - 1) / out;
        in.tile_begin = (int)tiles.size();
        const int rows = b->rows[i];
        const int groups = (in.strips + kWavesPerGroup - 1) / kWavesPerGroup;
        const int bands = (in.ny + rows - 1) / rows;
        for (int blk = 0; blk < bands; blk += 2)
            for (int gr = 0; gr < groups; ++gr)
                for (int bd = blk; bd < blk + 2 && bd < bands; ++bd) {
                    BatchTile t;
                    std::memset(&t, 0, sizeof t);
                    t.hp = in.hp;
                    for (int buf = 0; buf < 2; ++buf)
                        for (int f = 0; f < 3; ++f) t.state[buf][f] = in.state[buf][f];
                    t.nx = in.nx;
                    t.ny = in.ny;
                    t.strips = in.strips;
                    t.j0 = bd * rows;
                    t.j1 = (t.j0 + rows < in.ny) ? t.j0 + rows : in.ny;
                    t.group2 = 2 * gr + (bd & 1);
                    t.inst = i;
                    t.k = in.k;
                    tiles.push_back(t);
                    const int strips_here = in.strips - kWavesPerGroup * gr;
                    cost.push_back((t.j1 - t.j0 + 4 * K) *
                                   (strips_here < kWavesPerGroup ? strips_here : kWavesPerGroup));
                }
        in.tile_end = (int)tiles.size();
    }
    if (tiles.size() > b->tile_capacity) return SW2D_ENOSPC;
    b->n_tiles = (int)tiles.size();
    // hand-out order: costliest first (rows marched x strips); equal costs keep list order, so
    // the neighbouring bands of a member go out together
    std::vector<int> order(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    SW2D_BHIP(hipMemcpyAsync(b->d_inst, b->inst.data(), b->n * sizeof(BatchInst), hipMemcpyHostToDevice, b->stream));
    SW2D_BHIP(hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice,
                             b->stream));
    if (!order.empty())
        SW2D_BHIP(hipMemcpyAsync(b->d_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice,
                                 b->stream));
    SW2D_BHIP(hipStreamSynchronize(b->stream));
    return SW2D_OK;
}

// Workgroups of the K-step kernel the device holds at once (capped, see kBatchWgPerCu).
int resident_grid(int K, int* out) {
    int dev = 0, cus = 0, per_cu = 0;
    SW2D_BHIP(hipGetDevice(&dev));
    SW2D_BHIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const void* fn = K == 1   ? reinterpret_cast<const void*>(&sw2d_batch_kernel<1>)
                     : K == 2 ? reinterpret_cast<const void*>(&sw2d_batch_kernel<2>)
                              : reinterpret_cast<const void*>(&sw2d_batch_kernel<3>);
    SW2D_BHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBatchThreads, 0));
    if (per_cu < 1 || cus < 1) return SW2D_EINVAL;
    if (per_cu > kBatchWgPerCu) per_cu = kBatchWgPerCu;
    int g = cus * per_cu;
    if (g > kMaxBatchGrid) g = kMaxBatchGrid;
    *out = g;
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
    b->n_tiles = L.n_tiles;
    char* w = static_cast<char*>(d_work);
    b->d_inst = reinterpret_cast<BatchInst*>(w + L.inst);
    b->d_tiles = reinterpret_cast<BatchTile*>(w + L.tiles);
    b->d_order = reinterpret_cast<int*>(w + L.order);
    b->d_flags = reinterpret_cast<unsigned long long*>(w + L.gflags);
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

    b->inst.assign(n, BatchInst{});
    b->rows.assign(n, 0);
    b->tile_capacity = (size_t)L.n_tiles;
    for (int i = 0; i < n; ++i) {
        if (flags[i].bad != 0 || flags[i].hmax_bits == 0) return fail(SW2D_EINVAL);
        float hmax;
        std::memcpy(&hmax, &flags[i].hmax_bits, sizeof hmax);
        const sw2d_params& q = p[i];
        const double courant =
            q.dt * std::sqrt(q.g * (double)hmax) * std::sqrt(1.0 / (q.dx * q.dx) + 1.0 / (q.dy * q.dy));
        if (!(courant <= 1.0)) return fail(SW2D_EINVAL);
        BatchInst& in = b->inst[i];
        in.hp = reinterpret_cast<const float*>(w + L.hp[i]);
        const size_t cells = (size_t)q.nx * q.ny;
        for (int buf = 0; buf < 2; ++buf)
            for (int f = 0; f < 3; ++f) in.state[buf][f] = d_state[i] + (size_t)(3 * buf + f) * cells;
        in.nx = q.nx;
        in.ny = q.ny;
        in.k = sw2d::detail::make_coef(&q);
        in.cell_area = q.dx * q.dy;
        in.h_sum = flags[i].h_sum;
        b->rows[i] = rows_for(q, band_rows, i);
    }
    b->steps_per_pass = 1;
    b->passes_done = 0;
    int rc = upload_tiles(b, 1);
    if (rc) return fail(rc);
    BatchControl ctl;
    std::memset(&ctl, 0, sizeof ctl);
    std::vector<unsigned long long> zero_flags((size_t)kMaxBatchGrid * kFlagStride, 0ull);
    e = hipMemcpyAsync(b->d_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_flags, zero_flags.data(), zero_flags.size() * sizeof(unsigned long long),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail(batch_hip_fail(e, "sw2d_batch_create upload"));

    // persistent grid: no more workgroups than the device can hold at once
    int dev = 0, clock_khz = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return fail(batch_hip_fail(e, "device query"));
    rc = resident_grid(1, &b->max_grid);
    if (rc) return fail(rc);
    b->grid = b->max_grid;
    if (clock_khz <= 0) clock_khz = 100000;
    b->timeout_ticks = (unsigned long long)clock_khz * 1000ull * 2ull;  // 2 s per barrier
    e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(batch_hip_fail(e, "hipStreamCreateWithFlags"));
    *out = b;
    return SW2D_OK;
}

int sw2d_batch_set_time_blocking(sw2d_batch_t b, int32_t steps_per_pass) {
    if (!b) return SW2D_ESTATE;
    if (steps_per_pass < 1 || steps_per_pass > kMaxBatchK) return SW2D_EINVAL;
    if (steps_per_pass == b->steps_per_pass) return SW2D_OK;
    SW2D_BHIP(hipStreamSynchronize(b->stream));  // launches in flight read the old tile list
    int max_grid = 0;
    int rc = resident_grid(steps_per_pass, &max_grid);
    if (rc) return rc;
    rc = upload_tiles(b, steps_per_pass);
    if (rc) return rc;
    b->steps_per_pass = steps_per_pass;
    b->max_grid = max_grid;
    if (b->grid > max_grid || b->grid <= 0) b->grid = max_grid;
    drop_graph(b);
    return SW2D_OK;
}

int32_t sw2d_batch_time_blocking(sw2d_batch_t b) { return b ? b->steps_per_pass : -1; }

int sw2d_batch_set_launch(sw2d_batch_t b, int32_t steps_per_launch, int32_t use_graph, int32_t grid) {
    if (!b) return SW2D_ESTATE;
    if (steps_per_launch < 1 || grid < 0) return SW2D_EINVAL;
    if (grid > b->max_grid) return SW2D_EINVAL;  // must stay co-resident
    b->grid = grid > 0 ? grid : b->max_grid;
    b->steps_per_launch = steps_per_launch;
    b->use_graph = use_graph != 0;
    drop_graph(b);
    return SW2D_OK;
}

int sw2d_batch_step(sw2d_batch_t b, int32_t nsteps) {
    if (!b || nsteps < 0) return SW2D_ESTATE;
    if (nsteps == 0) return SW2D_OK;
    if (nsteps % b->steps_per_pass != 0) return SW2D_EINVAL;
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
    b->passes_done += nsteps / b->steps_per_pass;
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
    (void)kBatchRing;
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
    const int cur = (int)(b->passes_done & 1);
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
