// sw2d_kernels.hip - gfx950 kernels for the 2DSW time step and its per-step folds.
//
// One step of the model of Sect. 6.2 (predictor "dyn", first-order Shapiro filter,
// velocity update) fused into a single pass over HBM, with the folds the paper's
// compiler would emit as reductions (Sect. 4.3). The paper's compiler produces three
// separate map kernels (Sect. 6.2); fusing them is the map-fusion rewrite it
// describes (Sect. 4.3), done here by hand so that each step reads
// eta, u, v, H (16 B/cell) and writes eta, u, v (12 B/cell) exactly once.
//
// Work decomposition of the fused step (sw2d_step_kernel):
//   * a wave (64 lanes) owns a strip of 64 consecutive columns; lane l holds column
//     c = 60*strip - 2 + l. Lanes 2..61 produce output, lanes 0,1 and 62,63 are the
//     two-column halo the radius-2 stencil needs, so strips tile the row with
//     stride 60 and no LDS tile or barrier is needed inside the stencil;
//   * east/west neighbours come from cross-lane shuffles of registers;
//   * the wave marches north through a band of rows. Row r is loaded once (one
//     coalesced 256 B row segment per field, the next row prefetched) and flows
//     through a register pipeline: row r gives the x-fluxes, row r-1 the y-fluxes
//     and the predicted surface es, row r-2 the Shapiro output;
//   * 4 waves (adjacent strips) form a workgroup; workgroups are mapped to bands and
//     strip groups XCD-contiguously so that neighbouring tiles share one L2.
// Folds: per-lane FP64 sums of eta and FP32 maxima -> wave butterfly -> workgroup
// (LDS, fixed order) -> one partial per workgroup and step; sw2d_fold_kernel later adds
// the partials of each step in a fixed order, so the folds are bitwise reproducible.
// The static part of the total volume, sum_wet H, is folded once per handle.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw2d_internal.h"
#include "sw2d_pair.h"
#include "sw2d_tile.h"

namespace sw2d {

// Band and strip group of workgroup b. Workgroup b is dispatched to XCD b % 8; each XCD
// gets a contiguous range of logical tiles so that halo rows and columns shared by
// neighbours hit the same L2. Logical tiles run through blocks of two vertically adjacent
// bands, strip group by strip group, so the two bands of a block are dispatched together.
constexpr int kBandBlock = 2;

__device__ __forceinline__ int2 band_and_group(int b, int nblocks, int groups_x, int bands) {
    const int q = nblocks / kXcds, r = nblocks % kXcds;
    const int x = b % kXcds, kq = b / kXcds;
    const int tile = x * q + min(x, r) + kq;
    const int per_block = groups_x * kBandBlock;
    const int blk = tile / per_block;
    const int rem = tile - blk * per_block;
    const int nb = min(kBandBlock, bands - blk * kBandBlock);
    const int group = rem / nb;
    return make_int2(blk * kBandBlock + (rem - group * nb), group);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, kWave));
    return x;
}

// Sum of a double over a 256-thread workgroup in a fixed order (result in thread 0).
__device__ __forceinline__ double block_sum_256(double x, double* lds) {
    lds[threadIdx.x] = x;
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) lds[threadIdx.x] += lds[threadIdx.x + half];
        __syncthreads();
    }
    return lds[0];
}

// Adds the per-wave partial folds of one workgroup in wave order and writes them.
__device__ __forceinline__ void workgroup_fold(double disp, float mu, float mv, FoldPartial* out) {
    __shared__ double s_disp[kWavesPerGroup];
    __shared__ float s_mu[kWavesPerGroup], s_mv[kWavesPerGroup];
    disp = wave_sum(disp);
    mu = wave_max(mu);
    mv = wave_max(mv);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) {
        s_disp[wave] = disp;
        s_mu[wave] = mu;
        s_mv[wave] = mv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        float c = 0.f, d = 0.f;
#pragma unroll
        for (int w = 0; w < kWavesPerGroup; ++w) {
            b += s_disp[w];
            c = fmaxf(c, s_mu[w]);
            d = fmaxf(d, s_mv[w]);
        }
        out->disp = b;
        out->mu = c;
        out->mv = d;
    }
}

template <int kVar>
__global__ __launch_bounds__(kGroupThreads) void sw2d_step_kernel(
    const float* __restrict__ eta, const float* __restrict__ u, const float* __restrict__ v,
    const float* __restrict__ hp, float* __restrict__ eta_o, float* __restrict__ u_o,
    float* __restrict__ v_o, FoldPartial* __restrict__ part, StepGeometry geo, StepCoef k) {
    const int2 bg = band_and_group(blockIdx.x, geo.nblocks, geo.groups_x, geo.bands);
    const int band = bg.x, group = bg.y;
    constexpr bool kAdv = (kVar & kVarAdvection) != 0;
    constexpr int kOut = kAdv ? kAdvStripOut : kStripOut;
    constexpr int kWest = kAdv ? kAdvHaloW : kHalo;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int strip = group * kWavesPerGroup + wave;
    const int c = strip * kOut - kWest + lane;
    const bool col_in = c >= 0 && c < geo.nx;
    const bool out_lane = col_in && lane >= kWest && lane < kWest + kOut;
    const int j0 = band * geo.rows;
    const int j1 = min(j0 + geo.rows, geo.ny);

    double f_disp = 0.0;
    float f_mu = 0.f, f_mv = 0.f;
    if (kAdv && strip < geo.strips) {
        march_adv<kVar>(eta, u, v, hp, eta_o, u_o, v_o, geo.nx, geo.ny, c, col_in, out_lane, j0, j1, k, f_disp,
                        f_mu, f_mv);
    } else if (strip < geo.strips) {
        // Odd bands march south, so each band boundary is read by both of its bands at
        // the same moment (both at their start or both at their end) and the second
        // read hits L2 instead of HBM.
        if (band & 1)
            march<false, kVar>(eta, u, v, hp, eta_o, u_o, v_o, geo.nx, geo.ny, c, col_in, out_lane, j0, j1,
                               k, f_disp, f_mu, f_mv);
        else
            march<true, kVar>(eta, u, v, hp, eta_o, u_o, v_o, geo.nx, geo.ny, c, col_in, out_lane, j0, j1,
                              k, f_disp, f_mu, f_mv);
    }
    workgroup_fold(f_disp, f_mu, f_mv, part + blockIdx.x);
}

// K steps per pass over HBM (temporal blocking): strips of 64 - 4K owned columns, bands
// with a 2K-row halo; the intermediate states stay in registers. kVar: plain or a variant
// without advection.
template <int K, int kVar = 0>
__global__ __launch_bounds__(kGroupThreads) void sw2d_stepk_kernel(
    const float* __restrict__ eta, const float* __restrict__ u, const float* __restrict__ v,
    const float* __restrict__ hp, float* __restrict__ eta_o, float* __restrict__ u_o,
    float* __restrict__ v_o, FoldPartial* __restrict__ part, int stride, StepGeometry geo, StepCoef k) {
    const int2 bg = band_and_group(blockIdx.x, geo.nblocks, geo.groups_x, geo.bands);
    const int band = bg.x, group = bg.y;
    constexpr int kOut = kWave - 4 * K;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int strip = group * kWavesPerGroup + wave;
    const int c = strip * kOut - 2 * K + lane;
    const bool col_in = c >= 0 && c < geo.nx;
    const bool out_lane = col_in && lane >= 2 * K && lane < kWave - 2 * K;
    const int j0 = band * geo.rows;
    const int j1 = min(j0 + geo.rows, geo.ny);

    LaneFolds F[K];
    if (strip < geo.strips) {
        if (band & 1)  // odd bands march south
            marchK<K, false, kVar>(eta, u, v, hp, eta_o, u_o, v_o, geo.nx, geo.ny, c, col_in, out_lane, j0, j1, k,
                                   F);
        else
            marchK<K, true, kVar>(eta, u, v, hp, eta_o, u_o, v_o, geo.nx, geo.ny, c, col_in, out_lane, j0, j1, k,
                                  F);
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
        if (s > 0) __syncthreads();
        workgroup_fold(F[s].disp, F[s].mu(), F[s].mv(), part + (size_t)s * stride + blockIdx.x);
    }
}

// The same with two adjacent columns per lane: strips of 128 - 4K owned columns; kWide when
// nx is even (8-byte row accesses). The register budget is held to 3 waves per SIMD.
template <int K, bool kWide>
__global__ __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(3))) void sw2d_stepk_pair_kernel(
    const float* __restrict__ eta, const float* __restrict__ u, const float* __restrict__ v,
    const float* __restrict__ hp, float* __restrict__ eta_o, float* __restrict__ u_o,
    float* __restrict__ v_o, FoldPartial* __restrict__ part, int stride, StepGeometry geo, StepCoef k) {
    const int2 bg = band_and_group(blockIdx.x, geo.nblocks, geo.groups_x, geo.bands);
    const int band = bg.x, group = bg.y;
    constexpr int kOut = 2 * kWave - 4 * K;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int strip = group * kWavesPerGroup + wave;
    const int c0 = strip * kOut - 2 * K + 2 * lane;
    const bool col_in = c0 >= 0 && c0 < geo.nx;
    const bool owned = col_in && lane >= K && lane < kWave - K;
    const int j0 = band * geo.rows;
    const int j1 = min(j0 + geo.rows, geo.ny);

    // per-lane FP64 surface sums of the K steps (see PairFolds)
    __shared__ double s_disp[K][kGroupThreads];
    PairFolds F[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
        s_disp[s][threadIdx.x] = 0.0;
        F[s].disp = &s_disp[s][threadIdx.x];
    }
    if (strip < geo.strips) {
        if (band & 1)  // odd bands march south
            marchK_pair<K, false, kWide>(eta, u, v, hp, eta_o, u_o, v_o, geo.nx, geo.ny, c0, col_in, owned, j0, j1,
                                         k, F);
        else
            marchK_pair<K, true, kWide>(eta, u, v, hp, eta_o, u_o, v_o, geo.nx, geo.ny, c0, col_in, owned, j0, j1,
                                        k, F);
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
        if (s > 0) __syncthreads();
        workgroup_fold(s_disp[s][threadIdx.x], F[s].max_u, F[s].max_v, part + (size_t)s * stride + blockIdx.x);
    }
}

// Final level of the folds: one workgroup per step adds that step's partials in a
// fixed order and writes the ring entry. h_sum = sum over water cells of H.
__global__ __launch_bounds__(kFoldThreads) void sw2d_fold_kernel(const FoldPartial* __restrict__ part,
                                                                 int nparts, int stride,
                                                                 int64_t first_step,
                                                                 sw2d_red* __restrict__ ring,
                                                                 int ring_cap, double cell_area,
                                                                 double h_sum) {
    __shared__ double s_disp[kFoldThreads];
    __shared__ float s_mu[kFoldThreads], s_mv[kFoldThreads];
    const FoldPartial* p = part + (size_t)blockIdx.x * stride;
    double disp = 0.0;
    float mu = 0.f, mv = 0.f;
    for (int i = threadIdx.x; i < nparts; i += kFoldThreads) {
        disp += p[i].disp;
        mu = fmaxf(mu, p[i].mu);
        mv = fmaxf(mv, p[i].mv);
    }
    const int t = threadIdx.x;
    s_disp[t] = disp;
    s_mu[t] = mu;
    s_mv[t] = mv;
    __syncthreads();
    for (int half = kFoldThreads / 2; half > 0; half >>= 1) {
        if (t < half) {
            s_disp[t] += s_disp[t + half];
            s_mu[t] = fmaxf(s_mu[t], s_mu[t + half]);
            s_mv[t] = fmaxf(s_mv[t], s_mv[t + half]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const int64_t step = first_step + blockIdx.x;
        sw2d_red* o = ring + (size_t)((step - 1) % ring_cap);
        o->step = step;
        o->vol_total = cell_area * (h_sum + s_disp[0]);
        o->vol_disp = cell_area * s_disp[0];
        o->max_abs_u = s_mu[0];
        o->max_abs_v = s_mv[0];
    }
}

// Static preparation, once per handle: validate the inputs, pack the land mask into the
// depth field (hp = wet ? H : 0, so wet == hp > 0) and find the deepest water cell. With
// wetting and drying (allow_dry) a water cell may start empty (H + eta = 0).
__global__ __launch_bounds__(256) void sw2d_prep_kernel(const float* __restrict__ H,
                                                        const uint8_t* __restrict__ mask,
                                                        const float* __restrict__ eta,
                                                        const float* __restrict__ u,
                                                        const float* __restrict__ v, int nx, int ny,
                                                        float* __restrict__ hp,
                                                        PrepFlags* __restrict__ flags, bool allow_dry) {
    const size_t n = (size_t)nx * ny;
    uint32_t bad = 0;
    uint32_t hmax = 0;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx / nx), i = (int)(idx - (size_t)j * nx);
        const bool wet = mask[idx] != 0;
        const float d = H[idx], e = eta[idx];
        if (!isfinite(e) || !isfinite(u[idx]) || !isfinite(v[idx])) bad |= kBadState;
        if (wet) {
            if (i == 0 || j == 0 || i == nx - 1 || j == ny - 1) bad |= kWetBorder;
            if (!(d > 0.f) || !isfinite(d)) bad |= kBadDepth;
            else {
                hmax = max(hmax, __float_as_uint(d));  // positive floats order like their bits
                if (allow_dry ? !(d + e >= 0.f) : !(d + e > 0.f)) bad |= kDryCell;
            }
        }
        hp[idx] = (wet && d > 0.f && isfinite(d)) ? d : 0.f;
    }
    // one atomic per wave
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        bad |= __shfl_xor(bad, off, kWave);
        hmax = max(hmax, (uint32_t)__shfl_xor((int)hmax, off, kWave));
    }
    if (threadIdx.x % kWave == 0) {
        if (bad) atomicOr(&flags->bad, bad);
        atomicMax(&flags->hmax_bits, hmax);
    }
}

// sum_wet H in a fixed order: workgroup b adds rows [b ny / G, (b+1) ny / G) of hp.
__global__ __launch_bounds__(256) void sw2d_hsum_kernel(const float* __restrict__ hp, int nx, int ny,
                                                        double* __restrict__ partial) {
    __shared__ double lds[256];
    const int G = gridDim.x;
    const int j0 = (int)((int64_t)blockIdx.x * ny / G), j1 = (int)((int64_t)(blockIdx.x + 1) * ny / G);
    double s = 0.0;
    for (int j = j0; j < j1; ++j)
        for (int i = threadIdx.x; i < nx; i += 256) s += (double)hp[(size_t)j * nx + i];
    s = block_sum_256(s, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sw2d_hsum_final_kernel(const double* __restrict__ partial, int n,
                                                              PrepFlags* __restrict__ flags) {
    __shared__ double lds[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    s = block_sum_256(s, lds);
    if (threadIdx.x == 0) flags->h_sum = s;
}

// ---------------------------------------------------------------------------------------
// Host-side launchers (called by the C ABI in sw2d_api.hip)

hipError_t launch_step(int kvar, const float* eta, const float* u, const float* v, const float* hp,
                       float* eta_o, float* u_o, float* v_o, FoldPartial* part,
                       const StepGeometry& geo, const StepCoef& k, hipStream_t s) {
    const dim3 grid(geo.nblocks), block(kGroupThreads);
#define SW2D_STEP_CASE(V)                                                                                   \
    case V:                                                                                                 \
        hipLaunchKernelGGL(sw2d_step_kernel<V>, grid, block, 0, s, eta, u, v, hp, eta_o, u_o, v_o, part, geo, k); \
        break;
    switch (kvar) {
        SW2D_STEP_CASE(0)
        SW2D_STEP_CASE(1)
        SW2D_STEP_CASE(2)
        SW2D_STEP_CASE(3)
        SW2D_STEP_CASE(4)
        SW2D_STEP_CASE(5)
        SW2D_STEP_CASE(6)
        SW2D_STEP_CASE(7)
        SW2D_STEP_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef SW2D_STEP_CASE
    return hipGetLastError();
}

hipError_t launch_stepk(int K, int kvar, const float* eta, const float* u, const float* v, const float* hp,
                        float* eta_o, float* u_o, float* v_o, FoldPartial* part, int stride,
                        const StepGeometry& geo, const StepCoef& k, hipStream_t s) {
    const dim3 grid(geo.nblocks), block(kGroupThreads);
    if (kvar != 0) {
        // the variants without advection: the one-column pipeline of their single-step kernel
#define SW2D_VARK_CASE(KK, V)                                                                                    \
    if (K == (KK) && kvar == (V)) {                                                                             \
        hipLaunchKernelGGL((sw2d_stepk_kernel<KK, (V)>), grid, block, 0, s, eta, u, v, hp, eta_o, u_o, v_o, part, \
                           stride, geo, k);                                                                     \
        return hipGetLastError();                                                                               \
    }
        SW2D_VARK_CASE(2, kVarFriction)
        SW2D_VARK_CASE(3, kVarFriction)
        SW2D_VARK_CASE(4, kVarFriction)
        SW2D_VARK_CASE(2, kVarFilterUV)
        SW2D_VARK_CASE(3, kVarFilterUV)
        SW2D_VARK_CASE(4, kVarFilterUV)
        SW2D_VARK_CASE(2, kVarFriction | kVarFilterUV)
        SW2D_VARK_CASE(3, kVarFriction | kVarFilterUV)
        SW2D_VARK_CASE(4, kVarFriction | kVarFilterUV)
        SW2D_VARK_CASE(2, kVarWetDry)
        SW2D_VARK_CASE(3, kVarWetDry)
        SW2D_VARK_CASE(4, kVarWetDry)
#undef SW2D_VARK_CASE
        return hipErrorInvalidValue;
    }
    const bool wide = (geo.nx % 2) == 0;
#define SW2D_PAIR_CASE(KK)                                                                                         \
    case KK:                                                                                                       \
        if (wide)                                                                                                  \
            hipLaunchKernelGGL((sw2d_stepk_pair_kernel<KK, true>), grid, block, 0, s, eta, u, v, hp, eta_o, u_o, v_o, \
                               part, stride, geo, k);                                                              \
        else                                                                                                       \
            hipLaunchKernelGGL((sw2d_stepk_pair_kernel<KK, false>), grid, block, 0, s, eta, u, v, hp, eta_o, u_o,   \
                               v_o, part, stride, geo, k);                                                         \
        break;
    switch (K) {
        SW2D_PAIR_CASE(2)
        SW2D_PAIR_CASE(3)
        SW2D_PAIR_CASE(4)
        default:
            return hipErrorInvalidValue;
    }
#undef SW2D_PAIR_CASE
    return hipGetLastError();
}

hipError_t launch_fold(const FoldPartial* part, int nparts, int stride, int nsteps,
                       int64_t first_step, sw2d_red* ring, int ring_cap, double cell_area,
                       double h_sum, hipStream_t s) {
    hipLaunchKernelGGL(sw2d_fold_kernel, dim3(nsteps), dim3(kFoldThreads), 0, s, part, nparts,
                       stride, first_step, ring, ring_cap, cell_area, h_sum);
    return hipGetLastError();
}

hipError_t launch_prep(const float* H, const uint8_t* mask, const float* eta, const float* u,
                       const float* v, int nx, int ny, float* hp, PrepFlags* flags,
                       double* scratch, hipStream_t s, bool allow_dry) {
    const size_t n = (size_t)nx * ny;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(sw2d_prep_kernel, dim3((unsigned)blocks), dim3(256), 0, s, H, mask, eta, u, v,
                       nx, ny, hp, flags, allow_dry);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int G = ny < kHsumBlocks ? ny : kHsumBlocks;
    hipLaunchKernelGGL(sw2d_hsum_kernel, dim3(G), dim3(256), 0, s, hp, nx, ny, scratch);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sw2d_hsum_final_kernel, dim3(1), dim3(256), 0, s, scratch, G, flags);
    return hipGetLastError();
}

}  // namespace sw2d
