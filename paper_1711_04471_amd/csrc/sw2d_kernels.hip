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
//
// Compile-time options (defaults are the tuned choice):
//   SW2D_PREFETCH  rows loaded ahead of the one being processed (1 or 2)
//   SW2D_DPP       1: neighbour exchange with wave-wide DPP row shifts, 0: ds_bpermute
//   SW2D_NT_STORE  1: non-temporal stores of the new state
//   SW2D_XCD_MAP   1: XCD-contiguous workgroup -> tile mapping
//   SW2D_ZIGZAG    1: odd bands march south (band-boundary rows are re-read from L2)
//   SW2D_BAND_BLOCK vertically adjacent bands dispatched back to back (1 = plain
//                  row-major tile order)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw2d_internal.h"

namespace sw2d {

#ifndef SW2D_PREFETCH
#define SW2D_PREFETCH 1
#endif
#ifndef SW2D_DPP
#define SW2D_DPP 1
#endif
#ifndef SW2D_NT_STORE
#define SW2D_NT_STORE 0
#endif
#ifndef SW2D_XCD_MAP
#define SW2D_XCD_MAP 1
#endif
#ifndef SW2D_ZIGZAG
#define SW2D_ZIGZAG 1
#endif
#ifndef SW2D_BAND_BLOCK
#define SW2D_BAND_BLOCK 2
#endif
static_assert(SW2D_PREFETCH >= 1 && SW2D_PREFETCH <= 4, "prefetch depth");

__device__ __forceinline__ int tile_of_block(int b, int n) {
#if SW2D_XCD_MAP
    // Workgroup b is dispatched to XCD b % 8; give each XCD a contiguous range of
    // logical tiles so halo rows and columns shared by neighbours hit the same L2.
    const int q = n / kXcds, r = n % kXcds;
    const int x = b % kXcds, k = b / kXcds;
    return x * q + min(x, r) + k;
#else
    (void)n;
    return b;
#endif
}

// Lane l receives lane l+1's value (its east neighbour); lane 63 receives 0.
__device__ __forceinline__ float from_east(float x) {
#if SW2D_DPP
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130 /* wave_shl:1 */,
                                                      0xf, 0xf, false));
#else
    return __shfl_down(x, 1, kWave);
#endif
}

// Lane l receives lane l-1's value (its west neighbour); lane 0 receives 0.
__device__ __forceinline__ float from_west(float x) {
#if SW2D_DPP
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138 /* wave_shr:1 */,
                                                      0xf, 0xf, false));
#else
    return __shfl_up(x, 1, kWave);
#endif
}

__device__ __forceinline__ void store(float* p, float x) {
#if SW2D_NT_STORE
    __builtin_nontemporal_store(x, p);
#else
    *p = x;
#endif
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

// Row r of the march: water flags, total depth, x-face predictor and flux, and the
// x-part of the surface update (pe = eta - dt/dx (Fx - Fx_W)).
struct RowX {
    float e, h, pe, us;
    bool w, wE, wW;
};

__device__ __forceinline__ RowX row_x(float e, float hpr, float ur, const StepCoef& k) {
    RowX o;
    o.e = e;
    o.w = hpr > 0.f;
    o.h = hpr + e;
    const float eE = from_east(e);
    const float hpE = from_east(hpr);
    const float hpW = from_west(hpr);
    o.wE = hpE > 0.f;
    o.wW = hpW > 0.f;
    const bool au = o.w && o.wE;
    o.us = au ? ur - k.cx * (eE - e) : 0.f;
    const float fx = au ? o.us * (o.us > 0.f ? o.h : hpE + eE) : 0.f;
    const float fxW = from_west(fx);
    o.pe = e - k.rx * (fx - fxW);
    return o;
}

// The y-face between a southern cell (lo) and its northern neighbour (hi).
__device__ __forceinline__ void face_y(float v_lo, float e_lo, float h_lo, bool w_lo, float e_hi,
                                       float h_hi, bool w_hi, const StepCoef& k, float& vs, float& fy) {
    const bool av = w_lo && w_hi;
    vs = av ? v_lo - k.cy * (e_hi - e_lo) : 0.f;
    fy = av ? vs * (vs > 0.f ? h_lo : h_hi) : 0.f;
}

// First-order Shapiro filter of the predicted surface es_c across water neighbours
// (east, west, north, south, always added in that order).
__device__ __forceinline__ float shapiro(float es_c, bool w_c, bool wE, bool wW, float es_n, bool w_n,
                                         float es_s, bool w_s, float e4) {
    const float esE = from_east(es_c);
    const float esW = from_west(es_c);
    float s = 0.f;
    if (wE) s += esE - es_c;
    if (wW) s += esW - es_c;
    if (w_n) s += es_n - es_c;
    if (w_s) s += es_s - es_c;
    return w_c ? es_c + e4 * s : 0.f;
}

// One wave marches a band [j0, j1) of its strip, north (kNorth) or south, and writes
// the new state of its output lanes. Every output value is the same expression in
// either direction; only the order of the per-lane fold additions differs.
template <bool kNorth>
__device__ __forceinline__ void march(const float* __restrict__ eta, const float* __restrict__ u,
                                      const float* __restrict__ v, const float* __restrict__ hp,
                                      float* __restrict__ eta_o, float* __restrict__ u_o,
                                      float* __restrict__ v_o, int nx, int ny, int c, bool col_in,
                                      bool out_lane, int j0, int j1, const StepCoef& k,
                                      double& f_disp, float& f_mu, float& f_mv) {
    auto load = [&](const float* __restrict__ p, int r) -> float {
        return (col_in && r >= 0 && r < ny) ? p[(size_t)r * nx + c] : 0.f;
    };
    auto emit = [&](int q, float eta_new, float us_q, float vs_q) {
        if (out_lane) {
            const size_t o = (size_t)q * nx + c;
            store(eta_o + o, eta_new);
            store(u_o + o, us_q);
            store(v_o + o, vs_q);
            f_disp += (double)eta_new;  // zero on land
            f_mu = fmaxf(f_mu, fabsf(us_q));
            f_mv = fmaxf(f_mv, fabsf(vs_q));
        }
    };
    constexpr int step = kNorth ? 1 : -1;
    const int r_first = kNorth ? j0 - 2 : j1 + 1;
    const int n_rows = j1 - j0 + 4;

    // registers of the rows 1, 2 and 3 behind the one being loaded (in march order)
    float e1 = 0.f, h1 = 0.f, v1 = 0.f, pe1 = 0.f, us1 = 0.f, fy1 = 0.f, vs1 = 0.f;
    bool w1 = false, wE1 = false, wW1 = false;
    float es2 = 0.f, fy2 = 0.f, vs2 = 0.f, us2 = 0.f;
    bool w2 = false, wE2 = false, wW2 = false;
    float es3 = 0.f;
    bool w3 = false;

    float qe[SW2D_PREFETCH], qh[SW2D_PREFETCH], qu[SW2D_PREFETCH], qv[SW2D_PREFETCH];
#pragma unroll
    for (int d = 0; d < SW2D_PREFETCH; ++d) {
        const int rr = r_first + d * step;
        const bool ok = d < n_rows;
        qe[d] = ok ? load(eta, rr) : 0.f;
        qh[d] = ok ? load(hp, rr) : 0.f;
        qu[d] = ok ? load(u, rr) : 0.f;
        qv[d] = ok ? load(v, rr) : 0.f;
    }
    for (int i = 0; i < n_rows; ++i) {
        const int r = r_first + i * step;
        const float e = qe[0], hpr = qh[0], ur = qu[0], vr = qv[0];
#pragma unroll
        for (int d = 0; d + 1 < SW2D_PREFETCH; ++d) {
            qe[d] = qe[d + 1];
            qh[d] = qh[d + 1];
            qu[d] = qu[d + 1];
            qv[d] = qv[d + 1];
        }
        if (i + SW2D_PREFETCH < n_rows) {
            const int rr = r + SW2D_PREFETCH * step;
            qe[SW2D_PREFETCH - 1] = load(eta, rr);
            qh[SW2D_PREFETCH - 1] = load(hp, rr);
            qu[SW2D_PREFETCH - 1] = load(u, rr);
            qv[SW2D_PREFETCH - 1] = load(v, rr);
        }
        const RowX X = row_x(e, hpr, ur, k);
        if constexpr (kNorth) {
            // y-face between rows r-1 and r, then es of row r-1, then the output row r-2
            float vs, fy;
            face_y(v1, e1, h1, w1, X.e, X.h, X.w, k, vs, fy);
            const float es = w1 ? pe1 - k.ry * (fy - fy2) : 0.f;
            const float eta_new = shapiro(es2, w2, wE2, wW2, es, w1, es3, w3, k.e4);
            if (i >= 4) emit(r - 2, eta_new, us2, vs2);
            es3 = es2;
            w3 = w2;
            es2 = es;
            fy2 = fy;
            vs2 = vs;
            us2 = us1;
            w2 = w1;
            wE2 = wE1;
            wW2 = wW1;
            v1 = vr;
        } else {
            // y-face between rows r and r+1, then es of row r+1, then the output row r+2
            float vs, fy;
            face_y(vr, X.e, X.h, X.w, e1, h1, w1, k, vs, fy);
            const float es = w1 ? pe1 - k.ry * (fy1 - fy) : 0.f;
            const float eta_new = shapiro(es2, w2, wE2, wW2, es3, w3, es, w1, k.e4);
            if (i >= 4) emit(r + 2, eta_new, us2, vs2);
            es3 = es2;
            w3 = w2;
            es2 = es;
            us2 = us1;
            vs2 = vs1;
            w2 = w1;
            wE2 = wE1;
            wW2 = wW1;
            fy1 = fy;
            vs1 = vs;
        }
        e1 = X.e;
        h1 = X.h;
        pe1 = X.pe;
        us1 = X.us;
        w1 = X.w;
        wE1 = X.wE;
        wW1 = X.wW;
    }
}

__global__ __launch_bounds__(kGroupThreads) void sw2d_step_kernel(
    const float* __restrict__ eta, const float* __restrict__ u, const float* __restrict__ v,
    const float* __restrict__ hp, float* __restrict__ eta_o, float* __restrict__ u_o,
    float* __restrict__ v_o, FoldPartial* __restrict__ part, StepGeometry geo, StepCoef k) {
    const int tile = tile_of_block(blockIdx.x, geo.nblocks);
#if SW2D_BAND_BLOCK > 1
    // blocks of SW2D_BAND_BLOCK vertically adjacent bands are dispatched together
    const int per_block = geo.groups_x * SW2D_BAND_BLOCK;
    const int blk = tile / per_block;
    const int rem = tile - blk * per_block;
    const int nb = min(SW2D_BAND_BLOCK, geo.bands - blk * SW2D_BAND_BLOCK);
    const int group = rem / nb;
    const int band = blk * SW2D_BAND_BLOCK + (rem - group * nb);
#else
    const int band = tile / geo.groups_x;
    const int group = tile - band * geo.groups_x;
#endif
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int strip = group * kWavesPerGroup + wave;
    const int c = strip * kStripOut - kHalo + lane;
    const bool col_in = c >= 0 && c < geo.nx;
    const bool out_lane = col_in && lane >= kHalo && lane < kWave - kHalo;
    const int j0 = band * geo.rows;
    const int j1 = min(j0 + geo.rows, geo.ny);

    double f_disp = 0.0;
    float f_mu = 0.f, f_mv = 0.f;
    if (strip < geo.strips) {
#if SW2D_ZIGZAG
        // Odd bands march south, so each band boundary is read by both of its bands at
        // the same moment (both at their start or both at their end) and the second
        // read hits L2 instead of HBM.
        if (band & 1)
            march<false>(eta, u, v, hp, eta_o, u_o, v_o, geo.nx, geo.ny, c, col_in, out_lane, j0, j1,
                         k, f_disp, f_mu, f_mv);
        else
#endif
            march<true>(eta, u, v, hp, eta_o, u_o, v_o, geo.nx, geo.ny, c, col_in, out_lane, j0, j1,
                        k, f_disp, f_mu, f_mv);
    }
    workgroup_fold(f_disp, f_mu, f_mv, part + blockIdx.x);
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
// depth field (hp = wet ? H : 0, so wet == hp > 0) and find the deepest water cell.
__global__ __launch_bounds__(256) void sw2d_prep_kernel(const float* __restrict__ H,
                                                        const uint8_t* __restrict__ mask,
                                                        const float* __restrict__ eta,
                                                        const float* __restrict__ u,
                                                        const float* __restrict__ v, int nx, int ny,
                                                        float* __restrict__ hp,
                                                        PrepFlags* __restrict__ flags) {
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
                if (!(d + e > 0.f)) bad |= kDryCell;
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

hipError_t launch_step(const float* eta, const float* u, const float* v, const float* hp,
                       float* eta_o, float* u_o, float* v_o, FoldPartial* part,
                       const StepGeometry& geo, const StepCoef& k, hipStream_t s) {
    hipLaunchKernelGGL(sw2d_step_kernel, dim3(geo.nblocks), dim3(kGroupThreads), 0, s, eta, u, v, hp,
                       eta_o, u_o, v_o, part, geo, k);
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
                       double* scratch, hipStream_t s) {
    const size_t n = (size_t)nx * ny;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(sw2d_prep_kernel, dim3((unsigned)blocks), dim3(256), 0, s, H, mask, eta, u, v,
                       nx, ny, hp, flags);
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
