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
// Folds: per-lane FP64 sums and FP32 maxima -> wave butterfly -> workgroup (LDS,
// fixed order) -> one partial per workgroup and step; sw2d_fold_kernel later adds the
// partials of each step in a fixed order, so the folds are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw2d_internal.h"

namespace sw2d {

__device__ __forceinline__ int xcd_contiguous(int b, int n) {
    // Workgroup b is dispatched to XCD b % 8; give each XCD a contiguous range of
    // logical tiles so halo rows and columns shared by neighbours hit the same L2.
    const int q = n / kXcds, r = n % kXcds;
    const int x = b % kXcds, k = b / kXcds;
    return x * q + min(x, r) + k;
}

__device__ __forceinline__ float shfl_from_east(float x) { return __shfl_down(x, 1, kWave); }
__device__ __forceinline__ float shfl_from_west(float x) { return __shfl_up(x, 1, kWave); }

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

// Adds the per-wave partial folds of one workgroup in wave order and writes them.
__device__ __forceinline__ void workgroup_fold(double tot, double disp, float mu, float mv,
                                               FoldPartial* out) {
    __shared__ double s_tot[kWavesPerGroup], s_disp[kWavesPerGroup];
    __shared__ float s_mu[kWavesPerGroup], s_mv[kWavesPerGroup];
    tot = wave_sum(tot);
    disp = wave_sum(disp);
    mu = wave_max(mu);
    mv = wave_max(mv);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) {
        s_tot[wave] = tot;
        s_disp[wave] = disp;
        s_mu[wave] = mu;
        s_mv[wave] = mv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        float c = 0.f, d = 0.f;
#pragma unroll
        for (int w = 0; w < kWavesPerGroup; ++w) {
            a += s_tot[w];
            b += s_disp[w];
            c = fmaxf(c, s_mu[w]);
            d = fmaxf(d, s_mv[w]);
        }
        out->tot = a;
        out->disp = b;
        out->mu = c;
        out->mv = d;
    }
}

__global__ __launch_bounds__(kGroupThreads) void sw2d_step_kernel(
    const float* __restrict__ eta, const float* __restrict__ u, const float* __restrict__ v,
    const float* __restrict__ hp, float* __restrict__ eta_o, float* __restrict__ u_o,
    float* __restrict__ v_o, FoldPartial* __restrict__ part, StepGeometry geo, StepCoef k) {
    const int tile = xcd_contiguous(blockIdx.x, geo.nblocks);
    const int band = tile / geo.groups_x;
    const int group = tile - band * geo.groups_x;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int strip = group * kWavesPerGroup + wave;
    const int nx = geo.nx, ny = geo.ny;
    const int c = strip * kStripOut - kHalo + lane;
    const bool col_in = c >= 0 && c < nx;
    const bool out_lane = col_in && lane >= kHalo && lane < kWave - kHalo;
    const int j0 = band * geo.rows;
    const int j1 = min(j0 + geo.rows, ny);

    double f_tot = 0.0, f_disp = 0.0;
    float f_mu = 0.f, f_mv = 0.f;

    if (strip < geo.strips) {
        auto load = [&](const float* __restrict__ p, int r) -> float {
            return (col_in && r >= 0 && r < ny) ? p[(size_t)r * nx + c] : 0.f;
        };
        // lag 1 (row r-1), lag 2 (row r-2), lag 3 (row r-3) registers of the pipeline
        float e1 = 0.f, h1 = 0.f, hp1 = 0.f, v1 = 0.f, pe1 = 0.f, us1 = 0.f;
        bool w1 = false, wE1 = false, wW1 = false;
        float es2 = 0.f, fy2 = 0.f, vs2 = 0.f, us2 = 0.f, hp2 = 0.f;
        bool w2 = false, wE2 = false, wW2 = false;
        float es3 = 0.f;
        bool w3 = false;

        int r = j0 - 2;
        float e_n = load(eta, r), hp_n = load(hp, r), u_n = load(u, r), v_n = load(v, r);
        for (; r <= j1 + 1; ++r) {
            const float e = e_n, hpr = hp_n, ur = u_n, vr = v_n;
            if (r + 1 <= j1 + 1) {
                e_n = load(eta, r + 1);
                hp_n = load(hp, r + 1);
                u_n = load(u, r + 1);
                v_n = load(v, r + 1);
            }
            // row r: x-face predictor and flux (dyn), partial surface update
            const bool w = hpr > 0.f;
            const float h = hpr + e;
            const float eE = shfl_from_east(e);
            const float hpE = shfl_from_east(hpr);
            const float hpW = shfl_from_west(hpr);
            const bool wE = hpE > 0.f, wW = hpW > 0.f;
            const bool au = w && wE;
            const float us = au ? ur - k.cx * (eE - e) : 0.f;
            const float fx = au ? us * (us > 0.f ? h : hpE + eE) : 0.f;
            const float fxW = shfl_from_west(fx);
            const float pe = e - k.rx * (fx - fxW);
            // row r-1: y-face predictor and flux, predicted surface es
            const bool av = w1 && w;
            const float vs = av ? v1 - k.cy * (e - e1) : 0.f;
            const float fy = av ? vs * (vs > 0.f ? h1 : h) : 0.f;
            const float es = w1 ? pe1 - k.ry * (fy - fy2) : 0.f;
            // row r-2: first-order Shapiro filter across water neighbours
            const float esE = shfl_from_east(es2);
            const float esW = shfl_from_west(es2);
            float s = 0.f;
            if (wE2) s += esE - es2;
            if (wW2) s += esW - es2;
            if (w1) s += es - es2;
            if (w3) s += es3 - es2;
            const float eta_new = w2 ? es2 + k.e4 * s : 0.f;

            const int q = r - 2;
            if (q >= j0 && out_lane) {
                const size_t o = (size_t)q * nx + c;
                eta_o[o] = eta_new;
                u_o[o] = us2;
                v_o[o] = vs2;
                if (w2) {
                    f_disp += (double)eta_new;
                    f_tot += (double)hp2 + (double)eta_new;
                }
                f_mu = fmaxf(f_mu, fabsf(us2));
                f_mv = fmaxf(f_mv, fabsf(vs2));
            }
            // advance the pipeline
            es3 = es2;
            w3 = w2;
            es2 = es;
            fy2 = fy;
            vs2 = vs;
            us2 = us1;
            hp2 = hp1;
            w2 = w1;
            wE2 = wE1;
            wW2 = wW1;
            e1 = e;
            h1 = h;
            hp1 = hpr;
            v1 = vr;
            pe1 = pe;
            us1 = us;
            w1 = w;
            wE1 = wE;
            wW1 = wW;
        }
    }
    workgroup_fold(f_tot, f_disp, f_mu, f_mv, part + blockIdx.x);
}

// Final level of the folds: one workgroup per step adds that step's partials in a
// fixed order and writes the ring entry.
__global__ __launch_bounds__(kFoldThreads) void sw2d_fold_kernel(const FoldPartial* __restrict__ part,
                                                                 int nparts, int stride,
                                                                 int64_t first_step,
                                                                 sw2d_red* __restrict__ ring,
                                                                 int ring_cap, double cell_area) {
    __shared__ double s_tot[kFoldThreads], s_disp[kFoldThreads];
    __shared__ float s_mu[kFoldThreads], s_mv[kFoldThreads];
    const FoldPartial* p = part + (size_t)blockIdx.x * stride;
    double tot = 0.0, disp = 0.0;
    float mu = 0.f, mv = 0.f;
    for (int i = threadIdx.x; i < nparts; i += kFoldThreads) {
        tot += p[i].tot;
        disp += p[i].disp;
        mu = fmaxf(mu, p[i].mu);
        mv = fmaxf(mv, p[i].mv);
    }
    const int t = threadIdx.x;
    s_tot[t] = tot;
    s_disp[t] = disp;
    s_mu[t] = mu;
    s_mv[t] = mv;
    __syncthreads();
    for (int half = kFoldThreads / 2; half > 0; half >>= 1) {
        if (t < half) {
            s_tot[t] += s_tot[t + half];
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
        o->vol_total = cell_area * s_tot[0];
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
                       hipStream_t s) {
    hipLaunchKernelGGL(sw2d_fold_kernel, dim3(nsteps), dim3(kFoldThreads), 0, s, part, nparts,
                       stride, first_step, ring, ring_cap, cell_area);
    return hipGetLastError();
}

hipError_t launch_prep(const float* H, const uint8_t* mask, const float* eta, const float* u,
                       const float* v, int nx, int ny, float* hp, PrepFlags* flags, hipStream_t s) {
    const size_t n = (size_t)nx * ny;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(sw2d_prep_kernel, dim3((unsigned)blocks), dim3(256), 0, s, H, mask, eta, u, v,
                       nx, ny, hp, flags);
    return hipGetLastError();
}

}  // namespace sw2d
