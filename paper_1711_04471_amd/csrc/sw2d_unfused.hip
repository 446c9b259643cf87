// sw2d_unfused.hip - the step split the way the paper's compiler splits it (Sect. 6.2:
// three map kernels: the predictor "dyn", the Shapiro filter, the velocity update), plus the
// folds as a separate reduction, kept as an in-repository comparison for the fused pass.
//
// dyn writes the predicted face velocities and the predicted surface to scratch arrays,
// shapiro reads the predicted surface and writes the new surface, update copies the
// predicted velocities into the new state, and the fold kernel reads the new state again:
// 16 + 12, 8 + 4, 8 + 8 and 12 bytes per cell, 68 B per cell-step against the fused 28 B.
// Same arithmetic per cell as the fused pass (the state agrees to FP32 rounding).
#include <hip/hip_runtime.h>

#include "sw2d_internal.h"

namespace sw2d {

namespace {

constexpr int kTX = 64, kTY = 4;

__device__ __forceinline__ float at(const float* __restrict__ a, int nx, int ny, int j, int i) {
    return (i >= 0 && j >= 0 && i < nx && j < ny) ? a[(size_t)j * nx + i] : 0.f;
}

// x-face between (j,i) and (j,i+1): predicted velocity and upwind flux
__device__ __forceinline__ void xface(const float* __restrict__ eta, const float* __restrict__ u,
                                      const float* __restrict__ hp, int nx, int ny, int j, int i,
                                      const StepCoef& k, float& us, float& fx) {
    const float e = at(eta, nx, ny, j, i), eE = at(eta, nx, ny, j, i + 1);
    const float h = at(hp, nx, ny, j, i), hE = at(hp, nx, ny, j, i + 1);
    const bool au = h > 0.f && hE > 0.f;
    us = au ? at(u, nx, ny, j, i) - k.cx * (eE - e) : 0.f;
    fx = au ? us * (us > 0.f ? h + e : hE + eE) : 0.f;
}

__device__ __forceinline__ void yface(const float* __restrict__ eta, const float* __restrict__ v,
                                      const float* __restrict__ hp, int nx, int ny, int j, int i,
                                      const StepCoef& k, float& vs, float& fy) {
    const float e = at(eta, nx, ny, j, i), eN = at(eta, nx, ny, j + 1, i);
    const float h = at(hp, nx, ny, j, i), hN = at(hp, nx, ny, j + 1, i);
    const bool av = h > 0.f && hN > 0.f;
    vs = av ? at(v, nx, ny, j, i) - k.cy * (eN - e) : 0.f;
    fy = av ? vs * (vs > 0.f ? h + e : hN + eN) : 0.f;
}

__global__ __launch_bounds__(kTX* kTY) void dyn_kernel(const float* __restrict__ eta, const float* __restrict__ u,
                                                      const float* __restrict__ v, const float* __restrict__ hp,
                                                      int nx, int ny, StepCoef k, float* __restrict__ us_o,
                                                      float* __restrict__ vs_o, float* __restrict__ es_o) {
    const int i = blockIdx.x * kTX + threadIdx.x, j = blockIdx.y * kTY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    float us, fx, usW, fxW, vs, fy, vsS, fyS;
    xface(eta, u, hp, nx, ny, j, i, k, us, fx);
    xface(eta, u, hp, nx, ny, j, i - 1, k, usW, fxW);
    yface(eta, v, hp, nx, ny, j, i, k, vs, fy);
    yface(eta, v, hp, nx, ny, j - 1, i, k, vsS, fyS);
    const size_t o = (size_t)j * nx + i;
    const float e = eta[o];
    us_o[o] = us;
    vs_o[o] = vs;
    es_o[o] = hp[o] > 0.f ? (e - k.rx * (fx - fxW)) - k.ry * (fy - fyS) : 0.f;
}

__global__ __launch_bounds__(kTX* kTY) void shapiro_kernel(const float* __restrict__ es, const float* __restrict__ hp,
                                                          int nx, int ny, float e4, float* __restrict__ eta_o) {
    const int i = blockIdx.x * kTX + threadIdx.x, j = blockIdx.y * kTY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const size_t o = (size_t)j * nx + i;
    const float c = es[o];
    float s = 0.f;
    if (at(hp, nx, ny, j, i + 1) > 0.f) s += at(es, nx, ny, j, i + 1) - c;
    if (at(hp, nx, ny, j, i - 1) > 0.f) s += at(es, nx, ny, j, i - 1) - c;
    if (at(hp, nx, ny, j + 1, i) > 0.f) s += at(es, nx, ny, j + 1, i) - c;
    if (at(hp, nx, ny, j - 1, i) > 0.f) s += at(es, nx, ny, j - 1, i) - c;
    eta_o[o] = hp[o] > 0.f ? c + e4 * s : 0.f;
}

__global__ __launch_bounds__(256) void update_kernel(const float* __restrict__ us, const float* __restrict__ vs,
                                                     size_t n, float* __restrict__ u_o, float* __restrict__ v_o) {
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (size_t)gridDim.x * 256) {
        u_o[p] = us[p];
        v_o[p] = vs[p];
    }
}

__global__ __launch_bounds__(256) void fold_state_kernel(const float* __restrict__ eta, const float* __restrict__ u,
                                                         const float* __restrict__ v, size_t n,
                                                         FoldPartial* __restrict__ part) {
    __shared__ double sd[256];
    __shared__ float su[256], sv[256];
    double d = 0.0;
    float mu = 0.f, mv = 0.f;
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (size_t)gridDim.x * 256) {
        d += (double)eta[p];  // zero on land
        mu = fmaxf(mu, fabsf(u[p]));
        mv = fmaxf(mv, fabsf(v[p]));
    }
    const int t = threadIdx.x;
    sd[t] = d;
    su[t] = mu;
    sv[t] = mv;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            sd[t] += sd[t + h];
            su[t] = fmaxf(su[t], su[t + h]);
            sv[t] = fmaxf(sv[t], sv[t + h]);
        }
        __syncthreads();
    }
    if (t == 0) {
        part[blockIdx.x].disp = sd[0];
        part[blockIdx.x].mu = su[0];
        part[blockIdx.x].mv = sv[0];
    }
}

}  // namespace

hipError_t launch_unfused_step(const float* eta, const float* u, const float* v, const float* hp, float* eta_o,
                               float* u_o, float* v_o, float* scratch, int nx, int ny, const StepCoef& k,
                               FoldPartial* part, int nparts, hipStream_t s) {
    const size_t n = (size_t)nx * ny;
    float* us = scratch;
    float* vs = scratch + n;
    float* es = scratch + 2 * n;
    const dim3 grid((nx + kTX - 1) / kTX, (ny + kTY - 1) / kTY), block(kTX, kTY);
    hipLaunchKernelGGL(dyn_kernel, grid, block, 0, s, eta, u, v, hp, nx, ny, k, us, vs, es);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(shapiro_kernel, grid, block, 0, s, es, hp, nx, ny, k.e4, eta_o);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(update_kernel, dim3((unsigned)blocks), dim3(256), 0, s, us, vs, n, u_o, v_o);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fold_state_kernel, dim3(nparts), dim3(256), 0, s, eta_o, u_o, v_o, n, part);
    return hipGetLastError();
}

}  // namespace sw2d
