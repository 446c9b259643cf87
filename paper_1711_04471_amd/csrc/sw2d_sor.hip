// sw2d_sor.hip - red-black successive over-relaxation for the pressure Poisson equation of
// the paper's second workload (Sect. 6.3: SOR takes most of its GPU time), with the residual
// of every iteration folded on the device.
//
// Arrays [nz][ny][nx] FP32; the outermost layer holds fixed (Dirichlet) values. One
// iteration = a sweep over the red cells ((i + j + k) even), then over the black ones; a
// cell becomes p + omega (g - p), g = (cx (pE + pW) + cy (pN + pS) + cz (pU + pD) - f) / d,
// d = 2 (cx + cy + cz), c_ = 1 / spacing^2.
//
// Layout: the solver works on the two colours stored apart (red and black arrays of
// [nz][ny][w] with w = ceil(nx / 2); cell (i, j, k) lives in its colour's array at i / 2), so a
// sweep reads one whole array of its own colour, the other colour's array and its own half of
// f, and writes its own array - 16 B per cell and iteration, no half-used cache lines. The
// split and the merge back to [nz][ny][nx] are one pass each per solve. A sweep thread owns one
// position of its colour per plane (threads run along the rows of a plane, so they coalesce
// across row ends) and walks kSorPlanes planes. The residual r = f - L p of
// the state after iteration m is folded without an extra pass: a black cell's neighbours
// are all red, so the black sweep of iteration m knows its residual right after the update;
// a red cell's residual needs the black values of iteration m, which the red sweep of
// iteration m + 1 reads before it overwrites the red cell. One residual-only pass per colour
// covers the initial black cells and the final red cells. Workgroup partials (FP64 sum of
// r^2, max |r| as magnitude bits) are added per iteration in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "sw2d_internal.h"

namespace sw2d {
namespace {

#ifndef SW2D_SOR_PLANES
#define SW2D_SOR_PLANES 8
#endif
#ifndef SW2D_SOR_THREADS
#define SW2D_SOR_THREADS 512
#endif
constexpr int kSorThreads = SW2D_SOR_THREADS, kSorPlanes = SW2D_SOR_PLANES;
constexpr int kSorFoldThreads = 256;
enum SorMode { kSorUpdate = 0, kSorResidualOnly = 1 };

struct SorCoef {
    float cx, cy, cz, diag, inv_diag, omega;
};

struct alignas(16) SorPartial {
    double sum_r2;
    unsigned max_bits;
    unsigned pad;
};

struct SorGeometry {
    int nx, ny, nz, w, rows_q, gx, gz, nblocks;  // w = ceil(nx / 2); rows_q = (ny - 2) w
};

SorGeometry sor_geometry(int nx, int ny, int nz) {
    SorGeometry g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.w = (nx + 1) / 2;
    g.rows_q = (ny - 2) * g.w;
    g.gx = (g.rows_q + kSorThreads - 1) / kSorThreads;
    g.gz = (nz - 2 + kSorPlanes - 1) / kSorPlanes;
    g.nblocks = g.gx * g.gz;
    return g;
}

// [nz][ny][nx] -> the two colour arrays (dir = 0), or back (dir = 1)
__global__ __launch_bounds__(256) void sor_split_kernel(float* __restrict__ nat, float* __restrict__ red,
                                                        float* __restrict__ black, SorGeometry g, int dir) {
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
        const int i = (int)(q % g.nx);
        const size_t jk = q / g.nx;  // = k ny + j
        const int j = (int)(jk % g.ny), k = (int)(jk / g.ny);
        float* arr = ((i + j + k) & 1) ? black : red;
        const size_t o = jk * g.w + (i >> 1);
        if (dir == 0)
            arr[o] = nat[q];
        else
            nat[q] = arr[o];
    }
}

template <int COLOR, int MODE>
__global__ __launch_bounds__(kSorThreads) void sor_sweep_kernel(float* __restrict__ own,
                                                                const float* __restrict__ other,
                                                                const float* __restrict__ f_own, SorGeometry geo,
                                                                SorCoef c, SorPartial* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double s_sum[kSorThreads];
    __shared__ unsigned s_max[kSorThreads];
    const int nx = geo.nx, ny = geo.ny, nz = geo.nz, w = geo.w;
    const int q = blockIdx.x * kSorThreads + threadIdx.x;
    const int jj = q / w;
    const int m = q - jj * w;
    const int j = 1 + jj;
    const bool row_ok = q < geo.rows_q;
    const int k0 = 1 + blockIdx.y * kSorPlanes;
    const size_t plane = (size_t)ny * w;
    double acc = 0.0;
    unsigned mx = 0u;
    // The thread walks the planes at one position m of the other colour's array: its z
    // neighbours are that array's values at m one plane down and up, and one of its x
    // neighbours in a plane is the value at m itself, so each plane loads the upper z value
    // and the outer x value only and passes the rest on.
    const size_t o_m0 = ((size_t)k0 * ny + (row_ok ? j : 1)) * w + m;
    float zd = 0.f, xm = 0.f;
    if (row_ok && k0 <= nz - 2) {
        zd = other[o_m0 - plane];
        xm = other[o_m0];
    }
    for (int kk = 0; kk < kSorPlanes; ++kk) {
        const int k = k0 + kk;
        if (k > nz - 2 || !row_ok) break;
        const size_t o = o_m0 + (size_t)kk * plane;
        const float zu = other[o + plane];
        const int s = (COLOR + j + k) & 1;  // i = s + 2 m has the sweep's colour
        const int i = s + 2 * m;
        if (i >= 1 && i <= nx - 2) {
            const float xo = s ? other[o + 1] : other[o - 1];  // the outer x neighbour
            const float pE = s ? xo : xm, pW = s ? xm : xo;
            const float pc = own[o];
            const float fc = f_own[o];
            const float sx = pE + pW;
            const float sy = other[o + w] + other[o - w];
            const float sz = zu + zd;
            const float nb = fmaf(c.cz, sz, fmaf(c.cy, sy, c.cx * sx));
            float r = 0.f;
            if constexpr (MODE == kSorResidualOnly || COLOR == 0) r = fc - fmaf(-c.diag, pc, nb);
            if constexpr (MODE == kSorUpdate) {
                const float g = (nb - fc) * c.inv_diag;
                const float pn = fmaf(c.omega, g - pc, pc);
                own[o] = pn;
                if constexpr (COLOR == 1) r = fc - fmaf(-c.diag, pn, nb);
            }
            acc += (double)r * (double)r;
            mx = max(mx, __float_as_uint(r) & 0x7fffffffu);
        }
        zd = xm;
        xm = zu;
    }
    // fixed-order tree over the workgroup
    const int t = threadIdx.x;
    s_sum[t] = acc;
    s_max[t] = mx;
    __syncthreads();
    for (int h = kSorThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            s_sum[t] += s_sum[t + h];
            s_max[t] = max(s_max[t], s_max[t + h]);
        }
        __syncthreads();
    }
    if (t == 0) {
        const int b = blockIdx.y * gridDim.x + blockIdx.x;
        part[b].sum_r2 = s_sum[0];
        part[b].max_bits = s_max[0];
        part[b].pad = 0u;
    }
}

// Residual of state m = red partials of slot m + black partials of slot m, each added in
// block order by a fixed tree; one workgroup per m.
__global__ __launch_bounds__(kSorFoldThreads) void sor_fold_kernel(const SorPartial* __restrict__ red,
                                                                   const SorPartial* __restrict__ black,
                                                                   int nblocks, sw2d_sor_res* __restrict__ out) {
    __shared__ double s_sum[kSorFoldThreads];
    __shared__ unsigned s_max[kSorFoldThreads];
    const int m = blockIdx.x, t = threadIdx.x;
    const SorPartial* slots[2] = {red + (size_t)m * nblocks, black + (size_t)m * nblocks};
    double acc = 0.0;
    unsigned mx = 0u;
    for (int c = 0; c < 2; ++c)
        for (int b = t; b < nblocks; b += kSorFoldThreads) {
            acc += slots[c][b].sum_r2;
            mx = max(mx, slots[c][b].max_bits);
        }
    s_sum[t] = acc;
    s_max[t] = mx;
    __syncthreads();
    for (int h = kSorFoldThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            s_sum[t] += s_sum[t + h];
            s_max[t] = max(s_max[t], s_max[t + h]);
        }
        __syncthreads();
    }
    if (t == 0) {
        out[m].iter = m;
        out[m].max_abs_r = __uint_as_float(s_max[0]);
        out[m].sum_r2 = s_sum[0];
    }
}

thread_local char g_sor_msg[256] = "";

int sor_fail(hipError_t e, const char* what) {
    if (e == hipSuccess) return SW2D_OK;
    std::snprintf(g_sor_msg, sizeof g_sor_msg, "%s: %s", what, hipGetErrorString(e));
    detail::set_hip_message(g_sor_msg);
    return SW2D_EHIP;
}

bool sor_params_ok(const sw2d_sor_params* p) {
    if (!p) return false;
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return false;
    if ((int64_t)p->nx * p->ny * p->nz >= ((int64_t)1 << 31)) return false;
    for (double h : {p->dx, p->dy, p->dz})
        if (!(h > 0.0) || !std::isfinite(h)) return false;
    return p->omega > 0.0 && p->omega < 2.0;
}

template <int COLOR, int MODE>
hipError_t launch_sweep(float* own, const float* other, const float* f_own, const SorGeometry& g, const SorCoef& c,
                        SorPartial* part, hipStream_t s) {
    hipLaunchKernelGGL((sor_sweep_kernel<COLOR, MODE>), dim3(g.gx, g.gz), dim3(kSorThreads), 0, s, own, other, f_own,
                       g, c, part);
    return hipGetLastError();
}

hipError_t launch_split(float* nat, float* red, float* black, const SorGeometry& g, int dir, hipStream_t s) {
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(sor_split_kernel, dim3((unsigned)blocks), dim3(256), 0, s, nat, red, black, g, dir);
    return hipGetLastError();
}

size_t colour_floats(const SorGeometry& g) { return (size_t)g.nz * g.ny * g.w; }

}  // namespace
}  // namespace sw2d

using namespace sw2d;

extern "C" {

size_t sw2d_sor_workspace_bytes(const sw2d_sor_params* p, int32_t iters) {
    if (!sor_params_ok(p) || iters < 0) return 0;
    const SorGeometry g = sor_geometry(p->nx, p->ny, p->nz);
    // red, black, f red, f black (16 B aligned each), then the residual partials
    const size_t arr = (colour_floats(g) * sizeof(float) + 255) / 256 * 256;
    return 4 * arr + 2 * (size_t)(iters + 1) * g.nblocks * sizeof(SorPartial);
}

int sw2d_sor_run(const sw2d_sor_params* p, float* d_p, const float* d_f, int32_t iters, sw2d_sor_res* d_res,
                 void* d_work, size_t work_bytes, void* stream) {
    if (!sor_params_ok(p) || !d_p || !d_f || iters < 0 || !d_work) return SW2D_EINVAL;
    if (work_bytes < sw2d_sor_workspace_bytes(p, iters)) return SW2D_ENOSPC;
    const SorGeometry g = sor_geometry(p->nx, p->ny, p->nz);
    SorCoef c;
    const double cx = 1.0 / (p->dx * p->dx), cy = 1.0 / (p->dy * p->dy), cz = 1.0 / (p->dz * p->dz);
    c.cx = (float)cx;
    c.cy = (float)cy;
    c.cz = (float)cz;
    c.diag = (float)(2.0 * (cx + cy + cz));
    c.inv_diag = (float)(1.0 / (2.0 * (cx + cy + cz)));
    c.omega = (float)p->omega;
    const size_t arr = (colour_floats(g) * sizeof(float) + 255) / 256 * 256;
    char* base = static_cast<char*>(d_work);
    float* R = reinterpret_cast<float*>(base);
    float* B = reinterpret_cast<float*>(base + arr);
    float* FR = reinterpret_cast<float*>(base + 2 * arr);
    float* FB = reinterpret_cast<float*>(base + 3 * arr);
    auto* red = reinterpret_cast<SorPartial*>(base + 4 * arr);
    SorPartial* black = red + (size_t)(iters + 1) * g.nblocks;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_split(d_p, R, B, g, 0, s);
    if (e == hipSuccess) e = launch_split(const_cast<float*>(d_f), FR, FB, g, 0, s);  // read only (dir 0)
    if (e == hipSuccess) e = launch_sweep<1, kSorResidualOnly>(B, R, FB, g, c, black, s);  // black part of state 0
    for (int32_t n = 0; n < iters && e == hipSuccess; ++n) {
        e = launch_sweep<0, kSorUpdate>(R, B, FR, g, c, red + (size_t)n * g.nblocks, s);
        if (e == hipSuccess) e = launch_sweep<1, kSorUpdate>(B, R, FB, g, c, black + (size_t)(n + 1) * g.nblocks, s);
    }
    if (e == hipSuccess) e = launch_sweep<0, kSorResidualOnly>(R, B, FR, g, c, red + (size_t)iters * g.nblocks, s);
    if (e == hipSuccess) e = launch_split(d_p, R, B, g, 1, s);
    if (e == hipSuccess && d_res) {
        hipLaunchKernelGGL(sor_fold_kernel, dim3(iters + 1), dim3(kSorFoldThreads), 0, s, red, black, g.nblocks,
                           d_res);
        e = hipGetLastError();
    }
    return sor_fail(e, "sw2d_sor_run");
}

}  // extern "C"
