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

#include <algorithm>
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

// ---------------------------------------------------------------------------------------
// One whole iteration per launch (fused = 1): a workgroup owns a tile of kFuM colour positions
// x kFuJ rows and a chunk of kFuZ planes, reads the old red and black arrays and writes the
// new ones into the other pair (ping-pong, so no workgroup reads a value another one has
// already replaced). Walking up its planes, it computes the new red values of the next plane
// over the tile grown by one position and one row (the red neighbours of its black cells),
// keeps three planes of them in LDS, and updates the black cells of the plane below from
// them. Every red and black value is the expression of the two-sweep iteration, so the
// state is bitwise that of sor_sweep_kernel<0> then <1>; the red residual of the previous
// state and the black residual of the new one are folded as there (owned cells only).
constexpr int kFuM = 32, kFuJ = 16, kFuZ = 16;
constexpr int kFuThreads = kFuM * kFuJ;                    // one black cell per thread
constexpr int kFuHm = kFuM + 2, kFuHj = kFuJ + 2;          // red halo region of a plane
constexpr int kFuHalo = kFuHm * kFuHj;
constexpr int kFuRedPer = (kFuHalo + kFuThreads - 1) / kFuThreads;

struct SorFuGeometry {
    int tm, tj, tz, nblocks;  // tiles along positions, rows, plane chunks
};

SorFuGeometry sor_fu_geometry(const SorGeometry& g) {
    SorFuGeometry f;
    f.tm = (g.w + kFuM - 1) / kFuM;
    f.tj = (g.ny - 2 + kFuJ - 1) / kFuJ;
    f.tz = (g.nz - 2 + kFuZ - 1) / kFuZ;
    f.nblocks = f.tm * f.tj * f.tz;
    return f;
}

__global__ __launch_bounds__(kFuThreads) void sor_iter_kernel(const float* __restrict__ R, const float* __restrict__ B,
                                                              const float* __restrict__ FR, const float* __restrict__ FB,
                                                              float* __restrict__ Rn, float* __restrict__ Bn,
                                                              SorGeometry g, SorFuGeometry fg, SorCoef c,
                                                              SorPartial* __restrict__ red_part,
                                                              SorPartial* __restrict__ black_part) {
#pragma clang fp contract(off)
    __shared__ float s_red[3][kFuHalo];
    __shared__ double s_sum[kFuThreads];
    __shared__ unsigned s_max[kFuThreads];
    const int nx = g.nx, ny = g.ny, nz = g.nz, w = g.w;
    const size_t plane = (size_t)ny * w;
    const int b = blockIdx.x;
    const int tm = b % fg.tm, tj = (b / fg.tm) % fg.tj, tz = b / (fg.tm * fg.tj);
    const int m0 = tm * kFuM, j0 = 1 + tj * kFuJ, k0 = 1 + tz * kFuZ;
    const int k1 = min(k0 + kFuZ, nz - 1);  // planes [k0, k1) are this chunk's
    const int t = threadIdx.x;
    double acc_r = 0.0, acc_b = 0.0;
    unsigned mx_r = 0u, mx_b = 0u;

    // New red value of cell (m, j, k) (position m of the red array), from the old arrays;
    // cells on the boundary layer keep their value. *res: its residual in the old state.
    auto red_new = [&](int m, int j, int k, float* res) -> float {
        const size_t o = ((size_t)k * ny + j) * w + m;
        const float pc = R[o];
        const int s = (j + k) & 1;
        const int i = s + 2 * m;
        if (i < 1 || i > nx - 2 || j < 1 || j > ny - 2 || k < 1 || k > nz - 2) return pc;
        const float xm = B[o];
        const float xo = s ? B[o + 1] : B[o - 1];
        const float pE = s ? xo : xm, pW = s ? xm : xo;
        const float fc = FR[o];
        const float sx = pE + pW;
        const float sy = B[o + w] + B[o - w];
        const float sz = B[o + plane] + B[o - plane];
        const float nb = fmaf(c.cz, sz, fmaf(c.cy, sy, c.cx * sx));
        *res = fc - fmaf(-c.diag, pc, nb);
        const float gs = (nb - fc) * c.inv_diag;
        return fmaf(c.omega, gs - pc, pc);
    };

    // red halo items of this thread: item q -> (m, j) = (m0 - 1 + q % kFuHm, j0 - 1 + q / kFuHm)
    auto red_plane = [&](int k) {
        float* dst = s_red[(k + 3) % 3];
#pragma unroll
        for (int r = 0; r < kFuRedPer; ++r) {
            const int q = t + r * kFuThreads;
            if (q >= kFuHalo) break;
            const int hm = q % kFuHm, hj = q / kFuHm;
            const int m = m0 - 1 + hm, j = j0 - 1 + hj;
            float v = 0.f;
            if (m >= 0 && m < w && j >= 0 && j < ny && k >= 0 && k < nz) {
                float res = 0.f;
                v = red_new(m, j, k, &res);
                const bool owned = hm >= 1 && hm <= kFuM && hj >= 1 && hj <= kFuJ && k >= k0 && k < k1;
                const int i = ((j + k) & 1) + 2 * m;
                if (owned && i >= 1 && i <= nx - 2 && j <= ny - 2) {
                    Rn[((size_t)k * ny + j) * w + m] = v;
                    acc_r += (double)res * (double)res;
                    mx_r = max(mx_r, __float_as_uint(res) & 0x7fffffffu);
                }
            }
            dst[q] = v;
        }
    };

    // the black cell of this thread in plane k, from the new red values in LDS
    const int bm = t % kFuM, bj = t / kFuM;
    const int m = m0 + bm, j = j0 + bj;
    auto black_plane = [&](int k) {
        if (m >= w || j > ny - 2) return;
        const size_t o = ((size_t)k * ny + j) * w + m;
        const int s = (1 + j + k) & 1;
        const int i = s + 2 * m;
        if (i < 1 || i > nx - 2) return;
        const float* rc = s_red[(k + 3) % 3];
        const float* rd = s_red[(k + 2) % 3];
        const float* ru = s_red[(k + 4) % 3];
        const int h = (bj + 1) * kFuHm + (bm + 1);  // this position in the halo region
        const float xm = rc[h];
        const float xo = s ? rc[h + 1] : rc[h - 1];
        const float pE = s ? xo : xm, pW = s ? xm : xo;
        const float pc = B[o];
        const float fc = FB[o];
        const float sx = pE + pW;
        const float sy = rc[h + kFuHm] + rc[h - kFuHm];
        const float sz = ru[h] + rd[h];
        const float nb = fmaf(c.cz, sz, fmaf(c.cy, sy, c.cx * sx));
        const float gs = (nb - fc) * c.inv_diag;
        const float pn = fmaf(c.omega, gs - pc, pc);
        Bn[o] = pn;
        const float r = fc - fmaf(-c.diag, pn, nb);
        acc_b += (double)r * (double)r;
        mx_b = max(mx_b, __float_as_uint(r) & 0x7fffffffu);
    };

    red_plane(k0 - 1);
    red_plane(k0);
    for (int k = k0; k < k1; ++k) {
        __syncthreads();  // planes k - 1 and k are in LDS; the slot of k + 1 is free
        red_plane(k + 1);
        __syncthreads();
        black_plane(k);
    }

    // fixed-order trees: red residual (previous state) and black residual (new state)
    for (int pass = 0; pass < 2; ++pass) {
        __syncthreads();
        s_sum[t] = pass ? acc_b : acc_r;
        s_max[t] = pass ? mx_b : mx_r;
        __syncthreads();
        for (int hh = kFuThreads / 2; hh > 0; hh >>= 1) {
            if (t < hh) {
                s_sum[t] += s_sum[t + hh];
                s_max[t] = max(s_max[t], s_max[t + hh]);
            }
            __syncthreads();
        }
        if (t == 0) {
            SorPartial* q = (pass ? black_part : red_part) + b;
            q->sum_r2 = s_sum[0];
            q->max_bits = s_max[0];
            q->pad = 0u;
        }
    }
}

__global__ __launch_bounds__(256) void sor_zero_kernel(SorPartial* __restrict__ p, size_t n) {
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256)
        p[e] = SorPartial{0.0, 0u, 0u};
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
    return p->omega > 0.0 && p->omega < 2.0 && (p->fused == 0 || p->fused == 1);
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

// partials per residual slot: the sweep grid's, or with fused = 1 the larger of both grids
int part_stride(const sw2d_sor_params* p, const SorGeometry& g) {
    if (!p->fused) return g.nblocks;
    const int f = sor_fu_geometry(g).nblocks;
    return f > g.nblocks ? f : g.nblocks;
}

}  // namespace
}  // namespace sw2d

using namespace sw2d;

extern "C" {

size_t sw2d_sor_workspace_bytes(const sw2d_sor_params* p, int32_t iters) {
    if (!sor_params_ok(p) || iters < 0) return 0;
    const SorGeometry g = sor_geometry(p->nx, p->ny, p->nz);
    // red, black, f red, f black (and with fused = 1 a second red and black, 256 B aligned
    // each), then the residual partials: iters + 1 slots per colour
    const size_t arr = (colour_floats(g) * sizeof(float) + 255) / 256 * 256;
    return (p->fused ? 6 : 4) * arr + 2 * (size_t)(iters + 1) * part_stride(p, g) * sizeof(SorPartial);
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
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->fused) {
        // one launch per iteration, ping-pong between (R, B) and (R2, B2)
        float* R2 = reinterpret_cast<float*>(base + 4 * arr);
        float* B2 = reinterpret_cast<float*>(base + 5 * arr);
        const int stride = part_stride(p, g);
        const SorFuGeometry fg = sor_fu_geometry(g);
        auto* red = reinterpret_cast<SorPartial*>(base + 6 * arr);
        SorPartial* black = red + (size_t)(iters + 1) * stride;
        const size_t nparts = 2 * (size_t)(iters + 1) * stride;
        hipLaunchKernelGGL(sor_zero_kernel, dim3((unsigned)std::min<size_t>((nparts + 255) / 256, 1024)), dim3(256), 0, s,
                           red, nparts);
        hipError_t e = hipGetLastError();
        // both pairs start as the split state: the boundary layer is never written again
        if (e == hipSuccess) e = launch_split(d_p, R, B, g, 0, s);
        if (e == hipSuccess) e = launch_split(d_p, R2, B2, g, 0, s);
        if (e == hipSuccess) e = launch_split(const_cast<float*>(d_f), FR, FB, g, 0, s);  // read only (dir 0)
        if (e == hipSuccess) e = launch_sweep<1, kSorResidualOnly>(B, R, FB, g, c, black, s);  // black part of state 0
        for (int32_t n = 0; n < iters && e == hipSuccess; ++n) {
            hipLaunchKernelGGL(sor_iter_kernel, dim3(fg.nblocks), dim3(kFuThreads), 0, s, R, B, FR, FB, R2, B2, g, fg,
                               c, red + (size_t)n * stride, black + (size_t)(n + 1) * stride);
            e = hipGetLastError();
            std::swap(R, R2);
            std::swap(B, B2);
        }
        if (e == hipSuccess) e = launch_sweep<0, kSorResidualOnly>(R, B, FR, g, c, red + (size_t)iters * stride, s);
        if (e == hipSuccess) e = launch_split(d_p, R, B, g, 1, s);
        if (e == hipSuccess && d_res) {
            hipLaunchKernelGGL(sor_fold_kernel, dim3(iters + 1), dim3(kSorFoldThreads), 0, s, red, black, stride, d_res);
            e = hipGetLastError();
        }
        return sor_fail(e, "sw2d_sor_run");
    }
    auto* red = reinterpret_cast<SorPartial*>(base + 4 * arr);
    SorPartial* black = red + (size_t)(iters + 1) * g.nblocks;
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
