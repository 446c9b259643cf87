// sw2d_tile.h - the per-wave tile routine of the fused 2DSW step, shared by the
// single-grid kernel and the batched persistent kernel (one arithmetic path, so a
// batched instance is bitwise equal to the same basin stepped alone).
#pragma once

#include <hip/hip_runtime.h>

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

}  // namespace sw2d
