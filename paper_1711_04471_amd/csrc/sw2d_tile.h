// sw2d_tile.h - the per-wave tile routine of the fused 2DSW step, shared by the
// single-grid kernel and the batched persistent kernel (one arithmetic path, so a
// batched instance is bitwise equal to the same basin stepped alone).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "sw2d_internal.h"

namespace sw2d {

// Lane l receives lane l+1's value (its east neighbour); lane 63 receives 0 (the DPP
// bound control writes zero where the source lane lies outside the wave).
__device__ __forceinline__ float from_east(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x130 /* wave_shl:1 */, 0xf, 0xf, true));
}

// Lane l receives lane l-1's value (its west neighbour); lane 0 receives 0.
__device__ __forceinline__ float from_west(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x138 /* wave_shr:1 */, 0xf, 0xf, true));
}

// Formulas of the plain step (Sect. 6.2), written once and used by every row pipeline
// whatever its lane layout. Contraction is off and each fused multiply-add is explicit.

// Predicted velocity of an x-face from the surface of its west (e) and east (eE) cell:
// u* = u - g dt/dx (eta_E - eta), zero on an inactive face.
__device__ __forceinline__ float x_pred(float e, float eE, float ur, bool au, const StepCoef& k) {
#pragma clang fp contract(off)
    return au ? fmaf(-k.cx, eE - e, ur) : 0.f;
}

// Predicted velocity of a y-face from the surface of its south (e_lo) and north (e_hi) cell.
__device__ __forceinline__ float y_pred(float e_lo, float e_hi, float v_lo, bool av, const StepCoef& k) {
#pragma clang fp contract(off)
    return av ? fmaf(-k.cy, e_hi - e_lo, v_lo) : 0.f;
}

// Upwind flux through a face: the velocity times the total depth of the cell it comes from
// (h_lo for a positive velocity, h_hi otherwise); zero velocity gives zero flux.
__device__ __forceinline__ float upwind_flux(float vel, float h_lo, float h_hi) {
#pragma clang fp contract(off)
    return vel * (vel > 0.f ? h_lo : h_hi);
}

// x-part of the surface update: pe = eta - dt/dx (Fx - Fx_W).
__device__ __forceinline__ float x_update(float e, float fx, float fxW, const StepCoef& k) {
#pragma clang fp contract(off)
    return fmaf(-k.rx, fx - fxW, e);
}

// Predicted surface of a water cell: pe - dt/dy (Fy_N - Fy_S); zero on land.
__device__ __forceinline__ float y_update(bool w, float fyN, float fyS, float pe, const StepCoef& k) {
#pragma clang fp contract(off)
    return w ? fmaf(-k.ry, fyN - fyS, pe) : 0.f;
}

// First-order Shapiro filter of the predicted surface es_c of a water cell across its
// water neighbours, added east, west, north, south in that order; zero on land.
__device__ __forceinline__ float shapiro_nb(float es_c, bool w_c, float esE, bool wE, float esW, bool wW,
                                            float es_n, bool w_n, float es_s, bool w_s, float e4) {
#pragma clang fp contract(off)
    float s = wE ? esE - es_c : 0.f;
    if (wW) s += esW - es_c;
    if (w_n) s += es_n - es_c;
    if (w_s) s += es_s - es_c;
    return w_c ? fmaf(e4, s, es_c) : 0.f;
}

// Row r of the march: water flags, total depth, x-face predictor and flux, and the
// x-part of the surface update (pe = eta - dt/dx (Fx - Fx_W)).
struct RowX {
    float e, h, pe, us;
    bool w, wE, wW, au;
    bool d, dE, dW;  // wetting and drying: wet now (total depth above the threshold)
};

// Wetting and drying: a face between two water cells a and b carries flow when both are
// wet, or when one is wet and its surface stands above the other's.
__device__ __forceinline__ bool face_open(bool da, bool db, float ea, float eb) {
    return (da && db) || (da && ea > eb) || (db && eb > ea);
}

// Quadratic bottom friction (variant): the predictor divided by 1 + dt cd |u_old| / h_face,
// h_face the mean total depth of the face's two cells.
__device__ __forceinline__ float friction(float pred, float u_old, float h_a, float h_b, const StepCoef& k) {
#pragma clang fp contract(off)
    const float hf = 0.5f * (h_a + h_b);
    return pred / (1.f + k.kf * fabsf(u_old) / hf);
}

// Floating-point contraction is off in the step's arithmetic and every fused multiply-add
// is written out, so each kernel that inlines these routines rounds alike, bit for bit.
template <int kVar = 0>
__device__ __forceinline__ RowX row_x(float e, float hpr, float ur, const StepCoef& k) {
#pragma clang fp contract(off)
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
    o.au = au;
    if constexpr ((kVar & kVarWetDry) != 0) {
        // every lane takes the exchange before any select
        const float hW = from_west(o.h);
        o.d = o.h > k.hmin;
        o.dE = hpE + eE > k.hmin;
        o.dW = hW > k.hmin;
        o.us = (au && face_open(o.d, o.dE, e, eE)) ? fmaf(-k.cx, eE - e, ur) : 0.f;
    } else {
        o.us = x_pred(e, eE, ur, au, k);
    }
    if constexpr ((kVar & kVarFriction) != 0) o.us = au ? friction(o.us, ur, o.h, hpE + eE, k) : 0.f;
    // an inactive face has us = 0, so its flux is 0 without a second select
    const float fx = upwind_flux(o.us, o.h, hpE + eE);
    const float fxW = from_west(fx);
    o.pe = x_update(e, fx, fxW, k);
    return o;
}

// The y-face between a southern cell (lo) and its northern neighbour (hi).
template <int kVar = 0>
__device__ __forceinline__ void face_y(float v_lo, float e_lo, float h_lo, bool w_lo, float e_hi,
                                       float h_hi, bool w_hi, const StepCoef& k, float& vs, float& fy,
                                       bool& av) {
#pragma clang fp contract(off)
    av = w_lo && w_hi;
    if constexpr ((kVar & kVarWetDry) != 0) {
        vs = (av && face_open(h_lo > k.hmin, h_hi > k.hmin, e_lo, e_hi)) ? fmaf(-k.cy, e_hi - e_lo, v_lo) : 0.f;
    } else {
        vs = y_pred(e_lo, e_hi, v_lo, av, k);
    }
    if constexpr ((kVar & kVarFriction) != 0) vs = av ? friction(vs, v_lo, h_lo, h_hi, k) : 0.f;
    fy = upwind_flux(vs, h_lo, h_hi);  // vs = 0 on an inactive face
}

// First-order Shapiro filter of the predicted surface es_c across water neighbours
// (east, west, north, south, always added in that order).
__device__ __forceinline__ float shapiro(float es_c, bool w_c, bool wE, bool wW, float es_n, bool w_n,
                                         float es_s, bool w_s, float e4) {
#pragma clang fp contract(off)
    return shapiro_nb(es_c, w_c, from_east(es_c), wE, from_west(es_c), wW, es_n, w_n, es_s, w_s, e4);
}

// Wetting and drying: the filter acts on wet cells (d_c) across wet neighbours; a dry
// cell keeps its predicted surface (0 on land, where es is 0).
__device__ __forceinline__ float shapiro_wd(float es_c, bool d_c, bool dE, bool dW, float es_n, bool d_n,
                                            float es_s, bool d_s, float e4) {
#pragma clang fp contract(off)
    const float esE = from_east(es_c);
    const float esW = from_west(es_c);
    float s = dE ? esE - es_c : 0.f;
    if (dW) s += esW - es_c;
    if (d_n) s += es_n - es_c;
    if (d_s) s += es_s - es_c;
    return d_c ? fmaf(e4, s, es_c) : es_c;
}

// The same filter on face velocities (variant): c on an active face, neighbours east and
// west (lane exchange) and north and south, each counted only when active.
__device__ __forceinline__ float shapiro_face(float c, bool act, float n_val, bool n_act, float s_val, bool s_act,
                                              float e4) {
#pragma clang fp contract(off)
    const float cE = from_east(c), cW = from_west(c);
    const float a = act ? 1.f : 0.f;
    const bool actE = from_east(a) > 0.f, actW = from_west(a) > 0.f;
    float s = actE ? cE - c : 0.f;
    if (actW) s += cW - c;
    if (n_act) s += n_val - c;
    if (s_act) s += s_val - c;
    return act ? fmaf(e4, s, c) : 0.f;
}

// One time step of one wave's strip as a row pipeline. push() consumes input row r (in
// march order) and returns the new state of the row two behind it: row r gives the x-face
// predictor, flux and partial surface update; row r-1 (r+1 marching south) its y-face and
// the predicted surface es; row r-2 (r+2) the Shapiro filter. Every output value is the
// same expression in either direction.
// Wet flags of the old surface for rows 1, 2 and 3 behind (wetting and drying only; an
// empty base otherwise, so the other pipelines carry no unused state).
struct StageWetFlags {
    bool d1 = false, dE1 = false, dW1 = false, d2 = false, dE2 = false, dW2 = false, d3 = false;
};
struct StageNoFlags {};

template <bool kNorth, int kVar = 0>
struct Stage : std::conditional_t<(kVar & kVarWetDry) != 0, StageWetFlags, StageNoFlags> {
    static constexpr bool kFilterUV = (kVar & kVarFilterUV) != 0;
    static constexpr bool kWetDry = (kVar & kVarWetDry) != 0;
    // rows 1, 2 and 3 behind the one being consumed (in march order)
    float e1 = 0.f, h1 = 0.f, hp1 = 0.f, v1 = 0.f, pe1 = 0.f, us1 = 0.f, fy1 = 0.f, vs1 = 0.f;
    bool w1 = false, wE1 = false, wW1 = false;
    float es2 = 0.f, fy2 = 0.f, vs2 = 0.f, us2 = 0.f, hp2 = 0.f;
    bool w2 = false, wE2 = false, wW2 = false;
    float es3 = 0.f;
    bool w3 = false;
    // velocity-filter variant: face activity travelling with the face values, one more row
    bool au1 = false, au2 = false, au3 = false, av1 = false, av2 = false, av3 = false;
    float us3 = 0.f, vs3 = 0.f;

    __device__ __forceinline__ void push(float e, float hpr, float ur, float vr, const StepCoef& k,
                                         float& eta_o, float& u_o, float& v_o, float& hp_o) {
        const RowX X = row_x<kVar>(e, hpr, ur, k);
        if constexpr (kNorth) {
            // y-face between rows r-1 and r, then es of row r-1, then the output row r-2
            float vs, fy;
            bool av;
            face_y<kVar>(v1, e1, h1, w1, X.e, X.h, X.w, k, vs, fy, av);
            const float es = y_update(w1, fy, fy2, pe1, k);
            if constexpr (kWetDry) eta_o = shapiro_wd(es2, this->d2, this->dE2, this->dW2, es, this->d1, es3, this->d3, k.e4);
            else eta_o = shapiro(es2, w2, wE2, wW2, es, w1, es3, w3, k.e4);
            if constexpr (kFilterUV) {
                // north neighbour: row r-1 (u) and the face r-1|r (v); south: row r-3, face r-3|r-2
                u_o = shapiro_face(us2, au2, us1, au1, us3, au3, k.e4);
                v_o = shapiro_face(vs2, av2, vs, av, vs3, av3, k.e4);
                us3 = us2;
                au3 = au2;
                vs3 = vs2;
                av3 = av2;
                av2 = av;
            } else {
                u_o = us2;
                v_o = vs2;
            }
            hp_o = hp2;
            es3 = es2;
            w3 = w2;
            es2 = es;
            fy2 = fy;
            vs2 = vs;
            v1 = vr;
        } else {
            // y-face between rows r and r+1, then es of row r+1, then the output row r+2
            float vs, fy;
            bool av;
            face_y<kVar>(vr, X.e, X.h, X.w, e1, h1, w1, k, vs, fy, av);
            const float es = y_update(w1, fy1, fy, pe1, k);
            if constexpr (kWetDry) eta_o = shapiro_wd(es2, this->d2, this->dE2, this->dW2, es3, this->d3, es, this->d1, k.e4);
            else eta_o = shapiro(es2, w2, wE2, wW2, es3, w3, es, w1, k.e4);
            if constexpr (kFilterUV) {
                // north neighbour: row r+3 (u) and the face r+3|r+4 (v); south: row r+1, face r+1|r+2
                u_o = shapiro_face(us2, au2, us3, au3, us1, au1, k.e4);
                v_o = shapiro_face(vs2, av2, vs3, av3, vs1, av1, k.e4);
                us3 = us2;
                au3 = au2;
                vs3 = vs2;
                av3 = av2;
                av2 = av1;
                av1 = av;
            } else {
                u_o = us2;
                v_o = vs2;
            }
            hp_o = hp2;
            es3 = es2;
            w3 = w2;
            es2 = es;
            vs2 = vs1;
            fy1 = fy;
            vs1 = vs;
        }
        if constexpr (kFilterUV) {
            au2 = au1;
            au1 = X.au;
        }
        if constexpr (kWetDry) {
            this->d3 = this->d2;
            this->d2 = this->d1;
            this->dE2 = this->dE1;
            this->dW2 = this->dW1;
            this->d1 = X.d;
            this->dE1 = X.dE;
            this->dW1 = X.dW;
        }
        us2 = us1;
        hp2 = hp1;
        w2 = w1;
        wE2 = wE1;
        wW2 = wW1;
        e1 = X.e;
        h1 = X.h;
        hp1 = hpr;
        pe1 = X.pe;
        us1 = X.us;
        w1 = X.w;
        wE1 = X.wE;
        wW1 = X.wW;
    }
};

// ---------------------------------------------------------------------------------------
// Variant with nonlinear momentum advection (first-order upwind). The x-face predictor of a
// row needs u of the rows above and below it, so the pipeline computes it one row later
// than the plain Stage: push(row r) predicts the x-faces of row r-1 and the y-face r-1|r,
// completes es of row r-1 and returns row r-2 as before. The y-face's upwind difference
// reads v one row further south, so a band starts 3 rows below its first output row and
// marches north only; the x-face reads u one face further west, so strips keep 3 halo
// lanes on their west side.
template <int kVar>
struct StageAdv {
    static constexpr bool kFilterUV = (kVar & kVarFilterUV) != 0;
    // row r-1
    float e1 = 0.f, h1 = 0.f, hp1 = 0.f, u1 = 0.f, v1 = 0.f;
    bool w1 = false, wE1 = false, wW1 = false;
    // row r-2 (and the faces computed at the previous push)
    float u2 = 0.f, v2 = 0.f, es2 = 0.f, fy2 = 0.f, us2 = 0.f, vs2 = 0.f, hp2 = 0.f;
    bool w2 = false, wE2 = false, wW2 = false, au2 = false, av2 = false;
    // row r-3
    float es3 = 0.f, us3 = 0.f, vs3 = 0.f;
    bool w3 = false, au3 = false, av3 = false;

    __device__ __forceinline__ void push(float e, float hpr, float ur, float vr, const StepCoef& k,
                                         float& eta_o, float& u_o, float& v_o, float& hp_o) {
#pragma clang fp contract(off)
        const bool w = hpr > 0.f;
        const float h = hpr + e;
        const bool wE = from_east(hpr) > 0.f;
        const bool wW = from_west(hpr) > 0.f;
        // x-faces of row r-1: pressure gradient, advection, friction; flux and partial update
        const float eE1 = from_east(e1), hpE1 = from_east(hp1);
        // Lane exchanges are taken by every lane before any select: a DPP read from a lane
        // that sits out a divergent branch returns 0, not its value.
        const float uW1 = from_west(u1), uE1 = from_east(u1), vW1 = from_west(v1), vE1 = from_east(v1);
        const float uWr = from_west(ur);
        const bool au1 = w1 && wE1;
        const float vbar = 0.25f * ((v1 + vE1) + (v2 + from_east(v2)));
        // dt (u du/dx + vbar du/dy) = (u du) dt/dx + (vbar du) dt/dy, upstream differences
        const float tx = u1 > 0.f ? u1 * (u1 - uW1) : u1 * (uE1 - u1);
        const float ty = vbar > 0.f ? vbar * (u1 - u2) : vbar * (ur - u1);
        float pu = fmaf(-k.cx, eE1 - e1, u1);
        pu = pu - (tx * k.rx + ty * k.ry);
        if constexpr ((kVar & kVarFriction) != 0) pu = friction(pu, u1, h1, hpE1 + eE1, k);
        const float us1 = au1 ? pu : 0.f;
        const float fx1 = us1 * (us1 > 0.f ? h1 : hpE1 + eE1);
        const float pe1 = fmaf(-k.rx, fx1 - from_west(fx1), e1);
        // y-face r-1|r
        const bool av = w1 && w;
        const float ubar = 0.25f * ((u1 + uW1) + (ur + uWr));
        const float tbx = ubar > 0.f ? ubar * (v1 - vW1) : ubar * (vE1 - v1);
        const float tby = v1 > 0.f ? v1 * (v1 - v2) : v1 * (vr - v1);
        float pv = fmaf(-k.cy, e - e1, v1);
        pv = pv - (tbx * k.rx + tby * k.ry);
        if constexpr ((kVar & kVarFriction) != 0) pv = friction(pv, v1, h1, h, k);
        const float vs = av ? pv : 0.f;
        const float fy = vs * (vs > 0.f ? h1 : h);
        // surface of row r-1, then the output row r-2
        const float es = w1 ? fmaf(-k.ry, fy - fy2, pe1) : 0.f;
        eta_o = shapiro(es2, w2, wE2, wW2, es, w1, es3, w3, k.e4);
        if constexpr (kFilterUV) {
            u_o = shapiro_face(us2, au2, us1, au1, us3, au3, k.e4);
            v_o = shapiro_face(vs2, av2, vs, av, vs3, av3, k.e4);
        } else {
            u_o = us2;
            v_o = vs2;
        }
        hp_o = hp2;
        // shift: rows r-2 -> r-3, r-1 -> r-2, r -> r-1
        es3 = es2;
        w3 = w2;
        us3 = us2;
        au3 = au2;
        vs3 = vs2;
        av3 = av2;
        es2 = es;
        fy2 = fy;
        us2 = us1;
        au2 = au1;
        vs2 = vs;
        av2 = av;
        hp2 = hp1;
        w2 = w1;
        wE2 = wE1;
        wW2 = wW1;
        u2 = u1;
        v2 = v1;
        e1 = e;
        h1 = h;
        hp1 = hpr;
        u1 = ur;
        v1 = vr;
        w1 = w;
        wE1 = wE;
        wW1 = wW;
    }
};

// Rows go through buffer resources: one per field and row, whose size is the row's bytes,
// or zero for a row outside the grid. The hardware returns 0 for a load outside the
// resource and drops a store there, so a lane outside the grid (its byte offset, taken
// unsigned, lies past the row) or outside the band reads land and writes nothing, with no
// predication in the loop. Pointers and row numbers are wave-uniform.
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit dwords, gfx9 family
constexpr unsigned kNoLane = 0x80000000u;  // a byte offset past any row

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float* base, int r, int nx, int ny) {
    const bool in = r >= 0 && r < ny;
    const float* p = base + (ptrdiff_t)(in ? r : 0) * nx;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), 0, in ? nx * 4 : 0, kRsrcWord3);
}

__device__ __forceinline__ float row_load(const float* base, int r, int nx, int ny, unsigned off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(row_rsrc(base, r, nx, ny), (int)off, 0, 0));
}

// off: this lane's byte offset, or kNoLane for a lane that must not write
__device__ __forceinline__ void row_store(float* base, int r, int nx, unsigned off, float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), row_rsrc(base, r, nx, r + 1), (int)off, 0, 0);
}

// Rows requested ahead of the one being processed (deeper queues measured no faster).
constexpr int kRowsAhead = 1;

// Loads rows of one lane's column through a queue of kRowsAhead rows. A band's outermost
// rows feed its output only through some fields: the row two below the band only through its
// surface, depth and v (its y-face with the row above), the row above the band only through
// its surface and depth (the y-face below it). Their other fields are read through a
// zero-size resource (zeros, no memory traffic) when kTrim: skip_u and skip_uv name those
// rows. (The K-step marches keep every field: there the extra scalar work costs more than the
// outermost halo rows' traffic.)
template <bool kTrim = false>
struct RowLoader {
    const float* __restrict__ eta;
    const float* __restrict__ u;
    const float* __restrict__ v;
    const float* __restrict__ hp;
    int nx, ny, c;
    bool col_in;
    int skip_u = 0, skip_uv = 0;
    float qe[kRowsAhead], qh[kRowsAhead], qu[kRowsAhead], qv[kRowsAhead];

    __device__ __forceinline__ float load(const float* __restrict__ p, int r, int rows) const {
        return row_load(p, r, nx, rows, col_in ? (unsigned)c * 4u : kNoLane);
    }
    __device__ __forceinline__ float load(const float* __restrict__ p, int r) const { return load(p, r, ny); }
    __device__ __forceinline__ float load_u(int r) const {
        return load(u, r, kTrim && (r == skip_u || r == skip_uv) ? 0 : ny);
    }
    __device__ __forceinline__ float load_v(int r) const { return load(v, r, kTrim && r == skip_uv ? 0 : ny); }
    __device__ __forceinline__ void fill(int r_first, int step, int n_rows) {
#pragma unroll
        for (int d = 0; d < kRowsAhead; ++d) {
            const int rr = r_first + d * step;
            const bool ok = d < n_rows;
            qe[d] = ok ? load(eta, rr) : 0.f;
            qh[d] = ok ? load(hp, rr) : 0.f;
            qu[d] = ok ? load_u(rr) : 0.f;
            qv[d] = ok ? load_v(rr) : 0.f;
        }
    }
    // Row i (at r) out of the queue; row i + kRowsAhead requested.
    __device__ __forceinline__ void next(int i, int r, int step, int n_rows, float& e, float& h, float& uu,
                                         float& vv) {
        e = qe[0];
        h = qh[0];
        uu = qu[0];
        vv = qv[0];
#pragma unroll
        for (int d = 0; d + 1 < kRowsAhead; ++d) {
            qe[d] = qe[d + 1];
            qh[d] = qh[d + 1];
            qu[d] = qu[d + 1];
            qv[d] = qv[d + 1];
        }
        if (i + kRowsAhead < n_rows) {
            const int rr = r + kRowsAhead * step;
            qe[kRowsAhead - 1] = load(eta, rr);
            qh[kRowsAhead - 1] = load(hp, rr);
            qu[kRowsAhead - 1] = load_u(rr);
            qv[kRowsAhead - 1] = load_v(rr);
        }
    }
};

// Writes one output row of the new state.
struct RowStorer {
    float* __restrict__ eta;
    float* __restrict__ u;
    float* __restrict__ v;
    int nx, c;
    bool out_lane;
    __device__ __forceinline__ void put(int r, float e, float uu, float vv) const {
        const unsigned off = out_lane ? (unsigned)c * 4u : kNoLane;
        row_store(eta, r, nx, off, e);
        row_store(u, r, nx, off, uu);
        row_store(v, r, nx, off, vv);
    }
};

// Folds of one step over this lane's owned cells. The maxima take the magnitude as a source
// modifier of the float maximum (no separate instruction); a non-finite state shows in the
// FP64 surface sum, which every non-finite velocity reaches in the same step.
struct LaneFolds {
    double disp = 0.0;
    float max_u = 0.f, max_v = 0.f;
    __device__ __forceinline__ void add(float eta_new, float u_new, float v_new) {
        disp += (double)eta_new;  // zero on land
        max_u = fmaxf(max_u, fabsf(u_new));
        max_v = fmaxf(max_v, fabsf(v_new));
    }
    __device__ __forceinline__ float mu() const { return max_u; }
    __device__ __forceinline__ float mv() const { return max_v; }
};

// One wave marches a band [j0, j1) of its strip, north (kNorth) or south, and writes the
// new state of its output lanes.
template <bool kNorth, int kVar = 0>
__device__ __forceinline__ void march(const float* __restrict__ eta, const float* __restrict__ u,
                                      const float* __restrict__ v, const float* __restrict__ hp,
                                      float* __restrict__ eta_o, float* __restrict__ u_o,
                                      float* __restrict__ v_o, int nx, int ny, int c, bool col_in,
                                      bool out_lane, int j0, int j1, const StepCoef& k,
                                      double& f_disp, float& f_mu, float& f_mv) {
    constexpr int step = kNorth ? 1 : -1;
    const int r_first = kNorth ? j0 - 2 : j1 + 1;
    const int n_rows = j1 - j0 + 4;
    RowLoader<true> L{eta, u, v, hp, nx, ny, c, col_in};
    L.skip_u = j0 - 2;
    L.skip_uv = j1 + 1;
    const RowStorer W{eta_o, u_o, v_o, nx, c, out_lane};
    L.fill(r_first, step, n_rows);
    Stage<kNorth, kVar> A;
    LaneFolds F;
    for (int i = 0; i < n_rows; ++i) {
        const int r = r_first + i * step;
        float e, hpr, ur, vr;
        L.next(i, r, step, n_rows, e, hpr, ur, vr);
        float en, un, vn, hn;
        A.push(e, hpr, ur, vr, k, en, un, vn, hn);
        if (i >= 4) {
            W.put(r - 2 * step, en, un, vn);
            if (out_lane) F.add(en, un, vn);
        }
    }
    f_disp = F.disp;
    f_mu = F.mu();
    f_mv = F.mv();
}

// One step of a band with the advection pipeline (north only): rows j0-3 .. j1+1.
template <int kVar>
__device__ __forceinline__ void march_adv(const float* __restrict__ eta, const float* __restrict__ u,
                                          const float* __restrict__ v, const float* __restrict__ hp,
                                          float* __restrict__ eta_o, float* __restrict__ u_o,
                                          float* __restrict__ v_o, int nx, int ny, int c, bool col_in,
                                          bool out_lane, int j0, int j1, const StepCoef& k, double& f_disp,
                                          float& f_mu, float& f_mv) {
    const int r_first = j0 - 3;
    const int n_rows = j1 - j0 + 5;
    RowLoader<> L{eta, u, v, hp, nx, ny, c, col_in};
    const RowStorer W{eta_o, u_o, v_o, nx, c, out_lane};
    L.fill(r_first, 1, n_rows);
    StageAdv<kVar> A;
    LaneFolds F;
    for (int i = 0; i < n_rows; ++i) {
        const int r = r_first + i;
        float e, hpr, ur, vr;
        L.next(i, r, 1, n_rows, e, hpr, ur, vr);
        float en, un, vn, hn;
        A.push(e, hpr, ur, vr, k, en, un, vn, hn);
        if (i >= 5) {
            W.put(r - 2, en, un, vn);
            if (out_lane) F.add(en, un, vn);
        }
    }
    f_disp = F.disp;
    f_mu = F.mu();
    f_mv = F.mv();
}

// K time steps in one pass (temporal blocking): stage k+1 steps the rows stage k has just
// produced, so the intermediate states never leave the registers. Each step's stencil
// reaches two more columns into the garbage of the strip edges, so owned lanes shrink to
// 2K .. 63-2K, and bands need a 2K-row halo; the folds of every step are taken over the
// owned cells. kVar: the plain model or a variant whose step reaches no further than the
// plain step's (friction, the velocity filter, both, or wetting and drying; not advection).
template <int K, bool kNorth, int kVar = 0>
__device__ __forceinline__ void marchK(const float* __restrict__ eta, const float* __restrict__ u,
                                       const float* __restrict__ v, const float* __restrict__ hp,
                                       float* __restrict__ eta_o, float* __restrict__ u_o,
                                       float* __restrict__ v_o, int nx, int ny, int c, bool col_in,
                                       bool out_lane, int j0, int j1, const StepCoef& k, LaneFolds* F) {
    constexpr int step = kNorth ? 1 : -1;
    const int r_first = kNorth ? j0 - 2 * K : j1 + 2 * K - 1;
    const int n_rows = j1 - j0 + 4 * K;
    RowLoader<> L{eta, u, v, hp, nx, ny, c, col_in};
    const RowStorer W{eta_o, u_o, v_o, nx, c, out_lane};
    L.fill(r_first, step, n_rows);
    static_assert((kVar & kVarAdvection) == 0, "advection reaches too far for K-step passes");
    Stage<kNorth, kVar> S[K];
    int i = 0;
    // Priming: stage s starts at row 4s (march order) and has valid output from row 4(s+1).
    for (; i < 4 * K; ++i) {
        const int r = r_first + i * step;
        float e, hpr, ur, vr;
        L.next(i, r, step, n_rows, e, hpr, ur, vr);
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (s > 0 && i < 4 * s) break;
            float en, un, vn, hn;
            S[s].push(e, hpr, ur, vr, k, en, un, vn, hn);
            if (i < 4 * (s + 1)) break;
            const int ro = r - 2 * (s + 1) * step;  // row of stage s's output
            if (ro >= j0 && ro < j1 && out_lane) F[s].add(en, un, vn);
            e = en;
            hpr = hn;
            ur = un;
            vr = vn;
        }
    }
    // Steady state: every stage has valid output; the last one's rows are the band's own.
    for (; i < n_rows; ++i) {
        const int r = r_first + i * step;
        float e, hpr, ur, vr;
        L.next(i, r, step, n_rows, e, hpr, ur, vr);
#pragma unroll
        for (int s = 0; s < K; ++s) {
            float en, un, vn, hn;
            S[s].push(e, hpr, ur, vr, k, en, un, vn, hn);
            const int ro = r - 2 * (s + 1) * step;
            if (s == K - 1) {
                W.put(ro, en, un, vn);
                if (out_lane) F[s].add(en, un, vn);
            } else if (ro >= j0 && ro < j1 && out_lane) {
                F[s].add(en, un, vn);
            }
            e = en;
            hpr = hn;
            ur = un;
            vr = vn;
        }
    }
}

}  // namespace sw2d
