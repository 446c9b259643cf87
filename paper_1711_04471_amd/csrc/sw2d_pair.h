// sw2d_pair.h - the temporally blocked plain step with two adjacent columns per lane.
//
// Lane l of a wave holds columns c0 = base + 2l ("a") and c0 + 1 ("b"). The east neighbour
// of a is b of the same lane and that of b is a of lane l + 1; the west neighbour of a is b
// of lane l - 1 and that of b is a. A strip is then 128 columns wide and K steps per pass
// still cost 2K garbage columns on each side, so 128 - 4K of its columns are owned against
// 64 - 4K with one column per lane, and a row needs half the lane exchanges per cell. Every
// value is computed by the same formulas as in the one-column pipeline (sw2d_tile.h), in the
// same order, so the state is bitwise the same.
#pragma once

#include "sw2d_tile.h"

namespace sw2d {

// x-part of one cell of the input row (plain model).
struct PairX {
    float e, h, pe, us;
    bool w;
};

// Pipeline state of one column: rows 1, 2 and 3 behind the one being consumed (march order).
template <bool kNorth>
struct PairCol {
    // The water flags of rows 1 and 2 and the total depth of row 1 are taken again from their
    // depths where they are used (lane masks kept across the loop would not fit the scalar
    // registers, and the total depth saves a vector register); the flag of row 3 comes from
    // the caller, which takes it from the next stage's row 1 once every stage runs.
    float e1 = 0.f, hp1 = 0.f, v1 = 0.f, pe1 = 0.f, us1 = 0.f, fy1 = 0.f, vs1 = 0.f;
    float es2 = 0.f, fy2 = 0.f, vs2 = 0.f, us2 = 0.f, hp2 = 0.f;
    float es3 = 0.f, hp3 = 0.f;

    // y-face, predicted surface of the row one behind, filter output of the row two behind;
    // esE2, wE2, esW2 and wW2 are the predicted surfaces and water flags east and west of the
    // latter, w3 the water flag of the row three behind.
    __device__ __forceinline__ void advance(const PairX& X, float hpr, float vr, float esE2, bool wE2, float esW2,
                                            bool wW2, bool w3, const StepCoef& k, float& eta_o, float& u_o,
                                            float& v_o, float& hp_o) {
        u_o = us2;
        v_o = vs2;
        hp_o = hp2;
        const bool w1 = hp1 > 0.f, w2 = hp2 > 0.f;
        const float h1 = hp1 + e1;  // total depth of row 1, as the x-part computed it
        float vs, fy;
        bool av;
        if constexpr (kNorth) {
            face_y<0>(v1, e1, h1, w1, X.e, X.h, X.w, k, vs, fy, av);
            const float es = y_update(w1, fy, fy2, pe1, k);
            eta_o = shapiro_nb(es2, w2, esE2, wE2, esW2, wW2, es, w1, es3, w3, k.e4);
            es3 = es2;
            es2 = es;
            fy2 = fy;
            vs2 = vs;
            v1 = vr;
        } else {
            face_y<0>(vr, X.e, X.h, X.w, e1, h1, w1, k, vs, fy, av);
            const float es = y_update(w1, fy1, fy, pe1, k);
            eta_o = shapiro_nb(es2, w2, esE2, wE2, esW2, wW2, es3, w3, es, w1, k.e4);
            es3 = es2;
            es2 = es;
            vs2 = vs1;
            fy1 = fy;
            vs1 = vs;
        }
        us2 = us1;
        hp3 = hp2;
        hp2 = hp1;
        e1 = X.e;
        hp1 = hpr;
        pe1 = X.pe;
        us1 = X.us;
    }
};

// The east flag of column a is the flag of b and the west flag of b that of a; the flags
// across lanes (west of a, east of b) are taken by the caller: those of the input row, and
// those of the row two behind, which is the next stage's input row.
template <bool kNorth>
struct PairStage {
    PairCol<kNorth> a, b;

    // Consumes the input row (columns a and b of this lane) and returns the new state of the
    // row two behind it. aW, bE: flags west of a and east of b in the input row; aW2, bE2: in
    // the row two behind; aw3, bw3: the flags of columns a and b three rows behind.
    __device__ __forceinline__ void push(const float (&e)[2], const float (&hp)[2], const float (&ur)[2],
                                         const float (&vr)[2], bool aW, bool bE, bool aW2, bool bE2, bool aw3,
                                         bool bw3, const StepCoef& k, float (&eta_o)[2], float (&u_o)[2],
                                         float (&v_o)[2], float (&hp_o)[2]) {
        PairX xa, xb;
        xa.e = e[0];
        xb.e = e[1];
        xa.w = hp[0] > 0.f;
        xb.w = hp[1] > 0.f;
        xa.h = hp[0] + e[0];
        xb.h = hp[1] + e[1];
        // lane exchanges, taken by every lane before any select
        const float eEb = from_east(e[0]), hpEb = from_east(hp[0]);
        const float esEb = from_east(a.es2), esWa = from_west(b.es2);
        xa.us = x_pred(e[0], e[1], ur[0], xa.w && xb.w, k);
        xb.us = x_pred(e[1], eEb, ur[1], xb.w && bE, k);
        const float fxa = upwind_flux(xa.us, xa.h, xb.h);
        const float fxb = upwind_flux(xb.us, xb.h, hpEb + eEb);
        xa.pe = x_update(e[0], fxa, from_west(fxb), k);
        xb.pe = x_update(e[1], fxb, fxa, k);
        const float aes2 = a.es2;
        const bool aw2 = a.hp2 > 0.f, bw2 = b.hp2 > 0.f;
        a.advance(xa, hp[0], vr[0], b.es2, bw2, esWa, aW2, aw3, k, eta_o[0], u_o[0], v_o[0], hp_o[0]);
        b.advance(xb, hp[1], vr[1], esEb, bE2, aes2, aw2, bw3, k, eta_o[1], u_o[1], v_o[1], hp_o[1]);
    }
};

// Flags west of column a and east of column b of a row, from the row's depths.
__device__ __forceinline__ void cross_flags(float hp_a, float hp_b, bool& aW, bool& bE) {
    aW = from_west(hp_b) > 0.f;
    bE = from_east(hp_a) > 0.f;
}

// Rows of a column pair. kWide: nx is even, so a pair never straddles the end of a row and
// one 8-byte load or store moves it; otherwise each column goes through its own 4-byte
// access, and a b column past the row end reads 0 and is not written.
template <bool kWide>
struct PairIO {
    int nx, ny;
    unsigned off;  // byte offset of column a, or kNoLane

    __device__ __forceinline__ void load(const float* __restrict__ p, int r, float (&x)[2]) const {
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(p, r, nx, ny);
        if constexpr (kWide) {
            const auto q = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
            x[0] = __uint_as_float(q[0]);
            x[1] = __uint_as_float(q[1]);
        } else {
            x[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
            x[1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + 4u), 0, 0));
        }
    }
    // so: the byte offset of column a for an owned pair, kNoLane otherwise
    __device__ __forceinline__ void store(float* p, int r, unsigned so, const float (&x)[2]) const {
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(p, r, nx, r + 1);
        if constexpr (kWide) {
            __attribute__((ext_vector_type(2))) unsigned q;
            q[0] = __float_as_uint(x[0]);
            q[1] = __float_as_uint(x[1]);
            __builtin_amdgcn_raw_buffer_store_b64(q, rs, (int)so, 0, 0);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x[0]), rs, (int)so, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x[1]), rs, (int)(so + 4u), 0, 0);
        }
    }
};

// Folds of one step over this lane's owned pairs: the FP64 surface sum in an LDS slot of
// this lane (no other lane touches it), updated by an atomic that returns nothing, so it
// holds no registers across the march; the velocity maxima in registers.
struct PairFolds {
    double* disp;
    float max_u = 0.f, max_v = 0.f;
    __device__ __forceinline__ void add(const float (&e)[2], const float (&uu)[2], const float (&vv)[2]) {
        __hip_atomic_fetch_add(disp, (double)e[0] + (double)e[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        max_u = fmaxf(max_u, fmaxf(fabsf(uu[0]), fabsf(uu[1])));
        max_v = fmaxf(max_v, fmaxf(fabsf(vv[0]), fabsf(vv[1])));
    }
};

// Rows requested ahead by the two-column pass at 4 steps per pass. With the folds' FP64 sums in
// LDS and the flags and depths that neighbouring stages share taken once, two rows ahead fit
// the register budget of 3 waves per SIMD and measured faster there; at 2 and 3 steps per pass
// one row ahead measured faster (as in the one-column pipelines).
constexpr int kPairRowsAhead = 2;

// K steps of a band in one pass with two columns per lane (plain model). c0: column a of
// this lane; owned: both columns are this lane's output (the b column of a pair straddling
// an odd row end lies outside the grid, reads land and writes nothing).
template <int K, bool kNorth, bool kWide>
__device__ __forceinline__ void marchK_pair(const float* __restrict__ eta, const float* __restrict__ u,
                                            const float* __restrict__ v, const float* __restrict__ hp,
                                            float* __restrict__ eta_o, float* __restrict__ u_o,
                                            float* __restrict__ v_o, int nx, int ny, int c0, bool col_in,
                                            bool owned, int j0, int j1, const StepCoef& k, PairFolds* F) {
    constexpr int step = kNorth ? 1 : -1;
    constexpr int P = K >= 4 ? kPairRowsAhead : 1;
    const int r_first = kNorth ? j0 - 2 * K : j1 + 2 * K - 1;
    const int n_rows = j1 - j0 + 4 * K;
    const PairIO<kWide> io{nx, ny, col_in ? (unsigned)c0 * 4u : kNoLane};
    const unsigned so = owned ? (unsigned)c0 * 4u : kNoLane;
    float qe[P][2], qh[P][2], qu[P][2], qv[P][2];
#pragma unroll
    for (int d = 0; d < P; ++d) {
        const int rr = r_first + d * step;
        const int rl = d < n_rows ? rr : -1;  // a row outside the grid reads 0
        io.load(eta, rl, qe[d]);
        io.load(hp, rl, qh[d]);
        io.load(u, rl, qu[d]);
        io.load(v, rl, qv[d]);
    }
    PairStage<kNorth> S[K];
    bool lW1 = false, lE1 = false, lW2 = false, lE2 = false;  // last stage: rows 1 and 2 behind
    // One input row; in the priming rows (kSteady false) stage s starts at row 4s (march
    // order) and has valid output from row 4(s+1); in the steady state every stage has.
    auto row = [&](int i, auto steady) {
        constexpr bool kSteady = decltype(steady)::value;
        const int r = r_first + i * step;
        float e[2], h[2], uu[2], vv[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            e[c] = qe[0][c];
            h[c] = qh[0][c];
            uu[c] = qu[0][c];
            vv[c] = qv[0][c];
        }
#pragma unroll
        for (int d = 0; d + 1 < P; ++d) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                qe[d][c] = qe[d + 1][c];
                qh[d][c] = qh[d + 1][c];
                qu[d][c] = qu[d + 1][c];
                qv[d][c] = qv[d + 1][c];
            }
        }
        if (i + P < n_rows) {
            const int rr = r + P * step;
            io.load(eta, rr, qe[P - 1]);
            io.load(hp, rr, qh[P - 1]);
            io.load(u, rr, qu[P - 1]);
            io.load(v, rr, qv[P - 1]);
        }
        // Cross-lane flags of every stage's input row (stage s's row two behind is stage
        // s + 1's input row, whose depths it already holds), then the last stage's row two
        // behind, carried from two rows before.
        bool fW[K + 1], fE[K + 1];
        cross_flags(h[0], h[1], fW[0], fE[0]);
#pragma unroll
        for (int s = 1; s < K; ++s) cross_flags(S[s - 1].a.hp2, S[s - 1].b.hp2, fW[s], fE[s]);
        fW[K] = lW2;
        fE[K] = lE2;
        lW2 = lW1;
        lE2 = lE1;
        lW1 = fW[K - 1];
        lE1 = fE[K - 1];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if (!kSteady && s > 0 && i < 4 * s) break;
            float en[2], un[2], vn[2], hn[2];
            // Depth three rows behind stage s: its own in the priming rows, then (once every
            // stage runs) that of the row one behind stage s + 1, the same row.
            const PairStage<kNorth>& nxt = S[s + 1 < K ? s + 1 : s];
            const bool shared = kSteady && s + 1 < K;
            const float h3a = shared ? nxt.a.hp1 : S[s].a.hp3;
            const float h3b = shared ? nxt.b.hp1 : S[s].b.hp3;
            S[s].push(e, h, uu, vv, fW[s], fE[s], fW[s + 1], fE[s + 1], h3a > 0.f, h3b > 0.f, k, en, un, vn, hn);
            if (!kSteady && i < 4 * (s + 1)) break;
            const int ro = r - 2 * (s + 1) * step;  // row of stage s's output
            if (kSteady && s == K - 1) {
                // the last stage's steady rows are the band's own
                io.store(eta_o, ro, so, en);
                io.store(u_o, ro, so, un);
                io.store(v_o, ro, so, vn);
                if (owned) F[s].add(en, un, vn);
            } else if (ro >= j0 && ro < j1 && owned) {
                F[s].add(en, un, vn);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                e[c] = en[c];
                h[c] = hn[c];
                uu[c] = un[c];
                vv[c] = vn[c];
            }
        }
    };
    int i = 0;
    for (; i < 4 * K; ++i) row(i, std::false_type{});
    // Two rows per iteration: the pipeline's register shifts then mostly become renamings
    // instead of moves.
    for (; i + 1 < n_rows; i += 2) {
        row(i, std::true_type{});
        row(i + 1, std::true_type{});
    }
    if (i < n_rows) row(i, std::true_type{});
}

}  // namespace sw2d
