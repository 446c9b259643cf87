// sw2d_internal.h - types shared by the 2DSW kernels and the C ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw2d.h"

namespace sw2d {

constexpr int kWave = 64;                            // CDNA wavefront width
constexpr int kHalo = 2;                             // stencil radius of the fused step
constexpr int kStripOut = kWave - 2 * kHalo;         // output columns per wave strip (60)
constexpr int kMaxStepsPerPass = 4;                 // temporal blocking depth (K steps per pass)
// Owned columns of a strip at K steps per pass: the plain model at K >= 2 takes two adjacent
// columns per lane (120, 116, 112), one step per pass one column (60).
constexpr int strip_out_for(int K) { return (K >= 2 ? 2 * kWave : kWave) - 4 * K; }
constexpr int kWavesPerGroup = 4;                    // strips per workgroup
constexpr int kGroupThreads = kWave * kWavesPerGroup;
constexpr int kGroupCols = kStripOut * kWavesPerGroup;  // 240 output columns per workgroup
constexpr int kFoldThreads = 256;
constexpr int kXcds = 8;                             // MI355X: 8 XCDs, one L2 each
constexpr int kMinRows = 8;                          // smallest band height a handle may use
constexpr int kFoldChunk = 16;                       // steps whose partials are buffered
constexpr int kRingCap = 4096;                       // steps of folds kept for sw2d_reduce

// Per-workgroup fold partial of one step (16 B).
struct alignas(16) FoldPartial {
    double disp;  // sum over water cells of eta
    float mu;     // max |u|
    float mv;     // max |v|
};

struct StepGeometry {
    int nx, ny;
    int strips;    // ceil(nx / kStripOut)
    int groups_x;  // ceil(strips / kWavesPerGroup)
    int rows;      // rows per band
    int bands;     // ceil(ny / rows)
    int nblocks;   // groups_x * bands
};

// Step coefficients, computed in double on the host and rounded once to float.
struct StepCoef {
    float cx, cy;  // g dt / dx, g dt / dy
    float rx, ry;  // dt / dx, dt / dy
    float e4;      // eps / 4
    float kf;      // dt cd (bottom friction; 0 without it)
    float hmin;    // wet threshold on the total depth (wetting and drying; 0 without it)
};

// Model variants of the step (the flags of sw2d_params), as template arguments.
enum : int {
    kVarFriction = 1,
    kVarFilterUV = 2,
    kVarAdvection = 4,
    kVarAll = kVarFriction | kVarFilterUV | kVarAdvection,
    kVarWetDry = 8  // alone
};
// With advection the single-step strip keeps a 3-lane halo on its west side (the x-face
// predictor reads u one face further west) and 2 on its east side: 59 owned columns.
constexpr int kAdvHaloW = 3;
constexpr int kAdvStripOut = kWave - kAdvHaloW - kHalo;
constexpr int single_strip_out(uint32_t flags) { return (flags & kVarAdvection) ? kAdvStripOut : kStripOut; }
// Owned columns of a strip for K >= 2 steps per pass: the two-column pass for the plain
// model, the one-column pass for the variants that have one (all but advection).
constexpr int kstep_strip_out(int K, uint32_t flags) { return flags ? kWave - 4 * K : strip_out_for(K); }
// Variants that may advance several steps per pass: those whose step reaches no further than
// the plain step's two cells (advection reads one more face upstream).
constexpr bool kstep_variant_ok(uint32_t flags) { return (flags & kVarAdvection) == 0; }

enum : uint32_t {
    kWetBorder = 1u,
    kBadDepth = 2u,
    kBadState = 4u,
    kDryCell = 8u,
};

struct PrepFlags {
    uint32_t bad;        // OR of the k* bits above
    uint32_t hmax_bits;  // bit pattern of the largest water depth (positive float)
    double h_sum;        // sum over water cells of H (static part of the total volume)
};

constexpr int kHsumBlocks = 256;  // partials of the one-off sum_wet H

inline StepGeometry make_geometry(int nx, int ny, int rows, int strip_out = kStripOut) {
    StepGeometry g;
    g.nx = nx;
    g.ny = ny;
    g.strips = (nx + strip_out - 1) / strip_out;
    g.groups_x = (g.strips + kWavesPerGroup - 1) / kWavesPerGroup;
    g.rows = rows;
    g.bands = (ny + rows - 1) / rows;
    g.nblocks = g.groups_x * g.bands;
    return g;
}

// kvar: the model variants (0 for the plain step).
hipError_t launch_step(int kvar, const float* eta, const float* u, const float* v, const float* hp,
                       float* eta_o, float* u_o, float* v_o, FoldPartial* part,
                       const StepGeometry& geo, const StepCoef& k, hipStream_t s);
// K = 2..4 steps in one pass (geometry from make_geometry(..., kstep_strip_out(K, flags))),
// kvar 0 or a variant without advection; the partials of step s of the pass go to
// part[s * stride + 0..nblocks).
hipError_t launch_stepk(int K, int kvar, const float* eta, const float* u, const float* v, const float* hp,
                        float* eta_o, float* u_o, float* v_o, FoldPartial* part, int stride,
                        const StepGeometry& geo, const StepCoef& k, hipStream_t s);
// Partials of step s of the chunk start at part + s * stride; nparts of them are valid.
hipError_t launch_fold(const FoldPartial* part, int nparts, int stride, int nsteps,
                       int64_t first_step, sw2d_red* ring, int ring_cap, double cell_area,
                       double h_sum, hipStream_t s);
// Validation + packing, then sum_wet H; scratch holds kHsumBlocks doubles.
// The paper-shaped split: dyn, shapiro, velocity update, then a fold over the new state
// into part[0..nparts). scratch holds 3 nx ny floats.
hipError_t launch_unfused_step(const float* eta, const float* u, const float* v, const float* hp, float* eta_o,
                               float* u_o, float* v_o, float* scratch, int nx, int ny, const StepCoef& k,
                               FoldPartial* part, int nparts, hipStream_t s);
hipError_t launch_prep(const float* H, const uint8_t* mask, const float* eta, const float* u,
                       const float* v, int nx, int ny, float* hp, PrepFlags* flags,
                       double* scratch, hipStream_t s, bool allow_dry = false);

namespace detail {
// Shared by the single-grid and batched C ABI (defined in sw2d_api.hip).
bool params_valid(const sw2d_params* p);
StepCoef make_coef(const sw2d_params* p);
void set_hip_message(const char* msg);
}  // namespace detail

}  // namespace sw2d
