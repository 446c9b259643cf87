/*
 * sw2d.h - C ABI of the MI355X (gfx950) 2-D shallow-water (2DSW) step library.
 *
 * The model is the one of the paper's first auto-parallelisation test case
 * (Sect. 6.2, "Test Case 1: 2-D Shallow Water Model"): a time loop that calls a
 * predictor ("dyn"), then a first-order Shapiro filter ("shapiro"), then updates
 * the velocity; the paper's compiler turns its loop nests into maps and its
 * reductions into folds (Sect. 4.3) and keeps the data on the accelerator for the
 * whole run, copying only once (Sect. 4.3, last paragraph). The paper prints no
 * equations; this library implements the standard explicit Arakawa C-grid reading:
 *
 *   us  = a_u (u - g dt/dx (eta_E - eta))            a_u: both cells of the face wet
 *   vs  = a_v (v - g dt/dy (eta_N - eta))
 *   Fx  = us * (us > 0 ? H + eta : H_E + eta_E)        upwind total depth, old surface
 *   es  = wet (eta - dt/dx (Fx - Fx_W) - dt/dy (Fy - Fy_S))
 *   eta'= wet (es + eps/4 * sum over wet neighbours (es_nb - es))
 *   u'  = us, v' = vs
 *
 * and after every step the folds V_tot = dx dy sum_wet (H + eta'),
 * V_disp = dx dy sum_wet eta' (both accumulated in double), max|u'| and max|v'|.
 *
 * Layout: every field is a row-major [ny][nx] float32 array (i runs east along a
 * row, j runs north). u[j][i] sits on the east face of cell (j,i), v[j][i] on its
 * north face, so u[.][nx-1] and v[ny-1][.] are always zero. mask[j][i] != 0 means
 * water. The outermost ring of cells must be land (closed basin).
 *
 * Ownership: the caller owns every device buffer (state, depth, mask, workspace)
 * and the HIP stream; they must outlive the handle. The library owns only its
 * host-side handle and never allocates device memory; the one fixed device array it
 * holds is the staging buffer of sw2d_surrogate_advance_noalloc.
 *
 * Errors: every call returns an int status (SW2D_OK or a negative code below);
 * nothing throws or aborts across the ABI. Work is enqueued asynchronously on the
 * caller's stream; an asynchronous HIP error surfaces at a later call or at
 * sw2d_reduce, which synchronises the stream. A handle is not thread-safe.
 */
#ifndef SW2D_H
#define SW2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SW2D_OK = 0,
    SW2D_EINVAL = -1,    /* bad sizes/constants, wet border cell, bad depth, CFL > 1 */
    SW2D_EHIP = -2,      /* a HIP runtime call failed; see sw2d_strerror / sw2d_last_hip_error */
    SW2D_EUNSTABLE = -3, /* a fold came back non-finite: the run has blown up */
    SW2D_ESTATE = -4,    /* handle misuse (NULL handle, bad k, ...) */
    SW2D_ENOSPC = -5     /* workspace smaller than sw2d_workspace_bytes(), or a grid larger
                            than a fixed library array holds */
};

/* Model variants (flags of sw2d_params; the paper's model has neither - they are the
 * textbook family's options either side of it):
 *  SW2D_FRICTION:  quadratic bottom friction on the predictor,
 *                  us = (u - g dt/dx (eta_E - eta)) / (1 + dt cd |u| / h_face),
 *                  h_face = mean total depth (H + eta) of the face's two cells, |u| and the
 *                  depths of the old state; vs likewise.
 *  SW2D_FILTER_UV: the velocity update applies the Shapiro filter to the predicted
 *                  velocities as well: u' = us + eps/4 sum over active neighbouring u faces
 *                  (east, west, north, south) of (us_nb - us); v' likewise. The surface update
 *                  of the step uses the unfiltered us, vs.
 *  SW2D_ADVECTION: nonlinear momentum advection, first-order upwind, in the predictor:
 *                  us -= dt (u du/dx + vbar du/dy), vs -= dt (ubar dv/dx + v dv/dy), each
 *                  derivative a one-sided difference on the upstream side of its advecting
 *                  velocity (u > 0: backward), vbar the mean of the four v faces around the
 *                  u face, ubar likewise; faces off the grid or inactive count as 0. Applied
 *                  before the friction division.
 *  SW2D_WETDRY:    wetting and drying. A water cell is wet while its total depth H + eta
 *                  exceeds hmin (the old surface decides, once per step). A face between two
 *                  water cells carries flow when both are wet, or when one is wet and its
 *                  surface stands above the other's (the pressure gradient pushes water into
 *                  the dry cell); otherwise us (vs) = 0. Every water cell takes the flux
 *                  divergence; the Shapiro filter acts on wet cells across wet neighbours only,
 *                  and a dry cell keeps its predicted surface. H > 0 on water cells still
 *                  holds: H is the depth below the datum, which may sit above the still-water
 *                  level, so ground that can flood is a water cell whose surface starts at
 *                  eta = -H (zero total depth). Taken alone (no other flag).
 * A handle with SW2D_ADVECTION steps one step per pass (sw2d_set_time_blocking refuses
 * K > 1: its upwind differences reach one face further per step); every other combination
 * may take K steps per pass. The batched and unfused paths take flags = 0 only. */
#define SW2D_FRICTION 1u
#define SW2D_FILTER_UV 2u
#define SW2D_ADVECTION 4u
#define SW2D_WETDRY 8u

/* Grid and constants. nx, ny count every cell, land border included (>= 3 each), with
 * nx * ny <= 2^31 and nx <= 2^28 (a row is addressed with 32-bit byte offsets).
 * dx, dy, dt > 0 and finite; g >= 0 and finite; eps in [0, 1] (Shapiro weight);
 * flags: 0, a combination of SW2D_FRICTION, SW2D_FILTER_UV, SW2D_ADVECTION, or SW2D_WETDRY
 * alone; cd >= 0 and finite, the bottom-drag coefficient (used with SW2D_FRICTION, ignored
 * otherwise); hmin >= 0 and finite, the wet threshold on the total depth [m] (used with
 * SW2D_WETDRY, ignored otherwise; the kernels compare in FP32). */
typedef struct {
    int32_t nx, ny;
    double dx, dy, g, dt, eps;
    uint32_t flags;
    double cd;
    double hmin;
} sw2d_params;

/* The folds of the state after one step (32 bytes; the device writes this layout). */
typedef struct {
    int64_t step;      /* 1-based index of the step this entry follows */
    double vol_total;  /* dx dy sum_wet (H + eta) [m^3] */
    double vol_disp;   /* dx dy sum_wet eta        [m^3] */
    float max_abs_u;   /* max over all faces of |u| [m/s] */
    float max_abs_v;   /* max over all faces of |v| [m/s] */
} sw2d_red;

typedef struct sw2d_ctx *sw2d_t;

/* Device workspace (bytes) a handle needs for these params: the packed depth field,
 * per-workgroup fold partials, the fold ring and a few flags. 0 if params are bad. */
size_t sw2d_workspace_bytes(const sw2d_params *p);

/* Number of past steps whose folds sw2d_reduce can still return. */
int32_t sw2d_ring_capacity(void);

/* Validate and bind a problem. d_H (float32 [ny][nx], depth below the rest level,
 * ignored on land), d_mask (uint8 [ny][nx]) are read once; d_state holds 6*nx*ny
 * float32 = two (eta, u, v) buffers, buffer 0 holding the initial state; d_work is
 * the workspace. Checks (SW2D_EINVAL): sizes/constants; border cells must be land;
 * at least one cell must be water (an all-land grid has nothing to step); water cells
 * need finite H > 0 and H + eta > 0 (H + eta >= 0 with SW2D_WETDRY); the initial state
 * must be finite;
 * the Courant number dt sqrt(g H_max) sqrt(1/dx^2 + 1/dy^2) must not exceed 1.
 * Synchronises the stream once. On success *out is a new handle. */
int sw2d_create(const sw2d_params *p, const float *d_H, const uint8_t *d_mask, float *d_state,
                void *d_work, size_t work_bytes, void *hip_stream, sw2d_t *out);

/* Enqueue nsteps >= 0 time steps (and their folds) on the handle's stream. No host
 * synchronisation, no host-device copy. */
int sw2d_step(sw2d_t h, int32_t nsteps);

/* Benchmark form of sw2d_step: the same launches, with a HIP event pair recorded on the
 * handle's stream around every step kernel. Synchronises the stream and writes the mean
 * duration of one step kernel in milliseconds to *mean_step_ms. */
int sw2d_step_timed(sw2d_t h, int32_t nsteps, double *mean_step_ms);

/* Copy the folds of the last k steps (oldest first) into host_out[0..k-1]; k must be
 * in [1, min(steps done, sw2d_ring_capacity())]. Synchronises the stream. Returns
 * SW2D_EUNSTABLE (entries still written) when any returned fold is non-finite. */
int sw2d_reduce(sw2d_t h, sw2d_red *host_out, int32_t k);

/* Device pointers of the current (eta, u, v) buffers inside d_state. Valid until the
 * next sw2d_step / sw2d_set_state on this handle. */
int sw2d_state(sw2d_t h, float **d_eta, float **d_u, float **d_v);

/* Steps done so far (the restart counter). */
int64_t sw2d_steps_done(sw2d_t h);

/* Overwrite the current state with device arrays (float32 [ny][nx] each; they may be
 * the current buffers themselves) and set the step counter. Enqueued on the stream. */
int sw2d_set_state(sw2d_t h, const float *d_eta, const float *d_u, const float *d_v, int64_t step);

/* Band height (rows per workgroup) of the fused step, 8 (or ny if smaller) by default. Any
 * value in [8, ny] gives the same state bit for bit; it changes speed, and the grouping (not
 * the value) of fold sums. */
int sw2d_set_band_rows(sw2d_t h, int32_t rows);
int32_t sw2d_band_rows(sw2d_t h);

/* Temporal blocking: steps_per_pass = K in 2..4 makes sw2d_step advance K steps per pass
 * over HBM (the intermediate states stay in registers; a remainder of the step count takes
 * one shorter pass), with its own band height rows in [8, ny]; 1 (the default) restores one
 * step per pass. The state and folds are the same as with single steps (the state bit for
 * bit, the folds up to the order of their sums). SW2D_EINVAL for K or rows out of range, or
 * K > 1 on a handle with SW2D_ADVECTION. */
int sw2d_set_time_blocking(sw2d_t h, int32_t steps_per_pass, int32_t rows);
int32_t sw2d_time_blocking(sw2d_t h);

/* The same steps split the way the paper's compiler splits them (Sect. 6.2: three map
 * kernels - the predictor, the Shapiro filter, the velocity update - with the folds as a
 * separate reduction), for comparison with the fused pass: 68 B of HBM traffic per
 * cell-step instead of 28. d_scratch: caller-owned device memory of
 * sw2d_unfused_scratch_bytes(p) bytes (the predicted u, v and surface). The state agrees
 * with sw2d_step to FP32 rounding. */
size_t sw2d_unfused_scratch_bytes(const sw2d_params *p);
int sw2d_step_unfused(sw2d_t h, int32_t nsteps, float *d_scratch, size_t scratch_bytes);

/* ---------------------------------------------------------------------------------------
 * Red-black SOR for the pressure Poisson equation (the paper's second workload, Sect. 6.3:
 * its pressure solver, successive over-relaxation, 50 iterations on 300 x 300 x 90).
 *
 * Arrays are [nz][ny][nx] row-major FP32 device memory; the outermost layer of cells holds
 * fixed (Dirichlet) values that are read, never written. The equation on interior cells is
 * cx (pE + pW - 2p) + cy (pN + pS - 2p) + cz (pU + pD - 2p) = f, c_ = 1 / spacing^2. One
 * iteration updates every red cell ((i + j + k) even), then every black one, to
 * p + omega (g - p) with the Gauss-Seidel value g = (cx (pE + pW) + cy (pN + pS) +
 * cz (pU + pD) - f) / (2 (cx + cy + cz)).
 * ------------------------------------------------------------------------------------- */
typedef struct {
    int32_t nx, ny, nz; /* cells incl. the boundary layer, each >= 3, product < 2^31 */
    double dx, dy, dz;  /* spacings > 0 */
    double omega;       /* relaxation factor, 0 < omega < 2 */
    int32_t fused;      /* 0: a red sweep then a black sweep per iteration; 1: one pass per
                           iteration (new red values of a tile and its one-cell ring in on-chip
                           memory, ping-pong arrays); the same state bit for bit, residual sums
                           to rounding order */
} sw2d_sor_params;

/* Residual r = f - L p of the state after `iter` iterations (iter 0 = the initial state):
 * sum over interior cells of r^2 (FP64, fixed summation order) and max |r|. 16 bytes. */
typedef struct {
    int32_t iter;
    float max_abs_r;
    double sum_r2;
} sw2d_sor_res;

/* Device workspace for sw2d_sor_run with `iters` iterations (residual partials); 0 for
 * invalid parameters. */
size_t sw2d_sor_workspace_bytes(const sw2d_sor_params *p, int32_t iters);

/* Run `iters` iterations on d_p in place (asynchronous on `stream`, a hipStream_t or NULL).
 * d_f: the right-hand side (its boundary layer is not read). d_res: NULL, or device memory
 * for iters + 1 sw2d_sor_res entries, the residual after 0, 1, ..., iters iterations.
 * d_work: caller-owned device memory of sw2d_sor_workspace_bytes(p, iters) bytes. All
 * buffers stay the caller's. Returns SW2D_EINVAL for invalid parameters or NULL arrays,
 * SW2D_ENOSPC for a short workspace, SW2D_EHIP for a launch error. Deterministic: the same
 * inputs give the same bits. */
int sw2d_sor_run(const sw2d_sor_params *p, float *d_p, const float *d_f, int32_t iters, sw2d_sor_res *d_res,
                 void *d_work, size_t work_bytes, void *stream);

/* Release the host handle. Device buffers stay the caller's. NULL is accepted. */
int sw2d_destroy(sw2d_t h);

/* Static text for a status code. */
const char *sw2d_strerror(int code);

/* Text of the last HIP error seen by this library on the calling thread ("" if none). */
const char *sw2d_last_hip_error(void);

/* ---------------------------------------------------------------------------------------
 * Batched ensembles: n independent basins of any sizes advanced together by one
 * persistent launch per chunk of steps (a grid barrier between steps), the launch
 * sequence recorded once in a HIP graph and replayed. Each instance runs the same tile
 * routine as sw2d_step, so its state is bitwise equal to the same basin stepped alone;
 * its folds are equal up to the order of the sums. This is the same time loop
 * (Sect. 6.2) applied to many problems at once; the paper itself runs one grid at a time.
 * ------------------------------------------------------------------------------------ */
typedef struct sw2d_bctx *sw2d_batch_t;

/* Workspace bytes for n instances with params p[0..n-1] and band heights band_rows
 * (rows per work item, >= 8, one per instance; NULL = 16). 0 if any argument is bad. */
size_t sw2d_batch_workspace_bytes(int32_t n, const sw2d_params *p, const int32_t *band_rows);

/* Validate and bind n instances. Instance i has its own d_H[i], d_mask[i] and d_state[i]
 * (6*nx*ny float32: two (eta, u, v) buffers, buffer 0 holding its initial state), all laid
 * out as for sw2d_create and checked the same way (SW2D_EINVAL names no instance; the
 * caller can create instances alone to find it). Arrays of pointers are read during the
 * call only. Synchronises the stream. The library creates one private HIP stream per
 * handle, used only to record graphs. */
int sw2d_batch_create(int32_t n, const sw2d_params *p, const float *const *d_H,
                      const uint8_t *const *d_mask, float *const *d_state, const int32_t *band_rows,
                      void *d_work, size_t work_bytes, void *hip_stream, sw2d_batch_t *out);

/* Launch shape: steps per persistent launch (>= 1, default 50), whether sw2d_batch_step
 * records and replays a HIP graph (default 1), and the persistent grid size in
 * workgroups (0 = the most the device holds at once; larger values are rejected so the
 * grid barrier always has every workgroup resident). Drops any recorded graph. */
int sw2d_batch_set_launch(sw2d_batch_t b, int32_t steps_per_launch, int32_t use_graph, int32_t grid);

/* Steps per pass of the batched kernel (temporal blocking as sw2d_set_time_blocking): 1
 * (default), 2 or 3. Each member's strips then own 64 - 4K columns and its bands read a
 * 2K-row halo; the grid meets once per pass; the states equal single steps bit for bit and
 * the folds of every step are kept. Afterwards sw2d_batch_step takes multiples of K only.
 * Synchronises the stream, rebuilds the tile list, drops a recorded graph, and lowers the
 * grid to what the K-step kernel keeps resident. SW2D_EINVAL for K outside 1..3. */
int sw2d_batch_set_time_blocking(sw2d_batch_t b, int32_t steps_per_pass);
int32_t sw2d_batch_time_blocking(sw2d_batch_t b);

/* Enqueue nsteps steps of every instance on the stream (no host synchronisation). With
 * graphs on, the first call for a given nsteps records the graph; later calls with the
 * same nsteps replay it. */
int sw2d_batch_step(sw2d_batch_t b, int32_t nsteps);

/* sw2d_batch_step bracketed by HIP events on the stream; synchronises and writes the mean
 * wall time per step (ms) of the whole enqueued sequence. */
int sw2d_batch_step_timed(sw2d_batch_t b, int32_t nsteps, double *ms_per_step);

/* Folds of the last step of every instance into host_out[0..n-1]. Synchronises. Returns
 * SW2D_EHIP if a grid-barrier wait ran past its 2 s deadline (the kernel then stopped
 * early), SW2D_EUNSTABLE if a fold is non-finite. */
int sw2d_batch_reduce(sw2d_batch_t b, sw2d_red *host_out);

/* Current (eta, u, v) device buffers of instance k. */
int sw2d_batch_state(sw2d_batch_t b, int32_t k, float **d_eta, float **d_u, float **d_v);

int64_t sw2d_batch_steps_done(sw2d_batch_t b);

/* Deadline of one grid-barrier wait (default 2 s, at most 60 s). A wait past it sets the
 * error that sw2d_batch_reduce reports and makes every workgroup return; the tests use a
 * zero deadline to exercise that path. Drops any recorded graph. */
int sw2d_batch_set_barrier_timeout(sw2d_batch_t b, double seconds);

/* Persistent grid size in workgroups (256 threads each). */
int32_t sw2d_batch_grid(sw2d_batch_t b);

/* Release the handle, its graph and its private stream. NULL is accepted. */
int sw2d_batch_destroy(sw2d_batch_t b);

/* ---------------------------------------------------------------------------------------
 * Learned coarse-step surrogate: building blocks. The surrogate advances a 4x-coarsened
 * state with the same step on the coarse grid (sw2d_create/sw2d_step with 4 dx, 4 dt) and
 * adds a correction from a convolutional network: 3x3 'same' (zero padding) convolutions
 * 5 -> 32 -> 32 -> 32 -> 3, ReLU after the first three, BF16 weights and activations with
 * FP32 accumulation on the matrix cores. The plain fine model stays the judge and the
 * fallback. The training and rollout loops are sequenced by the caller.
 *
 * Feature maps are NHWC BF16 (uint16_t bit patterns) with C = 16 (the network input: the 5
 * normalised channels eta, u, v, H, mask, then zeros) or C = 32, a pixel's channels
 * contiguous: element (n, y, x, c) at ((n*ny + y)*nx + x)*C + c. The network output and
 * its targets are FP32 planes [n][3][ny][nx]. Weights of a layer with cin inputs are the
 * FP32 master [9][32][cin] (tap t = 3*ky + kx, then output channel, then input channel;
 * the last layer uses output rows 0..2 only, the rest stay zero) and its BF16 copies.
 * All pointers are device pointers; feature maps and weights need 16 B alignment. Every
 * call enqueues on `stream` and returns a status code; none synchronises.
 * ------------------------------------------------------------------------------------ */

/* 4x4 restriction of a fine state [ny_fine][nx_fine] (both multiples of 4) to the coarse
 * grid [ny_fine/4][nx_fine/4]: eta_c and H_c are means over the block's water cells, a
 * coarse cell is water when >= 8 of its 16 fine cells are, u_c (v_c) is the mean of the 4
 * fine u (v) on the coarse cell's east (north) face; land and inactive faces are 0. */
int sw2d_restrict4(const float *eta, const float *u, const float *v, const float *H, const uint8_t *mask,
                   int32_t nx_fine, int32_t ny_fine, float *eta_c, float *u_c, float *v_c, float *H_c,
                   uint8_t *mask_c, void *stream);

/* Network input: out[p][c] = bf16((x_c[p] - mean[c]) / std[c] + noise) for the channels
 * (eta, u, v, H, mask as 0/1), c = 0..4; channels 5..15 are 0. mean, std: host arrays of 5.
 * noise (training only; 0 when noise_amp = 0) is added to channels 0..2: noise_amp * U,
 * U uniform in [-1, 1) from SplitMix64 (Steele, Lea & Flood 2014): z = noise_seed +
 * (3 p + c + 1) * 0x9E3779B97F4A7C15, the SplitMix64 finaliser, U = (z >> 40) / 2^23 - 1. */
int sw2d_pack_input(const float *eta, const float *u, const float *v, const float *H, const uint8_t *mask,
                    int32_t nx, int32_t ny, const float *mean, const float *std_, float noise_amp,
                    uint64_t noise_seed, uint16_t *out, void *stream);

/* Forward 3x3 convolution of nimg images. relu = 1: cin in {16, 32}, out = BF16 NHWC with
 * 32 channels, bias then ReLU. relu = 0 (the last layer): cin = 32, out = FP32 planes
 * [nimg][3][ny][nx] of output channels 0..2 plus bias. wk: BF16 [9][32][cin]. */
int sw2d_conv3x3_fwd(const uint16_t *in, int32_t cin, const uint16_t *wk, const float *bias, int32_t relu,
                     void *out, int32_t nimg, int32_t ny, int32_t nx, void *stream);

/* The first layer (cin 16, bias, ReLU) of one image reading the raw coarse state: the
 * packing of sw2d_pack_input without noise is done while the input patch is staged, so the
 * packed input never goes to memory (inference). Same arguments as sw2d_pack_input (mean,
 * std: host arrays of 5) and sw2d_conv3x3_fwd; out: BF16 NHWC 32 channels. Bitwise equal to
 * sw2d_pack_input followed by sw2d_conv3x3_fwd. */
int sw2d_conv3x3_fwd_raw(const float *eta, const float *u, const float *v, const float *H, const uint8_t *mask,
                         int32_t nx, int32_t ny, const float *mean, const float *std_, const uint16_t *wk,
                         const float *bias, uint16_t *out, void *stream);

/* The whole network on one image in one pass (inference): the packing of the raw coarse
 * state, layers 1-3 (bias, ReLU) and layer 4 (channels 0..2 plus bias), with the
 * intermediate maps kept in on-chip memory. eta, u, v, H, mask, nx, ny, mean, std_: as
 * sw2d_conv3x3_fwd_raw; wk, bias: host arrays of 4 device pointers, wk[0] BF16 [9][32][16],
 * wk[1..3] BF16 [9][32][32], bias[l] FP32 [32], all 16 B aligned; out: FP32 planes
 * [3][ny][nx] (device). Bitwise equal to sw2d_pack_input (no noise), three sw2d_conv3x3_fwd
 * with relu = 1 and one with relu = 0. */
int sw2d_cnn_forward(const float *eta, const float *u, const float *v, const float *H, const uint8_t *mask,
                     int32_t nx, int32_t ny, const float *mean, const float *std_, const uint16_t *const *wk,
                     const float *const *bias, float *out, void *stream);

/* nsteps corrected coarse steps of the surrogate on a coarse-grid handle, all enqueued on the
 * handle's stream without host synchronisation: each step runs sw2d_cnn_forward on the
 * current state into delta (FP32 planes [3][ny][nx], device scratch of the caller), advances
 * the handle one step (sw2d_step) and adds the network's output to the new state as
 * sw2d_apply_correction does (t_std: host array of 3 scales). H, mask: the coarse grid's
 * depth and water mask (device); mean, std_, wk, bias: as sw2d_cnn_forward. The network sees
 * the state before the step and its output corrects the state after it. */
int sw2d_surrogate_advance(sw2d_t coarse, int32_t nsteps, const float *H, const uint8_t *mask, const float *mean,
                           const float *std_, const uint16_t *const *wk, const float *const *bias,
                           const float *t_std, float *delta);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sw2d_surrogate_advance without the delta
 * argument. The network output is staged in a fixed library array of 3 *
 * SW2D_NOALLOC_MAX_CELLS floats per device (24 MiB, taken when the library's code is loaded
 * on that device and held until the process ends), so the coarse grid may have at most
 * SW2D_NOALLOC_MAX_CELLS cells: a larger one returns SW2D_ENOSPC before anything is enqueued.
 * Every call on one device shares that array and the network overwrites every entry it later
 * reads, so no state carries over between calls; calls that overlap on one device (two
 * streams, two threads) race on it and must be serialised by the caller. Allocates nothing:
 * no hipMalloc, hipFree or allocating library routine (the first call on a device looks up
 * the array's device address once). Other arguments and errors as sw2d_surrogate_advance;
 * the resulting state is bitwise the same. */
#define SW2D_NOALLOC_MAX_CELLS 2097152
int sw2d_surrogate_advance_noalloc(sw2d_t coarse, int32_t nsteps, const float *H, const uint8_t *mask,
                                   const float *mean, const float *std_, const uint16_t *const *wk,
                                   const float *const *bias, const float *t_std);

/* The last layer (cin 32 -> channels 0..2 plus bias) of one image with its output added to
 * the state as sw2d_apply_correction does (t_std: host array of 3 scales), without the
 * output planes going to memory. Bitwise equal to sw2d_conv3x3_fwd (relu = 0) followed by
 * sw2d_apply_correction. */
int sw2d_conv3x3_correct(const uint16_t *in, const uint16_t *wk, const float *bias, const float *t_std,
                         const uint8_t *mask, float *eta, float *u, float *v, int32_t nx, int32_t ny,
                         void *stream);

/* Data gradient of a layer with 32 inputs: dx[p][c] = (act_in[p][c] > 0) *
 * sum_t sum_o dy[p - off_t][o] W[t][o][c], i.e. the gradient through the convolution and
 * through the ReLU that produced the layer input act_in. dy, act_in, dx: BF16 NHWC 32
 * channels; wd: BF16 [9][32][32] from sw2d_cast_weights (taps flipped, transposed). */
int sw2d_conv3x3_dgrad(const uint16_t *dy, const uint16_t *wd, const uint16_t *act_in, uint16_t *dx,
                       int32_t nimg, int32_t ny, int32_t nx, void *stream);

/* Weight gradient dW[t][o][c] = sum_p dy[p][o] x[p + off_t][c] and db[o] = sum_p dy[p][o]
 * (FP32 outputs [9][32][cin] and [32]), summed over pixel chunks in a fixed order. x: BF16
 * NHWC cin channels; dy: BF16 NHWC 32 channels. work: FP32 partials, sized by
 * sw2d_wgrad_workspace_bytes (0 for bad sizes). */
size_t sw2d_wgrad_workspace_bytes(int32_t cin, int32_t nimg, int32_t ny, int32_t nx);
int sw2d_conv3x3_wgrad(const uint16_t *x, int32_t cin, const uint16_t *dy, int32_t nimg, int32_t ny, int32_t nx,
                       float *dW, float *db, void *work, size_t work_bytes, void *stream);

/* Masked squared error: for each image and channel (eta on water cells, u on active east
 * faces, v on active north faces of mask), r = out - target_scale[c] * target; *loss_sum
 * (device double) = sum r^2 over active entries; d_out (BF16 NHWC 32 channels, 3..31
 * zero) = 2 r inv_n. target_scale: host array of 3. */
size_t sw2d_mse_workspace_bytes(void);
int sw2d_mse_grad(const float *out, const float *target, const float *target_scale, const uint8_t *mask,
                  int32_t nimg, int32_t ny, int32_t nx, float inv_n, uint16_t *d_out, double *loss_sum, void *work,
                  size_t work_bytes, void *stream);

/* Training targets: out[c][p] = a_c[p] - b_c[p] for c = 0, 1, 2 (out: FP32 [3][n]). */
int sw2d_sub3(const float *a0, const float *a1, const float *a2, const float *b0, const float *b1,
              const float *b2, int32_t n, float *out, void *stream);

/* out2[0] = sum x, out2[1] = sum x^2 (device doubles, fixed order) over the n entries with
 * mask != 0 (all entries if mask is NULL): the normalisation statistics. */
size_t sw2d_moments_workspace_bytes(void);
int sw2d_moments(const float *x, const uint8_t *mask, int64_t n, double *out2, void *work, size_t work_bytes,
                 void *stream);

/* Adam (Kingma & Ba) with bias correction on n FP32 parameters; t is the 1-based step. */
int sw2d_adam(float *theta, const float *grad, float *m, float *v, int32_t n, int32_t t, float lr, float beta1,
              float beta2, float eps, void *stream);

/* BF16 working copies of one layer's FP32 master [9][32][cin]: wk (same layout) and, when
 * wd is not NULL (cin = 32 only), the data-gradient layout wd[8 - t][c][o] = W[t][o][c]. */
int sw2d_cast_weights(const float *master, int32_t cin, uint16_t *wk, uint16_t *wd, void *stream);

/* state += t_std[c] * out[c] on active entries (eta: water cells, u/v: active faces). t_std:
 * host array of 3. */
int sw2d_apply_correction(float *eta, float *u, float *v, const float *out, const uint8_t *mask, int32_t nx,
                          int32_t ny, const float *t_std, void *stream);

/* *sum_sq (device double) = sum over mask != 0 of (a - b)^2, accumulated in double in a
 * fixed order (the RMSE of the judge is sqrt(sum_sq / count)). */
size_t sw2d_rmse_workspace_bytes(void);
int sw2d_rmse(const float *a, const float *b, const uint8_t *mask, int32_t n, double *sum_sq, void *work,
              size_t work_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SW2D_H */
