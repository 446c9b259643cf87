// sw2d_surrogate_api.hip - C ABI of the surrogate's building blocks (argument checks and
// launches only; the training and rollout loops are sequenced by the caller).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "sw2d_internal.h"
#include "sw2d_handle.h"
#include "sw2d_surrogate.h"

using namespace sw2d;
using namespace sw2d::sur;

namespace {

int fail(hipError_t e, const char* what) {
    if (e == hipSuccess) return SW2D_OK;
    char msg[256];
    std::snprintf(msg, sizeof msg, "%s: %s", what, hipGetErrorString(e));
    sw2d::detail::set_hip_message(msg);
    return SW2D_EHIP;
}

bool dims_ok(int nimg, int ny, int nx) {
    return nimg >= 1 && ny >= 1 && nx >= 1 && (int64_t)nimg * ny * nx < ((int64_t)1 << 31);
}

bool aligned16(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

constexpr int kMseBlocks = 1024;
constexpr int kRmseBlocks = 1024;

// Staging of the network output for sw2d_surrogate_advance_noalloc: three FP32 planes of a
// coarse grid of at most SW2D_NOALLOC_MAX_CELLS cells. Each device holds its own copy at its
// own address; host code uses only the address hipGetSymbolAddress returns for a device,
// never the array's name (which on the host is a stand-in, not a device address).
static __device__ __align__(256) float scratch[3 * (size_t)SW2D_NOALLOC_MAX_CELLS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the device that owns stream s, looked up once per device
// with that device current.
int scratch_for_stream(hipStream_t s, float** out) {
    int dev = -1;
    hipError_t e = hipStreamGetDevice(s, &dev);
    if (e != hipSuccess) return fail(e, "sw2d_surrogate_advance_noalloc: hipStreamGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return SW2D_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = -1;
        e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void* ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return fail(e, "sw2d_surrogate_advance_noalloc: hipGetSymbolAddress");
        if (!ptr) return SW2D_EHIP;
        g_scratch_dev[dev] = static_cast<float*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return SW2D_OK;
}

// n corrected coarse steps with the network output staged in `delta` (3 planes of the grid).
int advance_corrected(sw2d_t coarse, hipStream_t s, int nx, int ny, int32_t nsteps, const float* H,
                      const uint8_t* mask, const float* mean, const float* std_, const uint16_t* const* wk,
                      const float* const* bias, const float* t_std, float* delta) {
    for (int32_t n = 0; n < nsteps; ++n) {
        float *e, *u, *v;
        int rc = sw2d_state(coarse, &e, &u, &v);
        if (rc == SW2D_OK) rc = sw2d_cnn_forward(e, u, v, H, mask, nx, ny, mean, std_, wk, bias, delta, s);
        if (rc == SW2D_OK) rc = sw2d_step(coarse, 1);
        if (rc == SW2D_OK) rc = sw2d_state(coarse, &e, &u, &v);
        if (rc == SW2D_OK) rc = fail(launch_correct(e, u, v, delta, mask, ny, nx, t_std, s), "sw2d_surrogate_advance");
        if (rc != SW2D_OK) return rc;
    }
    return SW2D_OK;
}

}  // namespace

extern "C" {

int sw2d_restrict4(const float* eta, const float* u, const float* v, const float* H, const uint8_t* mask,
                   int32_t nx_fine, int32_t ny_fine, float* eta_c, float* u_c, float* v_c, float* H_c,
                   uint8_t* mask_c, void* stream) {
    if (!eta || !u || !v || !H || !mask || !eta_c || !u_c || !v_c || !H_c || !mask_c) return SW2D_EINVAL;
    if (nx_fine < 4 || ny_fine < 4 || nx_fine % 4 || ny_fine % 4 || !dims_ok(1, ny_fine, nx_fine))
        return SW2D_EINVAL;
    return fail(launch_restrict4(eta, u, v, H, mask, nx_fine, ny_fine, eta_c, u_c, v_c, H_c, mask_c,
                                 static_cast<hipStream_t>(stream)),
                "sw2d_restrict4");
}

int sw2d_pack_input(const float* eta, const float* u, const float* v, const float* H, const uint8_t* mask,
                    int32_t nx, int32_t ny, const float* mean, const float* std_, float noise_amp, uint64_t noise_seed,
                    uint16_t* out, void* stream) {
    if (!eta || !u || !v || !H || !mask || !mean || !std_ || !out || !aligned16(out)) return SW2D_EINVAL;
    if (!dims_ok(1, ny, nx) || !(noise_amp >= 0.f) || !std::isfinite(noise_amp)) return SW2D_EINVAL;
    InputNorm nrm;
    nrm.noise_amp = noise_amp;
    nrm.noise_seed = noise_seed;
    for (int c = 0; c < 5; ++c) {
        if (!(std_[c] > 0.f) || !std::isfinite(mean[c])) return SW2D_EINVAL;
        nrm.mean[c] = mean[c];
        nrm.inv_std[c] = 1.f / std_[c];
    }
    return fail(launch_pack_input(eta, u, v, H, mask, nx * ny, nrm, out, static_cast<hipStream_t>(stream)),
                "sw2d_pack_input");
}

int sw2d_conv3x3_fwd(const uint16_t* in, int32_t cin, const uint16_t* wk, const float* bias, int32_t relu,
                     void* out, int32_t nimg, int32_t ny, int32_t nx, void* stream) {
    if (!in || !wk || !bias || !out || !aligned16(in) || !aligned16(wk) || !aligned16(out)) return SW2D_EINVAL;
    if ((cin != 16 && cin != 32) || !dims_ok(nimg, ny, nx)) return SW2D_EINVAL;
    if (!relu && cin != 32) return SW2D_EINVAL;
    const int mode = relu ? kConvRelu : kConvLinear3;
    return fail(launch_conv3x3(cin, mode, in, wk, bias, relu ? static_cast<uint16_t*>(out) : nullptr,
                               relu ? nullptr : static_cast<float*>(out), nullptr, nimg, ny, nx,
                               static_cast<hipStream_t>(stream)),
                "sw2d_conv3x3_fwd");
}

int sw2d_conv3x3_fwd_raw(const float* eta, const float* u, const float* v, const float* H, const uint8_t* mask,
                         int32_t nx, int32_t ny, const float* mean, const float* std_, const uint16_t* wk,
                         const float* bias, uint16_t* out, void* stream) {
    if (!eta || !u || !v || !H || !mask || !mean || !std_ || !wk || !bias || !out || !aligned16(wk) ||
        !aligned16(out))
        return SW2D_EINVAL;
    if (!dims_ok(1, ny, nx)) return SW2D_EINVAL;
    InputNorm nrm;
    nrm.noise_amp = 0.f;
    nrm.noise_seed = 0;
    for (int c = 0; c < 5; ++c) {
        if (!(std_[c] > 0.f) || !std::isfinite(mean[c])) return SW2D_EINVAL;
        nrm.mean[c] = mean[c];
        nrm.inv_std[c] = 1.f / std_[c];
    }
    return fail(launch_conv3x3_raw(RawIn{eta, u, v, H, mask}, nrm, wk, bias, out, ny, nx,
                                   static_cast<hipStream_t>(stream)),
                "sw2d_conv3x3_fwd_raw");
}

int sw2d_cnn_forward(const float* eta, const float* u, const float* v, const float* H, const uint8_t* mask,
                     int32_t nx, int32_t ny, const float* mean, const float* std_, const uint16_t* const* wk,
                     const float* const* bias, float* out, void* stream) {
    if (!eta || !u || !v || !H || !mask || !mean || !std_ || !wk || !bias || !out) return SW2D_EINVAL;
    if (!dims_ok(1, ny, nx)) return SW2D_EINVAL;
    FusedNet net;
    for (int l = 0; l < 4; ++l) {
        if (!wk[l] || !bias[l] || !aligned16(wk[l]) || !aligned16(bias[l])) return SW2D_EINVAL;
        net.wk[l] = wk[l];
        net.bias[l] = bias[l];
    }
    InputNorm nrm;
    nrm.noise_amp = 0.f;
    nrm.noise_seed = 0;
    for (int c = 0; c < 5; ++c) {
        if (!(std_[c] > 0.f) || !std::isfinite(mean[c])) return SW2D_EINVAL;
        nrm.mean[c] = mean[c];
        nrm.inv_std[c] = 1.f / std_[c];
    }
    return fail(launch_cnn_fused(RawIn{eta, u, v, H, mask}, nrm, net, out, ny, nx, static_cast<hipStream_t>(stream)),
                "sw2d_cnn_forward");
}

int sw2d_surrogate_advance(sw2d_t coarse, int32_t nsteps, const float* H, const uint8_t* mask, const float* mean,
                           const float* std_, const uint16_t* const* wk, const float* const* bias, const float* t_std,
                           float* delta) {
    hipStream_t s = nullptr;
    int nx = 0, ny = 0;
    if (!sw2d::detail::handle_info(coarse, &s, &nx, &ny) || nsteps < 0) return SW2D_ESTATE;
    if (!H || !mask || !mean || !std_ || !wk || !bias || !t_std || !delta) return SW2D_EINVAL;
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(t_std[c])) return SW2D_EINVAL;
    return advance_corrected(coarse, s, nx, ny, nsteps, H, mask, mean, std_, wk, bias, t_std, delta);
}

int sw2d_surrogate_advance_noalloc(sw2d_t coarse, int32_t nsteps, const float* H, const uint8_t* mask,
                                   const float* mean, const float* std_, const uint16_t* const* wk,
                                   const float* const* bias, const float* t_std) {
    hipStream_t s = nullptr;
    int nx = 0, ny = 0;
    if (!sw2d::detail::handle_info(coarse, &s, &nx, &ny) || nsteps < 0) return SW2D_ESTATE;
    if (!H || !mask || !mean || !std_ || !wk || !bias || !t_std) return SW2D_EINVAL;
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(t_std[c])) return SW2D_EINVAL;
    if ((int64_t)nx * ny > SW2D_NOALLOC_MAX_CELLS) return SW2D_ENOSPC;
    float* delta = nullptr;
    const int rc = scratch_for_stream(s, &delta);
    if (rc != SW2D_OK) return rc;
    return advance_corrected(coarse, s, nx, ny, nsteps, H, mask, mean, std_, wk, bias, t_std, delta);
}

int sw2d_conv3x3_correct(const uint16_t* in, const uint16_t* wk, const float* bias, const float* t_std,
                         const uint8_t* mask, float* eta, float* u, float* v, int32_t nx, int32_t ny, void* stream) {
    if (!in || !wk || !bias || !t_std || !mask || !eta || !u || !v || !aligned16(in) || !aligned16(wk))
        return SW2D_EINVAL;
    if (!dims_ok(1, ny, nx)) return SW2D_EINVAL;
    const CorrectOut co{eta, u, v, mask, t_std[0], t_std[1], t_std[2]};
    return fail(launch_conv3x3_correct(in, wk, bias, co, ny, nx, static_cast<hipStream_t>(stream)),
                "sw2d_conv3x3_correct");
}

int sw2d_conv3x3_dgrad(const uint16_t* dy, const uint16_t* wd, const uint16_t* act_in, uint16_t* dx, int32_t nimg,
                       int32_t ny, int32_t nx, void* stream) {
    if (!dy || !wd || !act_in || !dx || !aligned16(dy) || !aligned16(wd) || !aligned16(dx) || !aligned16(act_in))
        return SW2D_EINVAL;
    if (!dims_ok(nimg, ny, nx)) return SW2D_EINVAL;
    return fail(launch_conv3x3(32, kConvDgradMask, dy, wd, nullptr, dx, nullptr, act_in, nimg, ny, nx,
                               static_cast<hipStream_t>(stream)),
                "sw2d_conv3x3_dgrad");
}

size_t sw2d_wgrad_workspace_bytes(int32_t cin, int32_t nimg, int32_t ny, int32_t nx) {
    if ((cin != 16 && cin != 32) || !dims_ok(nimg, ny, nx)) return 0;
    const size_t chunks = (size_t)wgrad_chunks(nimg, ny, nx);
    return chunks * (9 * 32 * (size_t)cin + 32) * sizeof(float);
}

int sw2d_conv3x3_wgrad(const uint16_t* x, int32_t cin, const uint16_t* dy, int32_t nimg, int32_t ny, int32_t nx,
                       float* dW, float* db, void* work, size_t work_bytes, void* stream) {
    if (!x || !dy || !dW || !db || !work || !aligned16(x) || !aligned16(dy) || !aligned16(work)) return SW2D_EINVAL;
    const size_t need = sw2d_wgrad_workspace_bytes(cin, nimg, ny, nx);
    if (need == 0) return SW2D_EINVAL;
    if (work_bytes < need) return SW2D_ENOSPC;
    const size_t chunks = (size_t)wgrad_chunks(nimg, ny, nx);
    float* part_w = static_cast<float*>(work);
    float* part_b = part_w + chunks * 9 * 32 * cin;
    return fail(launch_wgrad(cin, x, dy, nimg, ny, nx, part_w, part_b, dW, db, static_cast<hipStream_t>(stream)),
                "sw2d_conv3x3_wgrad");
}

size_t sw2d_mse_workspace_bytes(void) { return kMseBlocks * sizeof(double); }

int sw2d_mse_grad(const float* out, const float* target, const float* target_scale, const uint8_t* mask,
                  int32_t nimg, int32_t ny, int32_t nx, float inv_n, uint16_t* d_out, double* loss_sum, void* work,
                  size_t work_bytes, void* stream) {
    if (!out || !target || !target_scale || !mask || !d_out || !loss_sum || !work || !aligned16(d_out))
        return SW2D_EINVAL;
    if (!dims_ok(nimg, ny, nx) || !(inv_n >= 0.f) || !std::isfinite(inv_n)) return SW2D_EINVAL;
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(target_scale[c])) return SW2D_EINVAL;
    if (work_bytes < sw2d_mse_workspace_bytes()) return SW2D_ENOSPC;
    return fail(launch_mse_grad(out, target, mask, nimg, ny, nx, inv_n, target_scale, d_out,
                                static_cast<double*>(work), kMseBlocks, loss_sum, static_cast<hipStream_t>(stream)),
                "sw2d_mse_grad");
}

int sw2d_sub3(const float* a0, const float* a1, const float* a2, const float* b0, const float* b1, const float* b2,
              int32_t n, float* out, void* stream) {
    if (!a0 || !a1 || !a2 || !b0 || !b1 || !b2 || !out || n < 1) return SW2D_EINVAL;
    return fail(launch_sub3(a0, a1, a2, b0, b1, b2, n, out, static_cast<hipStream_t>(stream)), "sw2d_sub3");
}

size_t sw2d_moments_workspace_bytes(void) { return 2 * kRmseBlocks * sizeof(double); }

int sw2d_moments(const float* x, const uint8_t* mask, int64_t n, double* out2, void* work, size_t work_bytes,
                 void* stream) {
    if (!x || !out2 || !work || n < 1) return SW2D_EINVAL;
    if (work_bytes < sw2d_moments_workspace_bytes()) return SW2D_ENOSPC;
    return fail(launch_moments(x, mask, n, static_cast<double*>(work), kRmseBlocks, out2,
                               static_cast<hipStream_t>(stream)),
                "sw2d_moments");
}

int sw2d_adam(float* theta, const float* grad, float* m, float* v, int32_t n, int32_t t, float lr, float beta1,
              float beta2, float eps, void* stream) {
    if (!theta || !grad || !m || !v || n < 1 || t < 1) return SW2D_EINVAL;
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) || !(lr >= 0.f))
        return SW2D_EINVAL;
    AdamHyper hp;
    hp.lr = lr;
    hp.beta1 = beta1;
    hp.beta2 = beta2;
    hp.eps = eps;
    hp.inv_bc1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)t)));
    hp.inv_bc2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)t)));
    return fail(launch_adam(theta, grad, m, v, n, hp, static_cast<hipStream_t>(stream)), "sw2d_adam");
}

int sw2d_cast_weights(const float* master, int32_t cin, uint16_t* wk, uint16_t* wd, void* stream) {
    if (!master || !wk || (cin != 16 && cin != 32)) return SW2D_EINVAL;
    if (wd && cin != 32) return SW2D_EINVAL;  // data gradients exist for 32-channel inputs only
    return fail(launch_cast_weights(master, cin, 32, wk, wd, static_cast<hipStream_t>(stream)), "sw2d_cast_weights");
}

int sw2d_apply_correction(float* eta, float* u, float* v, const float* out, const uint8_t* mask, int32_t nx,
                          int32_t ny, const float* t_std, void* stream) {
    if (!eta || !u || !v || !out || !mask || !t_std || !dims_ok(1, ny, nx)) return SW2D_EINVAL;
    return fail(launch_correct(eta, u, v, out, mask, ny, nx, t_std, static_cast<hipStream_t>(stream)),
                "sw2d_apply_correction");
}

size_t sw2d_rmse_workspace_bytes(void) { return kRmseBlocks * sizeof(double); }

int sw2d_rmse(const float* a, const float* b, const uint8_t* mask, int32_t n, double* sum_sq, void* work,
              size_t work_bytes, void* stream) {
    if (!a || !b || !mask || !sum_sq || !work || n < 1) return SW2D_EINVAL;
    if (work_bytes < sw2d_rmse_workspace_bytes()) return SW2D_ENOSPC;
    return fail(launch_sqdiff(a, b, mask, n, static_cast<double*>(work), kRmseBlocks, sum_sq,
                              static_cast<hipStream_t>(stream)),
                "sw2d_rmse");
}

}  // extern "C"
