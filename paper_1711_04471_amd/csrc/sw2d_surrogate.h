// sw2d_surrogate.h - host-side launchers and shared types of the surrogate kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sw2d {
namespace sur {

enum : int { kConvRelu = 0, kConvLinear3 = 1, kConvDgradMask = 2, kConvCorrect = 3 };

struct InputNorm {
    float mean[5];
    float inv_std[5];
    float noise_amp;      // uniform noise in [-amp, amp) added to the normalised eta, u, v (training)
    uint64_t noise_seed;  // counter-based generator key
};

struct AdamHyper {
    float lr, beta1, beta2, eps;
    float inv_bc1, inv_bc2;  // 1 / (1 - beta^t), computed in double on the host
};

hipError_t launch_restrict4(const float* eta, const float* u, const float* v, const float* H,
                            const uint8_t* mask, int NX, int NY, float* eta_c, float* u_c, float* v_c,
                            float* H_c, uint8_t* mask_c, hipStream_t s);
hipError_t launch_pack_input(const float* eta, const float* u, const float* v, const float* H,
                             const uint8_t* mask, int npix, const InputNorm& nrm, uint16_t* out,
                             hipStream_t s);
// Raw state read by the first layer in place of a packed input (inference: no noise).
struct RawIn {
    const float* eta;
    const float* u;
    const float* v;
    const float* H;
    const uint8_t* mask;
};
// The last layer's output applied as the correction of the coarse state (mode kConvCorrect).
struct CorrectOut {
    float* eta;
    float* u;
    float* v;
    const uint8_t* mask;
    float s0, s1, s2;
};
// First layer (16 input channels, ReLU) with the packing of the raw state fused in.
hipError_t launch_conv3x3_raw(const RawIn& raw, const InputNorm& nrm, const uint16_t* Wk, const float* bias,
                              uint16_t* out_bf, int H, int W, hipStream_t s);
// Last layer (32 -> 3, linear) whose output is added to the state as the correction.
hipError_t launch_conv3x3_correct(const uint16_t* in, const uint16_t* Wk, const float* bias, const CorrectOut& co,
                                  int H, int W, hipStream_t s);
// The four layers of one image in one pass, the maps kept on chip (inference).
struct FusedNet {
    const uint16_t* wk[4];  // BF16 [9][32][cin], cin = 16, 32, 32, 32
    const float* bias[4];   // [32]
};
hipError_t launch_cnn_fused(const RawIn& raw, const InputNorm& nrm, const FusedNet& net, float* out_f, int H,
                            int W, hipStream_t s);
hipError_t launch_conv3x3(int kin, int mode, const uint16_t* in, const uint16_t* Wk, const float* bias,
                          uint16_t* out_bf, float* out_f, const uint16_t* relu_src, int nimg, int H, int W,
                          hipStream_t s);
int wgrad_chunks(int nimg, int H, int W);
hipError_t launch_wgrad(int kin, const uint16_t* x, const uint16_t* dy, int nimg, int H, int W, float* part_w,
                        float* part_b, float* dW, float* db, hipStream_t s);
hipError_t launch_mse_grad(const float* out, const float* target, const uint8_t* mask, int nimg, int H, int W,
                           float inv_n, const float* tscale, uint16_t* d_out, double* partial, int nblocks,
                           double* loss, hipStream_t s);
hipError_t launch_sub3(const float* a0, const float* a1, const float* a2, const float* b0, const float* b1,
                       const float* b2, int n, float* out, hipStream_t s);
hipError_t launch_moments(const float* x, const uint8_t* mask, int64_t n, double* partial, int nblocks, double* out,
                          hipStream_t s);
hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int n, const AdamHyper& hp,
                       hipStream_t s);
hipError_t launch_cast_weights(const float* master, int kin, int dkin, uint16_t* wk, uint16_t* wd, hipStream_t s);
hipError_t launch_correct(float* eta, float* u, float* v, const float* out, const uint8_t* mask, int H, int W,
                          const float* t_std, hipStream_t s);
hipError_t launch_sqdiff(const float* a, const float* b, const uint8_t* mask, int n, double* partial, int nblocks,
                         double* out, hipStream_t s);

}  // namespace sur
}  // namespace sw2d
