// sw2d_surrogate.hip - kernels of the learned coarse-step surrogate of the 2DSW model.
//
// The surrogate advances a 4x-coarsened state of the model of Sect. 6.2 with the same
// fused step on the coarse grid (4 dx, 4 dt) and adds a correction predicted by a small
// convolutional network: 3x3 'same' convolutions 5 -> 32 -> 32 -> 32 -> 3 with ReLU after
// the first three. The plain fine model is its judge and fallback.
//
// Kernels here:
//   * restrict4      fine (eta, u, v, H, mask) -> coarse, 4x4 blocks;
//   * pack_input     coarse state -> normalised BF16 NHWC input (5 channels padded to 16);
//   * conv3x3        implicit GEMM on BF16 MFMA (v_mfma_f32_32x32x16_bf16), FP32 accumulate:
//                    out[p][n] = sum over taps t and channels k of in[p + off_t][k] Wk[t][n][k];
//                    used for the forward layers (bias + ReLU + BF16 store, or bias + FP32
//                    planar store of 3 channels) and for the data gradient (flipped,
//                    transposed weights; fused ReLU-mask of the layer input);
//   * wgrad          dW[t][o][c] = sum_p dY[p][o] X[p + off_t][c], split over pixel
//                    chunks on MFMA, FP32 partials, then a fixed-order reduction;
//   * mse_grad       masked squared error and its gradient (BF16 NHWC, 32 channels);
//   * adam           Adam on FP32 master weights, then BF16 working copies in the forward
//                    and data-gradient layouts;
//   * correct        state += activity * t_std * out;
//   * rmse           sum over water of (a - b)^2 in FP64, fixed-order.
// Feature maps are NHWC BF16 with 16 or 32 channels: a pixel's channels are one 32/64 B
// row, so one lane's MFMA operand (8 consecutive channels) is one 16 B load.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sw2d_internal.h"
#include "sw2d_surrogate.h"

namespace sw2d {
namespace sur {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even (one hardware conversion).
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// Two values to BF16, packed with a in the low half.
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------------------------ restrict4
__global__ __launch_bounds__(256) void restrict4_kernel(const float* __restrict__ eta, const float* __restrict__ u,
                                                        const float* __restrict__ v, const float* __restrict__ H,
                                                        const uint8_t* __restrict__ mask, int NX, int NY,
                                                        float* __restrict__ eta_c, float* __restrict__ u_c,
                                                        float* __restrict__ v_c, float* __restrict__ H_c,
                                                        uint8_t* __restrict__ mask_c) {
    const int nx = NX / 4, ny = NY / 4;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nx * ny) return;
    const int J = idx / nx, I = idx - J * nx;
    auto wet_count = [&](int JJ, int II) -> int {
        if (JJ < 0 || II < 0 || JJ >= ny || II >= nx) return 0;
        int n = 0;
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) n += mask[(size_t)(4 * JJ + r) * NX + 4 * II + c] != 0;
        return n;
    };
    int n = 0;
    float se = 0.f, sh = 0.f;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            const size_t f = (size_t)(4 * J + r) * NX + 4 * I + c;
            if (mask[f]) {
                ++n;
                se += eta[f];
                sh += H[f];
            }
        }
    const bool wc = n >= 8;
    eta_c[idx] = wc ? se / (float)n : 0.f;
    H_c[idx] = n > 0 ? sh / (float)n : 0.f;
    mask_c[idx] = wc ? 1 : 0;
    const bool au = wc && wet_count(J, I + 1) >= 8;
    const bool av = wc && wet_count(J + 1, I) >= 8;
    float su = 0.f, sv = 0.f;
    for (int r = 0; r < 4; ++r) su += u[(size_t)(4 * J + r) * NX + 4 * I + 3];
    for (int c = 0; c < 4; ++c) sv += v[(size_t)(4 * J + 3) * NX + 4 * I + c];
    u_c[idx] = au ? 0.25f * su : 0.f;
    v_c[idx] = av ? 0.25f * sv : 0.f;
}

// ------------------------------------------------------------------------------ pack_input
// SplitMix64 (Steele, Lea & Flood, 2014) of the counter seed + (i + 1) * golden gamma, mapped
// to a uniform float in [-1, 1): the training-noise generator, keyed by (seed, element).
__device__ __forceinline__ float splitmix_uniform(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)(z >> 40) * (1.0f / 8388608.0f) - 1.0f;
}

// The 16 BF16 input channels of one pixel from its raw values x = (eta, u, v, H, mask):
// normalised, plus the training noise on channels 0..2, then 11 zero channels; two 16 B
// chunks. p is the pixel's index (the noise counter).
__device__ __forceinline__ void pack_values(const float (&x)[5], size_t p, const InputNorm& nrm, uint4& a,
                                            uint4& b) {
    uint16_t o[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) o[c] = 0;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        float y = (x[c] - nrm.mean[c]) * nrm.inv_std[c];
        if (c < 3 && nrm.noise_amp > 0.f) y += nrm.noise_amp * splitmix_uniform(nrm.noise_seed, (uint64_t)p * 3 + c);
        o[c] = f2bf(y);
    }
    a.x = o[0] | ((uint32_t)o[1] << 16);
    a.y = o[2] | ((uint32_t)o[3] << 16);
    a.z = o[4] | ((uint32_t)o[5] << 16);
    a.w = o[6] | ((uint32_t)o[7] << 16);
    b.x = o[8] | ((uint32_t)o[9] << 16);
    b.y = o[10] | ((uint32_t)o[11] << 16);
    b.z = o[12] | ((uint32_t)o[13] << 16);
    b.w = o[14] | ((uint32_t)o[15] << 16);
}

__device__ __forceinline__ void pack_pixel(const float* __restrict__ eta, const float* __restrict__ u,
                                           const float* __restrict__ v, const float* __restrict__ H,
                                           const uint8_t* __restrict__ mask, size_t p, const InputNorm& nrm,
                                           uint4& a, uint4& b) {
    const float x[5] = {eta[p], u[p], v[p], H[p], mask[p] ? 1.f : 0.f};
    pack_values(x, p, nrm, a, b);
}

__global__ __launch_bounds__(256) void pack_input_kernel(const float* __restrict__ eta, const float* __restrict__ u,
                                                         const float* __restrict__ v, const float* __restrict__ H,
                                                         const uint8_t* __restrict__ mask, int npix, InputNorm nrm,
                                                         uint16_t* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    uint4 a, b;
    pack_pixel(eta, u, v, H, mask, (size_t)p, nrm, a, b);
    uint4* dst = reinterpret_cast<uint4*>(out + (size_t)p * 16);
    dst[0] = a;
    dst[1] = b;
}

// ------------------------------------------------------------------------------ conv3x3
// Tile: kConvTH rows x 32 columns of output pixels per workgroup (4 waves, TH/4 rows each);
// the (TH+2) x 34 input patch is staged in LDS with a padded pixel stride.
constexpr int kConvTH = 8;
constexpr int kConvRowsPerWave = kConvTH / 4;
constexpr int kConvTW = 32;
constexpr int kConvThreads = 256;

template <int KIN>
struct ConvLds {
    static constexpr int kStride = KIN * 2 + 16;  // bytes per pixel, 16 B aligned, spreads banks
    static constexpr int kCols = kConvTW + 2;
    static constexpr int kRows = kConvTH + 2;
    static constexpr int kBytes = kRows * kCols * kStride;
};

template <int KIN, int MODE, bool kRaw = false>
__global__ __launch_bounds__(kConvThreads) void conv3x3_kernel(const uint16_t* __restrict__ in,
                                                               const uint16_t* __restrict__ Wk,
                                                               const float* __restrict__ bias,
                                                               uint16_t* __restrict__ out_bf,
                                                               float* __restrict__ out_f,
                                                               const uint16_t* __restrict__ relu_src, int H,
                                                               int W, int nimg, RawIn raw, InputNorm nrm,
                                                               CorrectOut co) {
    using L = ConvLds<KIN>;
    __shared__ __attribute__((aligned(16))) unsigned char patch[L::kBytes];
    const int tiles_x = (W + kConvTW - 1) / kConvTW;
    const int tiles_y = (H + kConvTH - 1) / kConvTH;
    const int per_img = tiles_x * tiles_y;
    const int total = per_img * nimg;

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int half = lane / 32;  // which 8-channel group of a 16-channel chunk
    const int j = lane % 32;     // pixel within the 32-column block; also the A row (n)

    // A operands (weights), one per tap and 16-channel chunk: Wk[t][n = j][k0 + 8 half + 0..7],
    // loaded once and kept in registers while the workgroup walks its tiles
    constexpr int kK = KIN / 16;
    bf16x8 a[9][kK];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int kc = 0; kc < kK; ++kc)
            a[t][kc] = *reinterpret_cast<const bf16x8*>(Wk + ((size_t)t * 32 + j) * KIN + kc * 16 + half * 8);
    // the bias is the accumulators' initial value (lane: output channels 8 q + 4 half + e)
    f32x16 binit;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) binit[4 * q + e] = MODE == kConvDgradMask ? 0.f : bias[8 * q + 4 * half + e];

    // The next tile's input patch is fetched into registers while the current one is
    // multiplied, then written to LDS: every load of a patch is in flight at once.
    constexpr int kChunks = KIN / 8;  // 16 B chunks per pixel
    constexpr int kPatchChunks = L::kRows * L::kCols * kChunks;
    constexpr int kPer = (kPatchChunks + kConvThreads - 1) / kConvThreads;
    uint4 pre[kPer];
    auto fetch = [&](int tile_g) {
        const int img = tile_g / per_img;
        const int tile = tile_g - img * per_img;
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        const int y0 = ty * kConvTH, x0 = tx * kConvTW;
        const size_t img_off = (size_t)img * H * W;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + q * kConvThreads;
            const int pix = e / kChunks, ch = e - pix * kChunks;
            const int r = pix / L::kCols, c = pix - r * L::kCols;
            const int gy = y0 + r - 1, gx = x0 + c - 1;
            pre[q] = make_uint4(0u, 0u, 0u, 0u);
            if (e < kPatchChunks && gy >= 0 && gy < H && gx >= 0 && gx < W) {
                if constexpr (kRaw) {  // pack the raw state here (KIN = 16: chunk 0 or 1)
                    uint4 a, b;
                    pack_pixel(raw.eta, raw.u, raw.v, raw.H, raw.mask, img_off + (size_t)gy * W + gx, nrm, a, b);
                    pre[q] = ch == 0 ? a : b;
                } else {
                    pre[q] = reinterpret_cast<const uint4*>(in + (img_off + (size_t)gy * W + gx) * KIN)[ch];
                }
            }
        }
    };
    auto commit = [&]() {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + q * kConvThreads;
            const int pix = e / kChunks, ch = e - pix * kChunks;
            if (e < kPatchChunks) *reinterpret_cast<uint4*>(patch + pix * L::kStride + ch * 16) = pre[q];
        }
    };

    if ((int)blockIdx.x < total) fetch(blockIdx.x);
    for (int tile_g = blockIdx.x; tile_g < total; tile_g += gridDim.x) {
        const int img = tile_g / per_img;
        const int tile = tile_g - img * per_img;
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        const int y0 = ty * kConvTH, x0 = tx * kConvTW;
        const size_t img_off = (size_t)img * H * W;

        __syncthreads();  // the previous tile's patch is no longer read
        commit();
        __syncthreads();
        if (tile_g + (int)gridDim.x < total) fetch(tile_g + gridDim.x);

        f32x16 acc[kConvRowsPerWave];
#pragma unroll
        for (int b = 0; b < kConvRowsPerWave; ++b) acc[b] = binit;

#pragma unroll
        for (int b = 0; b < kConvRowsPerWave; ++b) {
            const int r = wave * kConvRowsPerWave + b;  // output row within the tile
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int ky = t / 3, kx = t - 3 * (t / 3);
                const unsigned char* src = patch + ((r + ky) * L::kCols + (j + kx)) * L::kStride + half * 16;
#pragma unroll
                for (int kc = 0; kc < kK; ++kc) {
                    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(src + kc * 32);
                    acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[t][kc], bv, acc[b], 0, 0, 0);
                }
            }
        }

        // epilogue: lane holds pixel j, output channels n = 8 (q) + 4 half + (0..3), q = 0..3
#pragma unroll
        for (int b = 0; b < kConvRowsPerWave; ++b) {
            const int gy = y0 + wave * kConvRowsPerWave + b, gx = x0 + j;
            if (gy >= H || gx >= W) continue;
            const size_t p = img_off + (size_t)gy * W + gx;
            if constexpr (MODE == kConvRelu || MODE == kConvDgradMask) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int n0 = 8 * q + 4 * half;
                    uint16_t o[4];
                    if constexpr (MODE == kConvRelu) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) o[e] = f2bf(fmaxf(acc[b][4 * q + e], 0.f));
                    } else {
                        const uint2 m = *reinterpret_cast<const uint2*>(relu_src + p * 32 + n0);
                        const uint16_t mv[4] = {(uint16_t)(m.x & 0xffff), (uint16_t)(m.x >> 16),
                                                (uint16_t)(m.y & 0xffff), (uint16_t)(m.y >> 16)};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            o[e] = (bf2f(mv[e]) > 0.f) ? f2bf(acc[b][4 * q + e]) : (uint16_t)0;
                    }
                    uint2 w;
                    w.x = o[0] | ((uint32_t)o[1] << 16);
                    w.y = o[2] | ((uint32_t)o[3] << 16);
                    *reinterpret_cast<uint2*>(out_bf + p * 32 + n0) = w;
                }
            } else if constexpr (MODE == kConvCorrect) {
                // the state += activity * (output * scale), as the correction kernel does
                if (half == 0 && co.mask[p] != 0) {
                    co.eta[p] = fmaf(co.s0, acc[b][0], co.eta[p]);
                    if (gx + 1 < W && co.mask[p + 1]) co.u[p] = fmaf(co.s1, acc[b][1], co.u[p]);
                    if (gy + 1 < H && co.mask[p + W]) co.v[p] = fmaf(co.s2, acc[b][2], co.v[p]);
                }
            } else {  // kConvLinear3: channels 0..2 as FP32 planes [img][3][H][W]
                if (half == 0) {
#pragma unroll
                    for (int e = 0; e < 3; ++e)
                        out_f[((size_t)img * 3 + e) * H * W + (size_t)gy * W + gx] = acc[b][e];
                }
            }
        }
    }
}

// ------------------------------------------------------------------------------ fused forward
// The four layers of one image in one pass (inference). A workgroup owns a kFuTH x kFuTW tile
// of output pixels and computes every layer over the tile grown by the receptive field still
// ahead of it: layer 1 over (TH + 6) x (TW + 6) pixels of the (TH + 8) x (TW + 8) packed input,
// layer 2 over (TH + 4) x (TW + 4), layer 3 over (TH + 2) x (TW + 2), layer 4 over the tile.
// The maps stay in LDS, two buffers used in turn; a map's pixels outside the image are stored
// as 0, which is the next layer's zero padding. A layer's pixels are taken 32 at a time in
// row-major order of its region (the lane's address carries the row wrap), so the MFMA blocks
// do not depend on the region's width. Taps, channel chunks, the packing of the input and the
// epilogues are those of the layer-by-layer kernels: the output is bitwise theirs.
constexpr int kFuTH = 16;
constexpr int kFuTW = 32;
constexpr int kFuThreads = 512;
constexpr int kFuWaves = kFuThreads / 64;

template <int L>  // the region of layer L's output; L = 0 is the packed input
struct FuRegion {
    static constexpr int kHalo = 4 - L;
    static constexpr int kRows = kFuTH + 2 * kHalo;
    static constexpr int kCols = kFuTW + 2 * kHalo;
    static constexpr int kPix = kRows * kCols;
    static constexpr int kStride = (L == 0 ? 32 : 64) + 16;  // bytes per pixel, 16 B aligned, spreads banks
    static constexpr int kBytes = kPix * kStride;
};
// buffer A holds layer 1's map, then layer 3's; buffer B the packed input, then layer 2's map
constexpr int kFuBufA = FuRegion<1>::kBytes;
constexpr int kFuBufB = FuRegion<0>::kBytes > FuRegion<2>::kBytes ? FuRegion<0>::kBytes : FuRegion<2>::kBytes;
static_assert(FuRegion<3>::kBytes <= kFuBufA, "layer 3 map in buffer A");
constexpr int kFuWSlot = 9 * 32 * 32 * 2;  // one layer's BF16 weights (the widest)
constexpr int kFuBiasBytes = 4 * 32 * 4;
constexpr int kFuLds = kFuBufA + kFuBufB + 2 * kFuWSlot + kFuBiasBytes;
constexpr int kFuWPer = (kFuWSlot / 16 + kFuThreads - 1) / kFuThreads;  // 16 B weight chunks per thread
constexpr int kFuRawPer = (FuRegion<0>::kPix + kFuThreads - 1) / kFuThreads;  // input pixels per thread

typedef short i16x2 __attribute__((ext_vector_type(2)));

// ReLU of two packed BF16 values: a BF16 with its sign bit set is a negative 16-bit integer,
// so the signed maximum with 0 zeroes exactly the negative values (and -0). Rounding then
// clamping equals clamping then rounding, since rounding keeps the sign.
__device__ __forceinline__ uint32_t relu_bf2(uint32_t w) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16x2, w), (i16x2){0, 0}));
}

// The bias pattern of a lane (output channels 8 q + 4 half + e) as an accumulator value.
__device__ __forceinline__ f32x16 bias_pattern(const float* __restrict__ bias, int half) {
    f32x16 b;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) b[4 * q + e] = bias[8 * q + 4 * half + e];
    return b;
}

// One layer over its region: input map in_lds (region L - 1), output map out_lds (region L),
// or, for the last layer, channels 0..2 to the FP32 planes out_f [3][H][W]. bias: the layer's
// 32 biases in LDS; a lane's output channels start from theirs. A block's B
// operands (all taps and channel chunks) are read from LDS before its first product, so the
// reads overlap the products instead of waiting one by one.
template <int L, int KIN, bool kLast>
__device__ __forceinline__ void fused_layer(const unsigned char* __restrict__ in_lds, unsigned char* __restrict__ out_lds,
                                            const bf16x8 (&a)[9][2], const float* __restrict__ bias, float* __restrict__ out_f,
                                            int y0, int x0, int H, int W, int wave, int half, int j) {
    using In = FuRegion<L - 1>;
    using Out = FuRegion<L>;
    constexpr int kK = KIN / 16;
    constexpr int kBlocks = (Out::kPix + 31) / 32;
    const int oy = y0 - Out::kHalo, ox = x0 - Out::kHalo;  // image coordinates of the region's first pixel
    for (int blk = wave; blk < kBlocks; blk += kFuWaves) {
        const int P = blk * 32 + j;
        const bool valid = P < Out::kPix;
        const int Pc = valid ? P : Out::kPix - 1;  // the last block's spare lanes read a real pixel
        const int ry = Pc / Out::kCols, rx = Pc - ry * Out::kCols;
        const unsigned char* base = in_lds + (ry * In::kCols + rx) * In::kStride + half * 16;
        bf16x8 bv[9][kK];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ky = t / 3, kx = t - 3 * (t / 3);
#pragma unroll
            for (int kc = 0; kc < kK; ++kc)
                bv[t][kc] = *reinterpret_cast<const bf16x8*>(base + (ky * In::kCols + kx) * In::kStride + kc * 32);
        }
        f32x16 acc = bias_pattern(bias, half);
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int kc = 0; kc < kK; ++kc) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[t][kc], bv[t][kc], acc, 0, 0, 0);
        // the scheduler is told to issue the block's LDS reads before its products
        __builtin_amdgcn_sched_group_barrier(0x100, 9 * kK, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 9 * kK, 0);
        const int gy = oy + ry, gx = ox + rx;
        const bool inside = valid && gy >= 0 && gy < H && gx >= 0 && gx < W;
        if constexpr (!kLast) {
            // lane holds pixel P, output channels n = 8 q + 4 half + (0..3)
            if (valid) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int n0 = 8 * q + 4 * half;
                    uint2 w;
                    w.x = relu_bf2(f2bf2(acc[4 * q + 0], acc[4 * q + 1]));
                    w.y = relu_bf2(f2bf2(acc[4 * q + 2], acc[4 * q + 3]));
                    if (!inside) w = make_uint2(0u, 0u);
                    *reinterpret_cast<uint2*>(out_lds + P * Out::kStride + n0 * 2) = w;
                }
            }
        } else {
            if (inside && half == 0) {
#pragma unroll
                for (int e = 0; e < 3; ++e) out_f[(size_t)e * H * W + (size_t)gy * W + gx] = acc[e];
            }
        }
    }
}

// A operands of one layer (lane: output channel j, channels 8 half.. of each 16-chunk) from
// the layer's weights staged in LDS ([9][32][KIN] BF16).
template <int KIN>
__device__ __forceinline__ void fused_weights(bf16x8 (&a)[9][2], const unsigned char* __restrict__ slot, int half, int j) {
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int kc = 0; kc < KIN / 16; ++kc)
            a[t][kc] = *reinterpret_cast<const bf16x8*>(slot + (((t * 32 + j) * KIN) + kc * 16 + half * 8) * 2);
}

__global__ __launch_bounds__(kFuThreads) void cnn_fused_kernel(RawIn raw, InputNorm nrm, FusedNet net,
                                                               float* __restrict__ out_f, int H, int W) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[kFuLds];
    unsigned char* bufA = lds;
    unsigned char* bufB = lds + kFuBufA;
    unsigned char* wslot[2] = {lds + kFuBufA + kFuBufB, lds + kFuBufA + kFuBufB + kFuWSlot};
    float* bias_lds = reinterpret_cast<float*>(lds + kFuBufA + kFuBufB + 2 * kFuWSlot);
    const int tiles_x = (W + kFuTW - 1) / kFuTW;
    const int total = tiles_x * ((H + kFuTH - 1) / kFuTH);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int half = lane / 32, j = lane % 32;
    if (threadIdx.x < 128) bias_lds[threadIdx.x] = net.bias[threadIdx.x / 32][threadIdx.x % 32];

    // the packed input of a tile: raw values fetched into registers, packed into buffer B
    float rx_[kFuRawPer][5];
    bool rin[kFuRawPer];
    auto fetch = [&](int tile) {
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        const int y0 = ty * kFuTH - FuRegion<0>::kHalo, x0 = tx * kFuTW - FuRegion<0>::kHalo;
#pragma unroll
        for (int q = 0; q < kFuRawPer; ++q) {
            const int e = threadIdx.x + q * kFuThreads;
            const int r = e / FuRegion<0>::kCols, c = e - r * FuRegion<0>::kCols;
            const int gy = y0 + r, gx = x0 + c;
            rin[q] = e < FuRegion<0>::kPix && gy >= 0 && gy < H && gx >= 0 && gx < W;
            const size_t p = rin[q] ? (size_t)gy * W + gx : 0;
            rx_[q][0] = rin[q] ? raw.eta[p] : 0.f;
            rx_[q][1] = rin[q] ? raw.u[p] : 0.f;
            rx_[q][2] = rin[q] ? raw.v[p] : 0.f;
            rx_[q][3] = rin[q] ? raw.H[p] : 0.f;
            rx_[q][4] = rin[q] ? (raw.mask[p] ? 1.f : 0.f) : 0.f;
        }
    };
    auto commit = [&]() {
#pragma unroll
        for (int q = 0; q < kFuRawPer; ++q) {
            const int e = threadIdx.x + q * kFuThreads;
            if (e < FuRegion<0>::kPix) {
                uint4 ca = make_uint4(0u, 0u, 0u, 0u), cb = make_uint4(0u, 0u, 0u, 0u);
                if (rin[q]) pack_values(rx_[q], 0, nrm, ca, cb);  // no noise at inference
                uint4* dst = reinterpret_cast<uint4*>(bufB + e * FuRegion<0>::kStride);
                dst[0] = ca;
                dst[1] = cb;
            }
        }
    };
    // The next layer's weights go from global memory straight into the free LDS slot while
    // the current layer runs (a wave copies 64 consecutive 16 B chunks per load; the chunk
    // counts are multiples of 64); the wait and the barrier after the layer publish them, and
    // each wave then reads its A operands from LDS.
    auto wstage = [&](int layer, unsigned char* slot) {
        const int chunks = 9 * 32 * (layer == 0 ? 16 : 32) / 8;
        const uint4* src = reinterpret_cast<const uint4*>(net.wk[layer]);
#pragma unroll
        for (int q = 0; q < kFuWPer; ++q) {
            const int first = q * kFuThreads + wave * 64;  // wave-uniform
            if (first < chunks)
                __builtin_amdgcn_global_load_lds(src + first + lane, reinterpret_cast<uint4*>(slot) + first, 16, 0, 0);
        }
    };
    auto publish = [&]() {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies (and loads) have landed
        __syncthreads();
    };

    bf16x8 w[9][2];
    wstage(0, wslot[0]);
    if ((int)blockIdx.x < total) {
        fetch(blockIdx.x);
        commit();
    }
    __builtin_amdgcn_s_waitcnt(0);
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        const int y0 = ty * kFuTH, x0 = tx * kFuTW;
        const int next = tile + (int)gridDim.x;
        __syncthreads();  // packed input and layer 1's weights in place; the last tile's layer 4 done
        fused_weights<16>(w, wslot[0], half, j);
        wstage(1, wslot[1]);
        fused_layer<1, 16, false>(bufB, bufA, w, bias_lds, nullptr, y0, x0, H, W, wave, half, j);
        publish();
        fused_weights<32>(w, wslot[1], half, j);
        wstage(2, wslot[0]);
        if (next < total) fetch(next);
        fused_layer<2, 32, false>(bufA, bufB, w, bias_lds + 32, nullptr, y0, x0, H, W, wave, half, j);
        publish();
        fused_weights<32>(w, wslot[0], half, j);
        wstage(3, wslot[1]);
        fused_layer<3, 32, false>(bufB, bufA, w, bias_lds + 64, nullptr, y0, x0, H, W, wave, half, j);
        publish();
        fused_weights<32>(w, wslot[1], half, j);
        wstage(0, wslot[0]);
        if (next < total) commit();  // buffer B is free: layer 4 reads buffer A only
        fused_layer<4, 32, true>(bufA, nullptr, w, bias_lds + 96, out_f, y0, x0, H, W, wave, half, j);
        __builtin_amdgcn_s_waitcnt(0);
    }
}

// ------------------------------------------------------------------------------ wgrad
// dW[t][o][c] = sum_p dY[p][o] X[p + off_t][c] on the MFMA with K = pixels: A = dY (32
// outputs x 16 pixels), B = X shifted by the tap (16 pixels x 32 channels). Both operands
// take 8 consecutive pixels of one channel per lane while the maps are NHWC (channels
// contiguous), so a tile is staged in LDS pair-packed: a dword holds two horizontally
// adjacent pixels of one channel, dword (r * pairs + q) * 32 + c for row r, pair q,
// channel c. A lane reads one row's pixels c0 - 1 .. c0 + 8 of its channel as 5 dwords and
// forms the three horizontal taps' operands from them (the odd tap by byte alignment); the
// dY operand is 4 dwords. Workgroup g takes tiles g * kWgTiles ... of all images' 4 x 128
// pixel tiles, fetching the next tile into registers while the current one is multiplied.
// Its 12 waves (3 per SIMD) split the work by tile row and tap row: wave w accumulates the
// three taps of tap row ky = w / 4 over tile row w % 4 (3 accumulators of 32 x 32); the four
// tile rows of a tap are added in LDS in row order, and the chunk's partial [9][32][KIN]
// (and the bias partial [32]) goes to global memory.
constexpr int kWgTH = 4;                    // rows per tile
constexpr int kWgTW = 128;                  // pixels per tile row
constexpr int kWgTiles = 8;                 // tiles per chunk
constexpr int kWgWaves = 12;                // (tile row, tap row) pairs
constexpr int kWgThreads = 64 * kWgWaves;
constexpr int kWgXPairs = (kWgTW + 2) / 2;  // pairs of the input rows: pixels -1 .. kWgTW
constexpr int kWgDPairs = kWgTW / 2;        // pairs of the dY rows
constexpr int kWgXRows = kWgTH + 2;
constexpr int kWgXItems = kWgXRows * kWgXPairs * 4;  // (row, pair, 8-channel group), 32 channels
constexpr int kWgDItems = kWgTH * kWgDPairs * 4;
constexpr int kWgXPer = (kWgXItems + kWgThreads - 1) / kWgThreads;
constexpr int kWgDPer = (kWgDItems + kWgThreads - 1) / kWgThreads;

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Channels 2m, 2m+1 of pixels p0 (x) and p1 (y) -> dwords (p0 c, p1 c) for c = 2m and 2m+1.
__device__ __forceinline__ void pair_pack(const uint4& x, const uint4& y, uint4& lo, uint4& hi) {
    lo.x = __builtin_amdgcn_perm(y.x, x.x, 0x05040100u);
    lo.y = __builtin_amdgcn_perm(y.x, x.x, 0x07060302u);
    lo.z = __builtin_amdgcn_perm(y.y, x.y, 0x05040100u);
    lo.w = __builtin_amdgcn_perm(y.y, x.y, 0x07060302u);
    hi.x = __builtin_amdgcn_perm(y.z, x.z, 0x05040100u);
    hi.y = __builtin_amdgcn_perm(y.z, x.z, 0x07060302u);
    hi.z = __builtin_amdgcn_perm(y.w, x.w, 0x05040100u);
    hi.w = __builtin_amdgcn_perm(y.w, x.w, 0x07060302u);
}

__device__ __forceinline__ bf16x8 as_bf16x8(unsigned a, unsigned b, unsigned c, unsigned d) {
    return __builtin_bit_cast(bf16x8, (u32x4){a, b, c, d});
}

template <int KIN>
__global__ __launch_bounds__(kWgThreads) void wgrad_kernel(const uint16_t* __restrict__ x,
                                                           const uint16_t* __restrict__ dy, int nimg, int H, int W,
                                                           float* __restrict__ part_w, float* __restrict__ part_b) {
    constexpr int G = KIN / 8;  // 8-channel groups of the input map
    __shared__ __attribute__((aligned(16))) unsigned xs[kWgXRows * kWgXPairs * 32];
    __shared__ __attribute__((aligned(16))) unsigned ds[kWgTH * kWgDPairs * 32];
    __shared__ float red[kWgTH][2][32];
    __shared__ float tapsum[3][32 * 32];
    const int tiles_x = (W + kWgTW - 1) / kWgTW, tiles_y = (H + kWgTH - 1) / kWgTH;
    const int tiles = tiles_x * tiles_y * nimg;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int half = lane / 32, j = lane % 32;
    const int row = wave % kWgTH, ky = wave / kWgTH;  // this wave's tile row and tap row
    const int first = blockIdx.x * kWgTiles;
    const int ntiles = min(kWgTiles, tiles - first);

    if constexpr (KIN < 32) {
        // channels KIN .. 31 of the input rows stay zero: they are the B columns j >= KIN
        for (int e = threadIdx.x; e < kWgXRows * kWgXPairs * 32; e += kWgThreads)
            if (e % 32 >= KIN) xs[e] = 0u;
    }

    // the tile's rows in registers: input items (row, pair, group) and dY items
    uint4 rx[kWgXPer][2], rd[kWgDPer][2];
    auto fetch = [&](int k) {
        const int tile = first + k;
        const int img = tile / (tiles_x * tiles_y);
        const int tt = tile - img * tiles_x * tiles_y;
        const int ty = tt / tiles_x, tx = tt - ty * tiles_x;
        const int y0 = ty * kWgTH, x0 = tx * kWgTW;
        const size_t img_off = (size_t)img * H * W;
#pragma unroll
        for (int i = 0; i < kWgXPer; ++i) {
            const int e = threadIdx.x + kWgThreads * i;
            const int g = e % 4, rq = e / 4;
            const int r = rq / kWgXPairs, q = rq - r * kWgXPairs;
            const int gy = y0 - 1 + r, gx = x0 - 1 + 2 * q;
            const bool row_ok = e < kWgXItems && g < G && gy >= 0 && gy < H;
            const uint4* src = reinterpret_cast<const uint4*>(x + (img_off + (size_t)gy * W + gx) * KIN) + g;
            rx[i][0] = (row_ok && gx >= 0 && gx < W) ? src[0] : make_uint4(0u, 0u, 0u, 0u);
            rx[i][1] = (row_ok && gx + 1 < W) ? src[G] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int i = 0; i < kWgDPer; ++i) {
            const int e = threadIdx.x + kWgThreads * i;
            const int g = e % 4, rq = e / 4;
            const int r = rq / kWgDPairs, q = rq - r * kWgDPairs;
            const int gy = y0 + r, gx = x0 + 2 * q;
            const bool row_ok = e < kWgDItems && gy < H;
            const uint4* src = reinterpret_cast<const uint4*>(dy + (img_off + (size_t)gy * W + gx) * 32) + g;
            rd[i][0] = (row_ok && gx < W) ? src[0] : make_uint4(0u, 0u, 0u, 0u);
            rd[i][1] = (row_ok && gx + 1 < W) ? src[4] : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int i = 0; i < kWgXPer; ++i) {
            const int e = threadIdx.x + kWgThreads * i;
            const int g = e % 4, rq = e / 4;
            if (e < kWgXItems && g < G) {
                uint4 lo, hi;
                pair_pack(rx[i][0], rx[i][1], lo, hi);
                uint4* dst = reinterpret_cast<uint4*>(xs + rq * 32 + 8 * g);
                dst[0] = lo;
                dst[1] = hi;
            }
        }
#pragma unroll
        for (int i = 0; i < kWgDPer; ++i) {
            const int e = threadIdx.x + kWgThreads * i;
            const int g = e % 4, rq = e / 4;
            if (e < kWgDItems) {
                uint4 lo, hi;
                pair_pack(rd[i][0], rd[i][1], lo, hi);
                uint4* dst = reinterpret_cast<uint4*>(ds + rq * 32 + 8 * g);
                dst[0] = lo;
                dst[1] = hi;
            }
        }
    };

    f32x16 acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[t][e] = 0.f;
    float bsum = 0.f;  // bias gradient: channel j over this lane's pixels (tap row 0 only)

    if (ntiles > 0) fetch(0);
    for (int k = 0; k < ntiles; ++k) {
        __syncthreads();  // every wave is done with the previous tile
        stage();
        __syncthreads();
        if (k + 1 < ntiles) fetch(k + 1);
        // K steps of 16 pixels along the tile row; lane: pixels c0 .. c0 + 7
#pragma unroll 2
        for (int ks = 0; ks < kWgTW / 16; ++ks) {
            const int q0 = ks * 8 + half * 4;  // pair of pixel c0 = 16 ks + 8 half
            const unsigned* dq = ds + (row * kWgDPairs + q0) * 32 + j;
            const unsigned a0 = dq[0], a1 = dq[32], a2 = dq[64], a3 = dq[96];
            // input pixels c0 - 1 .. c0 + 8 of image row row + ky - 1 (pairs q0 .. q0 + 4)
            const unsigned* xq = xs + ((row + ky) * kWgXPairs + q0) * 32 + j;
            const unsigned d0 = xq[0], d1 = xq[32], d2 = xq[64], d3 = xq[96], d4 = xq[128];
            const bf16x8 av = as_bf16x8(a0, a1, a2, a3);
            if (ky == 0) {
                bsum += __uint_as_float(a0 << 16);
                bsum += __uint_as_float(a0 & 0xffff0000u);
                bsum += __uint_as_float(a1 << 16);
                bsum += __uint_as_float(a1 & 0xffff0000u);
                bsum += __uint_as_float(a2 << 16);
                bsum += __uint_as_float(a2 & 0xffff0000u);
                bsum += __uint_as_float(a3 << 16);
                bsum += __uint_as_float(a3 & 0xffff0000u);
            }
            const bf16x8 b0 = as_bf16x8(d0, d1, d2, d3);
            const bf16x8 b1 = as_bf16x8(__builtin_amdgcn_alignbyte(d1, d0, 2), __builtin_amdgcn_alignbyte(d2, d1, 2),
                                        __builtin_amdgcn_alignbyte(d3, d2, 2), __builtin_amdgcn_alignbyte(d4, d3, 2));
            const bf16x8 b2 = as_bf16x8(d1, d2, d3, d4);
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b0, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b1, acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b2, acc[2], 0, 0, 0);
        }
    }
    // for each horizontal tap kx: the four tile rows of every tap row added in row order in
    // LDS, then the three taps 3 ky + kx written out
    float* out = part_w + (size_t)blockIdx.x * 9 * 32 * KIN;
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
        for (int r = 0; r < kWgTH; ++r) {
            __syncthreads();
            if (row == r) {
                // acc[kx][e]: o = 8 (e / 4) + 4 half + e % 4, c = j
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int o = 8 * (e / 4) + 4 * half + (e % 4);
                    if (r == 0) tapsum[ky][o * 32 + j] = acc[kx][e];
                    else tapsum[ky][o * 32 + j] += acc[kx][e];
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 3 * 32 * KIN; e += kWgThreads) {
            const int yy = e / (32 * KIN), rem = e - yy * 32 * KIN;
            const int o = rem / KIN, c = rem - o * KIN;
            out[(size_t)(3 * yy + kx) * 32 * KIN + rem] = tapsum[yy][o * 32 + c];
        }
    }
    if (ky == 0) red[row][half][j] = bsum;
    __syncthreads();
    if (threadIdx.x < 32) {
        float b = 0.f;
#pragma unroll
        for (int r = 0; r < kWgTH; ++r) b += red[r][0][threadIdx.x] + red[r][1][threadIdx.x];
        part_b[(size_t)blockIdx.x * 32 + threadIdx.x] = b;
    }
}

// dW[i] = sum over chunks of part[chunk][i], in a fixed order: a workgroup takes 32
// weights, its 32 slices of 32 threads add the chunks k = slice (mod 32) in increasing k, and
// the 32 slice sums are added in slice order. Entries nw .. nw+31 are the bias.
constexpr int kRedW = 32, kRedSlices = 32;

__global__ __launch_bounds__(kRedW* kRedSlices) void wgrad_reduce_kernel(const float* __restrict__ part_w,
                                                                        const float* __restrict__ part_b,
                                                                        int chunks, int nw, float* __restrict__ dW,
                                                                        float* __restrict__ db) {
    __shared__ float red[kRedSlices][kRedW];
    const int w = threadIdx.x % kRedW, slice = threadIdx.x / kRedW;
    const int i = blockIdx.x * kRedW + w;
    float acc = 0.f;
    if (i < nw) {
#pragma unroll 8
        for (int k = slice; k < chunks; k += kRedSlices) acc += part_w[(size_t)k * nw + i];
    } else if (i < nw + 32) {
        for (int k = slice; k < chunks; k += kRedSlices) acc += part_b[(size_t)k * 32 + (i - nw)];
    }
    red[slice][w] = acc;
    __syncthreads();
    if (slice == 0) {
        float t = red[0][w];
#pragma unroll
        for (int q = 1; q < kRedSlices; ++q) t += red[q][w];
        if (i < nw)
            dW[i] = t;
        else if (i < nw + 32)
            db[i - nw] = t;
    }
}

// ------------------------------------------------------------------------------ mse_grad
// out, target: FP32 planes [img][3][H][W]; mask: coarse water mask [img][H][W].
// d_out (BF16 NHWC, 32 channels, 3..31 zero) = 2 act (out - target) * inv_n;
// partial[block] = sum act (out - target)^2.
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ out, const float* __restrict__ target,
                                                       const uint8_t* __restrict__ mask, int nimg, int H, int W,
                                                       float inv_n, float ts0, float ts1, float ts2,
                                                       uint16_t* __restrict__ d_out, double* __restrict__ partial) {
    const float tscale[3] = {ts0, ts1, ts2};
    __shared__ double lds[256];
    const size_t npix = (size_t)nimg * H * W;
    double s = 0.0;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < npix; q += (size_t)gridDim.x * 256) {
        const size_t img = q / ((size_t)H * W);
        const size_t pin = q - img * H * W;
        const int y = (int)(pin / W), x = (int)(pin - (size_t)y * W);
        const uint8_t* m = mask + img * H * W;
        const bool wet = m[pin] != 0;
        const bool act[3] = {wet, wet && x + 1 < W && m[pin + 1] != 0, wet && y + 1 < H && m[pin + W] != 0};
        uint16_t o[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t f = (img * 3 + c) * H * W + pin;
            const float r = act[c] ? out[f] - target[f] * tscale[c] : 0.f;
            s += (double)r * (double)r;
            o[c] = f2bf(2.f * r * inv_n);
        }
        uint4* dst = reinterpret_cast<uint4*>(d_out + q * 32);
        dst[0] = make_uint4(o[0] | ((uint32_t)o[1] << 16), o[2], 0u, 0u);
        dst[1] = make_uint4(0u, 0u, 0u, 0u);
        dst[2] = make_uint4(0u, 0u, 0u, 0u);
        dst[3] = make_uint4(0u, 0u, 0u, 0u);
    }
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = lds[0];
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partial, int n,
                                                           double* __restrict__ out) {
    __shared__ double lds[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = lds[0];
}

// ------------------------------------------------------------------------------ adam
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ theta, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int n,
                                                   AdamHyper hp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = hp.beta1 * m[i] + (1.f - hp.beta1) * g;
    const float vi = hp.beta2 * v[i] + (1.f - hp.beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= hp.lr * (mi * hp.inv_bc1) / (sqrtf(vi * hp.inv_bc2) + hp.eps);
}

// BF16 working copies of one layer: forward Wk[t][n][k] and data-gradient Wd[t'][k][n] with
// t' = 8 - t (flipped taps), from the FP32 master in forward layout [9][32][kin].
__global__ __launch_bounds__(256) void cast_weights_kernel(const float* __restrict__ master, int kin, int dkin,
                                                           uint16_t* __restrict__ wk, uint16_t* __restrict__ wd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9 * 32 * kin) return;
    const int t = i / (32 * kin), rem = i - t * 32 * kin;
    const int n = rem / kin, k = rem - n * kin;
    const uint16_t b = f2bf(master[i]);
    wk[i] = b;
    // data gradient: output channels are the forward input channels k (32 of them, kin
    // may be 16 or 32), reduced channels are the forward outputs n (dkin of them)
    if (wd && n < dkin) wd[((size_t)(8 - t) * 32 + k) * dkin + n] = b;
}

// ------------------------------------------------------------------------------ correct
__global__ __launch_bounds__(256) void correct_kernel(float* __restrict__ eta, float* __restrict__ u,
                                                      float* __restrict__ v, const float* __restrict__ out,
                                                      const uint8_t* __restrict__ mask, int H, int W, float s0,
                                                      float s1, float s2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= H * W) return;
    const int y = p / W, x = p - y * W;
    const bool wet = mask[p] != 0;
    if (!wet) return;
    const size_t plane = (size_t)H * W;
    eta[p] = fmaf(s0, out[p], eta[p]);
    if (x + 1 < W && mask[p + 1]) u[p] = fmaf(s1, out[plane + p], u[p]);
    if (y + 1 < H && mask[p + W]) v[p] = fmaf(s2, out[2 * plane + p], v[p]);
}

// ------------------------------------------------------------------------------ rmse
__global__ __launch_bounds__(256) void sqdiff_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                     const uint8_t* __restrict__ mask, int n,
                                                     double* __restrict__ partial) {
    __shared__ double lds[256];
    double s = 0.0;
    // 64-bit index: n may come close to 2^31, and the stride would overflow an int
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        if (mask[i]) {
            const double d = (double)a[i] - (double)b[i];
            s += d * d;
        }
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = lds[0];
}

// ------------------------------------------------------------------------------ sub3
// out[c][p] = a_c[p] - b_c[p] for the three fields (training target: fine ahead minus coarse).
__global__ __launch_bounds__(256) void sub3_kernel(const float* __restrict__ a0, const float* __restrict__ a1,
                                                   const float* __restrict__ a2, const float* __restrict__ b0,
                                                   const float* __restrict__ b1, const float* __restrict__ b2,
                                                   int n, float* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    out[p] = a0[p] - b0[p];
    out[(size_t)n + p] = a1[p] - b1[p];
    out[2 * (size_t)n + p] = a2[p] - b2[p];
}

// ------------------------------------------------------------------------------ moments
// partial[block] = (sum x, sum x^2) in double over entries with mask != 0 (all if no mask).
__global__ __launch_bounds__(256) void moments_kernel(const float* __restrict__ x, const uint8_t* __restrict__ mask,
                                                      int64_t n, double* __restrict__ partial) {
    __shared__ double l1[256], l2[256];
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        if (!mask || mask[i]) {
            const double v = (double)x[i];
            s1 += v;
            s2 += v * v;
        }
    l1[threadIdx.x] = s1;
    l2[threadIdx.x] = s2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            l1[threadIdx.x] += l1[threadIdx.x + h];
            l2[threadIdx.x] += l2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = l1[0];
        partial[2 * blockIdx.x + 1] = l2[0];
    }
}

__global__ __launch_bounds__(256) void moments_final_kernel(const double* __restrict__ partial, int n,
                                                            double* __restrict__ out) {
    __shared__ double l1[256], l2[256];
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        s1 += partial[2 * i];
        s2 += partial[2 * i + 1];
    }
    l1[threadIdx.x] = s1;
    l2[threadIdx.x] = s2;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            l1[threadIdx.x] += l1[threadIdx.x + h];
            l2[threadIdx.x] += l2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = l1[0];
        out[1] = l2[0];
    }
}

// ------------------------------------------------------------------------------ launchers
hipError_t launch_sub3(const float* a0, const float* a1, const float* a2, const float* b0, const float* b1,
                       const float* b2, int n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(sub3_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a0, a1, a2, b0, b1, b2, n, out);
    return hipGetLastError();
}

hipError_t launch_moments(const float* x, const uint8_t* mask, int64_t n, double* partial, int nblocks, double* out,
                          hipStream_t s) {
    hipLaunchKernelGGL(moments_kernel, dim3(nblocks), dim3(256), 0, s, x, mask, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(moments_final_kernel, dim3(1), dim3(256), 0, s, partial, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_restrict4(const float* eta, const float* u, const float* v, const float* H,
                            const uint8_t* mask, int NX, int NY, float* eta_c, float* u_c, float* v_c,
                            float* H_c, uint8_t* mask_c, hipStream_t s) {
    const int n = (NX / 4) * (NY / 4);
    hipLaunchKernelGGL(restrict4_kernel, dim3((n + 255) / 256), dim3(256), 0, s, eta, u, v, H, mask, NX, NY,
                       eta_c, u_c, v_c, H_c, mask_c);
    return hipGetLastError();
}

hipError_t launch_pack_input(const float* eta, const float* u, const float* v, const float* H,
                             const uint8_t* mask, int npix, const InputNorm& nrm, uint16_t* out,
                             hipStream_t s) {
    hipLaunchKernelGGL(pack_input_kernel, dim3((npix + 255) / 256), dim3(256), 0, s, eta, u, v, H, mask, npix, nrm,
                       out);
    return hipGetLastError();
}

// Workgroups of `kernel` the current device holds at once (CUs x occupancy), cached per
// device and kernel; 0 when the query fails.
int resident_groups(const void* kernel, int threads) {
    constexpr int kDevs = 16, kSlots = 8;
    static thread_local const void* keys[kDevs][kSlots] = {};
    static thread_local int vals[kDevs][kSlots] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevs) return 0;
    for (int i = 0; i < kSlots; ++i)
        if (keys[dev][i] == kernel) return vals[dev][i];
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess) return 0;
    const int v = cus * (per_cu > 0 ? per_cu : 1);
    for (int i = 0; i < kSlots; ++i)
        if (!keys[dev][i]) {
            keys[dev][i] = kernel;
            vals[dev][i] = v;
            break;
        }
    return v;
}

hipError_t launch_conv3x3_raw(const RawIn& raw, const InputNorm& nrm, const uint16_t* Wk, const float* bias,
                              uint16_t* out_bf, int H, int W, hipStream_t s) {
    const int tiles = ((W + kConvTW - 1) / kConvTW) * ((H + kConvTH - 1) / kConvTH);
    const int cap = resident_groups(reinterpret_cast<const void*>(&conv3x3_kernel<16, kConvRelu, true>), kConvThreads);
    if (cap < 1) return hipErrorInvalidDeviceFunction;
    hipLaunchKernelGGL((conv3x3_kernel<16, kConvRelu, true>), dim3(tiles < cap ? tiles : cap), dim3(kConvThreads), 0, s,
                       nullptr, Wk, bias, out_bf, nullptr, nullptr, H, W, 1, raw, nrm, CorrectOut{});
    return hipGetLastError();
}

hipError_t launch_conv3x3_correct(const uint16_t* in, const uint16_t* Wk, const float* bias, const CorrectOut& co,
                                  int H, int W, hipStream_t s) {
    const int tiles = ((W + kConvTW - 1) / kConvTW) * ((H + kConvTH - 1) / kConvTH);
    const int cap = resident_groups(reinterpret_cast<const void*>(&conv3x3_kernel<32, kConvCorrect>), kConvThreads);
    if (cap < 1) return hipErrorInvalidDeviceFunction;
    hipLaunchKernelGGL((conv3x3_kernel<32, kConvCorrect>), dim3(tiles < cap ? tiles : cap), dim3(kConvThreads), 0, s,
                       in, Wk, bias, nullptr, nullptr, nullptr, H, W, 1, RawIn{}, InputNorm{}, co);
    return hipGetLastError();
}

hipError_t launch_cnn_fused(const RawIn& raw, const InputNorm& nrm, const FusedNet& net, float* out_f, int H,
                            int W, hipStream_t s) {
    const int tiles = ((W + kFuTW - 1) / kFuTW) * ((H + kFuTH - 1) / kFuTH);
    const int cap = resident_groups(reinterpret_cast<const void*>(&cnn_fused_kernel), kFuThreads);
    if (cap < 1) return hipErrorInvalidDeviceFunction;
    hipLaunchKernelGGL(cnn_fused_kernel, dim3(tiles < cap ? tiles : cap), dim3(kFuThreads), 0, s, raw, nrm, net, out_f,
                       H, W);
    return hipGetLastError();
}

hipError_t launch_conv3x3(int kin, int mode, const uint16_t* in, const uint16_t* Wk, const float* bias,
                          uint16_t* out_bf, float* out_f, const uint16_t* relu_src, int nimg, int H, int W,
                          hipStream_t s) {
    // A persistent grid of as many workgroups as the device holds at once: each loads the
    // weights once and walks tiles (measured faster than a second round of workgroups).
    const int tiles = ((W + kConvTW - 1) / kConvTW) * ((H + kConvTH - 1) / kConvTH) * nimg;
    const dim3 block(kConvThreads);
#define SW2D_CONV_CASE(K, M)                                                                          \
    if (kin == K && mode == M) {                                                                      \
        const int cap = resident_groups(reinterpret_cast<const void*>(&conv3x3_kernel<K, M>), kConvThreads); \
        if (cap < 1) return hipErrorInvalidDeviceFunction;                                            \
        const dim3 grid(tiles < cap ? tiles : cap);                                                   \
        hipLaunchKernelGGL((conv3x3_kernel<K, M>), grid, block, 0, s, in, Wk, bias, out_bf, out_f, relu_src, H, \
                           W, nimg, RawIn{}, InputNorm{}, CorrectOut{});                              \
        return hipGetLastError();                                                                      \
    }
    SW2D_CONV_CASE(16, kConvRelu)
    SW2D_CONV_CASE(32, kConvRelu)
    SW2D_CONV_CASE(32, kConvLinear3)
    SW2D_CONV_CASE(32, kConvDgradMask)
#undef SW2D_CONV_CASE
    return hipErrorInvalidValue;
}

int wgrad_chunks(int nimg, int H, int W) {
    const int tiles = ((W + kWgTW - 1) / kWgTW) * ((H + kWgTH - 1) / kWgTH) * nimg;
    return (tiles + kWgTiles - 1) / kWgTiles;
}

hipError_t launch_wgrad(int kin, const uint16_t* x, const uint16_t* dy, int nimg, int H, int W, float* part_w,
                        float* part_b, float* dW, float* db, hipStream_t s) {
    const int chunks = wgrad_chunks(nimg, H, W);
    if (kin == 16)
        hipLaunchKernelGGL(wgrad_kernel<16>, dim3(chunks), dim3(kWgThreads), 0, s, x, dy, nimg, H, W, part_w, part_b);
    else if (kin == 32)
        hipLaunchKernelGGL(wgrad_kernel<32>, dim3(chunks), dim3(kWgThreads), 0, s, x, dy, nimg, H, W, part_w, part_b);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nw = 9 * 32 * kin;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((nw + 32 + kRedW - 1) / kRedW), dim3(kRedW * kRedSlices), 0, s, part_w,
                       part_b, chunks, nw, dW, db);
    return hipGetLastError();
}

hipError_t launch_mse_grad(const float* out, const float* target, const uint8_t* mask, int nimg, int H, int W,
                           float inv_n, const float* tscale, uint16_t* d_out, double* partial, int nblocks,
                           double* loss, hipStream_t s) {
    hipLaunchKernelGGL(mse_grad_kernel, dim3(nblocks), dim3(256), 0, s, out, target, mask, nimg, H, W, inv_n,
                       tscale[0], tscale[1], tscale[2], d_out, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial, nblocks, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int n, const AdamHyper& hp,
                       hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, theta, grad, m, v, n, hp);
    return hipGetLastError();
}

hipError_t launch_cast_weights(const float* master, int kin, int dkin, uint16_t* wk, uint16_t* wd, hipStream_t s) {
    const int n = 9 * 32 * kin;
    hipLaunchKernelGGL(cast_weights_kernel, dim3((n + 255) / 256), dim3(256), 0, s, master, kin, dkin, wk, wd);
    return hipGetLastError();
}

hipError_t launch_correct(float* eta, float* u, float* v, const float* out, const uint8_t* mask, int H, int W,
                          const float* t_std, hipStream_t s) {
    hipLaunchKernelGGL(correct_kernel, dim3((H * W + 255) / 256), dim3(256), 0, s, eta, u, v, out, mask, H, W,
                       t_std[0], t_std[1], t_std[2]);
    return hipGetLastError();
}

hipError_t launch_sqdiff(const float* a, const float* b, const uint8_t* mask, int n, double* partial, int nblocks,
                         double* out, hipStream_t s) {
    hipLaunchKernelGGL(sqdiff_kernel, dim3(nblocks), dim3(256), 0, s, a, b, mask, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial, nblocks, out);
    return hipGetLastError();
}

}  // namespace sur
}  // namespace sw2d
