// mc_mlp.h -- the importance network on gfx950: 4 -> 64 -> 64 -> 1 with SiLU
// hidden activations, predicting ln I from (x/L, y/L, z/L, normalised ln E).
// Weight matrices are BF16, the 64x64 products run on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), everything else is FP32.
// Rounding points: inputs, W1, W2, w3 and the first hidden activation are
// BF16; biases and accumulations are FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mc {

constexpr int MLP_IN = 4, MLP_HID = 64;
// flat parameter order: W1[4][64], b1[64], W2[64][64], b2[64], w3[64], b3
constexpr int MLP_W1 = 0, MLP_B1 = 256, MLP_W2 = 320, MLP_B2 = 4416, MLP_W3 = 4480, MLP_B3 = 4544;
constexpr int MLP_NPAR = 4545;
constexpr int H1_STRIDE = 72;  // padded LDS row of 64 BF16 activations (fewer bank conflicts)

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// Device copies of the network: FP32 biases (and master weights for
// training) plus BF16 copies of the matrices in the layouts the matrix-core
// fragments read.
struct MlpDev {
    const float *theta;      // [MLP_NPAR] FP32 parameters (flat order above)
    const uint16_t *W1;      // BF16 [4][64]
    const uint16_t *W2;      // BF16 [64][64], W2[k][n]: input k -> output n
    const uint16_t *W2t;     // BF16 [64][64], W2t[n][k] = W2[k][n]
    const uint16_t *w3;      // BF16 [64]
};

// FP32 -> BF16 bits, round to nearest even (NaN kept a NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float bf16_round(float x) { return bf16_to_f32(f32_to_bf16(x)); }

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad_f(float z)
{
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

// Matrix-core tile: D[16x16] += A[16x32] B[32x16], one wave.  Fragment layout
// of v_mfma_f32_16x16x32_bf16: lane l holds A[l % 16][8 (l / 16) + 0..7],
// B[8 (l / 16) + 0..7][l % 16] and D[4 (l / 16) + r][l % 16], r = 0..3.
__device__ __forceinline__ f32x4 mfma_16x16x32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// First layer of one sample (VALU): h1 = bf16(silu(bf16(f) W1 + b1)), written
// as BF16 into row `row` of the LDS activation block.
__device__ __forceinline__ void mlp_layer1(const MlpDev &m, const float (&f)[4], uint16_t *h1row)
{
    float x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = bf16_round(f[k]);
    for (int j = 0; j < MLP_HID; ++j) {
        float z = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) z = z + x[k] * bf16_to_f32(m.W1[k * MLP_HID + j]);
        z = z + m.theta[MLP_B1 + j];
        h1row[j] = f32_to_bf16(silu_f(z));
    }
}

// ln I of the 64 samples held one per lane of the calling wave.  Every lane
// of every wave of the workgroup must call it (it synchronises the
// workgroup); h1s is this wave's LDS block of 64 * H1_STRIDE BF16 and ys its
// 64 floats.
__device__ inline float wave_mlp(const MlpDev &m, const float (&f)[4], uint16_t *h1s, float *ys)
{
    const int lane = threadIdx.x & 63;
    mlp_layer1(m, f, h1s + lane * H1_STRIDE);
    __syncthreads();
    const int r16 = lane & 15, g4 = lane >> 4;
    const float b3 = m.theta[MLP_B3];
    for (int rt = 0; rt < 4; ++rt) {
        f32x4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const bf16x8 a = load_bf16x8(h1s + (rt * 16 + r16) * H1_STRIDE + kk * 32 + 8 * g4);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const bf16x8 b = load_bf16x8(m.W2t + (ct * 16 + r16) * MLP_HID + kk * 32 + 8 * g4);
                acc[ct] = mfma_16x16x32(a, b, acc[ct]);
            }
        }
        // y = sum over the 64 outputs of silu(z2 + b2) * w3, per row
        float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int col = ct * 16 + r16;
            const float b2 = m.theta[MLP_B2 + col], w3 = bf16_to_f32(m.w3[col]);
#pragma unroll
            for (int r = 0; r < 4; ++r) part[r] = part[r] + silu_f(acc[ct][r] + b2) * w3;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) part[r] = part[r] + __shfl_xor(part[r], o, 64);
        }
        if (r16 == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) ys[rt * 16 + 4 * g4 + r] = part[r] + b3;
        }
    }
    __syncthreads();
    return ys[lane];
}

// Importance features of a point, computed in FP64 and handed over as FP32:
// (x/L, clip(y/L, -1, 1), clip(z/L, -1, 1), (ln E - ln_emin) / ln_erange).
__device__ __forceinline__ void mlp_features(double x, double y, double z, double E, double L, double ln_emin,
                                             double ln_erange, float (&f)[4])
{
    f[0] = (float)(x / L);
    f[1] = (float)fmin(1.0, fmax(-1.0, y / L));
    f[2] = (float)fmin(1.0, fmax(-1.0, z / L));
    f[3] = (float)((log(E) - ln_emin) / ln_erange);
}

}  // namespace mc
