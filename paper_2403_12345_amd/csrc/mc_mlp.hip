// mc_mlp.hip -- inference and training kernels of the importance network.
//
// Training is full-batch: every sample is a (features, target ln I, weight)
// triple; the loss is sum_i w_i (y_i - t_i)^2 / sum_i w_i.  One wave handles 64
// samples: forward (first layer on the vector units, 64x64 layer on the matrix
// cores), backward (dW2 = H1^T dZ2 and dH1 = dZ2 W2^T on the matrix cores with
// dZ2 rounded to BF16, the rest on the vector units), and writes its partial
// gradient row; rows are summed in a fixed order, then one Adam step updates
// the FP32 master parameters and their BF16 copies.
#include "mc_mlp.h"
#include "mc_internal.h"

#pragma clang fp contract(off)

namespace mc {

// ---------------------------------------------------------------------------
// inference over a list of feature vectors
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_forward(MlpDev m, uint32_t n, const float *X, float *Y)
{
    __shared__ __attribute__((aligned(16))) uint16_t h1s[4][64 * H1_STRIDE];
    __shared__ float ys[4][64];
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    const int wave = threadIdx.x >> 6;
    float f[4] = {0.f, 0.f, 0.f, 0.f};
    if (i < n) {
#pragma unroll
        for (int k = 0; k < 4; ++k) f[k] = X[(size_t)i * 4 + k];
    }
    const float y = wave_mlp(m, f, h1s[wave], ys[wave]);
    if (i < n) Y[i] = y;
}

// ---------------------------------------------------------------------------
// gradient of the weighted loss: one wave per 64 samples
// ---------------------------------------------------------------------------
constexpr int PROW = MLP_NPAR + 1;  // partial row: gradient, then the loss term
constexpr int Z2_STRIDE = 65;

__global__ void __launch_bounds__(64) k_mlp_grad(MlpDev m, uint32_t n, const float *X, const float *T,
                                                 const float *Wt, const float *inv_wsum_p, float *partial)
{
    const float inv_wsum = *inv_wsum_p;
    __shared__ __attribute__((aligned(16))) uint16_t h1s[64 * H1_STRIDE];
    __shared__ __attribute__((aligned(16))) uint16_t dz2s[64 * H1_STRIDE];
    __shared__ float z2s[64 * Z2_STRIDE];
    __shared__ float xs[64 * 4];
    __shared__ float dys[64];
    __shared__ float lossv[64];
    const int lane = threadIdx.x, r16 = lane & 15, g4 = lane >> 4;
    const uint32_t s = blockIdx.x * 64 + lane;
    const bool valid = s < n;
    float f[4] = {0.f, 0.f, 0.f, 0.f};
    float t = 0.f, w = 0.f;
    if (valid) {
#pragma unroll
        for (int k = 0; k < 4; ++k) f[k] = X[(size_t)s * 4 + k];
        t = T[s];
        w = Wt[s];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) xs[lane * 4 + k] = bf16_round(f[k]);
    mlp_layer1(m, f, h1s + lane * H1_STRIDE);
    __syncthreads();
    // z2 = h1 W2 (without b2)
    for (int rt = 0; rt < 4; ++rt) {
        for (int ct = 0; ct < 4; ++ct) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const bf16x8 a = load_bf16x8(h1s + (rt * 16 + r16) * H1_STRIDE + kk * 32 + 8 * g4);
                const bf16x8 b = load_bf16x8(m.W2t + (ct * 16 + r16) * MLP_HID + kk * 32 + 8 * g4);
                acc = mfma_16x16x32(a, b, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) z2s[(rt * 16 + 4 * g4 + r) * Z2_STRIDE + ct * 16 + r16] = acc[r];
        }
    }
    __syncthreads();
    // output and dL/dy of this lane's sample
    float y = m.theta[MLP_B3];
    for (int c = 0; c < MLP_HID; ++c)
        y = y + silu_f(z2s[lane * Z2_STRIDE + c] + m.theta[MLP_B2 + c]) * bf16_to_f32(m.w3[c]);
    const float dy = valid ? 2.0f * w * (y - t) * inv_wsum : 0.0f;
    lossv[lane] = valid ? w * (y - t) * (y - t) * inv_wsum : 0.0f;
    dys[lane] = dy;
    // dz2 (rounded to BF16 for the two products it feeds)
    for (int c = 0; c < MLP_HID; ++c) {
        const float zz = z2s[lane * Z2_STRIDE + c] + m.theta[MLP_B2 + c];
        dz2s[lane * H1_STRIDE + c] = f32_to_bf16(dy * bf16_to_f32(m.w3[c]) * silu_grad_f(zz));
    }
    __syncthreads();
    float *row = partial + (size_t)blockIdx.x * PROW;
    // per output unit c = lane: dw3[c], db2[c] (samples in order)
    {
        const int c = lane;
        const float b2 = m.theta[MLP_B2 + c], w3 = bf16_to_f32(m.w3[c]);
        float gw3 = 0.f, gb2 = 0.f;
        for (int q = 0; q < 64; ++q) {
            const float zz = z2s[q * Z2_STRIDE + c] + b2;
            gw3 = gw3 + silu_f(zz) * dys[q];
            gb2 = gb2 + dys[q] * w3 * silu_grad_f(zz);
        }
        row[MLP_W3 + c] = gw3;
        row[MLP_B2 + c] = gb2;
    }
    if (lane == 0) {
        float gb3 = 0.f, l = 0.f;
        for (int q = 0; q < 64; ++q) {
            gb3 = gb3 + dys[q];
            l = l + lossv[q];
        }
        row[MLP_B3] = gb3;
        row[MLP_NPAR] = l;
    }
    // dW2[i][c] = sum over samples of h1[s][i] dz2[s][c]
    for (int it = 0; it < 4; ++it) {
        for (int ct = 0; ct < 4; ++ct) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                uint16_t av[8], bv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int q = kk * 32 + 8 * g4 + e;  // sample
                    av[e] = h1s[q * H1_STRIDE + it * 16 + r16];
                    bv[e] = dz2s[q * H1_STRIDE + ct * 16 + r16];
                }
                acc = mfma_16x16x32(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) row[MLP_W2 + (it * 16 + 4 * g4 + r) * MLP_HID + ct * 16 + r16] = acc[r];
        }
    }
    // dh1 = dz2 W2^T, then dz1 = dh1 silu'(z1); dW1, db1
    for (int it = 0; it < 4; ++it) {
        const int i = it * 16 + r16;
        float gw1[4] = {0.f, 0.f, 0.f, 0.f}, gb1 = 0.f;
        const float b1 = m.theta[MLP_B1 + i];
        float w1[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w1[k] = bf16_to_f32(m.W1[k * MLP_HID + i]);
        for (int st = 0; st < 4; ++st) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const bf16x8 a = load_bf16x8(dz2s + (st * 16 + r16) * H1_STRIDE + kk * 32 + 8 * g4);
                const bf16x8 b = load_bf16x8(m.W2 + (it * 16 + r16) * MLP_HID + kk * 32 + 8 * g4);
                acc = mfma_16x16x32(a, b, acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = st * 16 + 4 * g4 + r;
                float z1 = 0.f;
#pragma unroll
                for (int k = 0; k < 4; ++k) z1 = z1 + xs[q * 4 + k] * w1[k];
                z1 = z1 + b1;
                const float dz1 = acc[r] * silu_grad_f(z1);
#pragma unroll
                for (int k = 0; k < 4; ++k) gw1[k] = gw1[k] + xs[q * 4 + k] * dz1;
                gb1 = gb1 + dz1;
            }
        }
        // sum the four lane groups holding the same unit i
#pragma unroll
        for (int o = 16; o < 64; o <<= 1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) gw1[k] = gw1[k] + __shfl_xor(gw1[k], o, 64);
            gb1 = gb1 + __shfl_xor(gb1, o, 64);
        }
        if (g4 == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) row[MLP_W1 + k * MLP_HID + i] = gw1[k];
            row[MLP_B1 + i] = gb1;
        }
    }
}

// out = 1 / (sum of the n weights), one workgroup (fixed summation order)
__global__ void __launch_bounds__(256) k_mlp_wsum(const float *W, uint32_t n, float *out)
{
    __shared__ float part[256];
    float s = 0.f;
    for (uint32_t i = threadIdx.x; i < n; i += 256) s = s + W[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] = part[threadIdx.x] + part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 1.0f / part[0];
}

// grad[j] = sum over rows of partial[row][j], rows in order
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *partial, uint32_t rows, float *grad)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= PROW) return;
    float s = 0.f;
    for (uint32_t r = 0; r < rows; ++r) s = s + partial[(size_t)r * PROW + j];
    grad[j] = s;
}

__device__ __forceinline__ void refresh_bf16(uint32_t j, float v, uint16_t *W1, uint16_t *W2, uint16_t *W2t,
                                             uint16_t *w3)
{
    if (j < (uint32_t)MLP_B1) {
        W1[j] = f32_to_bf16(v);
    } else if (j >= (uint32_t)MLP_W2 && j < (uint32_t)MLP_B2) {
        const uint32_t e = j - MLP_W2, k = e / MLP_HID, nn = e % MLP_HID;
        const uint16_t b = f32_to_bf16(v);
        W2[k * MLP_HID + nn] = b;
        W2t[nn * MLP_HID + k] = b;
    } else if (j >= (uint32_t)MLP_W3 && j < (uint32_t)MLP_B3) {
        w3[j - MLP_W3] = f32_to_bf16(v);
    }
}

// Adam (Kingma & Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); then the BF16 copies.
__global__ void __launch_bounds__(256) k_mlp_adam(float *theta, float *mom, float *vel, const float *grad, float t,
                                                  float lr, uint16_t *W1, uint16_t *W2, uint16_t *W2t, uint16_t *w3)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= (uint32_t)MLP_NPAR) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = grad[j];
    const float mm = b1 * mom[j] + (1.0f - b1) * g;
    const float vv = b2 * vel[j] + (1.0f - b2) * g * g;
    mom[j] = mm;
    vel[j] = vv;
    const float mh = mm / (1.0f - powf(b1, t));
    const float vh = vv / (1.0f - powf(b2, t));
    const float th = theta[j] - lr * mh / (sqrtf(vh) + eps);
    theta[j] = th;
    refresh_bf16(j, th, W1, W2, W2t, w3);
}

__global__ void __launch_bounds__(256) k_mlp_sync(const float *theta, uint16_t *W1, uint16_t *W2, uint16_t *W2t,
                                                  uint16_t *w3)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j < (uint32_t)MLP_NPAR) refresh_bf16(j, theta[j], W1, W2, W2t, w3);
}

// ---------------------------------------------------------------------------
// initial parameters: W1 ~ U(-1/2, 1/2), W2 and w3 ~ U(-1/8, 1/8) (uniform in
// +-1/sqrt(fan in)), biases 0; draw j of the key `seed` from the Philox stream
// of pid j, lineage MLP_INIT_LINEAGE
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_init(float *theta, uint64_t seed)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= (uint32_t)MLP_NPAR) return;
    Rng rng(seed, (uint64_t)j, MLP_INIT_LINEAGE, 0u);
    const double u = 2.0 * rng.next() - 1.0;
    double v = 0.0;
    if (j < (uint32_t)MLP_B1) v = 0.5 * u;
    else if (j >= (uint32_t)MLP_W2 && j < (uint32_t)MLP_B2) v = 0.125 * u;
    else if (j >= (uint32_t)MLP_W3 && j < (uint32_t)MLP_B3) v = 0.125 * u;
    theta[j] = (float)v;
}

// ---------------------------------------------------------------------------
// training samples from the forward importance sums: every cell with at least
// min_credits detector credits gives `replicas` samples (cells in index
// order): features (x centre / L, f_y, f_z, ln E-bin centre), target
// ln(num / den), weight 1 / (1 / cnt + rel_floor^2).  The slab is invariant
// in y and z: f_y and f_z are drawn uniform on [-1, 1] (draws 2r and 2r + 1 of
// pid = cell, lineage IMP_SAMPLE_LINEAGE) so the network learns that.  One
// workgroup, a running block scan over the cells.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_imp_samples(ImpSampleArgs a)
{
    __shared__ uint32_t wsum[4];
    __shared__ float wmin[4], wmax[4];
    __shared__ uint32_t base;
    __shared__ float tmin, tmax;
    if (threadIdx.x == 0) {
        base = 0;
        tmin = INFINITY;
        tmax = -INFINITY;
    }
    __syncthreads();
    const int32_t cells = a.nx * a.ne;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int32_t c0 = 0; c0 < cells; c0 += 256) {
        const int32_t g = c0 + (int32_t)threadIdx.x;
        bool ok = false;
        if (g < cells) ok = a.cnt[g] >= a.min_credits && a.num[g] > 0.0 && a.den[g] > 0.0;
        const uint64_t m = __ballot(ok);
        float tg = 0.f;
        if (ok) tg = (float)log(a.num[g] / a.den[g]);
        float lo = ok ? tg : INFINITY, hi = ok ? tg : -INFINITY;
        for (int o = 32; o > 0; o >>= 1) {
            lo = fminf(lo, __shfl_xor(lo, o, 64));
            hi = fmaxf(hi, __shfl_xor(hi, o, 64));
        }
        if (lane == 0) {
            wsum[wave] = (uint32_t)__popcll(m);
            wmin[wave] = lo;
            wmax[wave] = hi;
        }
        __syncthreads();
        uint32_t pre = base;
        for (int w = 0; w < wave; ++w) pre += wsum[w];
        pre += (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (ok) {
            const int32_t ix = g % a.nx, e = g / a.nx;
            const double xc = a.x0 + (a.x1 - a.x0) * ((double)ix + 0.5) / (double)a.nx;
            const float fx = (float)(xc / a.length);
            const float fe = (float)(((double)e + 0.5) / (double)a.ne);
            const float wt = (float)(1.0 / (1.0 / a.cnt[g] + a.rel_floor * a.rel_floor));
            Rng rng(a.seed, (uint64_t)g, IMP_SAMPLE_LINEAGE, 0u);
            for (int32_t r = 0; r < a.replicas; ++r) {
                const size_t k = (size_t)pre * a.replicas + r;
                const double uy = rng.next(), uz = rng.next();
                a.X[k * 4 + 0] = fx;
                a.X[k * 4 + 1] = (float)(2.0 * uy - 1.0);
                a.X[k * 4 + 2] = (float)(2.0 * uz - 1.0);
                a.X[k * 4 + 3] = fe;
                a.T[k] = tg;
                a.W[k] = wt;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
            for (int w = 0; w < 4; ++w) {
                tmin = fminf(tmin, wmin[w]);
                tmax = fmaxf(tmax, wmax[w]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *a.n_out = (int32_t)(base * (uint32_t)a.replicas);
        if (a.range_out) {
            a.range_out[0] = tmin;
            a.range_out[1] = tmax;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_mlp_init(float *theta, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_init, dim3((MLP_NPAR + 255) / 256), dim3(256), 0, st, theta, seed);
    return hipGetLastError();
}

hipError_t launch_imp_samples(const ImpSampleArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_imp_samples, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}
hipError_t launch_mlp_forward(const MlpDev &m, uint32_t n, const float *X, float *Y, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, st, m, n, X, Y);
    return hipGetLastError();
}

size_t mlp_partial_floats(uint32_t n) { return (size_t)((n + 63) / 64) * PROW; }

hipError_t launch_mlp_wsum(const float *W, uint32_t n, float *inv_wsum, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_wsum, dim3(1), dim3(256), 0, st, W, n, inv_wsum);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpDev &m, uint32_t n, const float *X, const float *T, const float *W,
                           const float *inv_wsum, float *partial, float *grad_and_loss, hipStream_t st)
{
    const uint32_t rows = (n + 63) / 64;
    hipLaunchKernelGGL(k_mlp_grad, dim3(rows), dim3(64), 0, st, m, n, X, T, W, inv_wsum, partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((PROW + 255) / 256), dim3(256), 0, st, partial, rows, grad_and_loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *theta, float *mom, float *vel, const float *grad, int step, float lr, uint16_t *W1,
                           uint16_t *W2, uint16_t *W2t, uint16_t *w3, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPAR + 255) / 256), dim3(256), 0, st, theta, mom, vel, grad, (float)step,
                       lr, W1, W2, W2t, w3);
    return hipGetLastError();
}

hipError_t launch_mlp_sync(const float *theta, uint16_t *W1, uint16_t *W2, uint16_t *W2t, uint16_t *w3, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_sync, dim3((MLP_NPAR + 255) / 256), dim3(256), 0, st, theta, W1, W2, W2t, w3);
    return hipGetLastError();
}

}  // namespace mc
