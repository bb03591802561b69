// mlp.hpp -- kernels of the surrogate network: a fully connected
// 5 -> 128 -> 128 -> 128 -> 16 network with tanh hidden activations, FP32.
//
// Every matrix product runs on the matrix cores: one wave computes a 16x16
// output tile with v_mfma_f32_16x16x4_f32, walking the contraction four at a
// time.  Operand layout of that instruction (per lane l of the wave):
//   A (16x4): A[l % 16][l / 16]   B (4x16): B[l / 16][l % 16]
//   D (16x16): four values, D[4 (l / 16) + r][l % 16], r = 0..3.
// Products are written by exactly one wave per element and every sum has a
// fixed order, so training is bitwise reproducible.
#pragma once

#include "device_common.hpp"

namespace odk {

constexpr int kMlpIn = 5, kMlpHid = 128, kMlpOut = 16, kMlpLayers = 4;
constexpr int kMlpParams = kMlpIn * kMlpHid + kMlpHid + 2 * (kMlpHid * kMlpHid + kMlpHid) +
                           kMlpHid * kMlpOut + kMlpOut;   // 35,856

enum : int { kEpiNone = 0, kEpiBias = 1, kEpiBiasTanh = 2, kEpiTanhGrad = 3 };

struct Strided {
    const float* p;
    long long s0, s1;   // element (i, j) at p[i * s0 + j * s1]
    __device__ __forceinline__ float at(int i, int j) const { return p[i * s0 + j * s1]; }
};

// C(m, n) = epilogue(sum_k A(m, k) B(k, n)) for an M x N output; one wave per
// 16x16 tile (grid = ceil(M/16) * ceil(N/16) waves, 64 threads per block).
//   kEpiBias:      + bias[n]
//   kEpiBiasTanh:  tanh(. + bias[n])
//   kEpiTanhGrad:  . * (1 - Y(m, n)^2)   (Y: the tanh output of the layer)
template <int EPI>
__global__ __launch_bounds__(64) void mfma_gemm(Strided A, Strided B, float* __restrict__ C,
                                                long long ldc, int M, int N, int K,
                                                const float* __restrict__ bias, Strided Y)
{
    const int tiles_n = (N + 15) / 16;
    const int m0 = (blockIdx.x / tiles_n) * 16, n0 = (blockIdx.x % tiles_n) * 16;
    const int l = threadIdx.x;
    const int ra = m0 + (l & 15), kq = l >> 4, cb = n0 + (l & 15);
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + kq;
        const float a = (ra < M && k < K) ? A.at(ra, k) : 0.0f;
        const float b = (k < K && cb < N) ? B.at(k, cb) : 0.0f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = m0 + 4 * kq + r, n = cb;
        if (m < M && n < N) {
            float c = acc[r];
            if (EPI == kEpiBias || EPI == kEpiBiasTanh) c += bias[n];
            if (EPI == kEpiBiasTanh) c = tanhf(c);
            if (EPI == kEpiTanhGrad) {
                const float y = Y.at(m, n);
                c *= 1.0f - y * y;
            }
            C[m * ldc + n] = c;
        }
    }
}

// Column sums of a B x N matrix (bias gradients), one thread per column,
// rows in order.
__global__ void colsum_kernel(const float* __restrict__ D, int B, int N, float* __restrict__ out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += D[(long long)b * N + n];
    out[n] = s;
}

// Minibatch gather with input normalisation to [-1, 1] (per-feature box lo..hi)
// and target standardisation (per-output mean, std).
__global__ void gather_kernel(const float* __restrict__ X, const float* __restrict__ T,
                              const int* __restrict__ idx, int B, const float* __restrict__ norm,
                              float* __restrict__ Xb, float* __restrict__ Tb)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B) return;
    const int r = idx[t];
    for (int c = 0; c < kMlpIn; ++c) {
        const float lo = norm[c], hi = norm[kMlpIn + c];
        Xb[t * kMlpIn + c] = 2.0f * (X[(long long)r * kMlpIn + c] - lo) / (hi - lo) - 1.0f;
    }
    if (T)
        for (int c = 0; c < kMlpOut; ++c) {
            const float mu = norm[2 * kMlpIn + c], sd = norm[2 * kMlpIn + kMlpOut + c];
            Tb[t * kMlpOut + c] = (T[(long long)r * kMlpOut + c] - mu) / sd;
        }
}

// Input normalisation of n rows in place order; flags rows outside the box.
__global__ void normalize_kernel(const float* __restrict__ X, int n, const float* __restrict__ norm,
                                 float* __restrict__ Xn, int* __restrict__ inside)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int ok = 1;
    for (int c = 0; c < kMlpIn; ++c) {
        const float lo = norm[c], hi = norm[kMlpIn + c];
        const float z = 2.0f * (X[(long long)t * kMlpIn + c] - lo) / (hi - lo) - 1.0f;
        ok &= (z >= -1.0f && z <= 1.0f) ? 1 : 0;
        Xn[t * kMlpIn + c] = z;
    }
    inside[t] = ok;
}

// Standardised outputs back to target units: y * std + mean.
__global__ void denormalize_kernel(float* __restrict__ Y, int n, const float* __restrict__ norm)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * kMlpOut) return;
    const int c = t % kMlpOut;
    Y[t] = Y[t] * norm[2 * kMlpIn + kMlpOut + c] + norm[2 * kMlpIn + c];
}

// Mean-squared-error gradient dL/dY = 2 (Y - T) / (B * outputs) and the
// per-row squared error (summed by the host for the loss history).
__global__ void mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T, int B,
                                float* __restrict__ dY, float* __restrict__ row_err)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float e = 0.0f;
    const float s = 2.0f / (float)(B * kMlpOut);
    for (int c = 0; c < kMlpOut; ++c) {
        const float d = Y[b * kMlpOut + c] - T[b * kMlpOut + c];
        dY[b * kMlpOut + c] = s * d;
        e += d * d;
    }
    row_err[b] = e;
}

// Adam update of the flat parameter vector (bias-corrected moments).
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace odk
