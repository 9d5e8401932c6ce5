// bz_mlp.hpp -- the work predictor: a 4 -> 64 -> 64 -> 1 multilayer
// perceptron in FP32 with ReLU hidden layers, its forward pass, the gradient
// of the mean squared error and an Adam step, as HIP kernels.
//
// Parameter vector (BZ_MLP_PARAMS floats, row-major weight matrices):
//   W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3
// The network maps features of a code (field, length, dimension, rank
// deficit of the last information set) to log10 of the combinations the
// method evaluates on it; it only orders work, it never changes a result.
//
// Every sum runs in a fixed order (no atomics), so a training run is
// reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bz {

constexpr int MLP_IN = 4, MLP_H = 64;

// The network's inputs for a code: field, length, dimension and the rank
// deficit k - k_m of its last information set, normalised as in training.
__host__ __device__ inline void mlp_features(int p, int n, int k, int deficit, float *f) {
    f[0] = ((float)p - 5.0f) / 2.0f;
    f[1] = ((float)n - 60.0f) / 30.0f;
    f[2] = ((float)k - 25.0f) / 15.0f;
    f[3] = (float)deficit / 8.0f;
}
constexpr int MLP_W1 = 0, MLP_B1 = MLP_W1 + MLP_H * MLP_IN, MLP_W2 = MLP_B1 + MLP_H, MLP_B2 = MLP_W2 + MLP_H * MLP_H,
              MLP_W3 = MLP_B2 + MLP_H, MLP_B3 = MLP_W3 + MLP_H, MLP_NPARAM = MLP_B3 + 1;

// One sample per thread; the parameters are staged in LDS once per workgroup.
// cache (optional): per sample the post-activation h1[64] and h2[64].
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ prm, const float *__restrict__ x,
                                                          int n, float *__restrict__ y, float *__restrict__ cache) {
    __shared__ float sp[MLP_NPARAM];
    for (int i = threadIdx.x; i < MLP_NPARAM; i += blockDim.x) sp[i] = prm[i];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float in[MLP_IN];
#pragma unroll
    for (int j = 0; j < MLP_IN; j++) in[j] = x[(size_t)s * MLP_IN + j];
    float h1[MLP_H];
#pragma unroll
    for (int i = 0; i < MLP_H; i++) {
        float a = sp[MLP_B1 + i];
#pragma unroll
        for (int j = 0; j < MLP_IN; j++) a = fmaf(sp[MLP_W1 + i * MLP_IN + j], in[j], a);
        h1[i] = fmaxf(a, 0.0f);
    }
    float out = sp[MLP_B3];
    for (int i = 0; i < MLP_H; i++) {
        float a = sp[MLP_B2 + i];
#pragma unroll
        for (int j = 0; j < MLP_H; j++) a = fmaf(sp[MLP_W2 + i * MLP_H + j], h1[j], a);
        const float h2 = fmaxf(a, 0.0f);
        out = fmaf(sp[MLP_W3 + i], h2, out);
        if (cache) cache[(size_t)s * 2 * MLP_H + MLP_H + i] = h2;
    }
    if (cache) {
#pragma unroll
        for (int i = 0; i < MLP_H; i++) cache[(size_t)s * 2 * MLP_H + i] = h1[i];
    }
    y[s] = out;
}

// Per sample: dL/dy = 2 (y - t) / n for L = mean (y - t)^2, then the
// pre-activation gradients of both hidden layers (ReLU passes the gradient
// where the unit is positive).  dz: per sample dz1[64], dz2[64], dy.
__global__ __launch_bounds__(256) void mlp_delta_kernel(const float *__restrict__ prm, const float *__restrict__ t,
                                                        int n, const float *__restrict__ y,
                                                        const float *__restrict__ cache, float *__restrict__ dz) {
    __shared__ float sp[MLP_NPARAM];
    for (int i = threadIdx.x; i < MLP_NPARAM; i += blockDim.x) sp[i] = prm[i];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float *h = cache + (size_t)s * 2 * MLP_H;
    const float dy = 2.0f * (y[s] - t[s]) / (float)n;
    float d2[MLP_H];
#pragma unroll
    for (int i = 0; i < MLP_H; i++) d2[i] = h[MLP_H + i] > 0.0f ? dy * sp[MLP_W3 + i] : 0.0f;
    float *o = dz + (size_t)s * (2 * MLP_H + 1);
    for (int j = 0; j < MLP_H; j++) {
        float a = 0.0f;
#pragma unroll
        for (int i = 0; i < MLP_H; i++) a = fmaf(sp[MLP_W2 + i * MLP_H + j], d2[i], a);
        o[j] = h[j] > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < MLP_H; i++) o[MLP_H + i] = d2[i];
    o[2 * MLP_H] = dy;
}

// One thread per parameter: its gradient summed over the samples in order.
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float *__restrict__ x, int n,
                                                       const float *__restrict__ cache, const float *__restrict__ dz,
                                                       float *__restrict__ grad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= MLP_NPARAM) return;
    const int DZ = 2 * MLP_H + 1, CH = 2 * MLP_H;
    float acc = 0.0f;
    if (q < MLP_B1) {  // W1[i][j]: dz1_i x_j
        const int i = q / MLP_IN, j = q % MLP_IN;
        for (int s = 0; s < n; s++) acc = fmaf(dz[(size_t)s * DZ + i], x[(size_t)s * MLP_IN + j], acc);
    } else if (q < MLP_W2) {  // b1[i]
        const int i = q - MLP_B1;
        for (int s = 0; s < n; s++) acc += dz[(size_t)s * DZ + i];
    } else if (q < MLP_B2) {  // W2[i][j]: dz2_i h1_j
        const int i = (q - MLP_W2) / MLP_H, j = (q - MLP_W2) % MLP_H;
        for (int s = 0; s < n; s++) acc = fmaf(dz[(size_t)s * DZ + MLP_H + i], cache[(size_t)s * CH + j], acc);
    } else if (q < MLP_W3) {  // b2[i]
        const int i = q - MLP_B2;
        for (int s = 0; s < n; s++) acc += dz[(size_t)s * DZ + MLP_H + i];
    } else if (q < MLP_B3) {  // w3[i]: dy h2_i
        const int i = q - MLP_W3;
        for (int s = 0; s < n; s++) acc = fmaf(dz[(size_t)s * DZ + 2 * MLP_H], cache[(size_t)s * CH + MLP_H + i], acc);
    } else {  // b3
        for (int s = 0; s < n; s++) acc += dz[(size_t)s * DZ + 2 * MLP_H];
    }
    grad[q] = acc;
}

// Mean squared error over the samples, in order, by one thread (small n).
__global__ void mlp_loss_kernel(const float *__restrict__ y, const float *__restrict__ t, int n, float *loss) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    float acc = 0.0f;
    for (int s = 0; s < n; s++) {
        const float e = y[s] - t[s];
        acc = fmaf(e, e, acc);
    }
    *loss = acc / (float)n;
}

// Adam (Kingma and Ba) with bias correction; step counts from 1.
__global__ void mlp_adam_kernel(float *__restrict__ prm, const float *__restrict__ grad, float *__restrict__ m,
                                float *__restrict__ v, int step, float lr, float b1, float b2, float eps) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= MLP_NPARAM) return;
    const float g = grad[q];
    const float mq = b1 * m[q] + (1.0f - b1) * g;
    const float vq = b2 * v[q] + (1.0f - b2) * g * g;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / (1.0f - powf(b1, (float)step));
    const float vh = vq / (1.0f - powf(b2, (float)step));
    prm[q] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace bz
