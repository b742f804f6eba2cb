// Row-size predictor: a 3-32-32-1 ReLU network in FP32 that estimates
// log1p nnz(C(i,:)) from (log1p nnz(A(i,:)), log1p flops_i,
// log1p max_k nnz(B(k,:))), so accumulators can be sized without a symbolic
// pass.  Parameters are one flat float array: W1[32][3], b1[32], W2[32][32],
// b2[32], w3[32], b3.  Kernels: inference, gradient of the asymmetric
// squared loss a_i (y_i - t_i)^2 (a_i = alpha when y_i < t_i), Adam.
#pragma once
#include "common.hpp"

namespace spg {

constexpr int MLP_H = 32;
constexpr int MLP_W1 = 0, MLP_B1 = MLP_W1 + 3 * MLP_H, MLP_W2 = MLP_B1 + MLP_H,
              MLP_B2 = MLP_W2 + MLP_H * MLP_H, MLP_W3 = MLP_B2 + MLP_H, MLP_B3 = MLP_W3 + MLP_H,
              MLP_NPARAMS = MLP_B3 + 1;  // 1217

__device__ inline float mlp_eval(const float* P, float x0, float x1, float x2) {
    float h1[MLP_H];
#pragma unroll
    for (int j = 0; j < MLP_H; ++j) {
        float z = P[MLP_B1 + j] + P[MLP_W1 + 3 * j] * x0 + P[MLP_W1 + 3 * j + 1] * x1 + P[MLP_W1 + 3 * j + 2] * x2;
        h1[j] = z > 0.f ? z : 0.f;
    }
    float y = P[MLP_B3];
#pragma unroll 4
    for (int j = 0; j < MLP_H; ++j) {
        float z = P[MLP_B2 + j];
#pragma unroll
        for (int k = 0; k < MLP_H; ++k) z += P[MLP_W2 + MLP_H * j + k] * h1[k];
        y += P[MLP_W3 + j] * (z > 0.f ? z : 0.f);
    }
    return y;
}

__device__ inline void load_params(float* s_p, const float* params) {
    for (int t = threadIdx.x; t < MLP_NPARAMS; t += blockDim.x) s_p[t] = params[t];
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_mlp_forward(const float* params, const float* x, int64_t n, float* y) {
    __shared__ float s_p[MLP_NPARAMS];
    load_params(s_p, params);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = mlp_eval(s_p, x[3 * i], x[3 * i + 1], x[3 * i + 2]);
}

// Gradient of (1/n) sum a_i (y_i - t_i)^2 for the block's 256 samples,
// added into grad (and the loss into *loss).  Per-sample backward vectors
// are staged in LDS; thread t then forms parameter entries t, t+256, ... as
// sums over the block's samples and adds each with one atomic.
constexpr int MLP_BS = 256;
struct MlpGradLds {
    float p[MLP_NPARAMS];
    float x[MLP_BS][4];
    float gz1[MLP_BS][MLP_H];
    float h1[MLP_BS][MLP_H];
    float gz2[MLP_BS][MLP_H];
    float h2[MLP_BS][MLP_H];
    float gy[MLP_BS];
    float red[MLP_BS / SPG_WAVE + 1];
};

__global__ void __launch_bounds__(MLP_BS) k_mlp_grad(const float* params, const float* x, const float* t,
                                                     int64_t n, float alpha, float* grad, float* loss) {
    __shared__ MlpGradLds L;
    load_params(L.p, params);
    const float* P = L.p;
    const int s = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * MLP_BS + s;
    const bool ok = i < n;
    const float inv_n = 1.0f / (float)n;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f;
    if (ok) {
        x0 = x[3 * i];
        x1 = x[3 * i + 1];
        x2 = x[3 * i + 2];
    }
    L.x[s][0] = x0;
    L.x[s][1] = x1;
    L.x[s][2] = x2;
    float z1[MLP_H], h1[MLP_H], z2[MLP_H];
#pragma unroll
    for (int j = 0; j < MLP_H; ++j) {
        z1[j] = P[MLP_B1 + j] + P[MLP_W1 + 3 * j] * x0 + P[MLP_W1 + 3 * j + 1] * x1 + P[MLP_W1 + 3 * j + 2] * x2;
        h1[j] = z1[j] > 0.f ? z1[j] : 0.f;
        L.h1[s][j] = h1[j];
    }
    float y = P[MLP_B3];
#pragma unroll
    for (int j = 0; j < MLP_H; ++j) {
        float z = P[MLP_B2 + j];
#pragma unroll
        for (int k = 0; k < MLP_H; ++k) z += P[MLP_W2 + MLP_H * j + k] * h1[k];
        z2[j] = z;
        const float h2 = z > 0.f ? z : 0.f;
        L.h2[s][j] = h2;
        y += P[MLP_W3 + j] * h2;
    }
    float gy = 0.f, l = 0.f;
    if (ok) {
        const float d = y - t[i];
        const float a = d < 0.f ? alpha : 1.f;
        gy = 2.f * a * d * inv_n;
        l = a * d * d * inv_n;
    }
    L.gy[s] = gy;
    float gz2[MLP_H];
#pragma unroll
    for (int j = 0; j < MLP_H; ++j) {
        gz2[j] = z2[j] > 0.f ? gy * P[MLP_W3 + j] : 0.f;
        L.gz2[s][j] = gz2[j];
    }
#pragma unroll 4
    for (int k = 0; k < MLP_H; ++k) {
        float g = 0.f;
#pragma unroll
        for (int j = 0; j < MLP_H; ++j) g += gz2[j] * P[MLP_W2 + MLP_H * j + k];
        L.gz1[s][k] = z1[k] > 0.f ? g : 0.f;
    }
    float lsum = block_reduce_add<MLP_BS, float>(l, L.red);  // barriers: staging complete
    if (threadIdx.x == 0 && loss) atomicAdd(loss, lsum);
    const int nb = (int)min((int64_t)MLP_BS, n - (int64_t)blockIdx.x * MLP_BS);
    for (int p = threadIdx.x; p < MLP_NPARAMS; p += MLP_BS) {
        float g = 0.f;
        if (p < MLP_B1) {
            const int j = p / 3, c = p % 3;
            for (int q = 0; q < nb; ++q) g += L.gz1[q][j] * L.x[q][c];
        } else if (p < MLP_W2) {
            const int j = p - MLP_B1;
            for (int q = 0; q < nb; ++q) g += L.gz1[q][j];
        } else if (p < MLP_B2) {
            const int j = (p - MLP_W2) / MLP_H, k = (p - MLP_W2) % MLP_H;
            for (int q = 0; q < nb; ++q) g += L.gz2[q][j] * L.h1[q][k];
        } else if (p < MLP_W3) {
            const int j = p - MLP_B2;
            for (int q = 0; q < nb; ++q) g += L.gz2[q][j];
        } else if (p < MLP_B3) {
            const int j = p - MLP_W3;
            for (int q = 0; q < nb; ++q) g += L.gy[q] * L.h2[q][j];
        } else {
            for (int q = 0; q < nb; ++q) g += L.gy[q];
        }
        atomicAdd(&grad[p], g);
    }
}

// Adam update (bias-corrected), one thread per parameter; the gradient
// buffer is cleared afterwards.
__global__ void __launch_bounds__(256) k_mlp_adam(float* params, float* grad, float* m, float* v,
                                                  int64_t step, float lr, float beta1, float beta2, float eps) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= MLP_NPARAMS) return;
    const float g = grad[p];
    const float mm = beta1 * m[p] + (1.f - beta1) * g;
    const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(beta1, (float)step));
    const float vh = vv / (1.f - powf(beta2, (float)step));
    params[p] -= lr * mh / (sqrtf(vh) + eps);
    grad[p] = 0.f;  // ready for the next accumulation
}

}  // namespace spg
