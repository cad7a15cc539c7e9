// Neural run-time surrogate of the execution planner (paper Sec. IV-D,
// Eqs. nn_surrogate, nn_pred_time, nn_loss): f(z) predicts the logarithm of
// the measured time from a normalised feature vector and is trained by
// minimising the mean squared error of log time.  This library's network has
// 8 inputs and two hidden layers of 64 ReLU units:
//     a1 = z W1 + b1, h1 = relu(a1), a2 = h1 W2 + b2, h2 = relu(a2),
//     f = h2 W3 + b3.
// Forward and per-sample backward run one thread per sample; parameter
// gradients are summed over samples by one thread per parameter in a fixed
// order (deterministic); Adam updates elementwise.
#include "kernels.h"

namespace procmv {

namespace {

constexpr int NI = kMlpIn, NH = kMlpHidden;
constexpr int OW1 = 0, OB1 = OW1 + NI * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH,
              OW3 = OB2 + NH, OB3 = OW3 + NH;

__global__ __launch_bounds__(64) void mlp_forward_kernel(const float* __restrict__ p,
                                                         const float* __restrict__ z, int n,
                                                         float* y, float* a1s, float* a2s)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float zi[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) zi[i] = z[(size_t)s * NI + i];
    float h1[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        float a = p[OB1 + j];
#pragma unroll
        for (int i = 0; i < NI; ++i) a = __builtin_fmaf(zi[i], p[OW1 + i * NH + j], a);
        if (a1s) a1s[(size_t)s * NH + j] = a;
        h1[j] = a > 0.f ? a : 0.f;
    }
    float out = p[OB3];
    for (int j = 0; j < NH; ++j) {
        float a = p[OB2 + j];
#pragma unroll
        for (int i = 0; i < NH; ++i) a = __builtin_fmaf(h1[i], p[OW2 + i * NH + j], a);
        if (a2s) a2s[(size_t)s * NH + j] = a;
        const float h = a > 0.f ? a : 0.f;
        out = __builtin_fmaf(h, p[OW3 + j], out);
    }
    y[s] = out;
}

// Per-sample backward: gy = 2 (y - t) / n, ga2 = gy W3 relu'(a2),
// ga1 = (ga2 W2^T) relu'(a1).
__global__ __launch_bounds__(64) void mlp_backward_kernel(const float* __restrict__ p,
                                                          const float* __restrict__ y,
                                                          const float* __restrict__ t, int n,
                                                          const float* __restrict__ a1s,
                                                          const float* __restrict__ a2s,
                                                          float* gys, float* ga1s, float* ga2s)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float gy = 2.0f * (y[s] - t[s]) / (float)n;
    gys[s] = gy;
    float ga2[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        ga2[j] = a2s[(size_t)s * NH + j] > 0.f ? gy * p[OW3 + j] : 0.f;
        ga2s[(size_t)s * NH + j] = ga2[j];
    }
    for (int i = 0; i < NH; ++i) {
        float g = 0.f;
#pragma unroll
        for (int j = 0; j < NH; ++j) g = __builtin_fmaf(ga2[j], p[OW2 + i * NH + j], g);
        ga1s[(size_t)s * NH + i] = a1s[(size_t)s * NH + i] > 0.f ? g : 0.f;
    }
}

// One thread per parameter: sum of the per-sample contributions, samples in
// index order.
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ z, int n,
                                                       const float* __restrict__ a1s,
                                                       const float* __restrict__ a2s,
                                                       const float* __restrict__ gys,
                                                       const float* __restrict__ ga1s,
                                                       const float* __restrict__ ga2s,
                                                       float* g)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kMlpParams) return;
    float acc = 0.f;
    if (q < OB1) {                       // W1[i][j] += z_i ga1_j
        const int i = q / NH, j = q - (q / NH) * NH;
        for (int s = 0; s < n; ++s)
            acc = __builtin_fmaf(z[(size_t)s * NI + i], ga1s[(size_t)s * NH + j], acc);
    } else if (q < OW2) {                // b1[j] += ga1_j
        const int j = q - OB1;
        for (int s = 0; s < n; ++s) acc += ga1s[(size_t)s * NH + j];
    } else if (q < OB2) {                // W2[i][j] += h1_i ga2_j
        const int r = q - OW2, i = r / NH, j = r - (r / NH) * NH;
        for (int s = 0; s < n; ++s) {
            const float a = a1s[(size_t)s * NH + i];
            acc = __builtin_fmaf(a > 0.f ? a : 0.f, ga2s[(size_t)s * NH + j], acc);
        }
    } else if (q < OW3) {                // b2[j] += ga2_j
        const int j = q - OB2;
        for (int s = 0; s < n; ++s) acc += ga2s[(size_t)s * NH + j];
    } else if (q < OB3) {                // W3[j] += h2_j gy
        const int j = q - OW3;
        for (int s = 0; s < n; ++s) {
            const float a = a2s[(size_t)s * NH + j];
            acc = __builtin_fmaf(a > 0.f ? a : 0.f, gys[s], acc);
        }
    } else {                             // b3 += gy
        for (int s = 0; s < n; ++s) acc += gys[s];
    }
    g[q] = acc;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr mhat / (sqrt(vhat) + eps).
__global__ void mlp_adam_kernel(float* p, const float* __restrict__ g, float* m, float* v,
                                float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kMlpParams) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// Mean squared error, one workgroup, fixed order.
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float* __restrict__ y,
                                                       const float* __restrict__ t, int n,
                                                       float* loss)
{
    __shared__ float part[256];
    float s = 0.f;
    for (int q = threadIdx.x; q < n; q += 256) {
        const float r = y[q] - t[q];
        s = __builtin_fmaf(r, r, s);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] / (float)n;
}

}  // namespace

hipError_t launch_mlp_forward(const float* p, const float* z, int n, float* y, float* a1s,
                              float* a2s, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, z, n, y,
                       a1s, a2s);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* p, const float* z, const float* y,
                               const float* t, int n, const float* a1s, const float* a2s,
                               float* gys, float* ga1s, float* ga2s, float* g, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_backward_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, y, t, n,
                       a1s, a2s, gys, ga1s, ga2s);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, z, n,
                       a1s, a2s, gys, ga1s, ga2s, g);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, float lr, int step,
                           hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, p, g,
                       m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(const float* y, const float* t, int n, float* loss, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, s, y, t, n, loss);
    return hipGetLastError();
}

}  // namespace procmv
