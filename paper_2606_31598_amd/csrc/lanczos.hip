// Vector kernels of the matrix-free Lanczos iteration that estimates the
// spectral bounds before the centered Chebyshev propagation (paper Sec. VII).
// The products H v run in the tile kernels; these kernels do the rest of each
// step: the binary64 inner product alpha_j = Re <v_j, H v_j>, the three-term
// update w <- w - alpha_j v_j - beta_{j-1} v_{j-1}, the binary64 norm
// beta_j = ||w|| and the normalisation v_{j+1} = w / beta_j.  Every sum is a
// fixed-order reduction: per-block partials, then every block that needs the
// total re-reduces the partials in the same order, so all blocks (and runs)
// see identical alpha and beta and nothing waits on another block.
#include "kernels.h"

namespace procmv {

namespace {

constexpr int kLzThreads = 256;

// Block-wide sum of one double per thread, fixed order; result in part[0].
__device__ inline void block_sum(double* part, double s)
{
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = kLzThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
}

// Sum of the nparts partials, identical in every block.
__device__ inline double total_of(double* part, const double* partials, int nparts)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kLzThreads) s += partials[i];
    block_sum(part, s);
    const double t = part[0];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kLzThreads) void lz_norm_partial_kernel(
    int32_t D, const float2* __restrict__ x, double* __restrict__ partials)
{
    __shared__ double part[kLzThreads];
    double s = 0.0;
    for (int i = blockIdx.x * kLzThreads + threadIdx.x; i < D; i += gridDim.x * kLzThreads) {
        const float2 a = x[i];
        s += (double)a.x * (double)a.x + (double)a.y * (double)a.y;
    }
    block_sum(part, s);
    if (threadIdx.x == 0) partials[blockIdx.x] = part[0];
}

// out = x / sqrt(sum of partials); block 0 stores the norm in *norm_out.
__global__ __launch_bounds__(kLzThreads) void lz_scale_kernel(
    int32_t D, const float2* __restrict__ x, float2* __restrict__ out,
    const double* __restrict__ partials, int32_t nparts, double* norm_out)
{
    __shared__ double part[kLzThreads];
    const double nrm = sqrt(total_of(part, partials, nparts));
    if (blockIdx.x == 0 && threadIdx.x == 0 && norm_out != nullptr) *norm_out = nrm;
    const double inv = 1.0 / nrm;
    for (int i = blockIdx.x * kLzThreads + threadIdx.x; i < D; i += gridDim.x * kLzThreads) {
        const float2 a = x[i];
        out[i] = make_float2((float)((double)a.x * inv), (float)((double)a.y * inv));
    }
}

// Partials of Re <v, w> = sum Re(conj(v_i) w_i).
__global__ __launch_bounds__(kLzThreads) void lz_dot_partial_kernel(
    int32_t D, const float2* __restrict__ v, const float2* __restrict__ w,
    double* __restrict__ partials)
{
    __shared__ double part[kLzThreads];
    double s = 0.0;
    for (int i = blockIdx.x * kLzThreads + threadIdx.x; i < D; i += gridDim.x * kLzThreads) {
        const float2 a = v[i], b = w[i];
        s += (double)a.x * (double)b.x + (double)a.y * (double)b.y;
    }
    block_sum(part, s);
    if (threadIdx.x == 0) partials[blockIdx.x] = part[0];
}

// alpha = total of the dot partials (stored by block 0 in *alpha_out);
// w <- w - alpha v - beta_prev v_prev (beta_prev null on the first step),
// computed in binary64 and rounded once; partials of ||w||^2.
__global__ __launch_bounds__(kLzThreads) void lz_update_kernel(
    int32_t D, const float2* __restrict__ v, const float2* __restrict__ v_prev,
    float2* __restrict__ w, const double* __restrict__ dot_partials, int32_t nparts,
    const double* beta_prev, double* alpha_out, double* __restrict__ norm_partials)
{
    __shared__ double part[kLzThreads];
    const double alpha = total_of(part, dot_partials, nparts);
    if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
    const double bp = beta_prev != nullptr ? *beta_prev : 0.0;
    double s = 0.0;
    for (int i = blockIdx.x * kLzThreads + threadIdx.x; i < D; i += gridDim.x * kLzThreads) {
        const float2 a = v[i], c = w[i];
        double rx = (double)c.x - alpha * (double)a.x;
        double ry = (double)c.y - alpha * (double)a.y;
        if (beta_prev != nullptr) {
            const float2 p = v_prev[i];
            rx -= bp * (double)p.x;
            ry -= bp * (double)p.y;
        }
        const float2 o = make_float2((float)rx, (float)ry);
        w[i] = o;
        s += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
    }
    block_sum(part, s);
    if (threadIdx.x == 0) norm_partials[blockIdx.x] = part[0];
}

}  // namespace

int32_t lanczos_blocks(int32_t D)
{
    const int64_t b = ((int64_t)D + 4 * kLzThreads - 1) / (4 * kLzThreads);
    return (int32_t)(b < 1 ? 1 : b > kLanczosMaxBlocks ? kLanczosMaxBlocks : b);
}

hipError_t launch_lanczos_normalise(int32_t D, const float2* x, float2* out,
                                    double* partials, double* norm_out, hipStream_t s)
{
    const int g = lanczos_blocks(D);
    hipLaunchKernelGGL(lz_norm_partial_kernel, dim3(g), dim3(kLzThreads), 0, s, D, x, partials);
    hipLaunchKernelGGL(lz_scale_kernel, dim3(g), dim3(kLzThreads), 0, s, D, x, out, partials,
                       g, norm_out);
    return hipGetLastError();
}

hipError_t launch_lanczos_scale(int32_t D, const float2* x, float2* out,
                                const double* partials, double* norm_out, hipStream_t s)
{
    const int g = lanczos_blocks(D);
    hipLaunchKernelGGL(lz_scale_kernel, dim3(g), dim3(kLzThreads), 0, s, D, x, out, partials,
                       g, norm_out);
    return hipGetLastError();
}

hipError_t launch_lanczos_orthogonalise(int32_t D, const float2* v, const float2* v_prev,
                                        float2* w, double* dot_partials,
                                        double* norm_partials, const double* beta_prev,
                                        double* alpha_out, hipStream_t s)
{
    const int g = lanczos_blocks(D);
    hipLaunchKernelGGL(lz_dot_partial_kernel, dim3(g), dim3(kLzThreads), 0, s, D, v, w,
                       dot_partials);
    hipLaunchKernelGGL(lz_update_kernel, dim3(g), dim3(kLzThreads), 0, s, D, v, v_prev, w,
                       dot_partials, g, beta_prev, alpha_out, norm_partials);
    return hipGetLastError();
}

}  // namespace procmv
