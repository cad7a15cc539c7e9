// Chebyshev step completion: psi = e^{-i c dt} acc (binary64 -> complex64)
// and the binary64 norm of every vector (paper Sec. VII; binary64 is kept for
// the coefficient accumulation and the norms).
#include "kernels.h"

namespace procmv {

namespace {

// One workgroup per vector: write psi and reduce |psi|^2 in a fixed order.
__global__ __launch_bounds__(1024) void cheb_finish_kernel(
    int32_t D, const double2* acc, int64_t ldacc, double2 phase, float2* psi,
    int64_t ld, double* norm2)
{
    __shared__ double part[1024];
    const int v = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < D; i += blockDim.x) {
        const double2 r = acc[v * ldacc + i];
        const double px = phase.x * r.x - phase.y * r.y;
        const double py = phase.x * r.y + phase.y * r.x;
        const float2 o = make_float2((float)px, (float)py);
        psi[v * ld + i] = o;
        s += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && norm2 != nullptr) norm2[v] = part[0];
}

__global__ void copy_vectors_kernel(int32_t D, int32_t nv, const float2* src,
                                    int64_t lds, float2* dst, int64_t ldd)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nv * D) return;
    const int v = (int)(t / D);
    const int i = (int)(t - (int64_t)v * D);
    dst[v * ldd + i] = src[v * lds + i];
}

}  // namespace

hipError_t launch_cheb_finish(int32_t D, int32_t nv, const double2* acc,
                              int64_t ldacc, double2 phase, float2* psi,
                              int64_t ld, double* norm2, hipStream_t s)
{
    hipLaunchKernelGGL(cheb_finish_kernel, dim3(nv), dim3(1024), 0, s, D, acc,
                       ldacc, phase, psi, ld, norm2);
    return hipGetLastError();
}

hipError_t launch_copy_vectors(int32_t D, int32_t nv, const float2* src,
                               int64_t lds, float2* dst, int64_t ldd,
                               hipStream_t s)
{
    const int64_t total = (int64_t)nv * D;
    hipLaunchKernelGGL(copy_vectors_kernel, dim3((unsigned)((total + 255) / 256)),
                       dim3(256), 0, s, D, nv, src, lds, dst, ldd);
    return hipGetLastError();
}

}  // namespace procmv
