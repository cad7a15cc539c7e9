// System-side mixing of the system-bath Kronecker product (paper Sec. VII
// example: H = H_S (x) I + I (x) H_B + g sum_a A_a (x) B_a).  With psi as the
// d_S x d_B matrix X, the bath operators have already been applied to the
// d_S rows of X by the tile kernels (Z_0 = H_B rows, Z_a = B_a rows); this
// kernel adds the d_S x d_S system matrices:
//   Y[s, j] = Z_0[s, j] + sum_t M_0[s, t] X[t, j] + sum_a sum_t M_a[s, t] Z_a[t, j]
// with M_0 = H_S and M_a = g A_a.  One thread per bath index j, all s; the
// column of X and of every Z_a is read once (coalesced across j), HBM-bound.
#include "kernels.h"

namespace procmv {

namespace {

__global__ __launch_bounds__(256) void kron_mix_kernel(KronMixArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.dB) return;
    const int dS = a.dS;
    float2 acc[kKronMaxSys];
    float2 col[kKronMaxSys];
#pragma unroll
    for (int s = 0; s < kKronMaxSys; ++s) {
        acc[s] = s < dS ? a.Z[s * a.dB + j] : make_float2(0.f, 0.f);
        col[s] = s < dS ? a.X[s * a.dB + j] : make_float2(0.f, 0.f);
    }
    for (int op = 0; op <= a.n_int; ++op) {
        if (op > 0) {
#pragma unroll
            for (int t = 0; t < kKronMaxSys; ++t)
                if (t < dS) col[t] = a.Z[((int64_t)op * dS + t) * a.dB + j];
        }
        const float2* M = a.M + op * kKronMaxSys * kKronMaxSys;
#pragma unroll
        for (int s = 0; s < kKronMaxSys; ++s) {
            float re = acc[s].x, im = acc[s].y;
#pragma unroll
            for (int t = 0; t < kKronMaxSys; ++t) {
                // rows and columns beyond dS hold zeros in M and in col
                const float2 m = M[s * kKronMaxSys + t];
                re = fmaf(m.x, col[t].x, re);
                re = fmaf(-m.y, col[t].y, re);
                im = fmaf(m.x, col[t].y, im);
                im = fmaf(m.y, col[t].x, im);
            }
            acc[s] = make_float2(re, im);
        }
    }
#pragma unroll
    for (int s = 0; s < kKronMaxSys; ++s)
        if (s < dS) a.Y[s * a.dB + j] = acc[s];
}

}  // namespace

hipError_t launch_kron_mix(const KronMixArgs& a, hipStream_t s)
{
    const unsigned grid = (unsigned)((a.dB + 255) / 256);
    hipLaunchKernelGGL(kron_mix_kernel, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace procmv

namespace procmv {

namespace {

// One Chebyshev term of the system-bath propagation (paper Sec. VII,
// Ht = (H - c)/R), in binary32 like the single-operator epilogue: with
// Y = H q_k, h = alpha Y + (bhi + blo) q_k (alpha = 1/R exact in binary32,
// bhi + blo = -alpha c as a hi + lo pair),
//   first:  q_new = h
//   later:  q_new = 2 h - q_prev
// written over q_prev, and acc += coef q_new in binary64 (the coefficient
// sum is the only binary64 arithmetic).
__global__ __launch_bounds__(256) void kron_cheb_term_kernel(
    int64_t n, const float2* __restrict__ Y, const float2* __restrict__ qk,
    float2* __restrict__ qprev, double2* __restrict__ acc, float alpha, float bhi, float blo,
    double2 coef, int first)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 y = Y[i], q = qk[i];
    const float bx = __builtin_fmaf(bhi, q.x, blo * q.x);
    const float by = __builtin_fmaf(bhi, q.y, blo * q.y);
    float2 o = make_float2(__builtin_fmaf(alpha, y.x, bx), __builtin_fmaf(alpha, y.y, by));
    if (!first) {
        const float2 p = qprev[i];
        o.x = __builtin_fmaf(2.0f, o.x, -p.x);
        o.y = __builtin_fmaf(2.0f, o.y, -p.y);
    }
    qprev[i] = o;
    double2 a = acc[i];
    a.x += coef.x * (double)o.x - coef.y * (double)o.y;
    a.y += coef.x * (double)o.y + coef.y * (double)o.x;
    acc[i] = a;
}

// acc = coef q (start of a step).
__global__ __launch_bounds__(256) void kron_cheb_init_kernel(
    int64_t n, const float2* __restrict__ q, double2* __restrict__ acc, double2 coef)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 v = q[i];
    acc[i] = double2{coef.x * (double)v.x - coef.y * (double)v.y,
                     coef.x * (double)v.y + coef.y * (double)v.x};
}

}  // namespace

hipError_t launch_kron_cheb_init(int64_t n, const float2* q, double2* acc, double2 coef,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(kron_cheb_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       s, n, q, acc, coef);
    return hipGetLastError();
}

hipError_t launch_kron_cheb_term(int64_t n, const float2* Y, const float2* qk, float2* qprev,
                                 double2* acc, float alpha, float bhi, float blo, double2 coef,
                                 int first, hipStream_t s)
{
    hipLaunchKernelGGL(kron_cheb_term_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       s, n, Y, qk, qprev, acc, alpha, bhi, blo, coef, first);
    return hipGetLastError();
}

}  // namespace procmv
