// Batched reduction and Chebyshev completion over many independent operators
// (the single-GPU form of parameter-parallel execution, paper Sec. IV-G).
//
// The vectors of all instances are packed into one buffer: instance k holds
// nv vectors of length D_k starting at element off_k = sum_{l<k} nv D_l, so
// element t of the packed buffer belongs to the instance whose range
// [off_k, off_{k+1}) contains t.
#include "kernels.h"

namespace procmv {

namespace {

__device__ __forceinline__ int find_instance(const int64_t* __restrict__ off, int n,
                                             int64_t t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <Epi MODE>
__global__ __launch_bounds__(256) void reduce_batched_kernel(BatchReduceArgs a)
{
    __shared__ float2 part[4][64];
    const int g = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 64 + l;
    const bool live = t < a.total;
    int k = 0;
    float sx = 0.f, sy = 0.f;
    BatchReduceItem it{};
    if (live) {
        k = find_instance(a.off, a.n, t);
        it = a.items[k];
        const int64_t local = t - it.off;
        const int v = (int)(local / it.D);
        const int i = (int)(local - (int64_t)v * it.D);
        const float2* p = it.P + (size_t)v * it.ldp + i;
        const size_t stride = (size_t)a.nv * it.ldp;
        const int k0 = (it.n_slots * g) / 4, k1 = (it.n_slots * (g + 1)) / 4;
        for (int q = k0; q < k1; ++q) {
            const float2 u = p[(size_t)q * stride];
            sx += u.x;
            sy += u.y;
        }
    }
    part[g][l] = make_float2(sx, sy);
    __syncthreads();
    if (g != 0 || !live) return;
    sx = part[0][l].x; sy = part[0][l].y;
    sx += part[1][l].x; sy += part[1][l].y;
    sx += part[2][l].x; sy += part[2][l].y;
    sx += part[3][l].x; sy += part[3][l].y;
    const float2 x = a.X[t];
    const float bx = __builtin_fmaf(it.beta_hi, x.x, it.beta_lo * x.x);
    const float by = __builtin_fmaf(it.beta_hi, x.y, it.beta_lo * x.y);
    const float hx = __builtin_fmaf(it.alpha, sx, bx);
    const float hy = __builtin_fmaf(it.alpha, sy, by);
    if (MODE == Epi::kApply) {
        a.Y[t] = make_float2(hx, hy);
    } else if (MODE == Epi::kChebFirst) {
        a.Yq1[t] = make_float2(hx, hy);
        double2 r;
        r.x = a.a0.x * (double)x.x - a.a0.y * (double)x.y;
        r.y = a.a0.x * (double)x.y + a.a0.y * (double)x.x;
        r.x += a.a1.x * (double)hx - a.a1.y * (double)hy;
        r.y += a.a1.x * (double)hy + a.a1.y * (double)hx;
        a.acc[t] = r;
    } else {
        const float2 prev = a.Y[t];
        const float nx = __builtin_fmaf(2.0f, hx, -prev.x);
        const float ny = __builtin_fmaf(2.0f, hy, -prev.y);
        a.Y[t] = make_float2(nx, ny);
        double2 r = a.acc[t];
        r.x += a.a0.x * (double)nx - a.a0.y * (double)ny;
        r.y += a.a0.x * (double)ny + a.a0.y * (double)nx;
        a.acc[t] = r;
    }
}

// One workgroup per (instance, vector): psi = phase acc, |psi|^2 in a fixed order.
__global__ __launch_bounds__(256) void finish_batched_kernel(
    const BatchReduceItem* __restrict__ items, int nv, const double2* acc,
    float2* psi, double* norm2)
{
    __shared__ double red[256];
    const int k = blockIdx.x / nv;
    const int v = blockIdx.x - k * nv;
    const BatchReduceItem it = items[k];
    const int64_t base = it.off + (int64_t)v * it.D;
    double s = 0.0;
    for (int i = threadIdx.x; i < it.D; i += 256) {
        const double2 r = acc[base + i];
        const double px = it.phase.x * r.x - it.phase.y * r.y;
        const double py = it.phase.x * r.y + it.phase.y * r.x;
        const float2 o = make_float2((float)px, (float)py);
        psi[base + i] = o;
        s += (double)o.x * (double)o.x + (double)o.y * (double)o.y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) norm2[blockIdx.x] = red[0];
}

}  // namespace

hipError_t launch_reduce_batched(const BatchReduceArgs& a, Epi mode, hipStream_t s)
{
    const dim3 grid((unsigned)((a.total + 63) / 64));
    switch (mode) {
    case Epi::kApply:
        hipLaunchKernelGGL(reduce_batched_kernel<Epi::kApply>, grid, dim3(256), 0, s, a);
        break;
    case Epi::kChebFirst:
        hipLaunchKernelGGL(reduce_batched_kernel<Epi::kChebFirst>, grid, dim3(256), 0, s, a);
        break;
    case Epi::kChebStep:
        hipLaunchKernelGGL(reduce_batched_kernel<Epi::kChebStep>, grid, dim3(256), 0, s, a);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_finish_batched(const BatchReduceItem* items, int n, int nv,
                                 const double2* acc, float2* psi, double* norm2,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(finish_batched_kernel, dim3(n * nv), dim3(256), 0, s, items, nv,
                       acc, psi, norm2);
    return hipGetLastError();
}

}  // namespace procmv
