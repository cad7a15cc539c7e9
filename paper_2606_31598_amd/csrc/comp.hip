// Compensated binary32 arithmetic for the sinc-DVR operator (paper Sec. VII
// centered Chebyshev propagation; Sec. III analytic generation).
//
// The kinetic stencil of the sinc-DVR operator has entries of order 1/dx^2
// whose row sums vanish, while the states it propagates are smooth: a plain
// binary32 sum of t(i-j) x_j loses the result to cancellation, and binary32
// storage of the recurrence vectors adds a relative rounding of 2^-24 per
// term, which the K ~ R dt terms of one step accumulate.  This reduction
// completes the block product and the recurrence in a form that avoids both
// while every operation stays binary32:
//   * the tile kernels apply only the far part |i - j| >= W of the operator
//     (entries inside the band are zero in their tables);
//   * the band 0 < |i - j| < W is summed here in difference form,
//     sum t(i-j) ((x_j - x_i)), whose terms are small for a smooth x, and the
//     rest of the row is the per-row constant C_i = d + sum_band t + v_i,
//     applied to x_i as a hi + lo pair;
//   * the recurrence vectors are double-binary32 pairs (hi + lo), and the
//     step q' = 2 alpha (y - c q) - q_prev is evaluated with exact products
//     and two-sums (Knuth's TwoSum, the FMA-based exact product), so the
//     only rounding left is that of the small term alpha y.
// The coefficient sum stays in binary64 as in the plain epilogue.
#include <hip/hip_ext.h>

#include "kernels.h"

namespace procmv {

namespace {

// s + e = a + b exactly (Knuth's branch-free two-sum).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// One component of the double-binary32 step: (nh, nl) = f (alpha y - gamma x)
// - prev with x = xh + xl, gamma = ghi + glo, prev = ph + pl; first = no prev.
template <bool FIRST>
__device__ __forceinline__ void comp_step(float f, float alpha, float ghi, float glo, float y,
                                          float xh, float xl, float ph, float pl, float& nh,
                                          float& nl)
{
    const float p = ghi * xh;                   // ghi xh = p + pe exactly
    const float pe = __builtin_fmaf(ghi, xh, -p);
    const float small = pe + __builtin_fmaf(ghi, xl, glo * xh);
    float t = f * __builtin_fmaf(alpha, y, -small);
    float s, e;
    if (FIRST) {
        s = -p;
    } else {
        two_sum(-f * p, -ph, s, e);             // f = 2: f p is exact
        t += e - pl;
    }
    two_sum(s, t, nh, nl);
}

template <Epi MODE>
__global__ __launch_bounds__(256) void reduce_comp_kernel(ReduceArgs a)
{
    constexpr int NS = 64 + 2 * (kNearBand - 1);
    static_assert(NS <= 256, "one staged element per thread");
    __shared__ float2 xh[NS], xl[NS];
    __shared__ float tks[kNearBand];
    __shared__ float2 part[4][64];
    const int W = a.W;                           // 1 <= W <= kNearBand
    const int D = a.D;
    const int v = blockIdx.y;
    const int r0 = reduce_row_block(a, blockIdx.x) * 64;
    const int g = threadIdx.x >> 6;
    const int l = threadIdx.x & 63;
    const int i = r0 + l;
    const bool live = i < D;
    const size_t e = (size_t)v * a.ldy + i;

    // Every global load is issued before the first barrier so that their
    // latencies overlap: the staged window, the epilogue operands (group 0)
    // and the group's partial slots.
    const float2* xv = a.X + (size_t)v * a.ldx;
    const float2* xlv = a.Xlo ? a.Xlo + (size_t)v * a.ldxl : nullptr;
    const int nst = 64 + 2 * (W - 1);
    const int js = r0 - (W - 1) + (int)threadIdx.x;
    const bool stage = (int)threadIdx.x < nst;
    const bool sin = stage && js >= 0 && js < D;
    const float2 sh = sin ? xv[js] : make_float2(0.f, 0.f);
    const float2 sl = (sin && xlv) ? xlv[js] : make_float2(0.f, 0.f);
    const float tkv = ((int)threadIdx.x < W && threadIdx.x > 0) ? a.tk[threadIdx.x] : 0.f;
    float2 cv = make_float2(0.f, 0.f), ph = cv, pl = cv;
    double2 acc0 = double2{0.0, 0.0};
    if (g == 0 && live) {
        cv = a.cv[i];
        if (MODE == Epi::kChebStep) {
            ph = a.Y[e];
            pl = a.Ylo[(size_t)v * a.ldylo + i];
            acc0 = a.acc[(size_t)v * a.ldacc + i];
        }
    }
    float sx = 0.f, sy = 0.f;
    if (live) {
        // far part: the group's share of the partial slots, in slot order
        const float2* p = a.P + (size_t)v * a.ldp + i;
        const size_t stride = (size_t)a.nv_stride * a.ldp;
        const int k0 = (a.n_slots * g) / 4, k1 = (a.n_slots * (g + 1)) / 4;
        int k = k0;
        for (; k + 4 <= k1; k += 4) {
            const float2 q0 = p[(size_t)(k + 0) * stride];
            const float2 q1 = p[(size_t)(k + 1) * stride];
            const float2 q2 = p[(size_t)(k + 2) * stride];
            const float2 q3 = p[(size_t)(k + 3) * stride];
            sx += q0.x; sy += q0.y;
            sx += q1.x; sy += q1.y;
            sx += q2.x; sy += q2.y;
            sx += q3.x; sy += q3.y;
        }
        for (; k < k1; ++k) {
            const float2 q = p[(size_t)k * stride];
            sx += q.x;
            sy += q.y;
        }
    }
    if (stage) {
        xh[threadIdx.x] = sh;
        xl[threadIdx.x] = sl;
    }
    if ((int)threadIdx.x < W) tks[threadIdx.x] = tkv;
    __syncthreads();

    if (live) {
        // band: the group's share of the offsets -(W-1)..-1, 1..W-1
        const int no = 2 * (W - 1);
        const int o0 = (no * g) / 4, o1 = (no * (g + 1)) / 4;
        const float2 ch = xh[l + W - 1], cl = xl[l + W - 1];
        float nx = 0.f, ny = 0.f;
        for (int q = o0; q < o1; ++q) {
            const int o = q < W - 1 ? q - (W - 1) : q - (W - 2);
            const int j = i + o;
            if (j < 0 || j >= D) continue;
            const float t = tks[o < 0 ? -o : o];
            const float2 h = xh[l + W - 1 + o], lo = xl[l + W - 1 + o];
            const float zx = (h.x - ch.x) + (lo.x - cl.x);
            const float zy = (h.y - ch.y) + (lo.y - cl.y);
            nx = __builtin_fmaf(t, zx, nx);
            ny = __builtin_fmaf(t, zy, ny);
        }
        sx += nx;
        sy += ny;
    }
    part[g][l] = make_float2(sx, sy);
    __syncthreads();
    if (g != 0 || !live) return;
    sx = part[0][l].x;
    sy = part[0][l].y;
    sx += part[1][l].x;
    sy += part[1][l].y;
    sx += part[2][l].x;
    sy += part[2][l].y;
    sx += part[3][l].x;
    sy += part[3][l].y;

    // y = far + band + C_i x (C as hi + lo, x as hi + lo)
    const float2 x = xh[l + W - 1], xlo = xl[l + W - 1];
    sx = __builtin_fmaf(cv.y, x.x, sx);
    sy = __builtin_fmaf(cv.y, x.y, sy);
    sx = __builtin_fmaf(cv.x, xlo.x, sx);
    sy = __builtin_fmaf(cv.x, xlo.y, sy);
    sx = __builtin_fmaf(cv.x, x.x, sx);
    sy = __builtin_fmaf(cv.x, x.y, sy);
    if (MODE == Epi::kApply) {
        a.Y[e] = make_float2(sx, sy);
        return;
    }
    float2 nh, nl;
    if (MODE == Epi::kChebFirst) {
        comp_step<true>(1.f, a.alpha, a.gamma_hi, a.gamma_lo, sx, x.x, xlo.x, 0.f, 0.f, nh.x,
                        nl.x);
        comp_step<true>(1.f, a.alpha, a.gamma_hi, a.gamma_lo, sy, x.y, xlo.y, 0.f, 0.f, nh.y,
                        nl.y);
        a.Yq1[e] = nh;
        a.Yq1lo[(size_t)v * a.ldylo + i] = nl;
        // q_0 enters with a zero lo part; its lo buffer starts the recurrence at zero
        a.Xlo_zero[(size_t)v * a.ldylo + i] = make_float2(0.f, 0.f);
        double2 r;
        r.x = a.a0.x * (double)x.x - a.a0.y * (double)x.y;
        r.y = a.a0.x * (double)x.y + a.a0.y * (double)x.x;
        const double qx = (double)nh.x + (double)nl.x, qy = (double)nh.y + (double)nl.y;
        r.x += a.a1.x * qx - a.a1.y * qy;
        r.y += a.a1.x * qy + a.a1.y * qx;
        a.acc[(size_t)v * a.ldacc + i] = r;
    } else {
        comp_step<false>(2.f, a.alpha, a.gamma_hi, a.gamma_lo, sx, x.x, xlo.x, ph.x, pl.x, nh.x,
                         nl.x);
        comp_step<false>(2.f, a.alpha, a.gamma_hi, a.gamma_lo, sy, x.y, xlo.y, ph.y, pl.y, nh.y,
                         nl.y);
        a.Y[e] = nh;
        a.Ylo[(size_t)v * a.ldylo + i] = nl;
        double2 r = acc0;
        const double qx = (double)nh.x + (double)nl.x, qy = (double)nh.y + (double)nl.y;
        r.x += a.a0.x * qx - a.a0.y * qy;
        r.y += a.a0.x * qy + a.a0.y * qx;
        a.acc[(size_t)v * a.ldacc + i] = r;
    }
}

}  // namespace

hipError_t launch_reduce_comp(const ReduceArgs& a, Epi mode, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1)
{
    if (a.W < 1 || a.W > kNearBand || a.nv < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.D + 63) / 64), (unsigned)a.nv), blk(256);
#define PROCMV_RED(M)                                                                        \
    if (e0) hipExtLaunchKernelGGL(reduce_comp_kernel<M>, grid, blk, 0, s, e0, e1, 0, a);     \
    else hipLaunchKernelGGL(reduce_comp_kernel<M>, grid, blk, 0, s, a);
    switch (mode) {
    case Epi::kApply: PROCMV_RED(Epi::kApply) break;
    case Epi::kChebFirst: PROCMV_RED(Epi::kChebFirst) break;
    case Epi::kChebStep: PROCMV_RED(Epi::kChebStep) break;
    }
#undef PROCMV_RED
    return hipGetLastError();
}

}  // namespace procmv
