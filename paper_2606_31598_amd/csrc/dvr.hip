// Sinc-DVR product on the VALU: analytic generation (paper Sec. III) of a
// Toeplitz-plus-diagonal operator fused with the block product.
//
// The off-diagonal entries depend only on k = i - j, so the block H^[n,m]
// restricted to a row band and a column chunk is read from a window of the
// symbol t(k) that is staged in LDS (band + chunk - 1 values) and never
// formed as a dense array.  Each lane owns RB consecutive rows; columns are
// walked CS at a time with the matching x values read as wave-wide LDS
// broadcasts (or through the scalar cache), and the CS new symbol values a
// lane needs per step are aligned 16-byte LDS reads, the other RB - 1 being
// carried in registers (a sliding window).  The zero-diagonal Toeplitz sum of each column chunk
// goes to one partial slot; the fixed-order reduction adds the chunks, the
// site potential v_i x_i and the constant diagonal.
#include <hip/hip_ext.h>

#include "kernels.h"

namespace procmv {

namespace {

template <int NV, int RB, int CHUNK, int CS, int XL>
__device__ __forceinline__ void dvr_band_chunk(const DvrToeplitzArgs& a)
{
    // CS columns per step; XL = 1 stages the chunk's x in LDS (broadcast
    // reads), XL = 0 reads it through the scalar cache.
    constexpr int BAND = 256 * RB;               // rows per workgroup
    constexpr int NSYM = BAND + CHUNK - 1;       // symbol window of the tile
    constexpr int NSYM4 = (NSYM + 3) / 4 + 2;
    static_assert(RB % 4 == 0 && CHUNK % CS == 0, "tile shape");
    __shared__ float4 sym4[NSYM4];
    __shared__ float2 xl[XL ? NV : 1][XL ? CHUNK : 1];
    float* sym = (float*)sym4;

    const int D = a.D;
    const int band = blockIdx.x;                 // row band
    const int chunk = blockIdx.y;                // column chunk (= partial slot)
    const int r0 = band * BAND;
    const int c0 = chunk * CHUNK;
    // sym[s] = t(k), k = s + kmin, kmin = r0 - (c0 + CHUNK - 1)
    const int kmin = r0 - (c0 + CHUNK - 1);
    for (int s = threadIdx.x; s < 4 * NSYM4; s += 256) {
        const int k = s + kmin;
        float t = 0.f;
        if (s < NSYM && k > -D && k < D) t = a.text[k + D - 1];
        sym[s] = t;
    }
    if (XL) {
        for (int q = threadIdx.x; q < NV * CHUNK; q += 256) {
            const int v = q / CHUNK, c = q - (q / CHUNK) * CHUNK;
            xl[v][c] = (c0 + c < D) ? a.X[v * a.ldx + c0 + c] : make_float2(0.f, 0.f);
        }
    }
    __syncthreads();

    const int i0 = r0 + threadIdx.x * RB;        // first row of this lane
    float2 acc[RB][NV];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[r][v] = make_float2(0.f, 0.f);

    // Window of the RB + CS - 1 symbol values t(i0 + r - (j + c)),
    // r in [0, RB), c in [0, CS): win[e], e = r - c + CS - 1, sits at LDS
    // position lbase - CS m + e - (CS - 1) for the step j = c0 + CS m.
    constexpr int NW = RB + CS - 1;
    float win[NW];
    const int lbase = threadIdx.x * RB + CHUNK - 1;   // i0 - c0 - kmin
#pragma unroll
    for (int e = CS; e < NW; ++e) win[e] = sym[lbase - (CS - 1) + e];

    const int ncol = min(CHUNK, D - c0);
    const int nfull = ncol / CS;                 // steps with every column in range
    const float2* __restrict__ xb = a.X + c0;
    for (int m = 0; m < (ncol + CS - 1) / CS; ++m) {
        const int pos = (lbase - CS * m - (CS - 1)) >> 2;
#pragma unroll
        for (int q = 0; q < CS / 4; ++q) {
            const float4 nw = sym4[pos + q];
            win[4 * q + 0] = nw.x;
            win[4 * q + 1] = nw.y;
            win[4 * q + 2] = nw.z;
            win[4 * q + 3] = nw.w;
        }
        const bool full = m < nfull;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            float2 x[CS];
            if (XL) {
#pragma unroll
                for (int c = 0; c < CS; ++c) x[c] = xl[v][CS * m + c];   // zero past the end
            } else {
                const float2* xv = xb + v * a.ldx;
                if (full) {
#pragma unroll
                    for (int c = 0; c < CS; ++c) x[c] = xv[CS * m + c];
                } else {
                    // ragged last step: clamped (in-range) reads, zero past the end
#pragma unroll
                    for (int c = 0; c < CS; ++c) {
                        const int cc = CS * m + c;
                        const float2 t = xv[cc < ncol ? cc : ncol - 1];
                        x[c] = cc < ncol ? t : make_float2(0.f, 0.f);
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < CS; ++c)
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const float t = win[r - c + CS - 1];
                    acc[r][v].x = __builtin_fmaf(t, x[c].x, acc[r][v].x);
                    acc[r][v].y = __builtin_fmaf(t, x[c].y, acc[r][v].y);
                }
        }
        // slide: the next step's e >= CS are this step's e - CS
#pragma unroll
        for (int e = NW - 1; e >= CS; --e) win[e] = win[e - CS];
    }

#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int i = i0 + r;
        if (i < D) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                a.P[((size_t)chunk * NV + v) * a.ldp + i] = acc[r][v];
        }
    }
}

template <int NV, int RB, int CHUNK, int CS, int XL>
__global__ __launch_bounds__(256) void dvr_toeplitz_kernel(DvrToeplitzArgs a)
{
    dvr_band_chunk<NV, RB, CHUNK, CS, XL>(a);
}

template <int NV, int RB, int CHUNK, int CS, int XL>
hipError_t launch_cfg(const DvrToeplitzArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid((unsigned)((a.D + 256 * RB - 1) / (256 * RB)),
                    (unsigned)((a.D + CHUNK - 1) / CHUNK));
    if (e0)   // events stamped by the dispatch itself (kernel start / end)
        hipExtLaunchKernelGGL((dvr_toeplitz_kernel<NV, RB, CHUNK, CS, XL>), grid, dim3(256), 0,
                              s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL((dvr_toeplitz_kernel<NV, RB, CHUNK, CS, XL>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// Variants: (rows per lane, chunk, columns per step, x in LDS).
template <int NV>
hipError_t launch_dvr_nv(const DvrToeplitzArgs& a, int variant, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1)
{
    switch (variant) {
    case 0: return launch_cfg<NV, 4, 256, 8, 0>(a, s, e0, e1);
    case 1: return launch_cfg<NV, 4, 1024, 8, 0>(a, s, e0, e1);
    case 2: return launch_cfg<NV, 4, 1024, 16, 0>(a, s, e0, e1);
    case 3: return launch_cfg<NV, 4, 1024, 8, 1>(a, s, e0, e1);
    case 4: return launch_cfg<NV, 8, 512, 8, 1>(a, s, e0, e1);
    case 5: return launch_cfg<NV, 8, 1024, 16, 0>(a, s, e0, e1);
    case 6: return launch_cfg<NV, 4, 512, 16, 1>(a, s, e0, e1);
    case 7: return launch_cfg<NV, 8, 512, 16, 1>(a, s, e0, e1);
    case 8: return launch_cfg<NV, 8, 256, 16, 1>(a, s, e0, e1);
    case 9: return launch_cfg<NV, 4, 256, 16, 1>(a, s, e0, e1);
    case 10: return launch_cfg<NV, 4, 1024, 16, 1>(a, s, e0, e1);
    case 11: return launch_cfg<NV, 8, 1024, 16, 1>(a, s, e0, e1);
    case 12: return launch_cfg<NV, 4, 1024, 32, 1>(a, s, e0, e1);
    case 13: return launch_cfg<NV, 4, 2048, 16, 1>(a, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int dvr_toeplitz_variant(int32_t D, int nv)
{
    // measured on MI355X: x staged in LDS, 4 rows per lane, 16 columns per
    // step; at large D 1024-column chunks for one vector (half the partial
    // slots of 512) and 512 for more; 256-column chunks below
    if (D < 16384) return 9;
    return nv == 1 ? 10 : 6;
}

int dvr_toeplitz_chunk_of(int variant)
{
    static const int chunk[14] = {256, 1024, 1024, 1024, 512, 1024, 512, 512, 256, 256,
                                  1024, 1024, 1024, 2048};
    return (variant >= 0 && variant < 14) ? chunk[variant] : 0;
}

hipError_t launch_dvr_toeplitz(const DvrToeplitzArgs& a, int nv, int variant,
                               hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    switch (nv) {
    case 1: return launch_dvr_nv<1>(a, variant, s, e0, e1);
    case 2: return launch_dvr_nv<2>(a, variant, s, e0, e1);
    case 4: return launch_dvr_nv<4>(a, variant, s, e0, e1);
    case 8: return launch_dvr_nv<8>(a, variant, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace procmv
