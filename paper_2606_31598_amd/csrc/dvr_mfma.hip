// Sinc-DVR Toeplitz product on the matrix cores (binary32 MFMA), one vector.
//
// The operator's off-diagonal part depends only on k = i - j (paper Sec. III,
// analytic generation), so with the rows and columns cut into blocks of 32,
// y_I = sum_J T_{I-J} x_J, where T_d[p][q] = t(32 d + p - q) is one 32 x 32
// Toeplitz block per block offset d.  For a fixed d the blocks T_d are shared
// by every output block I: y_I += T_d x_{I-d} for all I is a dense
// contraction (32 x 32 times 32 x N, N running over output blocks), which is
// what the matrix cores do.  Each wave owns 16 output blocks (the 32 MFMA
// columns are 16 blocks x {re, im}) and walks a chunk of block offsets d;
// per d it reads the 16 symbol values of its A fragment and the 16 x values
// of its B fragment from LDS and issues 16 v_mfma_f32_32x32x2_f32 (the whole
// K = 32 of the block).  A workgroup's 4 waves cover 64 consecutive output
// blocks with the same chunk of d (about one workgroup per compute unit in
// all: fewer chunks mean fewer partial slots to write and reduce and less
// staging, which measured faster than more resident workgroups); each
// chunk's sums go to one partial slot,
// reduced in a fixed order afterwards like the VALU kernel's column chunks.
// The symbol comes from the same table as the VALU kernel (binary32 entries,
// zero at k = 0 and, for the compensated arithmetic, inside the band).
#include <hip/hip_ext.h>

#include "kernels.h"

namespace procmv {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBlk = 32;           // Toeplitz block edge
constexpr int kWaveBlocks = 16;    // output blocks per wave (32 MFMA columns: re, im)
constexpr int kThreads = 256;      // 4 waves per workgroup
constexpr int kGroupBlocks = kWaveBlocks * (kThreads / 64);   // output blocks per workgroup
constexpr int kMaxChunk = 72;      // block offsets per workgroup (LDS sizing)
constexpr int kTargetGroups = 256; // about one workgroup per compute unit
// x blocks one workgroup reads: kGroupBlocks + chunk - 1
constexpr int kXBlocks = kGroupBlocks + kMaxChunk - 1;
constexpr int kXPitch = 16;        // floats per (component, parity, block)
constexpr int kSymLen = kBlk * kMaxChunk + 2 * (kBlk - 1) + 1;

__global__ __launch_bounds__(kThreads) void dvr_toeplitz_mfma_kernel(DvrToeplitzArgs a, int n_chunks)
{
    // x split by component (re, im) and by parity of the index within its
    // block: xs[c][kg][B][s] = x_c[32 B + 2 s + kg], so that the 16 values a
    // lane feeds its 16 MFMAs are contiguous
    __shared__ float xs[2][2][kXBlocks][kXPitch];
    __shared__ float sym[kSymLen];

    const int D = a.D;
    const int nblk = (D + kBlk - 1) / kBlk;
    const int I0 = blockIdx.x * kGroupBlocks;
    // block offsets d with some output block I in [I0, I0 + 64) and input
    // block I - d in [0, nblk): d in [I0 - (nblk - 1), I0 + 63]
    const int dlo = I0 - (nblk - 1);
    const int nd = kGroupBlocks + nblk - 1;
    const int per = (nd + n_chunks - 1) / n_chunks;
    const int d0 = dlo + (int)blockIdx.y * per;
    const int d1 = min(d0 + per, dlo + nd);           // exclusive
    const int chunk = blockIdx.y;                     // partial slot

    if (d0 < d1) {
        // symbol window: m = 32 d + p - q in [32 d0 - 31, 32 (d1 - 1) + 31];
        // x blocks B in [I0 - d1 + 1, I0 + 63 - d0].  Each thread issues all
        // its global loads before its LDS stores, so they are in flight together.
        const int mlo = kBlk * d0 - (kBlk - 1);
        const int nm = kBlk * (d1 - d0) + 2 * (kBlk - 1);
        const int Blo = I0 - d1 + 1;
        const int nx = (kGroupBlocks + (d1 - d0) - 1) * kBlk;
        constexpr int SPER = (kSymLen + kThreads - 1) / kThreads;
        constexpr int XPER = (kXBlocks * kBlk + kThreads - 1) / kThreads;
        float sv[SPER];
        float2 xv[XPER];
#pragma unroll
        for (int u = 0; u < SPER; ++u) {
            const int e = (int)threadIdx.x + kThreads * u;
            const int m = mlo + e;
            sv[u] = (e < nm && m > -D && m < D) ? a.text[m + D - 1] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            const int e = (int)threadIdx.x + kThreads * u;
            const int j = Blo * kBlk + e;
            xv[u] = (e < nx && j >= 0 && j < D) ? a.X[j] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < SPER; ++u) {
            const int e = (int)threadIdx.x + kThreads * u;
            if (e < nm) sym[e] = sv[u];
        }
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            const int e = (int)threadIdx.x + kThreads * u;
            if (e < nx) {
                const int bb = e / kBlk, r = e - bb * kBlk;
                xs[0][r & 1][bb][r >> 1] = xv[u].x;
                xs[1][r & 1][bb][r >> 1] = xv[u].y;
            }
        }
    }
    __syncthreads();
    // (an empty chunk still writes its slot: zeros)

    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int p = lane & 31;             // A row (output row in the block)
    const int kg = lane >> 5;            // k = 2 s + kg of this lane
    const int n = lane & 31;             // B / C column
    const int nb = n >> 1;               // output block within the wave
    const int comp = n & 1;              // re / im
    const int Iw = I0 + kWaveBlocks * w;
    const int mlo = kBlk * d0 - (kBlk - 1);
    const int Blo = I0 - d1 + 1;

    f32x16 acc0 = {}, acc1 = {};
    for (int d = d0; d < d1; ++d) {
        // A[p][2s + kg] = t(32 d + p - 2 s - kg); B[2s + kg][n] = x_comp[32 (Iw + nb - d) + 2s + kg]
        const float* ap = sym + (kBlk * d + p - kg - mlo);
        const float4* bp = (const float4*)&xs[comp][kg][Iw + nb - d - Blo][0];
        float av[16], bv[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) av[s] = ap[-2 * s];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 t = bp[q];
            bv[4 * q + 0] = t.x;
            bv[4 * q + 1] = t.y;
            bv[4 * q + 2] = t.z;
            bv[4 * q + 3] = t.w;
        }
#pragma unroll
        for (int s = 0; s < 16; s += 2) {
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], bv[s], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s + 1], bv[s + 1], acc1, 0, 0, 0);
        }
    }
    // C[row][n]: lane holds column n, rows 8 (r >> 2) + 4 kg + (r & 3)
    const int I = Iw + nb;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = kBlk * I + 8 * (r >> 2) + 4 * kg + (r & 3);
        if (i < D) ((float*)(a.P + (size_t)chunk * a.ldp + i))[comp] = acc0[r] + acc1[r];
    }
}

}  // namespace

int dvr_mfma_chunks(int32_t D)
{
    // about kTargetGroups workgroups in all (row groups x chunks), at least one
    const int groups = ((D + kBlk - 1) / kBlk + kGroupBlocks - 1) / kGroupBlocks;
    const int nd = kGroupBlocks + (D + kBlk - 1) / kBlk - 1;
    int s = (kTargetGroups + groups - 1) / groups;
    // each chunk at most kMaxChunk offsets (LDS window)
    const int smin = (nd + kMaxChunk - 1) / kMaxChunk;
    if (s < smin) s = smin;
    if (s > nd) s = nd;
    return s;
}

hipError_t launch_dvr_toeplitz_mfma(const DvrToeplitzArgs& a, hipStream_t s, hipEvent_t e0,
                                    hipEvent_t e1)
{
    const int groups = ((a.D + kBlk - 1) / kBlk + kGroupBlocks - 1) / kGroupBlocks;
    const int chunks = dvr_mfma_chunks(a.D);
    const dim3 grid((unsigned)groups, (unsigned)chunks);
    if (e0)
        hipExtLaunchKernelGGL(dvr_toeplitz_mfma_kernel, grid, dim3(kThreads), 0, s, e0, e1, 0, a,
                              chunks);
    else
        hipLaunchKernelGGL(dvr_toeplitz_mfma_kernel, grid, dim3(kThreads), 0, s, a, chunks);
    return hipGetLastError();
}

}  // namespace procmv
