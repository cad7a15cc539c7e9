// Sinc-DVR Toeplitz product on the bfloat16 matrix cores, one vector, with
// an exact three-piece split of the binary32 operands.
//
// The off-diagonal part of the operator depends only on k = i - j (paper
// Sec. III, analytic generation): with rows and columns cut into blocks of
// 32, y_I = sum_d T_d x_{I-d}, where T_d[p][q] = t(32 d + p - q) is one 32 x 32
// Toeplitz block per block offset d, shared by every output block I.
//
// Every binary32 value v (symbol entry or vector component) is written as
// v = hi + mid + lo with three bfloat16 pieces: hi = v rounded to the nearest
// bfloat16, mid = the remainder rounded likewise, lo = what is left (at most
// 8 significant bits), each subtraction exact.  Products of pieces are exact
// in binary32, so the six products whose piece levels sum to at most two
// (hh, hm, mh, hl, lh, mm) reproduce t x up to the dropped mid-lo, lo-mid and
// lo-lo terms, at most 2^-23 |t x| (|mid| <= 2^-8 |v|, |lo| <= 2^-16 |v|;
// root mean square about 2^-27) and of either sign: the rounding level of a
// binary32 product.  They run as v_mfma_f32_32x32x16_bf16 with binary32
// accumulation (the split-BF16 application of the paper's precision options,
// with a third piece so that nothing coarser than binary32 rounding enters),
// the hh products and the five smaller ones in separate sums (see the
// accumulators below).  Per 32 x 32 block and 16 columns of K that is six
// bf16 MFMAs of 32 cycles against eight binary32 32x32x2 MFMAs of 64 cycles:
// 2.7x fewer matrix-core cycles.
//
// Layout: a workgroup of 8 waves owns 64 consecutive output blocks and one
// chunk of block offsets d; each wave owns two column tiles of 16 blocks
// (32 MFMA columns: 16 blocks x {re, im}), so every A fragment it reads
// feeds two MFMAs, and shares them with three more waves that take the other
// phases of d mod 4 (two waves per SIMD hide each other's LDS latency; their
// sums meet in LDS, and the workgroup's rows leave in coalesced 16-byte
// stores).  64 blocks per workgroup keep the chunks long (16 partial slots at
// D = 32768): the slots are written, flushed at the end of the kernel and
// read again by the reduction, and fewer of them shorten all three.  The x
// window (3 pieces) sits in LDS with a row per (block, component) and an
// 80-byte row pitch, so the 16-byte B reads of 16 lanes hit 16 distinct
// groups of 4 banks.  A lane's A fragment is 8 consecutive symbol values
// starting at an offset that varies with its row p; the symbol window is kept
// in four copies shifted by 0..3 entries, and lane p reads the copy in which
// its run starts on an 8-byte boundary (two ds_read_b64, kept apart).  Each
// chunk's sums go to one partial slot, reduced in a fixed order afterwards.
// The symbol comes from the same binary32 table as the other Toeplitz kernels
// (zero at k = 0 and, for the compensated arithmetic, inside the band).
#include <hip/hip_ext.h>

#include "kernels.h"

namespace procmv {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBlk = 32;            // Toeplitz block edge
constexpr int kTileBlocks = 16;     // output blocks per MFMA column tile
constexpr int kWaveTiles = 2;       // column tiles per wave
constexpr int kTileGroups = 2;      // pairs of column tiles per workgroup
constexpr int kPhases = 4;          // waves per tile pair, each taking every 4th offset
constexpr int kThreads = 64 * kTileGroups * kPhases;   // 8 waves
constexpr int kGroupBlocks = kTileBlocks * kWaveTiles * kTileGroups;   // 64
constexpr int kOutPitch = 68;       // floats per output block in the LDS transpose
constexpr int kMaxChunk = 72;       // block offsets per workgroup (LDS sizing)
constexpr int kTargetGroups = 256;  // about one workgroup per compute unit
constexpr int kXBlocks = kGroupBlocks + kMaxChunk - 1;
constexpr int kXRow = 40;           // bf16 per (block, component) row: 32 + 8 pad
// symbol window: 32 L + 31 entries for a chunk of L offsets; each shifted
// copy padded to 16 mod 64 entries (8 mod 32 dwords: the four copies start
// 8 banks apart, so the 8-byte reads of 16 lanes, 4 rows x 4 copies, cover
// the 32 banks once)
constexpr int kSymLen = kBlk * kMaxChunk + kBlk - 1;
constexpr int kCopyPitch = ((kSymLen + 63 - 16) / 64) * 64 + 16;
static_assert(kCopyPitch >= kSymLen && kCopyPitch % 64 == 16, "copy pitch");

__device__ __forceinline__ uint32_t top16(float v)
{
    return __float_as_uint(v) >> 16;
}

// v rounded to the nearest bfloat16 (ties to even), as a binary32 value.
__device__ __forceinline__ float round_bf16(float v)
{
    const uint32_t u = __float_as_uint(v);
    return __uint_as_float((u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u);
}

// v = hi + mid + lo exactly (normal v): |v - hi| <= 2^-9 |v| has at most 16
// significant bits, |v - hi - mid| at most 8, so lo is a bfloat16 as it is.
__device__ __forceinline__ void split3(float v, uint32_t& h, uint32_t& m, uint32_t& l)
{
    const float vh = round_bf16(v);
    const float r1 = v - vh;
    const float vm = round_bf16(r1);
    const float r2 = r1 - vm;
    h = top16(vh);
    m = top16(vm);
    l = top16(r2);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v)
{
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ f32x16 mfma(uint4 a, uint4 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a), as_bf16x8(b), c, 0, 0, 0);
}

__global__ __launch_bounds__(kThreads) void dvr_toeplitz_bf16x6_kernel(DvrToeplitzArgs a,
                                                                       int n_chunks)
{
    // sa[piece][copy][e] = piece of V[e + copy], V[e] = t(ulo + e)
    __shared__ __attribute__((aligned(16))) unsigned short sa[3][4][kCopyPitch];
    // xs[piece][2 B + c][r] = piece of x_c[32 (Blo + B) + r]
    __shared__ __attribute__((aligned(16))) unsigned short xs[3][2 * kXBlocks][kXRow];

    const int D = a.D;
    const int nblk = (D + kBlk - 1) / kBlk;
    const int I0 = blockIdx.x * kGroupBlocks;
    // block offsets with some output block in [I0, I0 + 128) and its input
    // block in [0, nblk): d in [I0 - (nblk - 1), I0 + 127]
    const int dlo = I0 - (nblk - 1);
    const int nd = kGroupBlocks + nblk - 1;
    const int per = (nd + n_chunks - 1) / n_chunks;
    const int d0 = dlo + (int)blockIdx.y * per;
    const int d1 = min(d0 + per, dlo + nd);           // exclusive
    const int chunk = blockIdx.y;                     // partial slot
    // A runs t(u0 + j), u0 = -32 d - p + 16 h + 8 kg, over d in [d0, d1):
    // u in [ulo, ulo + nU)
    const int ulo = -kBlk * d1 + 1;
    const int Blo = I0 - d1 + 1;                      // first x block of the window

    if (d0 < d1) {
        const int nU = kBlk * (d1 - d0) + kBlk - 1;
        const int npair = (kGroupBlocks + (d1 - d0) - 1) * (kBlk / 2);
        constexpr int SPER = (kSymLen + kThreads - 1) / kThreads;
        constexpr int XPER = (kXBlocks * kBlk / 2 + kThreads - 1) / kThreads;
        float sv[SPER];
        float2 xv[XPER][2];
        // all global loads first, so that they are in flight together
#pragma unroll
        for (int u = 0; u < SPER; ++u) {
            const int e = (int)threadIdx.x + kThreads * u;
            const int m = ulo + e;
            sv[u] = (e < nU && m > -D && m < D) ? a.text[m + D - 1] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            const int q = (int)threadIdx.x + kThreads * u;
            const int j = Blo * kBlk + 2 * q;
            const bool in = q < npair;
            xv[u][0] = (in && j >= 0 && j < D) ? a.X[j] : make_float2(0.f, 0.f);
            xv[u][1] = (in && j + 1 >= 0 && j + 1 < D) ? a.X[j + 1] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < SPER; ++u) {
            const int e = (int)threadIdx.x + kThreads * u;
            if (e < nU) {
                uint32_t pc[3];
                split3(sv[u], pc[0], pc[1], pc[2]);
#pragma unroll
                for (int P = 0; P < 3; ++P)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (e >= c) sa[P][c][e - c] = (unsigned short)pc[P];
            }
        }
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            const int q = (int)threadIdx.x + kThreads * u;
            if (q < npair) {
                const int B = q / (kBlk / 2);
                const int r = 2 * (q - B * (kBlk / 2));
                uint32_t re0[3], re1[3], im0[3], im1[3];
                split3(xv[u][0].x, re0[0], re0[1], re0[2]);
                split3(xv[u][1].x, re1[0], re1[1], re1[2]);
                split3(xv[u][0].y, im0[0], im0[1], im0[2]);
                split3(xv[u][1].y, im1[0], im1[1], im1[2]);
#pragma unroll
                for (int P = 0; P < 3; ++P) {
                    *(uint32_t*)&xs[P][2 * B][r] = re0[P] | (re1[P] << 16);
                    *(uint32_t*)&xs[P][2 * B + 1][r] = im0[P] | (im1[P] << 16);
                }
            }
        }
    }
    __syncthreads();
    // (an empty chunk still writes its slot: zeros)

    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int tg = w % kTileGroups;   // tile pair of this wave
    const int dp = w / kTileGroups;   // phase of its block offsets
    const int p = lane & 31;             // A row; also the B / C column n
    const int kg = lane >> 5;            // K group: k = 8 kg + j
    const int nb = p >> 1;               // output block within a column tile
    const int comp = p & 1;              // re / im column
    const int cp = 3 - (p & 3);          // symbol copy with an aligned run for row p
    const int Iw = I0 + kWaveTiles * kTileBlocks * tg;
    // The two halves of a run are separate 8-byte reads: merged into one
    // 16-byte read at an 8-byte boundary they run at an eighth of the LDS
    // bandwidth.  An offset the compiler cannot see through keeps them apart.
    int half = 4;
    asm volatile("" : "+v"(half));

    // fragments of one step (d, h): A[p][8 kg + j] = t(32 d + p - q) with
    // q = 16 h + 8 kg + j, read as t(u0 + j) (t is even) from the copy in
    // which the run starts on an 8-byte boundary; B[8 kg + j][n] =
    // x_comp[32 (I - d) + q] for the lane's blocks I = Iw + nb, Iw + 16 + nb
    auto load_step = [&](int d, int h, uint4 (&A)[3], uint4 (&B0)[3], uint4 (&B1)[3]) {
        const int row0 = 2 * (Iw + nb - d - Blo) + comp;
        const int row1 = row0 + 2 * kTileBlocks;
        const int ea = kBlk * (d1 - d) - 1 - p + 16 * h + 8 * kg - cp;
#pragma unroll
        for (int P = 0; P < 3; ++P) {
            const uint2 lo = *(const uint2*)&sa[P][cp][ea];
            const uint2 hi = *(const uint2*)&sa[P][cp][ea + half];
            A[P] = make_uint4(lo.x, lo.y, hi.x, hi.y);
            B0[P] = *(const uint4*)&xs[P][row0][16 * h + 8 * kg];
            B1[P] = *(const uint4*)&xs[P][row1][16 * h + 8 * kg];
        }
    };
    // hh products and the five smaller ones in separate accumulators: added
    // to a sum of hh products, most of a smaller product falls below half a
    // unit of its last place and is rounded away, and what is lost is part of
    // t x with the sign of t x, not noise (a shift of the operator's energy,
    // about -8e-5 at D = 32768 for a smooth vector); in their own sum they keep
    // their digits, and the two sums meet once after the loop
    f32x16 acc0 = {}, acc1 = {}, low0 = {}, low1 = {};
    // hh | hm, mh, hl, lh, mm; the two tiles alternate
    auto products = [&](const uint4 (&A)[3], const uint4 (&B0)[3], const uint4 (&B1)[3]) {
        acc0 = mfma(A[0], B0[0], acc0);
        acc1 = mfma(A[0], B1[0], acc1);
        low0 = mfma(A[0], B0[1], low0);
        low1 = mfma(A[0], B1[1], low1);
        low0 = mfma(A[1], B0[0], low0);
        low1 = mfma(A[1], B1[0], low1);
        low0 = mfma(A[0], B0[2], low0);
        low1 = mfma(A[0], B1[2], low1);
        low0 = mfma(A[2], B0[0], low0);
        low1 = mfma(A[2], B1[0], low1);
        low0 = mfma(A[1], B0[1], low0);
        low1 = mfma(A[1], B1[1], low1);
    };
    // this wave's offsets: d0 + dp, d0 + dp + 4, ...; software pipeline: the
    // fragments of the next step are read while the matrix cores work on the
    // current one (the last pass re-reads a valid step and discards it)
    uint4 A0[3], B00[3], B10[3], A1[3], B01[3], B11[3];
    if (d0 + dp < d1) load_step(d0 + dp, 0, A0, B00, B10);
    for (int d = d0 + dp; d < d1; d += kPhases) {
        load_step(d, 1, A1, B01, B11);
        products(A0, B00, B10);
        load_step(d + kPhases < d1 ? d + kPhases : d, 0, A0, B00, B10);
        products(A1, B01, B11);
        // schedule as written: the 12 LDS reads of the next step issue ahead
        // of the 12 MFMAs of the current one, so they run under them
        __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);   // LDS reads
        __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);   // MFMAs
        __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 12, 0);
    }

#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc0[r] += low0[r];
        acc1[r] += low1[r];
    }

    // Sums of the four waves of a tile pair, then coalesced stores: the
    // workgroup's 64 x 32 rows go through LDS (the staging arrays are free
    // once every wave has left the loop), ob[block * kOutPitch + 2 row + c],
    // the phases adding in a fixed order.
    // C[row][n]: lane holds column n, rows 8 (r >> 2) + 4 kg + (r & 3).
    float* ob = reinterpret_cast<float*>(&xs[0][0][0]);
    static_assert(kGroupBlocks * kOutPitch * sizeof(float) <= sizeof(xs), "output staging");
    const int ob0 = (kWaveTiles * kTileBlocks * tg + nb) * kOutPitch + comp;
    const int ob1 = ob0 + kTileBlocks * kOutPitch;
#pragma unroll
    for (int ph = kPhases - 1; ph >= 0; --ph) {
        __syncthreads();
        if (dp == ph) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ro = 8 * (r >> 2) + 4 * kg + (r & 3);
                if (ph == kPhases - 1) {
                    ob[ob0 + 2 * ro] = acc0[r];
                    ob[ob1 + 2 * ro] = acc1[r];
                } else {
                    ob[ob0 + 2 * ro] += acc0[r];
                    ob[ob1 + 2 * ro] += acc1[r];
                }
            }
        }
    }
    __syncthreads();
    // each thread stores complex pairs (rows 2e, 2e + 1 of the workgroup)
    float2* slot = a.P + (size_t)chunk * a.ldp;
    const bool even_ld = (a.ldp & 1) == 0;   // 16-byte stores stay aligned
    constexpr int kPairs = kGroupBlocks * kBlk / 2;
#pragma unroll
    for (int k = 0; k < kPairs / kThreads; ++k) {
        const int e = (int)threadIdx.x + kThreads * k;
        const int blk = e / (kBlk / 2);
        const int rl = 2 * e - kBlk * blk;
        const float4 v = *(const float4*)&ob[blk * kOutPitch + 2 * rl];
        const int g = kBlk * I0 + 2 * e;
        if (g + 1 < D && even_ld) {
            *(float4*)(slot + g) = v;
        } else {
            if (g < D) slot[g] = make_float2(v.x, v.y);
            if (g + 1 < D) slot[g + 1] = make_float2(v.z, v.w);
        }
    }
}

}  // namespace

int dvr_bf16_chunks(int32_t D)
{
    // about kTargetGroups workgroups in all (row groups x chunks), at least one
    const int nblk = (D + kBlk - 1) / kBlk;
    const int groups = (nblk + kGroupBlocks - 1) / kGroupBlocks;
    const int nd = kGroupBlocks + nblk - 1;
    int s = (kTargetGroups + groups - 1) / groups;
    // each chunk at most kMaxChunk offsets (LDS window)
    const int smin = (nd + kMaxChunk - 1) / kMaxChunk;
    if (s < smin) s = smin;
    if (s > nd) s = nd;
    return s;
}

hipError_t launch_dvr_toeplitz_bf16(const DvrToeplitzArgs& a, hipStream_t s, hipEvent_t e0,
                                    hipEvent_t e1)
{
    const int nblk = (a.D + kBlk - 1) / kBlk;
    const int groups = (nblk + kGroupBlocks - 1) / kGroupBlocks;
    const int chunks = dvr_bf16_chunks(a.D);
    const dim3 grid((unsigned)groups, (unsigned)chunks);
    if (e0)
        hipExtLaunchKernelGGL(dvr_toeplitz_bf16x6_kernel, grid, dim3(kThreads), 0, s, e0, e1, 0,
                              a, chunks);
    else
        hipLaunchKernelGGL(dvr_toeplitz_bf16x6_kernel, grid, dim3(kThreads), 0, s, a, chunks);
    return hipGetLastError();
}

}  // namespace procmv
