// Kernel launch descriptors shared by the kernel files and the host API.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gen.h"

namespace procmv {

// Square super-tiles of E = 64 se entries (se = 1, 2 or 4 column tiles of 64)
// are the work units of the tile kernels (VALU and MFMA).  Output element i
// of band B = i / E receives exactly one partial per slot k in [0, N_s]:
// slot k >= B from the direct product of super-tile (B, k), slot k < B from
// the transposed product of super-tile (k, B), slot N_s from the transposed
// product of the diagonal super-tile (B, B).
constexpr int kSuper = 256;   // largest edge (se = 4)

// Edge in 64-column tiles for dimension D: the largest edge that still gives
// at least 45 super-tile bands (about 1000 super-tiles, four per compute
// unit), 64 below that.
inline int super_edge_tiles(int64_t D)
{
    for (int se = 4; se > 1; se /= 2)
        if ((D + 64 * se - 1) / (64 * se) >= 45) return se;
    return 1;
}

// VALU tile shape actually launched: the largest shape <= `shape` whose tile
// rows TR = 4 RW (RW = (8, 16, 32) / (2 nv) for shapes 0, 1, 2) fit the
// super-tile edge 64 se and, when tiles are read from a block cache of block
// size `cache_b` (0 = no cache), divide it, so that every cached tile lies
// inside one b x b slot.
inline int fit_tile_shape(int nv, int shape, int se, int cache_b)
{
    if (nv < 1) return 0;
    while (shape > 0) {
        const int tr = 4 * (16 << shape) / (2 * nv);
        if (tr <= 64 * se && (cache_b == 0 || cache_b % tr == 0)) break;
        --shape;
    }
    return shape;
}

// Where the entries of one tile come from.
struct SourceArgs {
    int gen;                   // 0 Philox-GUE, 1 sinc-DVR
    GueParams gue;
    DvrParams dvr;
    const int32_t* pair_slot;  // [n_blk * n_blk] slot of canonical pair or -1; null = no cache
    const void* slots;         // slot pool: b*b complex64 (GUE) or float (DVR) per slot
    int32_t b;
    int32_t n_blk;
    int32_t all_cached;        // every canonical pair has a slot
};

struct TileArgs {
    SourceArgs src;
    int32_t D;
    int32_t se;               // super-tile edge in 64-column tiles (1, 2, 4)
    int32_t n_super;          // N_s = ceil(D / (64 se))
    int32_t nv;               // vectors in this launch (MFMA kernel: <= 16)
    const int2* st_list;      // super-tile coordinates (sr, sc), sr <= sc
    const float2* X;          // nvec-chunk base, vector v at X + v * ldx
    int64_t ldx;
    int64_t xoff;             // batched launches: X = launch base + xoff
    float2* P;                // partials: slot s, vector v at P + (s * nv + v) * ldp
    int64_t ldp;
};

// One persistent launch over the (instance, super-tile) items of a batch.
struct BatchTileLaunch {
    const TileArgs* ops;      // device array, one per instance
    const int4* items;        // (instance, sr, sc, 0)
    int64_t n_items;
    const float2* xbase;      // packed vectors of all instances
    int gen, nv, shape, grid;
    int cached;               // some instance has cached block pairs
    int min_se;               // smallest super-tile edge (64-column tiles) of the instances
    int cache_b;              // common divisor of the cached instances' block sizes (0 = none)
    int mfma;                 // matrix-core kernel (binary32) instead of the VALU one
};

// Sinc-DVR Toeplitz product: row bands x column chunks, one partial slot per
// chunk.  text[k + D - 1] = t(k) for |k| < D, zero at k = 0.
struct DvrToeplitzArgs {
    int32_t D;
    const float* text;
    const float2* X;
    int64_t ldx;
    float2* P;                // slot = column chunk, vector v at P + (s * nv + v) * ldp
    int64_t ldp;
};

// Epilogue of the fixed-order partial reduction.
enum class Epi : int {
    kApply = 0,     // Y = alpha y + beta x
    kChebFirst = 1, // q1 = h;              acc = a0 q0 + a1 q1
    kChebStep = 2   // qn = 2 h - q_prev;   acc += a qn   (qn stored over q_prev)
};

struct ReduceArgs {
    int32_t D;
    int32_t nv;
    int32_t nv_stride;        // vector stride of the partial slots (>= nv)
    int32_t n_slots;          // N_s + 1
    const float2* P;
    int64_t ldp;
    const float2* X;          // the vectors the product was applied to
    int64_t ldx;
    const float* vdiag;       // optional site diagonal: y += vdiag[i] x_i first
    float2* Y;                // kApply: output; kChebStep: q_prev in, q_next out
    int64_t ldy;
    float2* Yq1;              // kChebFirst: q1 out
    double2* acc;             // binary64 accumulator (nv, ldacc)
    int64_t ldacc;
    float alpha;              // 1/R (Chebyshev) or 1 (apply)
    float beta_hi, beta_lo;   // constant-diagonal term, hi + lo binary32 pair
    double2 a0, a1;           // Chebyshev coefficients of the epilogue
    // compensated sinc-DVR epilogue (launch_reduce_comp); cv == null otherwise
    const float2* cv;         // per-row constant C_i as (hi, lo)
    const float* tk;          // binary32 kinetic symbol tk[k], k = 1..W-1
    int32_t W;                // band width: the tile kernels skip |i - j| < W
    const float2* Xlo;        // lo parts of X (ld ldxl); null = zero
    int64_t ldxl;
    float2* Ylo;              // kChebStep: lo of q_prev in, of q_next out (ld ldylo)
    float2* Yq1lo;            // kChebFirst: lo of q1 out
    float2* Xlo_zero;         // kChebFirst: lo buffer of q0, set to zero
    int64_t ldylo;
    float gamma_hi, gamma_lo; // alpha c as a hi + lo pair
    // > 0 (one vector): the partial slots come from the split-bf16 Toeplitz
    // kernel, whose row group g (xcd_groups of them, a multiple of 8; 32
    // blocks of 64 rows each, D = 2048 xcd_groups) ran every chunk on XCD
    // g mod 8: the reduction's workgroup b (XCD b mod 8) takes a 64-row
    // block of a group on its own XCD, so that it reads the slots through
    // that XCD's L2
    int32_t xcd_groups;
};

// Band of the compensated sinc-DVR arithmetic: entries with |i - j| < W are
// summed in difference form by the reduction, W = min(kNearBand, D).
constexpr int kNearBand = 32;

// 64-row block reduced by workgroup b: b itself, or with a.xcd_groups > 0 a
// block of a split-kernel row group that ran on b's XCD (workgroups go to the
// eight XCDs round robin by index; group g's 32 blocks sit on XCD g mod 8).
// A permutation of the 32 xcd_groups blocks.
__device__ __forceinline__ int reduce_row_block(const ReduceArgs& a, int b)
{
    if (a.xcd_groups <= 0) return b;
    const int x = b & 7, w = b >> 3;
    return (x + 8 * (w >> 5)) * 32 + (w & 31);
}

// Epilogue of the fixed-order reduction for output element (v, i) whose
// summed partials are (sx, sy): add the site diagonal, scale, add the
// constant diagonal, then store (product) or advance the Chebyshev
// recurrence and the binary64 accumulator.
template <Epi MODE>
__device__ __forceinline__ void reduce_epilogue(const ReduceArgs& a, int v, int i, float sx,
                                                float sy)
{
    const float2 x = a.X[v * a.ldx + i];
    if (a.vdiag != nullptr) {
        const float vd = a.vdiag[i];
        sx = __builtin_fmaf(vd, x.x, sx);
        sy = __builtin_fmaf(vd, x.y, sy);
    }
    // h = alpha * y + (beta_hi + beta_lo) * x
    const float bx = __builtin_fmaf(a.beta_hi, x.x, a.beta_lo * x.x);
    const float by = __builtin_fmaf(a.beta_hi, x.y, a.beta_lo * x.y);
    const float hx = __builtin_fmaf(a.alpha, sx, bx);
    const float hy = __builtin_fmaf(a.alpha, sy, by);
    if (MODE == Epi::kApply) {
        a.Y[v * a.ldy + i] = make_float2(hx, hy);
    } else if (MODE == Epi::kChebFirst) {
        a.Yq1[v * a.ldy + i] = make_float2(hx, hy);
        double2 r;
        r.x = a.a0.x * (double)x.x - a.a0.y * (double)x.y;
        r.y = a.a0.x * (double)x.y + a.a0.y * (double)x.x;
        r.x += a.a1.x * (double)hx - a.a1.y * (double)hy;
        r.y += a.a1.x * (double)hy + a.a1.y * (double)hx;
        a.acc[v * a.ldacc + i] = r;
    } else {
        float2* qp = a.Y + v * a.ldy + i;
        const float2 prev = *qp;
        const float nx = __builtin_fmaf(2.0f, hx, -prev.x);
        const float ny = __builtin_fmaf(2.0f, hy, -prev.y);
        *qp = make_float2(nx, ny);
        double2 r = a.acc[v * a.ldacc + i];
        r.x += a.a0.x * (double)nx - a.a0.y * (double)ny;
        r.y += a.a0.x * (double)ny + a.a0.y * (double)nx;
        a.acc[v * a.ldacc + i] = r;
    }
}

// Batched reduction: per-instance description and the launch arguments.
struct BatchReduceItem {
    int32_t D;
    int32_t n_slots;
    int64_t off;              // packed element offset of the instance
    const float2* P;          // its partial slots (vector stride nv)
    int64_t ldp;
    float alpha, beta_hi, beta_lo;
    double2 phase;            // e^{-i c dt} of the Chebyshev step
};

struct BatchReduceArgs {
    const BatchReduceItem* items;
    const int64_t* off;       // [n] packed offsets (sorted)
    int32_t n;
    int32_t nv;
    int64_t total;            // packed elements
    const float2* X;
    float2* Y;
    float2* Yq1;
    double2* acc;
    double2 a0, a1;
};

// Planner surrogate network: 8 inputs, two hidden layers of 64 ReLU units.
constexpr int kMlpIn = 8;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpHidden + 1;

// Launchers (defined in apply.hip).
hipError_t launch_tile_apply(const TileArgs& a, int nv, int shape, int n_st,
                             hipStream_t s);
hipError_t launch_tile_apply_batched(const BatchTileLaunch& b, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, Epi mode, hipStream_t s,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Static device workspace of the allocation-free product (defined in
// noalloc.hip): the current device's copy of a file-scope array, its
// address resolved once per device.
size_t static_workspace_bytes();
hipError_t static_workspace(void** ptr, size_t* bytes);
// Compensated reduction of the sinc-DVR operator (defined in comp.hip).
hipError_t launch_reduce_comp(const ReduceArgs& a, Epi mode, hipStream_t s,
                              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// MFMA multi-vector tile product, nv <= 16 (defined in mfma.hip);
// precision 0 = binary32 MFMA, 1 = split bfloat16.
hipError_t launch_tile_mfma(const TileArgs& a, int precision, int n_st,
                            hipStream_t s);
// Batched persistent matrix-core product (binary32) of the items of a batch.
hipError_t launch_tile_mfma_batched(const BatchTileLaunch& b, hipStream_t s);
hipError_t launch_cache_fill(const SourceArgs& src, int32_t D,
                             const int2* pairs, int64_t n_pairs, void* slots,
                             hipStream_t s);
hipError_t launch_get_entries(const SourceArgs& src, int64_t r0, int64_t c0,
                              int32_t nr, int32_t nc, float2* out,
                              hipStream_t s);
// Generator arithmetic self-test (defined in selftest.hip): count[0] = uniforms
// whose logarithm differs from the IEEE-division one, count[1] = square roots
// that differ from IEEE sqrt.
hipError_t launch_selftest_generator(unsigned* count, hipStream_t s);
// Sinc-DVR Toeplitz product (defined in dvr.hip).
int dvr_toeplitz_variant(int32_t D, int nv);
int dvr_toeplitz_chunk_of(int variant);
// e0/e1 (optional): start/stop events recorded by the kernel's dispatch.
hipError_t launch_dvr_toeplitz(const DvrToeplitzArgs& a, int nv, int variant,
                               hipStream_t s, hipEvent_t e0 = nullptr,
                               hipEvent_t e1 = nullptr);
// Sinc-DVR Toeplitz product of one vector on the matrix cores (defined in
// dvr_mfma.hip): partial slots = dvr_mfma_chunks(D), layout as above.
constexpr int32_t kDvrMfmaMinD = 16384;   // default routing: from this D on
int dvr_mfma_chunks(int32_t D);
hipError_t launch_dvr_toeplitz_mfma(const DvrToeplitzArgs& a, hipStream_t s,
                                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// The same product on the bfloat16 matrix cores with an exact three-piece
// split of the binary32 operands (defined in dvr_bf16.hip): partial slots =
// dvr_bf16_chunks(D), layout as above.
int dvr_bf16_chunks(int32_t D);
hipError_t launch_dvr_toeplitz_bf16(const DvrToeplitzArgs& a, hipStream_t s,
                                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Batched reduction and completion (defined in batch.hip).
hipError_t launch_reduce_batched(const BatchReduceArgs& a, Epi mode, hipStream_t s);
hipError_t launch_finish_batched(const BatchReduceItem* items, int n, int nv,
                                 const double2* acc, float2* psi, double* norm2,
                                 hipStream_t s);
// Surrogate network (defined in mlp.hip).
hipError_t launch_mlp_forward(const float* p, const float* z, int n, float* y, float* a1s,
                              float* a2s, hipStream_t s);
hipError_t launch_mlp_backward(const float* p, const float* z, const float* y,
                               const float* t, int n, const float* a1s, const float* a2s,
                               float* gys, float* ga1s, float* ga2s, float* g, hipStream_t s);
hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, float lr, int step,
                           hipStream_t s);
hipError_t launch_mlp_loss(const float* y, const float* t, int n, float* loss, hipStream_t s);
// Chebyshev helpers (defined in cheb.hip).
hipError_t launch_cheb_finish(int32_t D, int32_t nv, const double2* acc,
                              int64_t ldacc, double2 phase, float2* psi,
                              int64_t ld, double* norm2, hipStream_t s);
hipError_t launch_copy_vectors(int32_t D, int32_t nv, const float2* src,
                               int64_t lds, float2* dst, int64_t ldd,
                               hipStream_t s);
// System-side mixing of the system-bath Kronecker product (defined in kron.hip).
constexpr int kKronMaxSys = 8;     // d_S
constexpr int kKronMaxInt = 3;     // interaction terms
struct KronMixArgs {
    const float2* X;   // (dS, dB) input
    const float2* Z;   // (1 + n_int, dS, dB) bath products: H_B rows, then B_a rows
    float2* Y;         // (dS, dB) output
    int64_t dB;
    int32_t dS;
    int32_t n_int;
    // M_0 = H_S, M_a = g A_a, each kKronMaxSys x kKronMaxSys row-major (top-left dS x dS used)
    float2 M[(1 + kKronMaxInt) * kKronMaxSys * kKronMaxSys];
};
hipError_t launch_kron_mix(const KronMixArgs& a, hipStream_t s);
// Chebyshev propagation of the system-bath operator (defined in kron.hip):
// acc = coef q; and one binary32 term q_new = [2] (alpha Y + beta q_k)
// [- q_prev] over q_prev, beta = -alpha c as hi + lo, with acc += coef q_new
// (binary64).
hipError_t launch_kron_cheb_init(int64_t n, const float2* q, double2* acc, double2 coef,
                                 hipStream_t s);
hipError_t launch_kron_cheb_term(int64_t n, const float2* Y, const float2* qk, float2* qprev,
                                 double2* acc, float alpha, float bhi, float blo, double2 coef,
                                 int first, hipStream_t s);
// Lanczos vector steps (defined in lanczos.hip).  Partial buffers hold
// lanczos_blocks(D) <= kLanczosMaxBlocks doubles each.
constexpr int32_t kLanczosMaxBlocks = 512;
int32_t lanczos_blocks(int32_t D);
// out = x / ||x|| (binary64 norm, stored in *norm_out when not null).
hipError_t launch_lanczos_normalise(int32_t D, const float2* x, float2* out,
                                    double* partials, double* norm_out, hipStream_t s);
// out = x / sqrt(sum of partials), the partials of ||x||^2 being already
// written (by launch_lanczos_orthogonalise for the same x).
hipError_t launch_lanczos_scale(int32_t D, const float2* x, float2* out,
                                const double* partials, double* norm_out, hipStream_t s);
// *alpha_out = Re <v, w>; w <- w - alpha v - (*beta_prev) v_prev (beta_prev
// null: no v_prev term); norm_partials <- partials of ||w||^2.
hipError_t launch_lanczos_orthogonalise(int32_t D, const float2* v, const float2* v_prev,
                                        float2* w, double* dot_partials,
                                        double* norm_partials, const double* beta_prev,
                                        double* alpha_out, hipStream_t s);

}  // namespace procmv
