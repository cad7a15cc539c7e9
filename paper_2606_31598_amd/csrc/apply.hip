// Fused block source + two-sided block product on the VALU (gfx950).
//
// Paper Sec. III: phi^[n] = sum_m apply_H_block(n, m, psi^[m]) with blocks
// that are generated on the fly or read from a cache of canonical pairs
// (n <= m), using H^[m,n] = (H^[n,m])^dagger.  Each canonical entry is
// obtained once and applied twice: y_i += H_ij x_j and y_j += conj(H_ij) x_i.
//
// Work decomposition.  The canonical upper triangle is cut into square
// super-tiles of E x E (E = 64, 128 or 256 by dimension, see
// super_edge_tiles); one workgroup (4 waves of 64) owns one
// super-tile and walks its tiles of TR x 64 entries, TR = 4 * RW, each wave
// taking RW consecutive rows and each lane one column.  Direct sums for the
// wave's rows stay in registers across the super-tile row and are reduced
// across lanes once; transposed sums for each lane's columns stay in
// registers across the whole super-tile and are reduced across waves once.
// Both go to a partial buffer in which every output element has exactly one
// slot per super-tile band (see kernels.h), and a second kernel sums the slots
// in a fixed order: no atomics, bit-reproducible results.
#include <hip/hip_ext.h>

#include <type_traits>

#include "kernels.h"

namespace procmv {

namespace {

__device__ __forceinline__ float2 cmul(float2 h, float2 x)
{
    return make_float2(__builtin_fmaf(h.x, x.x, -h.y * x.y),
                       __builtin_fmaf(h.x, x.y, h.y * x.x));
}

// acc += h * x
__device__ __forceinline__ void cfma(float2& acc, float2 h, float2 x)
{
    acc.x = __builtin_fmaf(h.x, x.x, acc.x);
    acc.x = __builtin_fmaf(-h.y, x.y, acc.x);
    acc.y = __builtin_fmaf(h.x, x.y, acc.y);
    acc.y = __builtin_fmaf(h.y, x.x, acc.y);
}

// acc += conj(h) * x
__device__ __forceinline__ void cfma_conj(float2& acc, float2 h, float2 x)
{
    acc.x = __builtin_fmaf(h.x, x.x, acc.x);
    acc.x = __builtin_fmaf(h.y, x.y, acc.x);
    acc.y = __builtin_fmaf(h.x, x.y, acc.y);
    acc.y = __builtin_fmaf(-h.y, x.x, acc.y);
}

// acc += r * x (real entry)
__device__ __forceinline__ void rfma(float2& acc, float r, float2 x)
{
    acc.x = __builtin_fmaf(r, x.x, acc.x);
    acc.y = __builtin_fmaf(r, x.y, acc.y);
}

// Sum over the 64 lanes of a wave of N values per lane (N = 16, 32 or 64).
// Butterfly reduce-scatter: each halving step keeps half of the values and
// adds the partner lane's copy of them; afterwards every lane holds the wave
// total of value index lane / (64 / N) (the lanes of one group agree).
template <int N>
__device__ __forceinline__ float wave_reduce_scatter(float (&v)[N])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int half = N / 2, mask = 32; half >= 1; half /= 2, mask /= 2) {
#pragma unroll
        for (int k = 0; k < half; ++k) {
            const bool up = lane & mask;
            float keep, give;
            if (N <= 32) {
                // select values, not addresses: keeps the array in registers
                const float lo = v[k], hi = v[half + k];
                keep = up ? hi : lo;
                give = up ? lo : hi;
            } else {
                keep = up ? v[half + k] : v[k];
                give = up ? v[k] : v[half + k];
            }
            v[k] = keep + __shfl_xor(give, mask);
        }
    }
    float r = v[0];
#pragma unroll
    for (int mask = 32 / N; mask >= 1; mask /= 2) r += __shfl_xor(r, mask);
    return r;
}

// One entry h = H_ij of a tile row applied both ways: dir += h x_j for the
// row, tr += conj(h) x_i for the column (real entries for the sinc-DVR).  ok
// masks entries outside the canonical triangle or the matrix, upper keeps the
// diagonal out of the transposed sum.
template <int NV, int GEN>
__device__ __forceinline__ void apply_entry(float2 (&dir)[NV], float2 (&tr)[NV], float2 h,
                                            bool ok, bool upper, const float2 (&xj)[NV],
                                            const float2* xi)
{
    if (GEN == 0) {
        if (!ok) h = make_float2(0.f, 0.f);
        const float2 ht = upper ? h : make_float2(0.f, 0.f);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            cfma(dir[v], h, xj[v]);
            cfma_conj(tr[v], ht, xi[v]);
        }
    } else {
        const float hv = ok ? h.x : 0.f;
        const float hvt = upper ? hv : 0.f;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            rfma(dir[v], hv, xj[v]);
            rfma(tr[v], hvt, xi[v]);
        }
    }
}

// Block pair slot of the tile whose first row/column are (i0, j0).
__device__ __forceinline__ int32_t tile_slot(const SourceArgs& s, int i0, int j0)
{
    if (s.pair_slot == nullptr) return -1;
    int n = i0 / s.b, m = j0 / s.b;
    return s.pair_slot[n * s.n_blk + m];
}

// One super-tile (sr, sc) of one operator: everything the two-sided product
// of that super-tile contributes, written to its partial slots.
template <int NV, int RW, int GEN, int SRC>
__device__ __forceinline__ void super_tile(const TileArgs& a, int sr, int sc,
                                           float2 (*red)[64][NV], float2 (*xs)[NV])
{
    constexpr int TR = 4 * RW;          // rows per tile
    constexpr int SC = kSuper / 64;     // most column tiles per super-tile
    constexpr int NR = 2 * RW * NV;     // direct values reduced across lanes
    static_assert(NR == 16 || NR == 32 || NR == 64, "tile shape");
    const int sct = a.se;               // column tiles per super-tile here
    const int SR = 64 * sct / TR;       // tile rows (the launcher keeps TR <= edge)

    const int lane = threadIdx.x & 63;
    // wave index visibly uniform: a wave's row indices are scalars, and the
    // Philox products that depend on the row only run on the scalar unit
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool diag_st = (sr == sc);
    const int row0 = sr * 64 * sct, col0 = sc * 64 * sct;
    const int D = a.D;

    float2 tr[SC][NV];
#pragma unroll
    for (int c = 0; c < SC; ++c)
#pragma unroll
        for (int v = 0; v < NV; ++v) tr[c][v] = make_float2(0.f, 0.f);

    for (int rr = 0; rr < SR; ++rr) {
        const int trow0 = row0 + rr * TR;   // first row of the tile (WG-uniform)
        const int ib = trow0 + w * RW;      // first row of this wave
        float2 dir[RW][NV];
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int v = 0; v < NV; ++v) dir[r][v] = make_float2(0.f, 0.f);
        // x of the tile rows, staged in LDS and read back as wave broadcasts
        __syncthreads();
        for (int q = threadIdx.x; q < TR * NV; q += 256) {
            const int r = q / NV, v = q - (q / NV) * NV;
            const int i = trow0 + r;
            xs[r][v] = (i < D) ? a.X[v * a.ldx + i] : make_float2(0.f, 0.f);
        }
        __syncthreads();

#pragma unroll
        for (int cc = 0; cc < SC; ++cc) {
            if (cc >= sct) continue;
            const int tcol0 = col0 + cc * 64;
            if (trow0 >= D || tcol0 >= D) continue;
            // tiles strictly below the diagonal belong to the transpose
            if (diag_st && rr * TR > cc * 64 + 63) continue;
            const int j = tcol0 + lane;
            const bool jin = j < D;
            float2 xj[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                xj[v] = jin ? a.X[v * a.ldx + j] : make_float2(0.f, 0.f);

            const int32_t slot = SRC ? tile_slot(a.src, trow0, tcol0) : -1;
            if (SRC && slot >= 0) {
                // Cached tile: the RW row loads of this lane go out first.  A
                // tile lies inside one b x b block, whose slot is allocated in
                // full (rows/columns past D hold zeros): no bounds guard.
                const int bb = a.src.b;
                const int n0 = (trow0 / bb) * bb, m0 = (tcol0 / bb) * bb;
                const size_t base = (size_t)slot * bb * bb + (size_t)(ib - n0) * bb + (j - m0);
                float2 hc[RW];
                if (GEN == 0) {
                    const float2* sp = (const float2*)a.src.slots + base;
#pragma unroll
                    for (int r = 0; r < RW; ++r) hc[r] = sp[(size_t)r * bb];
                } else {
                    const float* sp = (const float*)a.src.slots + base;
#pragma unroll
                    for (int r = 0; r < RW; ++r) hc[r] = make_float2(sp[(size_t)r * bb], 0.f);
                }
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    const int i = ib + r;
                    const bool ok = jin && (i < D) && (i <= j);
                    const bool upper = ok && (i < j);
                    if (GEN == 0) {
                        const float2 h = ok ? hc[r] : make_float2(0.f, 0.f);
                        const float2 ht = upper ? h : make_float2(0.f, 0.f);
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            cfma(dir[r][v], h, xj[v]);
                            cfma_conj(tr[cc][v], ht, xs[w * RW + r][v]);
                        }
                    } else {
                        const float hv = ok ? hc[r].x : 0.f;
                        const float hvt = upper ? hv : 0.f;
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            rfma(dir[r][v], hv, xj[v]);
                            rfma(tr[cc][v], hvt, xs[w * RW + r][v]);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    const int i = ib + r;
                    const bool ok = jin && (i < D) && (i <= j);
                    const bool upper = ok && (i < j);
                    if (GEN == 0) {
                        // every lane draws at its own (i, j); entries outside the
                        // operator or below the diagonal are masked to zero below
                        uint32_t x0, x1;
                        philox_row((uint32_t)i, (uint32_t)j, a.src.gue.k0, a.src.gue.k1, x0, x1);
                        float z0, z1;
                        box_muller(x0, x1, z0, z1);
                        float2 h = (i == j) ? make_float2(a.src.gue.s_diag * z0, 0.f)
                                            : make_float2(a.src.gue.s_off * z0, a.src.gue.s_off * z1);
                        // keep at most two rows' generation chains in flight
                        if (r & 1) __builtin_amdgcn_sched_barrier(0);
                        if (!ok) h = make_float2(0.f, 0.f);
                        const float2 ht = upper ? h : make_float2(0.f, 0.f);
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            cfma(dir[r][v], h, xj[v]);
                            cfma_conj(tr[cc][v], ht, xs[w * RW + r][v]);
                        }
                    } else {
                        const float hv = ok ? dvr_entry(a.src.dvr, (uint32_t)i, (uint32_t)j) : 0.f;
                        const float hvt = upper ? hv : 0.f;
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            rfma(dir[r][v], hv, xj[v]);
                            rfma(tr[cc][v], hvt, xs[w * RW + r][v]);
                        }
                    }
                }
            }
        }

        // Direct partial of this tile row: reduce over the 64 lanes (columns),
        // slot sc.  Value index (v * RW + r) * 2 + {re, im}.
        float vals[NR];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                vals[(v * RW + r) * 2 + 0] = dir[r][v].x;
                vals[(v * RW + r) * 2 + 1] = dir[r][v].y;
            }
        const float tot = wave_reduce_scatter<NR>(vals);
        constexpr int G = 64 / NR;          // lanes holding the same total
        if ((lane % G) == 0) {
            const int idx = lane / G;
            const int comp = idx & 1;
            const int r = (idx >> 1) % RW;
            const int v = (idx >> 1) / RW;
            const int i = ib + r;
            if (i < D) {
                float* p = (float*)(a.P + ((size_t)sc * NV + v) * a.ldp + i);
                p[comp] = tot;
            }
        }
    }

    // Transposed partials: reduce over the 4 waves (rows), slot sr, or N_s for
    // the diagonal super-tile.
    const int slot_t = diag_st ? a.n_super : sr;
#pragma unroll
    for (int cc = 0; cc < SC; ++cc) {
        if (cc >= sct) continue;
#pragma unroll
        for (int v = 0; v < NV; ++v) red[w][lane][v] = tr[cc][v];
        __syncthreads();
        if (w == 0) {
            const int j = col0 + cc * 64 + lane;
            if (j < D) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    float2 s = red[0][lane][v];
                    s.x += red[1][lane][v].x; s.y += red[1][lane][v].y;
                    s.x += red[2][lane][v].x; s.y += red[2][lane][v].y;
                    s.x += red[3][lane][v].x; s.y += red[3][lane][v].y;
                    a.P[((size_t)slot_t * NV + v) * a.ldp + j] = s;
                }
            }
        }
        __syncthreads();
    }
}

// One super-tile of an operator whose canonical pairs are all cached: the
// same arithmetic, in the same order, as super_tile with a cached source (so
// the results are bit-identical), with the cache reads software-pipelined.
// The tiles of the super-tile are walked row by row, SC per tile row; the
// loads of tile t + PF (its RW entries per lane and the lane's x_j) are
// issued before tile t is applied, into one of 2 PF register buffers indexed
// by the tile column, and the x rows of the next tile row are fetched at the
// start of the current one into a second LDS buffer.  Every memory wait is
// then for data requested PF tiles earlier.  PF = 1 with three waves per SIMD
// measured fastest on MI355X (more buffers cost occupancy).
template <int NV, int RW, int GEN, int PF>
__device__ __forceinline__ void super_tile_cached(const TileArgs& a, int sr, int sc,
                                                  float2 (*red)[64][NV],
                                                  float2 (*xs2)[4 * RW][NV])
{
    constexpr int TR = 4 * RW;
    constexpr int SC = kSuper / 64;
    constexpr int NR = 2 * RW * NV;
    constexpr int NB = 2 * PF;           // register buffers (tiles in flight + 1)
    static_assert(SC % NB == 0, "buffer rotation");
    constexpr int sct = SC;              // largest super-tiles only (the launcher checks)
    constexpr int SR = 64 * sct / TR;
    using Entry = typename std::conditional<GEN == 0, float2, float>::type;

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const bool diag_st = (sr == sc);
    const int row0 = sr * 64 * sct, col0 = sc * 64 * sct;
    const int D = a.D;
    const int bb = a.src.b;
    const Entry* __restrict__ slots = (const Entry*)a.src.slots;
    const int n_rows = min(SR, (D - row0 + TR - 1) / TR);   // tile rows inside D

    float2 tr[SC][NV];
#pragma unroll
    for (int c = 0; c < SC; ++c)
#pragma unroll
        for (int v = 0; v < NV; ++v) tr[c][v] = make_float2(0.f, 0.f);

    Entry hb[NB][RW];
    float2 xb[NB][NV];
    // Issue the loads of tile (rr, cc) into buffer cc % NB.  Tiles that are not
    // applied (past D, or below the diagonal) read the first entries of slot 0.
    auto issue = [&](int rr, int cc) {
        const int trow0 = row0 + rr * TR, tcol0 = col0 + cc * 64;
        const bool live = tcol0 < D && !(diag_st && rr * TR > cc * 64 + 63);
        size_t base = 0;
        if (live) {
            const int n0 = (trow0 / bb) * bb, m0 = (tcol0 / bb) * bb;
            base = (size_t)tile_slot(a.src, trow0, tcol0) * bb * bb +
                   (size_t)(trow0 + w * RW - n0) * bb + (tcol0 + lane - m0);
        }
        const Entry* sp = slots + base;
#pragma unroll
        for (int r = 0; r < RW; ++r) hb[cc % NB][r] = sp[(size_t)r * bb];
        const int j = tcol0 + lane;
#pragma unroll
        for (int v = 0; v < NV; ++v)
            xb[cc % NB][v] = (live && j < D) ? a.X[v * a.ldx + j] : make_float2(0.f, 0.f);
    };
    auto stage = [&](int rr) {             // x of the rows of tile row rr
        const int q = threadIdx.x;
        float2 x = make_float2(0.f, 0.f);
        if (q < TR * NV) {
            const int i = row0 + rr * TR + q / NV;
            if (i < D) x = a.X[(q % NV) * a.ldx + i];
        }
        return x;
    };

    {
        const float2 x0 = stage(0);
        if (threadIdx.x < TR * NV) xs2[0][threadIdx.x / NV][threadIdx.x % NV] = x0;
    }
    if (n_rows > 0) {
#pragma unroll
        for (int c = 0; c < PF; ++c) issue(0, c);
    }
    __syncthreads();

    for (int rr = 0; rr < n_rows; ++rr) {
        const int trow0 = row0 + rr * TR;
        const int ib = trow0 + w * RW;
        const bool more = rr + 1 < n_rows;
        const float2 xnext = more ? stage(rr + 1) : make_float2(0.f, 0.f);
        const float2 (*xs)[NV] = xs2[rr & 1];
        float2 dir[RW][NV];
#pragma unroll
        for (int r = 0; r < RW; ++r)
#pragma unroll
            for (int v = 0; v < NV; ++v) dir[r][v] = make_float2(0.f, 0.f);

#pragma unroll
        for (int cc = 0; cc < SC; ++cc) {
            // prefetch PF tiles ahead: (rr, cc + PF) or (rr + 1, cc + PF - sct)
            if (cc + PF < sct) issue(rr, cc + PF);
            else if (more) issue(rr + 1, cc + PF - sct);
            const int tcol0 = col0 + cc * 64;
            if (tcol0 >= D || (diag_st && rr * TR > cc * 64 + 63)) continue;
            const int j = tcol0 + lane;
            const bool jin = j < D;
            float2 xj[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) xj[v] = xb[cc % NB][v];
            // interior tiles (inside D, strictly above the diagonal) need no masks
            const bool interior = tcol0 + 64 <= D && trow0 + TR <= D &&
                                  (!diag_st || rr * TR + TR - 1 < cc * 64);
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                float2 h;
                if (GEN == 0) h = *(const float2*)&hb[cc % NB][r];
                else h = make_float2(*(const float*)&hb[cc % NB][r], 0.f);
                if (interior) {
                    apply_entry<NV, GEN>(dir[r], tr[cc], h, true, true, xj, xs[w * RW + r]);
                } else {
                    const int i = ib + r;
                    const bool ok = jin && (i < D) && (i <= j);
                    apply_entry<NV, GEN>(dir[r], tr[cc], h, ok, ok && (i < j), xj,
                                         xs[w * RW + r]);
                }
            }
        }

        // direct partial of this tile row (as in super_tile)
        float vals[NR];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                vals[(v * RW + r) * 2 + 0] = dir[r][v].x;
                vals[(v * RW + r) * 2 + 1] = dir[r][v].y;
            }
        const float tot = wave_reduce_scatter<NR>(vals);
        constexpr int G = 64 / NR;
        if ((lane % G) == 0) {
            const int idx = lane / G;
            const int comp = idx & 1;
            const int r = (idx >> 1) % RW;
            const int v = (idx >> 1) / RW;
            const int i = ib + r;
            if (i < D) {
                float* p = (float*)(a.P + ((size_t)sc * NV + v) * a.ldp + i);
                p[comp] = tot;
            }
        }
        if (more && threadIdx.x < TR * NV)
            xs2[(rr + 1) & 1][threadIdx.x / NV][threadIdx.x % NV] = xnext;
        __syncthreads();
    }

    const int slot_t = diag_st ? a.n_super : sr;
#pragma unroll
    for (int cc = 0; cc < SC; ++cc) {
#pragma unroll
        for (int v = 0; v < NV; ++v) red[w][lane][v] = tr[cc][v];
        __syncthreads();
        if (w == 0) {
            const int j = col0 + cc * 64 + lane;
            if (j < D) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    float2 s = red[0][lane][v];
                    s.x += red[1][lane][v].x; s.y += red[1][lane][v].y;
                    s.x += red[2][lane][v].x; s.y += red[2][lane][v].y;
                    s.x += red[3][lane][v].x; s.y += red[3][lane][v].y;
                    a.P[((size_t)slot_t * NV + v) * a.ldp + j] = s;
                }
            }
        }
        __syncthreads();
    }
}

template <int NV, int RW, int GEN, int SRC>
__global__ __launch_bounds__(256) void tile_apply_kernel(TileArgs a)
{
    __shared__ float2 red[4][64][NV];
    __shared__ float2 xs[4 * RW][NV];
    const int2 st = a.st_list[blockIdx.x];
    super_tile<NV, RW, GEN, SRC>(a, st.x, st.y, red, xs);
}

// Single-vector products of a fully cached operator (tile shape 0, 256-wide
// super-tiles), one tile of prefetch.
template <int RW, int GEN, int PF>
__global__ __launch_bounds__(256, 3) void tile_apply_cached_kernel(TileArgs a)
{
    __shared__ float2 red[4][64][1];
    __shared__ float2 xs[2][4 * RW][1];
    const int2 st = a.st_list[blockIdx.x];
    super_tile_cached<1, RW, GEN, PF>(a, st.x, st.y, red, xs);
}

// Batched persistent form: every workgroup walks the flattened list of
// (instance, super-tile) items with a fixed stride; items are listed in an
// order that keeps neighbouring workgroups on comparable work.
template <int NV, int RW, int GEN, int SRC>
__global__ __launch_bounds__(256) void tile_apply_batched_kernel(
    const TileArgs* __restrict__ ops, const int4* __restrict__ items,
    int64_t n_items, const float2* xbase)
{
    __shared__ float2 red[4][64][NV];
    __shared__ float2 xs[4 * RW][NV];
    for (int64_t q = blockIdx.x; q < n_items; q += gridDim.x) {
        const int4 it = items[q];          // (instance, sr, sc, unused)
        TileArgs a = ops[it.x];
        a.X = xbase + a.xoff;
        super_tile<NV, RW, GEN, SRC>(a, it.y, it.z, red, xs);
    }
}

template <Epi MODE>
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a)
{
    // 64 elements per workgroup, 4 groups of slots per element; the group
    // sums are combined in a fixed order.
    __shared__ float2 part[4][64];
    const int g = threadIdx.x >> 6;
    const int64_t t = (int64_t)reduce_row_block(a, blockIdx.x) * 64 + (threadIdx.x & 63);
    const int64_t total = (int64_t)a.nv * a.D;
    const bool live = t < total;
    const int v = live ? (int)(t / a.D) : 0;
    const int i = live ? (int)(t - (int64_t)v * a.D) : 0;
    float sx = 0.f, sy = 0.f;
    if (live) {
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
    part[g][threadIdx.x & 63] = make_float2(sx, sy);
    __syncthreads();
    if (g != 0 || !live) return;
    {
        const int l = threadIdx.x & 63;
        sx = part[0][l].x; sy = part[0][l].y;
        sx += part[1][l].x; sy += part[1][l].y;
        sx += part[2][l].x; sy += part[2][l].y;
        sx += part[3][l].x; sy += part[3][l].y;
    }
    reduce_epilogue<MODE>(a, v, i, sx, sy);
}

template <int GEN>
__global__ void cache_fill_kernel(SourceArgs s, int32_t D, const int2* pairs,
                                  int64_t n_pairs, void* slots)
{
    const int64_t bb = (int64_t)s.b * s.b;
    const int64_t total = n_pairs * bb;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = t / bb;
        const int64_t e = t - p * bb;
        const int ii = (int)(e / s.b), jj = (int)(e - (int64_t)ii * s.b);
        const int2 nm = pairs[p];
        const int64_t i = (int64_t)nm.x * s.b + ii, j = (int64_t)nm.y * s.b + jj;
        const bool in = i < D && j < D;
        if (GEN == 0) {
            float2 h = in ? gue_entry(s.gue, (uint32_t)i, (uint32_t)j) : make_float2(0.f, 0.f);
            ((float2*)slots)[t] = h;
        } else {
            float h = in ? dvr_entry(s.dvr, (uint32_t)i, (uint32_t)j) : 0.f;
            ((float*)slots)[t] = h;
        }
    }
}

template <int GEN>
__global__ void get_entries_kernel(SourceArgs s, int64_t r0, int64_t c0,
                                   int32_t nr, int32_t nc, float2* out)
{
    const int64_t total = (int64_t)nr * nc;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = t / nc, b = t - a * nc;
        const uint32_t i = (uint32_t)(r0 + a), j = (uint32_t)(c0 + b);
        if (GEN == 0) out[t] = gue_entry(s.gue, i, j);
        else out[t] = make_float2(dvr_entry(s.dvr, i, j), 0.f);
    }
}

template <int NV, int RW>
hipError_t launch_nv(const TileArgs& a, int n_st, hipStream_t s)
{
    const bool cached = a.src.pair_slot != nullptr;
    const dim3 g(n_st), b(256);
    if constexpr (NV == 1 && RW == 8) {
        // single vector, fully cached, tile shape 0, 256-wide super-tiles:
        // pipelined reads
        if (cached && a.src.all_cached && a.se == kSuper / 64) {
            if (a.src.gen == 0)
                hipLaunchKernelGGL((tile_apply_cached_kernel<RW, 0, 1>), g, b, 0, s, a);
            else
                hipLaunchKernelGGL((tile_apply_cached_kernel<RW, 1, 1>), g, b, 0, s, a);
            return hipGetLastError();
        }
    }
    if (a.src.gen == 0) {
        if (cached) hipLaunchKernelGGL((tile_apply_kernel<NV, RW, 0, 1>), g, b, 0, s, a);
        else hipLaunchKernelGGL((tile_apply_kernel<NV, RW, 0, 0>), g, b, 0, s, a);
    } else {
        if (cached) hipLaunchKernelGGL((tile_apply_kernel<NV, RW, 1, 1>), g, b, 0, s, a);
        else hipLaunchKernelGGL((tile_apply_kernel<NV, RW, 1, 0>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

template <int NV, int RW>
hipError_t launch_nv_batched(const BatchTileLaunch& b, hipStream_t s)
{
    const dim3 g(b.grid), t(256);
    if (b.gen == 0) {
        if (b.cached)
            hipLaunchKernelGGL((tile_apply_batched_kernel<NV, RW, 0, 1>), g, t, 0, s, b.ops,
                               b.items, b.n_items, b.xbase);
        else
            hipLaunchKernelGGL((tile_apply_batched_kernel<NV, RW, 0, 0>), g, t, 0, s, b.ops,
                               b.items, b.n_items, b.xbase);
    } else {
        if (b.cached)
            hipLaunchKernelGGL((tile_apply_batched_kernel<NV, RW, 1, 1>), g, t, 0, s, b.ops,
                               b.items, b.n_items, b.xbase);
        else
            hipLaunchKernelGGL((tile_apply_batched_kernel<NV, RW, 1, 0>), g, t, 0, s, b.ops,
                               b.items, b.n_items, b.xbase);
    }
    return hipGetLastError();
}

}  // namespace

// Tile shapes: rows per wave RW = (8, 16, 32) / (2 NV) for shape 0, 1, 2.
hipError_t launch_tile_apply(const TileArgs& a, int nv, int shape, int n_st, hipStream_t s)
{
    shape = fit_tile_shape(nv, shape, a.se, a.src.pair_slot ? a.src.b : 0);
#define PROCMV_SHAPES(NV, R0, R1, R2)                                  \
    if (shape == 0) return launch_nv<NV, R0>(a, n_st, s);              \
    if (shape == 1) return launch_nv<NV, R1>(a, n_st, s);              \
    if (shape == 2) return launch_nv<NV, R2>(a, n_st, s);              \
    return hipErrorInvalidValue;
    switch (nv) {
    case 1: PROCMV_SHAPES(1, 8, 16, 32)
    case 2: PROCMV_SHAPES(2, 4, 8, 16)
    case 4: PROCMV_SHAPES(4, 2, 4, 8)
    case 8: PROCMV_SHAPES(8, 1, 2, 4)
    default: return hipErrorInvalidValue;
    }
#undef PROCMV_SHAPES
}

hipError_t launch_tile_apply_batched(const BatchTileLaunch& b0, hipStream_t s)
{
    BatchTileLaunch b = b0;
    b.shape = fit_tile_shape(b.nv, b.shape, b.min_se, b.cached ? b.cache_b : 0);
#define PROCMV_SHAPES(NV, R0, R1, R2)                                  \
    if (b.shape == 0) return launch_nv_batched<NV, R0>(b, s);          \
    if (b.shape == 1) return launch_nv_batched<NV, R1>(b, s);          \
    if (b.shape == 2) return launch_nv_batched<NV, R2>(b, s);          \
    return hipErrorInvalidValue;
    switch (b.nv) {
    case 1: PROCMV_SHAPES(1, 8, 16, 32)
    case 2: PROCMV_SHAPES(2, 4, 8, 16)
    case 4: PROCMV_SHAPES(4, 2, 4, 8)
    case 8: PROCMV_SHAPES(8, 1, 2, 4)
    default: return hipErrorInvalidValue;
    }
#undef PROCMV_SHAPES
}

hipError_t launch_reduce(const ReduceArgs& a, Epi mode, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1)
{
    const int64_t total = (int64_t)a.nv * a.D;
    const dim3 grid((unsigned)((total + 63) / 64)), blk(256);
#define PROCMV_RED(M)                                                                   \
    if (e0) hipExtLaunchKernelGGL(reduce_kernel<M>, grid, blk, 0, s, e0, e1, 0, a);     \
    else hipLaunchKernelGGL(reduce_kernel<M>, grid, blk, 0, s, a);
    switch (mode) {
    case Epi::kApply: PROCMV_RED(Epi::kApply) break;
    case Epi::kChebFirst: PROCMV_RED(Epi::kChebFirst) break;
    case Epi::kChebStep: PROCMV_RED(Epi::kChebStep) break;
    }
#undef PROCMV_RED
    return hipGetLastError();
}

hipError_t launch_cache_fill(const SourceArgs& src, int32_t D, const int2* pairs,
                             int64_t n_pairs, void* slots, hipStream_t s)
{
    const int64_t total = n_pairs * (int64_t)src.b * src.b;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (src.gen == 0)
        hipLaunchKernelGGL(cache_fill_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, s,
                           src, D, pairs, n_pairs, slots);
    else
        hipLaunchKernelGGL(cache_fill_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s,
                           src, D, pairs, n_pairs, slots);
    return hipGetLastError();
}

hipError_t launch_get_entries(const SourceArgs& src, int64_t r0, int64_t c0,
                              int32_t nr, int32_t nc, float2* out, hipStream_t s)
{
    const int64_t total = (int64_t)nr * nc;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (src.gen == 0)
        hipLaunchKernelGGL(get_entries_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, s,
                           src, r0, c0, nr, nc, out);
    else
        hipLaunchKernelGGL(get_entries_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s,
                           src, r0, c0, nr, nc, out);
    return hipGetLastError();
}

}  // namespace procmv
