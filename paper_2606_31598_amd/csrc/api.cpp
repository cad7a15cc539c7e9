// C ABI of libprocmv.so: operators, plans, products and propagation.
// The paper passages each call implements are cited in include/procmv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/procmv.h"
#include "kernels.h"

using namespace procmv;

namespace {

thread_local std::string g_err;

procmv_status fail(procmv_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                        \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess)                                                \
            return fail(e_ == hipErrorOutOfMemory ? PROCMV_ERR_OOM           \
                                                  : PROCMV_ERR_HIP,          \
                        "%s: %s", #expr, hipGetErrorString(e_));             \
    } while (0)

template <class T>
void dfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

}  // namespace

struct procmv_op {
    int gen = 0;
    uint64_t seed = 0;
    int64_t D = 0;
    procmv_dvr_params dvr{};
    // Philox-GUE scales (binary32, rounded once from binary64)
    float s_off = 0.f, s_diag = 0.f;
    // sinc-DVR: device tables and binary64 constants
    float* d_tk = nullptr;
    float* d_v = nullptr;
    float* d_text = nullptr;  // symmetric symbol t(k), k in (-D, D), zero at 0
    double d_const = 0.0;   // constant diagonal paired with the binary32 tables
    double dx = 0.0, vmax = 0.0;
    std::vector<float> h_tk, h_v;   // host copies of the binary32 tables
    // compensated arithmetic (precision PROCMV_FP32_COMPENSATED, sinc-DVR):
    // the tile kernels read tables without the band |i - j| < near_w, the
    // reduction adds the band in difference form and C_i x_i
    int32_t near_w = 0;
    float* d_text_far = nullptr;
    float* d_tk_far = nullptr;
    float* d_vzero = nullptr;
    float2* d_cv = nullptr;   // C_i = d + sum_{0<|k|<W, 0<=i+k<D} tk[|k|] + v_i as (hi, lo)
    float2* d_qlo = nullptr;  // lo parts of the two recurrence vectors
    size_t qlo_bytes = 0;
    // plan
    bool planned = false;
    int32_t b = 0, n_blk = 0;
    int strategy = 0, precision = 0;
    int tile_shape = -1;      // VALU tile shape (see launch_tile_apply); -1 = per class
    int dvr_kernel = 0;       // procedural sinc-DVR product: 0 auto, 1 VALU, 2 binary32
                              // matrix cores, 3 split-bf16 matrix cores
    double frac = 0.0;
    int64_t n_pair = 0, p_cache = 0;
    int32_t* d_pair_slot = nullptr;
    void* d_slots = nullptr;
    int2* d_pairs = nullptr;
    int32_t se = 4;             // super-tile edge in 64-column tiles
    int32_t n_super = 0;
    int64_t n_st = 0;
    int2* d_st = nullptr;       // cached super-tiles, then generated, then mixed
    int64_t n_st_cached = 0;    // super-tiles whose canonical pairs are all cached
    int64_t n_st_gen = 0;       // super-tiles with no cached pair
    // workspace
    float2* d_P = nullptr;
    size_t P_bytes = 0;
    float2* d_q = nullptr;
    size_t q_bytes = 0;
    double2* d_acc = nullptr;
    size_t acc_bytes = 0;
    double* d_norm = nullptr;
    size_t norm_bytes = 0;
    float2* d_kz = nullptr;     // Kronecker bath products (1 + n_int) x d_S x D
    size_t kz_bytes = 0;
    float2* d_kq = nullptr;     // Kronecker Chebyshev: q buffer and product (2 x d_S x D)
    size_t kq_bytes = 0;
    double2* d_kacc = nullptr;  // Kronecker Chebyshev accumulator (d_S x D) + norm
    size_t kacc_bytes = 0;
    float2* d_lz = nullptr;     // Lanczos vectors v_prev, v, w (D each)
    size_t lz_bytes = 0;
    double* d_lzs = nullptr;    // Lanczos partials (2 x kLanczosMaxBlocks), alpha, beta
    size_t lzs_bytes = 0;
    // measurement: event pairs around sampled launches
    int32_t prof_every = 0;
    int64_t prof_count[2] = {0, 0};
    std::vector<hipEvent_t> prof_ev[2];   // start, stop interleaved
    size_t prof_used[2] = {0, 0};

    size_t slot_elem() const { return gen == 0 ? sizeof(float2) : sizeof(float); }

    bool comp() const { return gen == 1 && precision == PROCMV_FP32_COMPENSATED; }

    // Block source of the products; `exact` = the operator's own entries
    // (the compensated products read the tables without the band).
    SourceArgs source(bool exact = false) const
    {
        SourceArgs s{};
        s.gen = gen;
        s.gue.k0 = (uint32_t)seed;
        s.gue.k1 = (uint32_t)(seed >> 32);
        s.gue.s_off = s_off;
        s.gue.s_diag = s_diag;
        s.dvr.tk = (comp() && !exact) ? d_tk_far : d_tk;
        s.dvr.v = (comp() && !exact) ? d_vzero : d_v;
        s.pair_slot = (planned && p_cache > 0) ? d_pair_slot : nullptr;
        s.slots = d_slots;
        s.b = b;
        s.n_blk = n_blk;
        s.all_cached = (planned && p_cache > 0 && p_cache == n_pair) ? 1 : 0;
        return s;
    }

    void release_plan()
    {
        dfree(d_pair_slot);
        dfree(d_slots);
        dfree(d_pairs);
        dfree(d_st);
        planned = false;
        p_cache = 0;
    }

    ~procmv_op()
    {
        release_plan();
        dfree(d_tk);
        dfree(d_v);
        dfree(d_text);
        dfree(d_text_far);
        dfree(d_tk_far);
        dfree(d_vzero);
        dfree(d_cv);
        dfree(d_qlo);
        dfree(d_P);
        dfree(d_q);
        dfree(d_acc);
        dfree(d_norm);
        dfree(d_lz);
        dfree(d_kz);
        dfree(d_kq);
        dfree(d_kacc);
        dfree(d_lzs);
        for (int k = 0; k < 2; ++k)
            for (hipEvent_t e : prof_ev[k]) (void)hipEventDestroy(e);
    }

    // Event pair for launch number prof_count[kind] if it is sampled.
    bool prof_pair(int kind, hipEvent_t& a, hipEvent_t& b)
    {
        if (prof_every <= 0) return false;
        const int64_t n = prof_count[kind]++;
        if (n % prof_every != 0) return false;
        std::vector<hipEvent_t>& ev = prof_ev[kind];
        if (prof_used[kind] + 2 > ev.size()) {
            hipEvent_t e0, e1;
            if (hipEventCreate(&e0) != hipSuccess) return false;
            if (hipEventCreate(&e1) != hipSuccess) {
                (void)hipEventDestroy(e0);
                return false;
            }
            ev.push_back(e0);
            ev.push_back(e1);
        }
        a = ev[prof_used[kind]];
        b = ev[prof_used[kind] + 1];
        prof_used[kind] += 2;
        return true;
    }
};

namespace {

// Grow a device buffer to at least `bytes`.
template <class T>
procmv_status ensure(T*& p, size_t& have, size_t bytes)
{
    if (have >= bytes) return PROCMV_OK;
    dfree(p);
    have = 0;
    HIP_TRY(hipMalloc((void**)&p, bytes));
    have = bytes;
    return PROCMV_OK;
}

// hi + lo binary32 pair of a binary64 value.
void split_f32(double v, float& hi, float& lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

// Largest binary32 value not above x (x > 0).
float f32_down(double x)
{
    float f = (float)x;
    if ((double)f > x) f = std::nextafter(f, 0.0f);
    return f;
}

// J_0(x) .. J_kmax(x), x >= 0, Miller's backward recurrence normalised by
// J_0 + 2 sum J_2k = 1.
std::vector<double> bessel_j(double x, int kmax)
{
    std::vector<double> out(kmax + 1, 0.0);
    if (x == 0.0) {
        out[0] = 1.0;
        return out;
    }
    const int top = (int)std::max((double)kmax, x) + 30 +
                    (int)(20.0 * std::cbrt(std::max(x, 1.0)));
    std::vector<double> j(top + 2, 0.0);
    j[top] = 1e-300;
    for (int k = top; k > 0; --k) {
        j[k - 1] = (2.0 * k / x) * j[k] - j[k + 1];
        if (std::fabs(j[k - 1]) > 1e250)
            for (int q = k - 1; q <= top; ++q) j[q] *= 1e-250;
    }
    double norm = j[0];
    for (int k = 2; k <= top; k += 2) norm += 2.0 * j[k];
    for (int k = 0; k <= kmax; ++k) out[k] = j[k] / norm;
    return out;
}

procmv_status check_op(procmv_op_t H)
{
    if (!H) return fail(PROCMV_ERR_INVALID_ARG, "null operator handle");
    return PROCMV_OK;
}

procmv_status upload_dvr(procmv_op* op)
{
    const int64_t D = op->D;
    const double dx = (op->dvr.x_max - op->dvr.x_min) / (double)(D - 1);
    const double inv_mdx2 = 1.0 / (op->dvr.mass * dx * dx);
    const double kpot = 0.5 * op->dvr.mass * op->dvr.omega * op->dvr.omega;
    std::vector<float> tk(D, 0.f), v(D, 0.f);
    double err = 0.0, vmax = 0.0;
    for (int64_t k = 1; k < D; ++k) {
        const double t = ((k & 1) ? -inv_mdx2 : inv_mdx2) / ((double)k * (double)k);
        tk[k] = (float)t;
        err += (double)tk[k] - t;
    }
    for (int64_t i = 0; i < D; ++i) {
        const double x = op->dvr.x_min + (double)i * dx;
        const double vv = kpot * (x * x);
        v[i] = (float)vv;
        vmax = std::max(vmax, vv);
    }
    const double d0 = (M_PI * M_PI / 6.0) * inv_mdx2;
    op->d_const = op->dvr.compensate ? d0 - 2.0 * err : d0;
    op->dx = dx;
    op->vmax = vmax;
    op->h_tk = tk;
    op->h_v = v;
    std::vector<float> text(2 * D - 1, 0.f);
    for (int64_t k = 1; k < D; ++k) text[D - 1 + k] = text[D - 1 - k] = tk[k];
    HIP_TRY(hipMalloc((void**)&op->d_text, (2 * D - 1) * sizeof(float)));
    HIP_TRY(hipMemcpy(op->d_text, text.data(), (2 * D - 1) * sizeof(float),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc((void**)&op->d_tk, D * sizeof(float)));
    HIP_TRY(hipMalloc((void**)&op->d_v, D * sizeof(float)));
    HIP_TRY(hipMemcpy(op->d_tk, tk.data(), D * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(op->d_v, v.data(), D * sizeof(float), hipMemcpyHostToDevice));
    return PROCMV_OK;
}

// Tables of the compensated arithmetic: symbol windows without the band
// 0 < |k| < W, a zero site potential for the tile kernels, and the per-row
// constant C_i = d + sum_{0<|k|<W, 0<=i+k<D} tk[|k|] + v_i (binary64 sum of
// the binary32 entries, stored as a hi + lo pair), so that
// (H x)_i = far_i + sum_band tk (x_j - x_i) + C_i x_i exactly.
procmv_status upload_comp(procmv_op* op)
{
    if (op->d_cv) return PROCMV_OK;
    const int64_t D = op->D;
    const int32_t W = (int32_t)std::min<int64_t>(kNearBand, D);
    std::vector<float> text(2 * D - 1, 0.f), tkf(D, 0.f);
    for (int64_t k = W; k < D; ++k) {
        text[D - 1 + k] = text[D - 1 - k] = op->h_tk[k];
        tkf[k] = op->h_tk[k];
    }
    std::vector<float2> cv(D);
    for (int64_t i = 0; i < D; ++i) {
        double c = op->d_const + (double)op->h_v[i];
        for (int32_t k = 1; k < W; ++k) {
            if (i - k >= 0) c += (double)op->h_tk[k];
            if (i + k < D) c += (double)op->h_tk[k];
        }
        float hi, lo;
        split_f32(c, hi, lo);
        cv[i] = make_float2(hi, lo);
    }
    const std::vector<float> zero(D, 0.f);
    HIP_TRY(hipMalloc((void**)&op->d_text_far, (2 * D - 1) * sizeof(float)));
    HIP_TRY(hipMalloc((void**)&op->d_tk_far, D * sizeof(float)));
    HIP_TRY(hipMalloc((void**)&op->d_vzero, D * sizeof(float)));
    HIP_TRY(hipMalloc((void**)&op->d_cv, D * sizeof(float2)));
    HIP_TRY(hipMemcpy(op->d_text_far, text.data(), (2 * D - 1) * sizeof(float),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(op->d_tk_far, tkf.data(), D * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(op->d_vzero, zero.data(), D * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(op->d_cv, cv.data(), D * sizeof(float2), hipMemcpyHostToDevice));
    op->near_w = W;
    return PROCMV_OK;
}

// The compensated reduction's operands (null cv = plain reduction).
void comp_fields(const procmv_op* op, ReduceArgs& r)
{
    if (!op->comp()) return;
    r.cv = op->d_cv;
    r.tk = op->d_tk;
    r.W = op->near_w;
}

// What the reduction of a tile product must add up.
struct TileOut {
    int32_t n_slots = 0;
    int32_t nv_stride = 0;
    const float* vdiag = nullptr;
    float2* P = nullptr;      // partial slots written by the tile kernels
    int32_t xcd_groups = 0;   // split-bf16 row groups pinned to XCDs (see ReduceArgs)
};

// Caller-provided partial buffer (the allocation-free product); null = the
// operator's own, grown on demand.
struct Scratch {
    float2* p = nullptr;
    size_t bytes = 0;
};

// Whether a block of `remaining` vectors goes to the matrix cores: always in
// split-bf16 precision, and in binary32 once there are enough vectors for the
// per-tile product to be a contraction worth a GEMM.
// Matrix-core path for vector blocks (measured on MI355X, D = 32768): always
// in split-bf16 precision; in binary32 for blocks of 8 or more vectors, and
// for 4 to 7 vectors when every canonical pair is cached (the VALU tile
// kernel generates faster up to 4 vectors: 2.0 against 3.1 ms for 4 GUE
// vectors, but streams a full cache slower: 3.1 against 2.0 ms).  The
// procedural sinc-DVR operator always takes the Toeplitz kernel (up to 8
// vectors per launch), 5-10 times faster than either.
bool mfma_path(int gen, bool procedural, bool all_cached, int precision, int nv)
{
    if (precision == PROCMV_SPLIT_BF16) return true;
    if (gen == 1 && procedural) return false;
    return nv >= 8 || (nv >= 4 && all_cached);
}

bool use_mfma(const procmv_op* op, int remaining)
{
    return mfma_path(op->gen, op->p_cache == 0, op->p_cache == op->n_pair, op->precision,
                     remaining);
}

// Vectors handled by one tile launch.
int chunk_vectors(const procmv_op* op, int remaining)
{
    if (use_mfma(op, remaining)) return remaining >= 16 ? 16 : remaining;
    return remaining >= 8 ? 8 : remaining >= 4 ? 4 : remaining >= 2 ? 2 : 1;
}

// Block product of one chunk of nv vectors into the partial buffer: the
// Toeplitz kernel for a procedural sinc-DVR operator in binary32 with few
// vectors, the MFMA kernel for vector blocks on the matrix cores, the generic
// two-sided VALU tile kernel otherwise.
procmv_status run_tiles(procmv_op* op, const float2* X, int64_t ldx, int nv,
                        hipStream_t s, TileOut& out, const Scratch& scr = Scratch{})
{
    const size_t ldp = (size_t)op->D;
    const bool mfma = use_mfma(op, nv);
    const bool toeplitz = !mfma && op->gen == 1 && op->p_cache == 0;
    // one vector of a large operator: the Toeplitz blocks on the matrix cores
    const bool tmfma = toeplitz && nv == 1 && op->dvr_kernel == 2;
    const bool tbf16 = toeplitz && nv == 1 &&
                       (op->dvr_kernel == 3 || (op->dvr_kernel == 0 && op->D >= kDvrMfmaMinD));
    const int variant = toeplitz ? dvr_toeplitz_variant((int32_t)op->D, nv) : 0;
    const int chunk = toeplitz ? dvr_toeplitz_chunk_of(variant) : 1;
    out.n_slots = tbf16 ? dvr_bf16_chunks((int32_t)op->D)
                : tmfma ? dvr_mfma_chunks((int32_t)op->D)
                : toeplitz ? (int32_t)((op->D + chunk - 1) / chunk) : op->n_super + 1;
    out.vdiag = (toeplitz && !op->comp()) ? op->d_v : nullptr;
    out.nv_stride = nv;
    const size_t need = (size_t)out.n_slots * out.nv_stride * ldp * sizeof(float2);
    if (scr.p) {
        if (need > scr.bytes)
            return fail(PROCMV_ERR_INVALID_ARG,
                        "partial slots need %zu bytes, above the %zu-byte static workspace",
                        need, scr.bytes);
        out.P = scr.p;
    } else {
        procmv_status st = ensure(op->d_P, op->P_bytes, need);
        if (st != PROCMV_OK) return st;
        out.P = op->d_P;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    // no timing events on the allocation-free path (it creates nothing)
    const bool timed = !scr.p && op->prof_pair(0, e0, e1);
    if (timed && !toeplitz) HIP_TRY(hipEventRecord(e0, s));
    if (toeplitz) {
        DvrToeplitzArgs a{};
        a.D = (int32_t)op->D;
        a.text = op->comp() ? op->d_text_far : op->d_text;
        a.X = X;
        a.ldx = ldx;
        a.P = out.P;
        a.ldp = (int64_t)ldp;
        if (tbf16) {
            HIP_TRY(launch_dvr_toeplitz_bf16(a, s, timed ? e0 : nullptr, e1));
            // 2048-row groups, a multiple of 8 of them: every chunk of group g
            // is workgroup g + groups c, on XCD g mod 8
            const int64_t groups = op->D / 2048;
            if (op->D % 2048 == 0 && groups % 8 == 0)
                out.xcd_groups = (int32_t)groups;
        }
        else if (tmfma)
            HIP_TRY(launch_dvr_toeplitz_mfma(a, s, timed ? e0 : nullptr, e1));
        else
            HIP_TRY(launch_dvr_toeplitz(a, nv, variant, s, timed ? e0 : nullptr, e1));
    } else {
        TileArgs a{};
        a.src = op->source();
        a.D = (int32_t)op->D;
        a.se = op->se;
        a.n_super = op->n_super;
        a.nv = nv;
        a.st_list = op->d_st;
        a.X = X;
        a.ldx = ldx;
        a.P = out.P;
        a.ldp = (int64_t)ldp;
        if (mfma) {
            HIP_TRY(launch_tile_mfma(a, op->precision == PROCMV_SPLIT_BF16 ? 1 : 0,
                                     (int)op->n_st, s));
        } else {
            // one launch per super-tile class (the cached class streams on
            // the pipelined kernel); default tile shape 0 for every class
            const int64_t n_c = op->n_st_cached, n_g = op->n_st_gen;
            const int64_t n_m = op->n_st - n_c - n_g;
            const SourceArgs src = a.src;
            if (n_c > 0) {
                a.src.all_cached = 1;
                HIP_TRY(launch_tile_apply(a, nv, op->tile_shape >= 0 ? op->tile_shape : 0,
                                          (int)n_c, s));
            }
            if (n_g > 0) {
                a.src = src;
                a.src.pair_slot = nullptr;
                a.src.all_cached = 0;
                a.st_list = op->d_st + n_c;
                HIP_TRY(launch_tile_apply(a, nv, op->tile_shape >= 0 ? op->tile_shape : 0,
                                          (int)n_g, s));
            }
            if (n_m > 0) {
                a.src = src;
                a.src.all_cached = 0;
                a.st_list = op->d_st + n_c + n_g;
                HIP_TRY(launch_tile_apply(a, nv, op->tile_shape >= 0 ? op->tile_shape : 0,
                                          (int)n_m, s));
            }
        }
    }
    if (timed && !toeplitz) HIP_TRY(hipEventRecord(e1, s));
    return PROCMV_OK;
}

procmv_status run_reduce(procmv_op* op, const ReduceArgs& r, Epi mode,
                         hipStream_t s, bool untimed = false)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = !untimed && op->prof_pair(1, e0, e1);
    if (r.cv)
        HIP_TRY(launch_reduce_comp(r, mode, s, timed ? e0 : nullptr, e1));
    else
        HIP_TRY(launch_reduce(r, mode, s, timed ? e0 : nullptr, e1));
    return PROCMV_OK;
}

ReduceArgs reduce_args(procmv_op* op, int nv, const TileOut& t)
{
    ReduceArgs r{};
    r.D = (int32_t)op->D;
    r.nv = nv;
    r.n_slots = t.n_slots;
    r.nv_stride = t.nv_stride;
    r.vdiag = t.vdiag;
    r.P = t.P;
    r.ldp = op->D;
    r.alpha = 1.0f;
    return r;
}

// One product H X of a vector block, reduced with the epilogue `mode`: tile
// kernel, then the fixed-order reduction.  r carries the epilogue operands
// (X, Y, acc, alpha, beta, coefficients); the partial-buffer fields are
// filled here.
procmv_status run_product(procmv_op* op, const float2* X, int64_t ldx, int nv, ReduceArgs r,
                          Epi mode, hipStream_t s, const Scratch& scr = Scratch{})
{
    TileOut to;
    procmv_status st = run_tiles(op, X, ldx, nv, s, to, scr);
    if (st != PROCMV_OK) return st;
    ReduceArgs base = reduce_args(op, nv, to);
    r.D = base.D;
    r.nv = base.nv;
    r.nv_stride = base.nv_stride;
    r.n_slots = base.n_slots;
    r.P = base.P;
    r.ldp = base.ldp;
    r.vdiag = base.vdiag;
    r.xcd_groups = to.xcd_groups;
    r.X = X;
    r.ldx = ldx;
    return run_reduce(op, r, mode, s, scr.p != nullptr);
}



}  // namespace

extern "C" {

const char* procmv_last_error(void) { return g_err.c_str(); }

procmv_status procmv_create_operator(procmv_generator gen, uint64_t seed,
                                     int64_t D, const void* gen_params,
                                     procmv_op_t* out)
{
    if (!out) return fail(PROCMV_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (gen != PROCMV_GEN_PHILOX_GUE && gen != PROCMV_GEN_SINC_DVR)
        return fail(PROCMV_ERR_INVALID_ARG, "unknown generator %d", (int)gen);
    if (D < 1 || D >= (int64_t(1) << 31))
        return fail(PROCMV_ERR_INVALID_ARG, "D = %lld outside [1, 2^31)", (long long)D);
    if (gen == PROCMV_GEN_SINC_DVR && D < 2)
        return fail(PROCMV_ERR_INVALID_ARG, "sinc-DVR needs D >= 2");
    procmv_op* op = new procmv_op();
    op->gen = (int)gen;
    op->seed = seed;
    op->D = D;
    if (gen == PROCMV_GEN_PHILOX_GUE) {
        op->s_off = (float)std::sqrt(1.0 / (2.0 * (double)D));
        op->s_diag = (float)std::sqrt(1.0 / (double)D);
    } else {
        if (gen_params) op->dvr = *(const procmv_dvr_params*)gen_params;
        else op->dvr = procmv_dvr_params{-20.0, 20.0, 1.0, 1.0, 1};
        if (!(op->dvr.x_max > op->dvr.x_min) || !(op->dvr.mass > 0)) {
            delete op;
            return fail(PROCMV_ERR_INVALID_ARG, "bad DVR parameters");
        }
        procmv_status st = upload_dvr(op);
        if (st != PROCMV_OK) {
            delete op;
            return st;
        }
    }
    *out = op;
    return PROCMV_OK;
}

void procmv_destroy(procmv_op_t H) { delete H; }

procmv_status procmv_plan(procmv_op_t H, int32_t block_size,
                          procmv_strategy strategy, double cache_fraction,
                          procmv_precision precision, void* stream)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (block_size < 64 || block_size % 64 != 0)
        return fail(PROCMV_ERR_INVALID_ARG, "block size %d: need a multiple of 64", block_size);
    if (strategy < PROCMV_PROCEDURAL || strategy > PROCMV_FULL)
        return fail(PROCMV_ERR_INVALID_ARG, "unknown strategy %d", (int)strategy);
    if (strategy == PROCMV_PARTIAL && !(cache_fraction >= 0.0 && cache_fraction <= 1.0))
        return fail(PROCMV_ERR_INVALID_ARG, "cache fraction %g outside [0, 1]", cache_fraction);
    if (precision != PROCMV_FP32 && precision != PROCMV_SPLIT_BF16 &&
        precision != PROCMV_FP32_COMPENSATED)
        return fail(PROCMV_ERR_INVALID_ARG, "unknown precision %d", (int)precision);
    if (precision == PROCMV_FP32_COMPENSATED && H->gen != PROCMV_GEN_SINC_DVR)
        return fail(PROCMV_ERR_INVALID_ARG,
                    "compensated arithmetic is defined for the sinc-DVR operator");
    hipStream_t s = (hipStream_t)stream;
    H->release_plan();
    if (precision == PROCMV_FP32_COMPENSATED) {
        st = upload_comp(H);
        if (st != PROCMV_OK) return st;
    }
    const int64_t D = H->D;
    H->b = block_size;
    H->n_blk = (int32_t)((D + block_size - 1) / block_size);
    H->strategy = (int)strategy;
    H->precision = (int)precision;
    H->frac = strategy == PROCMV_FULL ? 1.0 : strategy == PROCMV_PARTIAL ? cache_fraction : 0.0;
    const int64_t nb = H->n_blk;
    H->n_pair = nb * (nb + 1) / 2;
    // canonical pairs in row-major order; pair q is cached when
    // floor((q + 1) f) > floor(q f), which spreads the cached fraction evenly
    std::vector<int32_t> slot(nb * nb, -1);
    std::vector<int2> pairs;
    int64_t q = 0;
    for (int64_t n = 0; n < nb; ++n)
        for (int64_t m = n; m < nb; ++m, ++q) {
            bool take = false;
            if (strategy == PROCMV_FULL) take = true;
            else if (strategy == PROCMV_PARTIAL)
                take = std::floor((double)(q + 1) * H->frac) > std::floor((double)q * H->frac);
            if (take) {
                slot[n * nb + m] = (int32_t)pairs.size();
                pairs.push_back(make_int2((int)n, (int)m));
            }
        }
    H->p_cache = (int64_t)pairs.size();
    // VALU tile shape: per super-tile class unless set (procmv_autotune and
    // procmv_set_tile_shape override it)
    H->tile_shape = -1;
    // super-tile list, grouped by how its canonical pairs are stored: all
    // cached, none cached, or mixed (only when b < the super-tile edge)
    H->se = super_edge_tiles(D);
    const int64_t E = 64 * H->se;
    H->n_super = (int32_t)((D + E - 1) / E);
    std::vector<int2> st_cached, st_gen, st_mixed;
    for (int r = 0; r < H->n_super; ++r)
        for (int c = r; c < H->n_super; ++c) {
            const int64_t n_lo = (int64_t)r * E / block_size;
            const int64_t n_hi = (std::min<int64_t>(D, (int64_t)(r + 1) * E) - 1) / block_size;
            const int64_t m_lo = (int64_t)c * E / block_size;
            const int64_t m_hi = (std::min<int64_t>(D, (int64_t)(c + 1) * E) - 1) / block_size;
            int64_t n_cached = 0, n_canon = 0;
            for (int64_t n = n_lo; n <= n_hi; ++n)
                for (int64_t m = std::max(m_lo, n); m <= m_hi; ++m) {
                    ++n_canon;
                    n_cached += slot[n * nb + m] >= 0;
                }
            const int2 t = make_int2(r, c);
            if (n_cached == n_canon) st_cached.push_back(t);
            else if (n_cached == 0) st_gen.push_back(t);
            else st_mixed.push_back(t);
        }
    H->n_st_cached = (int64_t)st_cached.size();
    H->n_st_gen = (int64_t)st_gen.size();
    std::vector<int2> sts(st_cached);
    sts.insert(sts.end(), st_gen.begin(), st_gen.end());
    sts.insert(sts.end(), st_mixed.begin(), st_mixed.end());
    H->n_st = (int64_t)sts.size();
    HIP_TRY(hipMalloc((void**)&H->d_st, sts.size() * sizeof(int2)));
    HIP_TRY(hipMemcpy(H->d_st, sts.data(), sts.size() * sizeof(int2), hipMemcpyHostToDevice));
    if (H->p_cache > 0) {
        const size_t bytes = (size_t)H->p_cache * block_size * block_size * H->slot_elem();
        hipError_t e = hipMalloc(&H->d_slots, bytes);
        if (e != hipSuccess) {
            H->d_slots = nullptr;
            H->release_plan();
            (void)hipGetLastError();
            return fail(PROCMV_ERR_OOM, "cache of %lld pairs (%zu bytes) does not fit: %s",
                        (long long)H->p_cache, bytes, hipGetErrorString(e));
        }
        HIP_TRY(hipMalloc((void**)&H->d_pair_slot, slot.size() * sizeof(int32_t)));
        HIP_TRY(hipMemcpy(H->d_pair_slot, slot.data(), slot.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMalloc((void**)&H->d_pairs, pairs.size() * sizeof(int2)));
        HIP_TRY(hipMemcpy(H->d_pairs, pairs.data(), pairs.size() * sizeof(int2),
                          hipMemcpyHostToDevice));
        SourceArgs src = H->source();
        HIP_TRY(launch_cache_fill(src, (int32_t)D, H->d_pairs, H->p_cache, H->d_slots, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    H->planned = true;
    return PROCMV_OK;
}

procmv_status procmv_plan_info(procmv_op_t H, procmv_plan_info_t* info)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (!info) return fail(PROCMV_ERR_INVALID_ARG, "info is null");
    if (!H->planned) return fail(PROCMV_ERR_NOT_PLANNED, "operator has no plan");
    info->D = H->D;
    info->block_size = H->b;
    info->n_blk = H->n_blk;
    info->n_pair = H->n_pair;
    info->p_cache = H->p_cache;
    info->cache_bytes = H->p_cache * (int64_t)H->b * H->b * (int64_t)H->slot_elem();
    info->work_bytes = (int64_t)H->P_bytes;
    info->strategy = H->strategy;
    info->precision = H->precision;
    return PROCMV_OK;
}

}  // extern "C"

namespace {

// Y = H X with the partials in the operator's buffer or in `scr`.
procmv_status apply_impl(procmv_op_t H, const void* X, int64_t ldx, void* Y, int64_t ldy,
                         int32_t nvec, void* stream, const Scratch& scr)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (!H->planned) return fail(PROCMV_ERR_NOT_PLANNED, "procmv_apply before procmv_plan");
    if (!X || !Y) return fail(PROCMV_ERR_INVALID_ARG, "null vector pointer");
    if (nvec < 1) return fail(PROCMV_ERR_INVALID_ARG, "nvec = %d", nvec);
    if (ldx < H->D || ldy < H->D)
        return fail(PROCMV_ERR_INVALID_ARG, "leading dimensions must be >= D");
    const char* xb = (const char*)X;
    const char* yb = (const char*)Y;
    const size_t xs = ((size_t)(nvec - 1) * ldx + H->D) * sizeof(float2);
    const size_t ys = ((size_t)(nvec - 1) * ldy + H->D) * sizeof(float2);
    if (xb < yb + ys && yb < xb + xs)
        return fail(PROCMV_ERR_INVALID_ARG, "X and Y overlap");
    hipStream_t s = (hipStream_t)stream;
    float bhi = 0.f, blo = 0.f;
    if (H->gen == 1) split_f32(H->d_const, bhi, blo);
    for (int v0 = 0; v0 < nvec;) {
        const int nv = chunk_vectors(H, nvec - v0);
        const float2* Xc = (const float2*)X + (size_t)v0 * ldx;
        float2* Yc = (float2*)Y + (size_t)v0 * ldy;
        ReduceArgs r{};
        r.Y = Yc;
        r.ldy = ldy;
        r.alpha = 1.0f;
        r.beta_hi = bhi;
        r.beta_lo = blo;
        comp_fields(H, r);
        st = run_product(H, Xc, ldx, nv, r, Epi::kApply, s, scr);
        if (st != PROCMV_OK) return st;
        v0 += nv;
    }
    return PROCMV_OK;
}

}  // namespace

extern "C" {

procmv_status procmv_apply(procmv_op_t H, const void* X, int64_t ldx, void* Y,
                           int64_t ldy, int32_t nvec, void* stream)
{
    return apply_impl(H, X, ldx, Y, ldy, nvec, stream, Scratch{});
}

procmv_status procmv_apply_noalloc(procmv_op_t H, const void* X, int64_t ldx, void* Y,
                                   int64_t ldy, int32_t nvec, void* stream)
{
    // the device-resident static workspace of the current device (its
    // address is resolved once per device; no allocation here)
    Scratch scr;
    size_t bytes = 0;
    void* p = nullptr;
    HIP_TRY(static_workspace(&p, &bytes));
    scr.p = (float2*)p;
    scr.bytes = bytes;
    return apply_impl(H, X, ldx, Y, ldy, nvec, stream, scr);
}

procmv_status procmv_spectral_bounds(procmv_op_t H, double* c, double* R)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (!c || !R) return fail(PROCMV_ERR_INVALID_ARG, "null output");
    if (H->gen == 0) {
        *c = 0.0;
        *R = 2.5;
    } else {
        const double e_min = 0.0;
        const double e_max = M_PI * M_PI / (2.0 * H->dvr.mass * H->dx * H->dx) + H->vmax;
        *c = 0.5 * (e_max + e_min);
        *R = 0.5 * (e_max - e_min);
    }
    return PROCMV_OK;
}

namespace {

// Eigenvalues and eigenvectors of the symmetric tridiagonal T (diagonal a,
// off-diagonal b) by cyclic Jacobi rotations on a dense copy (Golub & Van
// Loan, symmetric Schur decomposition; m is small).  Returns the extreme
// eigenvalues and the last entries of their unit eigenvectors.
void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, int n,
                      double& th_min, double& s_min, double& th_max, double& s_max)
{
    std::vector<double> A((size_t)n * n, 0.0), V((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) {
        A[(size_t)i * n + i] = a[i];
        V[(size_t)i * n + i] = 1.0;
        if (i + 1 < n) A[(size_t)i * n + i + 1] = A[(size_t)(i + 1) * n + i] = b[i];
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) /
                                 (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
                // A <- J^T A J with J the rotation in the (p, q) plane
                for (int k = 0; k < n; ++k) {
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    int imin = 0, imax = 0;
    for (int i = 1; i < n; ++i) {
        if (A[(size_t)i * n + i] < A[(size_t)imin * n + imin]) imin = i;
        if (A[(size_t)i * n + i] > A[(size_t)imax * n + imax]) imax = i;
    }
    th_min = A[(size_t)imin * n + imin];
    th_max = A[(size_t)imax * n + imax];
    s_min = V[(size_t)(n - 1) * n + imin];
    s_max = V[(size_t)(n - 1) * n + imax];
}

}  // namespace

procmv_status procmv_lanczos_bounds(procmv_op_t H, const void* v0, int32_t m,
                                    double* bounds_out, double* alpha_out,
                                    double* beta_out, int32_t* steps_out, void* stream)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (!H->planned) return fail(PROCMV_ERR_NOT_PLANNED, "Lanczos before procmv_plan");
    if (!v0 || !bounds_out) return fail(PROCMV_ERR_INVALID_ARG, "null v0 or bounds_out");
    if (m < 1 || m > PROCMV_LANCZOS_MAX_STEPS || m > H->D)
        return fail(PROCMV_ERR_INVALID_ARG, "m = %d outside [1, min(D, %d)]", m,
                    PROCMV_LANCZOS_MAX_STEPS);
    const int32_t D = (int32_t)H->D;
    st = ensure(H->d_lz, H->lz_bytes, (size_t)3 * D * sizeof(float2));
    if (st != PROCMV_OK) return st;
    st = ensure(H->d_lzs, H->lzs_bytes,
                (size_t)(2 * kLanczosMaxBlocks + 2 * m) * sizeof(double));
    if (st != PROCMV_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    float2* vp = H->d_lz;
    float2* v = H->d_lz + D;
    float2* w = H->d_lz + 2 * (size_t)D;
    double* dotp = H->d_lzs;
    double* nrmp = H->d_lzs + kLanczosMaxBlocks;
    double* d_alpha = H->d_lzs + 2 * kLanczosMaxBlocks;
    double* d_beta = d_alpha + m;
    // v_1 = v0 / ||v0||
    HIP_TRY(launch_lanczos_normalise(D, (const float2*)v0, v, nrmp, nullptr, s));
    for (int j = 0; j < m; ++j) {
        st = procmv_apply(H, v, D, w, D, 1, stream);
        if (st != PROCMV_OK) return st;
        HIP_TRY(launch_lanczos_orthogonalise(D, v, vp, w, dotp, nrmp,
                                             j > 0 ? d_beta + j - 1 : nullptr, d_alpha + j, s));
        // v_{j+1} = w / beta_j overwrites v_{j-1} (the update wrote the norm partials)
        HIP_TRY(launch_lanczos_scale(D, w, vp, nrmp, d_beta + j, s));
        std::swap(vp, v);
    }
    std::vector<double> a(m), b(m);
    HIP_TRY(hipMemcpyAsync(a.data(), d_alpha, m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(b.data(), d_beta, m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // an exactly invariant Krylov space ends the recurrence (later steps divided by zero)
    int n = m;
    for (int j = 0; j < m; ++j)
        if (!(b[j] > 0.0)) { n = j + 1; b[j] = 0.0; break; }
    for (int j = 0; j < n; ++j)
        if (!std::isfinite(a[j]) || !std::isfinite(b[j]))
            return fail(PROCMV_ERR_INTERNAL, "Lanczos step %d is not finite", j);
    double th_min, s_min, th_max, s_max;
    tridiag_extremes(a, b, n, th_min, s_min, th_max, s_max);
    const double r_min = std::fabs(b[n - 1] * s_min), r_max = std::fabs(b[n - 1] * s_max);
    bounds_out[0] = th_min - r_min;
    bounds_out[1] = th_max + r_max;
    bounds_out[2] = th_min;
    bounds_out[3] = th_max;
    bounds_out[4] = r_min;
    bounds_out[5] = r_max;
    if (alpha_out) for (int j = 0; j < n; ++j) alpha_out[j] = a[j];
    if (beta_out) for (int j = 0; j < n; ++j) beta_out[j] = b[j];
    if (steps_out) *steps_out = n;
    return PROCMV_OK;
}

procmv_status procmv_kron_apply(procmv_op_t HB, const procmv_op_t* B, int32_t n_int,
                                int32_t dS, const double* HS, const double* A, double g,
                                const void* X, void* Y, void* stream)
{
    procmv_status st = check_op(HB);
    if (st != PROCMV_OK) return st;
    if (dS < 1 || dS > PROCMV_KRON_MAX_SYS || n_int < 0 || n_int > PROCMV_KRON_MAX_INT)
        return fail(PROCMV_ERR_INVALID_ARG, "d_S = %d or n_int = %d out of range", dS, n_int);
    if (!HS || !X || !Y || (n_int > 0 && (!B || !A)))
        return fail(PROCMV_ERR_INVALID_ARG, "null argument");
    const int64_t dB = HB->D;
    for (int a = 0; a < n_int; ++a) {
        st = check_op(B[a]);
        if (st != PROCMV_OK) return st;
        if (B[a]->D != dB)
            return fail(PROCMV_ERR_INVALID_ARG, "bath operator %d has D = %lld, H_B %lld", a,
                        (long long)B[a]->D, (long long)dB);
    }
    const size_t vec = (size_t)dS * dB;
    const char* xb = (const char*)X;
    const char* yb = (const char*)Y;
    if (xb < yb + vec * sizeof(float2) && yb < xb + vec * sizeof(float2))
        return fail(PROCMV_ERR_INVALID_ARG, "X and Y overlap");
    st = ensure(HB->d_kz, HB->kz_bytes, (size_t)(1 + n_int) * vec * sizeof(float2));
    if (st != PROCMV_OK) return st;
    // bath operators on the d_S rows of X (each checks its own plan)
    st = procmv_apply(HB, X, dB, HB->d_kz, dB, dS, stream);
    if (st != PROCMV_OK) return st;
    for (int a = 0; a < n_int; ++a) {
        st = procmv_apply(B[a], X, dB, HB->d_kz + (size_t)(1 + a) * vec, dB, dS, stream);
        if (st != PROCMV_OK) return st;
    }
    KronMixArgs k{};
    k.X = (const float2*)X;
    k.Z = HB->d_kz;
    k.Y = (float2*)Y;
    k.dB = dB;
    k.dS = dS;
    k.n_int = n_int;
    for (int op = 0; op <= n_int; ++op)
        for (int s = 0; s < dS; ++s)
            for (int t = 0; t < dS; ++t) {
                const double* m = op == 0 ? HS + 2 * (s * dS + t)
                                          : A + 2 * (((size_t)(op - 1) * dS + s) * dS + t);
                const double f = op == 0 ? 1.0 : g;
                k.M[(op * kKronMaxSys + s) * kKronMaxSys + t] =
                    make_float2((float)(f * m[0]), (float)(f * m[1]));
            }
    HIP_TRY(launch_kron_mix(k, (hipStream_t)stream));
    return PROCMV_OK;
}

procmv_status procmv_kron_propagate(procmv_op_t HB, const procmv_op_t* B, int32_t n_int,
                                    int32_t dS, const double* HS, const double* A, double g,
                                    void* psi, double dt, int32_t K, int32_t nsteps,
                                    double spec_c, double spec_R, double* norms_out,
                                    void* stream)
{
    procmv_status st = check_op(HB);
    if (st != PROCMV_OK) return st;
    if (!psi) return fail(PROCMV_ERR_INVALID_ARG, "psi is null");
    if (dS < 1 || dS > PROCMV_KRON_MAX_SYS || nsteps < 0 || !(dt >= 0.0) || !(spec_R > 0.0))
        return fail(PROCMV_ERR_INVALID_ARG, "bad d_S/nsteps/dt/R");
    const int64_t n = (int64_t)dS * HB->D;
    if (n > INT32_MAX) return fail(PROCMV_ERR_INVALID_ARG, "d_S d_B too large");
    // 1/R exact in binary32: the half-width is widened to 1/alpha
    const float alpha = f32_down(1.0 / spec_R);
    const double Reff = 1.0 / (double)alpha;
    if (K <= 0) K = procmv_cheb_order(Reff * dt, 1e-10);
    if (K < 1) return fail(PROCMV_ERR_INVALID_ARG, "Chebyshev order could not be set");
    st = ensure(HB->d_kq, HB->kq_bytes, (size_t)2 * n * sizeof(float2));
    if (st != PROCMV_OK) return st;
    st = ensure(HB->d_kacc, HB->kacc_bytes, (size_t)(n + 1) * sizeof(double2));
    if (st != PROCMV_OK) return st;
    const std::vector<double> j = bessel_j(Reff * dt, K);
    std::vector<double2> a(K + 1);
    for (int k = 0; k <= K; ++k) {
        const double m = (k == 0 ? 1.0 : 2.0) * j[k];
        const int q = k & 3;   // (-i)^k
        a[k] = q == 0 ? double2{m, 0.0} : q == 1 ? double2{0.0, -m}
             : q == 2 ? double2{-m, 0.0} : double2{0.0, m};
    }
    const double2 phase{std::cos(spec_c * dt), -std::sin(spec_c * dt)};
    float bhi, blo;
    split_f32(-(double)alpha * spec_c, bhi, blo);
    hipStream_t s = (hipStream_t)stream;
    float2* P0 = (float2*)psi;
    float2* qa = HB->d_kq;
    float2* Yb = HB->d_kq + n;
    double2* acc = HB->d_kacc;
    double* norm2 = (double*)(HB->d_kacc + n);
    for (int step = 0; step < nsteps; ++step) {
        HIP_TRY(launch_kron_cheb_init(n, P0, acc, a[0], s));
        st = procmv_kron_apply(HB, B, n_int, dS, HS, A, g, P0, Yb, stream);
        if (st != PROCMV_OK) return st;
        HIP_TRY(launch_kron_cheb_term(n, Yb, P0, qa, acc, alpha, bhi, blo, a[1], 1, s));
        // q_0 lives in psi, q_1 in qa; each term overwrites the older one
        float2* prev = P0;
        float2* cur = qa;
        for (int k = 1; k < K; ++k) {
            st = procmv_kron_apply(HB, B, n_int, dS, HS, A, g, cur, Yb, stream);
            if (st != PROCMV_OK) return st;
            HIP_TRY(launch_kron_cheb_term(n, Yb, cur, prev, acc, alpha, bhi, blo, a[k + 1], 0,
                                          s));
            std::swap(prev, cur);
        }
        HIP_TRY(launch_cheb_finish((int32_t)n, 1, acc, n, phase, P0, n, norm2, s));
        if (norms_out) {
            double v = 0.0;
            HIP_TRY(hipMemcpyAsync(&v, norm2, sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            norms_out[step] = std::sqrt(v);
        }
    }
    return PROCMV_OK;
}

int32_t procmv_cheb_order(double x, double tol)
{
    if (!(x >= 0.0) || !(tol > 0.0)) return -1;
    const int kmax = (int)x + 60 + (int)(30.0 * std::cbrt(std::max(x, 1.0)));
    std::vector<double> j = bessel_j(x, kmax + 1);
    for (int k = (int)std::ceil(x); k + 1 <= kmax + 1; ++k)
        if (2.0 * std::fabs(j[k]) < tol && 2.0 * std::fabs(j[k + 1]) < tol) return k;
    return -1;
}

namespace {

// nsteps applications of psi <- phase * sum_k a_k T_k(Ht) psi, Ht = alpha (H - c)
// (alpha (d - c) split into bhi + blo), in chunks of vectors; binary64 norms
// after each step when norms_out is given (synchronises then).
procmv_status cheb_run(procmv_op_t H, void* psi, int64_t ld, int32_t nvec, int32_t K,
                       int32_t nsteps, const std::vector<double2>& a, double2 phase,
                       float alpha, float bhi, float blo, float ghi, float glo,
                       double* norms_out, void* stream)
{
    procmv_status st = PROCMV_OK;
    hipStream_t s = (hipStream_t)stream;
    for (int v0 = 0; v0 < nvec;) {
        const int nv = chunk_vectors(H, nvec - v0);
        float2* P0 = (float2*)psi + (size_t)v0 * ld;
        const size_t D = (size_t)H->D;
        st = ensure(H->d_q, H->q_bytes, (size_t)nv * D * sizeof(float2));
        if (st != PROCMV_OK) return st;
        st = ensure(H->d_acc, H->acc_bytes, (size_t)nv * D * sizeof(double2));
        if (st != PROCMV_OK) return st;
        st = ensure(H->d_norm, H->norm_bytes, (size_t)nv * sizeof(double));
        if (st != PROCMV_OK) return st;
        const bool comp = H->comp();
        if (comp) {
            st = ensure(H->d_qlo, H->qlo_bytes, (size_t)2 * nv * D * sizeof(float2));
            if (st != PROCMV_OK) return st;
        }
        // lo parts (compensated arithmetic): lo_a goes with psi's slot, lo_b with d_q's
        float2* lo_a = comp ? H->d_qlo : nullptr;
        float2* lo_b = comp ? H->d_qlo + (size_t)nv * D : nullptr;
        for (int step = 0; step < nsteps; ++step) {
            // q0 lives in psi (ld), q1 in d_q (ld = D); the recurrence
            // overwrites the older of the two.
            float2* qa = P0;
            int64_t lda = ld;
            float2* qb = H->d_q;
            int64_t ldb = (int64_t)D;
            ReduceArgs r{};
            r.Yq1 = qb;
            r.ldy = ldb;
            r.acc = H->d_acc;
            r.ldacc = (int64_t)D;
            r.alpha = alpha;
            r.beta_hi = bhi;
            r.beta_lo = blo;
            r.a0 = a[0];
            r.a1 = a[1];
            if (comp) {
                comp_fields(H, r);
                r.Yq1lo = lo_b;
                r.Xlo_zero = lo_a;
                r.ldylo = (int64_t)D;
                r.gamma_hi = ghi;
                r.gamma_lo = glo;
            }
            st = run_product(H, qa, lda, nv, r, Epi::kChebFirst, s);
            if (st != PROCMV_OK) return st;
            // cur = qb (q1), prev = qa (q0)
            float2* cur = qb;
            int64_t ldc = ldb;
            float2* prev = qa;
            int64_t ldpv = lda;
            float2* cur_lo = lo_b;
            float2* prev_lo = lo_a;
            for (int k = 1; k < K; ++k) {
                ReduceArgs rs{};
                rs.Y = prev;   // q_{k-1} in, q_{k+1} out
                rs.ldy = ldpv;
                rs.acc = H->d_acc;
                rs.ldacc = (int64_t)D;
                rs.alpha = alpha;
                rs.beta_hi = bhi;
                rs.beta_lo = blo;
                rs.a0 = a[k + 1];
                if (comp) {
                    comp_fields(H, rs);
                    rs.Xlo = cur_lo;
                    rs.ldxl = (int64_t)D;
                    rs.Ylo = prev_lo;
                    rs.ldylo = (int64_t)D;
                    rs.gamma_hi = ghi;
                    rs.gamma_lo = glo;
                }
                st = run_product(H, cur, ldc, nv, rs, Epi::kChebStep, s);
                if (st != PROCMV_OK) return st;
                std::swap(cur, prev);
                std::swap(ldc, ldpv);
                std::swap(cur_lo, prev_lo);
            }
            HIP_TRY(launch_cheb_finish((int32_t)D, nv, H->d_acc, (int64_t)D, phase, P0, ld,
                                       H->d_norm, s));
            if (norms_out) {
                std::vector<double> n2(nv);
                HIP_TRY(hipMemcpyAsync(n2.data(), H->d_norm, nv * sizeof(double),
                                       hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                for (int v = 0; v < nv; ++v)
                    norms_out[(size_t)step * nvec + v0 + v] = std::sqrt(n2[v]);
            }
        }
        v0 += nv;
    }
    return PROCMV_OK;
}


}  // namespace

procmv_status procmv_chebyshev_propagate(procmv_op_t H, void* psi, int64_t ld,
                                         int32_t nvec, double dt, int32_t K,
                                         int32_t nsteps, double spec_c,
                                         double spec_R, double* norms_out,
                                         void* stream)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (!H->planned) return fail(PROCMV_ERR_NOT_PLANNED, "propagation before procmv_plan");
    if (!psi) return fail(PROCMV_ERR_INVALID_ARG, "psi is null");
    if (nvec < 1 || nsteps < 0 || ld < H->D || !(dt >= 0.0))
        return fail(PROCMV_ERR_INVALID_ARG, "bad nvec/nsteps/ld/dt");
    double c = spec_c, R = spec_R;
    if (!(R > 0.0)) {
        st = procmv_spectral_bounds(H, &c, &R);
        if (st != PROCMV_OK) return st;
    }
    // 1/R exact in binary32: the half-width is widened to 1/alpha.
    const float alpha = f32_down(1.0 / R);
    const double Reff = 1.0 / (double)alpha;
    if (K <= 0) K = procmv_cheb_order(Reff * dt, 1e-10);
    if (K < 1) return fail(PROCMV_ERR_INVALID_ARG, "Chebyshev order could not be set");
    const std::vector<double> j = bessel_j(Reff * dt, K);
    std::vector<double2> a(K + 1);
    for (int k = 0; k <= K; ++k) {
        const double m = (k == 0 ? 1.0 : 2.0) * j[k];
        // (-i)^k
        const int q = k & 3;
        a[k] = q == 0 ? double2{m, 0.0} : q == 1 ? double2{0.0, -m}
             : q == 2 ? double2{-m, 0.0} : double2{0.0, m};
    }
    const double2 phase{std::cos(c * dt), -std::sin(c * dt)};
    const double dconst = H->gen == 1 ? H->d_const : 0.0;
    float bhi, blo, ghi, glo;
    split_f32((double)alpha * (dconst - c), bhi, blo);
    split_f32((double)alpha * c, ghi, glo);
    return cheb_run(H, psi, ld, nvec, K, nsteps, a, phase, alpha, bhi, blo, ghi, glo, norms_out,
                    stream);
}

namespace {

// e^{-z} I_k(z), k = 0..kmax, z >= 0: Miller's backward recurrence
// I_{k-1} = (2k/z) I_k + I_{k+1} from far above, normalised by the sum rule
// e^{-z} (I_0 + 2 sum_{k>=1} I_k) = 1.
std::vector<double> bessel_i_scaled(double z, int kmax)
{
    std::vector<double> out(kmax + 1, 0.0);
    if (z == 0.0) {
        out[0] = 1.0;
        return out;
    }
    const int top = std::max(kmax, (int)std::sqrt(80.0 * std::max(z, 1.0)) + 40) + 30;
    std::vector<double> v(top + 2, 0.0);
    v[top] = 1e-300;
    for (int k = top; k > 0; --k) {
        v[k - 1] = (2.0 * k / z) * v[k] + v[k + 1];
        if (v[k - 1] > 1e250)
            for (int q = k - 1; q <= top; ++q) v[q] *= 1e-250;
    }
    double norm = v[0];
    for (int k = 1; k <= top; ++k) norm += 2.0 * v[k];
    for (int k = 0; k <= kmax; ++k) out[k] = v[k] / norm;
    return out;
}

}  // namespace

int32_t procmv_filter_order(double z, double tol)
{
    if (!(z >= 0.0) || !(tol > 0.0)) return -1;
    const int kmax = (int)std::sqrt(80.0 * std::max(z, 1.0)) + 60;
    const std::vector<double> v = bessel_i_scaled(z, kmax + 1);
    for (int k = 0; k + 1 <= kmax + 1; ++k)
        if (2.0 * v[k] < tol && 2.0 * v[k + 1] < tol) return std::max(k, 1);
    return -1;
}

procmv_status procmv_chebyshev_filter(procmv_op_t H, void* psi, int64_t ld, int32_t nvec,
                                      double tau, int32_t K, double spec_c, double spec_R,
                                      double* norms_out, void* stream)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (!H->planned) return fail(PROCMV_ERR_NOT_PLANNED, "filter before procmv_plan");
    if (!psi) return fail(PROCMV_ERR_INVALID_ARG, "psi is null");
    if (nvec < 1 || ld < H->D || !(tau >= 0.0))
        return fail(PROCMV_ERR_INVALID_ARG, "bad nvec/ld/tau");
    double c = spec_c, R = spec_R;
    if (!(R > 0.0)) {
        st = procmv_spectral_bounds(H, &c, &R);
        if (st != PROCMV_OK) return st;
    }
    const float alpha = f32_down(1.0 / R);
    const double Reff = 1.0 / (double)alpha;
    const double z = Reff * tau;
    if (K <= 0) K = procmv_filter_order(z, 1e-10);
    if (K < 1) return fail(PROCMV_ERR_INVALID_ARG, "filter order could not be set");
    // e^{-tau H} = e^{-tau (c - Reff)} sum_k (2 - delta_k0) (-1)^k e^{-z} I_k(z) T_k(Ht)
    const std::vector<double> iv = bessel_i_scaled(z, K);
    std::vector<double2> a(K + 1);
    for (int k = 0; k <= K; ++k)
        a[k] = double2{(k == 0 ? 1.0 : 2.0) * ((k & 1) ? -iv[k] : iv[k]), 0.0};
    const double scale = std::exp(-tau * (c - Reff));
    if (!std::isfinite(scale) || scale == 0.0)
        return fail(PROCMV_ERR_INVALID_ARG, "e^{-tau (c - R)} = %g is out of range", scale);
    const double2 phase{scale, 0.0};
    const double dconst = H->gen == 1 ? H->d_const : 0.0;
    float bhi, blo, ghi, glo;
    split_f32((double)alpha * (dconst - c), bhi, blo);
    split_f32((double)alpha * c, ghi, glo);
    return cheb_run(H, psi, ld, nvec, K, 1, a, phase, alpha, bhi, blo, ghi, glo, norms_out,
                    stream);
}

procmv_status procmv_get_entries(procmv_op_t H, int64_t r0, int64_t c0,
                                 int32_t nr, int32_t nc, void* out_dev,
                                 void* stream)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (!out_dev) return fail(PROCMV_ERR_INVALID_ARG, "out is null");
    if (nr < 0 || nc < 0 || r0 < 0 || c0 < 0 || r0 + nr > H->D || c0 + nc > H->D)
        return fail(PROCMV_ERR_INVALID_ARG, "window outside the matrix");
    if ((int64_t)nr * nc == 0) return PROCMV_OK;
    SourceArgs src = H->source(true);
    HIP_TRY(launch_get_entries(src, r0, c0, nr, nc, (float2*)out_dev, (hipStream_t)stream));
    return PROCMV_OK;
}

procmv_status procmv_selftest_generator(int32_t* ln_mismatches, int32_t* sqrt_mismatches,
                                        void* stream)
{
    if (!ln_mismatches || !sqrt_mismatches) return fail(PROCMV_ERR_INVALID_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    unsigned* d = nullptr;
    if (hipMalloc((void**)&d, 2 * sizeof(unsigned)) != hipSuccess)
        return fail(PROCMV_ERR_OOM, "self-test counters");
    unsigned h[2] = {0u, 0u};
    hipError_t e = launch_selftest_generator(d, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(PROCMV_ERR_HIP, "self-test: %s", hipGetErrorString(e));
    *ln_mismatches = (int32_t)h[0];
    *sqrt_mismatches = (int32_t)h[1];
    return PROCMV_OK;
}

procmv_status procmv_profile_enable(procmv_op_t H, int32_t every)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    H->prof_every = every > 0 ? every : 0;
    for (int k = 0; k < 2; ++k) {
        H->prof_count[k] = 0;
        H->prof_used[k] = 0;
    }
    return PROCMV_OK;
}

procmv_status procmv_profile_read(procmv_op_t H, double* tile_ms,
                                  int64_t* tile_launches, double* reduce_ms,
                                  int64_t* reduce_launches)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    double ms[2] = {0.0, 0.0};
    int64_t n[2] = {0, 0};
    for (int k = 0; k < 2; ++k) {
        for (size_t q = 0; q + 1 < H->prof_used[k]; q += 2) {
            HIP_TRY(hipEventSynchronize(H->prof_ev[k][q + 1]));
            float t = 0.f;
            HIP_TRY(hipEventElapsedTime(&t, H->prof_ev[k][q], H->prof_ev[k][q + 1]));
            ms[k] += (double)t;
            n[k] += 1;
        }
        H->prof_used[k] = 0;
        H->prof_count[k] = 0;
    }
    if (tile_ms) *tile_ms = ms[0];
    if (tile_launches) *tile_launches = n[0];
    if (reduce_ms) *reduce_ms = ms[1];
    if (reduce_launches) *reduce_launches = n[1];
    return PROCMV_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Batches of independent operators: one persistent launch per product.
// ------------------------------------------------------------------------
struct procmv_batch {
    std::vector<procmv_op*> ops;
    int n = 0, nv = 0, gen = 0;
    std::vector<int64_t> off;
    int64_t total = 0;
    std::vector<TileArgs> targs;
    std::vector<std::vector<int4>> per_inst;   // super-tile items of each instance
    TileArgs* d_ops = nullptr;
    int4* d_items = nullptr;
    int64_t n_items = 0;
    BatchReduceItem* d_ritems = nullptr;       // apply epilogue
    BatchReduceItem* d_citems = nullptr;       // Chebyshev epilogue
    std::vector<BatchReduceItem> h_citems;      // its host copy (outlives the async upload)
    int64_t* d_off = nullptr;
    float2* d_P = nullptr;
    float2* d_q = nullptr;
    double2* d_acc = nullptr;
    double* d_norm = nullptr;
    int shape = 1, grid = 1024, order = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap = nullptr;     // own stream for graph capture (the caller's
                                   // may be the legacy null stream)
    const void* g_psi = nullptr;
    double g_key[4] = {0, 0, 0, 0};
    int g_K = -1;

    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        g_psi = nullptr;
        g_K = -1;
    }

    ~procmv_batch()
    {
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
        dfree(d_ops);
        dfree(d_items);
        dfree(d_ritems);
        dfree(d_citems);
        dfree(d_off);
        dfree(d_P);
        dfree(d_q);
        dfree(d_acc);
        dfree(d_norm);
    }
};

namespace {

procmv_status batch_upload_items(procmv_batch* B)
{
    std::vector<int4> items;
    items.reserve((size_t)B->n_items);
    if (B->order == 0) {
        // round-robin over the instances, largest first
        std::vector<int> idx(B->n);
        for (int k = 0; k < B->n; ++k) idx[k] = k;
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
            return B->per_inst[x].size() > B->per_inst[y].size();
        });
        for (size_t q = 0;; ++q) {
            bool any = false;
            for (int k : idx)
                if (q < B->per_inst[k].size()) {
                    items.push_back(B->per_inst[k][q]);
                    any = true;
                }
            if (!any) break;
        }
    } else {
        for (int k = 0; k < B->n; ++k)
            items.insert(items.end(), B->per_inst[k].begin(), B->per_inst[k].end());
    }
    HIP_TRY(hipMemcpy(B->d_items, items.data(), items.size() * sizeof(int4),
                      hipMemcpyHostToDevice));
    return PROCMV_OK;
}

procmv_status batch_tiles(procmv_batch* B, const float2* xbase, hipStream_t s)
{
    BatchTileLaunch L{};
    L.ops = B->d_ops;
    L.items = B->d_items;
    L.n_items = B->n_items;
    L.xbase = xbase;
    L.gen = B->gen;
    L.nv = B->nv;
    L.shape = B->shape;
    L.grid = (int)std::min<int64_t>(B->grid, B->n_items);
    L.cached = 0;
    L.min_se = kSuper / 64;
    L.cache_b = 0;
    bool any_cached = false, all_full = true;
    for (procmv_op* op : B->ops) {
        L.cached |= (op->p_cache > 0) ? 1 : 0;
        any_cached = any_cached || op->p_cache > 0;
        all_full = all_full && op->p_cache == op->n_pair;
        // tiles of every cached instance must fit its slots: a common divisor
        if (op->p_cache > 0) L.cache_b = std::gcd(L.cache_b, (int)op->b);
    }
    // the single-operator routing rule, for the batch as a whole
    L.mfma = mfma_path(B->gen, !any_cached, all_full, PROCMV_FP32, B->nv) ? 1 : 0;
    if (L.mfma) HIP_TRY(launch_tile_mfma_batched(L, s));
    else HIP_TRY(launch_tile_apply_batched(L, s));
    return PROCMV_OK;
}

BatchReduceArgs batch_rargs(procmv_batch* B, const BatchReduceItem* items)
{
    BatchReduceArgs r{};
    r.items = items;
    r.off = B->d_off;
    r.n = B->n;
    r.nv = B->nv;
    r.total = B->total;
    return r;
}

procmv_status batch_enqueue_apply(procmv_batch* B, const float2* X, float2* Y, hipStream_t s)
{
    procmv_status st = batch_tiles(B, X, s);
    if (st != PROCMV_OK) return st;
    BatchReduceArgs r = batch_rargs(B, B->d_ritems);
    r.X = X;
    r.Y = Y;
    HIP_TRY(launch_reduce_batched(r, Epi::kApply, s));
    return PROCMV_OK;
}

}  // namespace

extern "C" {

procmv_status procmv_batch_create(const procmv_op_t* ops, int32_t n, int32_t nvec,
                                  procmv_batch_t* out)
{
    if (!out) return fail(PROCMV_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!ops || n < 1) return fail(PROCMV_ERR_INVALID_ARG, "empty batch");
    if (nvec != 1 && nvec != 2 && nvec != 4 && nvec != 8)
        return fail(PROCMV_ERR_INVALID_ARG, "batch nvec must be 1, 2, 4 or 8");
    for (int k = 0; k < n; ++k) {
        if (!ops[k]) return fail(PROCMV_ERR_INVALID_ARG, "operator %d is null", k);
        if (!ops[k]->planned) return fail(PROCMV_ERR_NOT_PLANNED, "operator %d has no plan", k);
        if (ops[k]->precision != PROCMV_FP32)
            return fail(PROCMV_ERR_INVALID_ARG, "batched products run in binary32");
        if (ops[k]->gen != ops[0]->gen)
            return fail(PROCMV_ERR_INVALID_ARG, "a batch holds one generator family");
    }
    procmv_batch* B = new procmv_batch();
    B->n = n;
    B->nv = nvec;
    B->gen = ops[0]->gen;
    B->ops.assign(ops, ops + n);
    B->off.resize(n);
    int64_t poff = 0;
    std::vector<int64_t> pstart(n);
    for (int k = 0; k < n; ++k) {
        B->off[k] = B->total;
        B->total += (int64_t)nvec * ops[k]->D;
        pstart[k] = poff;
        // batches take the largest super-tile edge for every instance: the
        // instances already fill the device, and big super-tiles carry less
        // per-item overhead
        poff += ((ops[k]->D + kSuper - 1) / kSuper + 1) * nvec * ops[k]->D;
    }
    hipError_t e = hipMalloc((void**)&B->d_P, (size_t)poff * sizeof(float2));
    if (e != hipSuccess) {
        delete B;
        return fail(PROCMV_ERR_OOM, "batch partial buffer: %s", hipGetErrorString(e));
    }
    B->targs.resize(n);
    B->per_inst.resize(n);
    std::vector<BatchReduceItem> ri(n);
    for (int k = 0; k < n; ++k) {
        procmv_op* op = ops[k];
        TileArgs& a = B->targs[k];
        a = TileArgs{};
        a.src = op->source();
        a.D = (int32_t)op->D;
        a.se = kSuper / 64;
        a.n_super = (int32_t)((op->D + kSuper - 1) / kSuper);
        a.nv = nvec;
        a.ldx = op->D;
        a.xoff = B->off[k];
        a.P = B->d_P + pstart[k];
        a.ldp = op->D;
        for (int r = 0; r < a.n_super; ++r)
            for (int c = r; c < a.n_super; ++c) B->per_inst[k].push_back(make_int4(k, r, c, 0));
        B->n_items += (int64_t)B->per_inst[k].size();
        ri[k] = BatchReduceItem{};
        ri[k].D = (int32_t)op->D;
        ri[k].n_slots = a.n_super + 1;
        ri[k].off = B->off[k];
        ri[k].P = a.P;
        ri[k].ldp = op->D;
        ri[k].alpha = 1.0f;
        if (op->gen == 1) split_f32(op->d_const, ri[k].beta_hi, ri[k].beta_lo);
        ri[k].phase = double2{1.0, 0.0};
    }
    procmv_status st = PROCMV_OK;
#define BTRY(expr)                                                           \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess) {                                              \
            st = fail(e_ == hipErrorOutOfMemory ? PROCMV_ERR_OOM : PROCMV_ERR_HIP, \
                      "%s: %s", #expr, hipGetErrorString(e_));               \
            delete B;                                                        \
            return st;                                                       \
        }                                                                    \
    } while (0)
    BTRY(hipMalloc((void**)&B->d_ops, n * sizeof(TileArgs)));
    BTRY(hipMemcpy(B->d_ops, B->targs.data(), n * sizeof(TileArgs), hipMemcpyHostToDevice));
    BTRY(hipMalloc((void**)&B->d_items, B->n_items * sizeof(int4)));
    BTRY(hipMalloc((void**)&B->d_ritems, n * sizeof(BatchReduceItem)));
    BTRY(hipMalloc((void**)&B->d_citems, n * sizeof(BatchReduceItem)));
    BTRY(hipMemcpy(B->d_ritems, ri.data(), n * sizeof(BatchReduceItem), hipMemcpyHostToDevice));
    BTRY(hipMalloc((void**)&B->d_off, n * sizeof(int64_t)));
    BTRY(hipMemcpy(B->d_off, B->off.data(), n * sizeof(int64_t), hipMemcpyHostToDevice));
#undef BTRY
    B->shape = 0;                   // same default as single operators
    st = batch_upload_items(B);
    if (st != PROCMV_OK) {
        delete B;
        return st;
    }
    *out = B;
    return PROCMV_OK;
}

void procmv_batch_destroy(procmv_batch_t B) { delete B; }

procmv_status procmv_batch_info(procmv_batch_t B, int64_t* total, int64_t* items,
                                int32_t* shape, int32_t* grid, int32_t* order)
{
    if (!B) return fail(PROCMV_ERR_INVALID_ARG, "null batch");
    if (total) *total = B->total;
    if (items) *items = B->n_items;
    if (shape) *shape = B->shape;
    if (grid) *grid = B->grid;
    if (order) *order = B->order;
    return PROCMV_OK;
}

procmv_status procmv_batch_configure(procmv_batch_t B, int32_t shape, int32_t grid,
                                     int32_t order)
{
    if (!B) return fail(PROCMV_ERR_INVALID_ARG, "null batch");
    if (shape < 0 || shape > 2 || grid < 1 || order < 0 || order > 1)
        return fail(PROCMV_ERR_INVALID_ARG, "bad launch configuration");
    B->shape = shape;
    B->grid = grid;
    if (order != B->order) {
        B->order = order;
        procmv_status st = batch_upload_items(B);
        if (st != PROCMV_OK) return st;
    }
    B->drop_graph();
    return PROCMV_OK;
}

// Packed X and Y of a batch must be disjoint.
bool batch_overlap(const procmv_batch* B, const void* X, const void* Y)
{
    const char* x = (const char*)X;
    const char* y = (const char*)Y;
    const size_t n = (size_t)B->total * sizeof(float2);
    return x < y + n && y < x + n;
}

procmv_status procmv_batch_apply(procmv_batch_t B, const void* X, void* Y, void* stream)
{
    if (!B) return fail(PROCMV_ERR_INVALID_ARG, "null batch");
    if (!X || !Y) return fail(PROCMV_ERR_INVALID_ARG, "bad vector pointers");
    if (batch_overlap(B, X, Y)) return fail(PROCMV_ERR_INVALID_ARG, "X and Y overlap");
    return batch_enqueue_apply(B, (const float2*)X, (float2*)Y, (hipStream_t)stream);
}

procmv_status procmv_batch_autotune(procmv_batch_t B, const void* X, void* Y, int32_t reps,
                                    void* stream, double* best_ms)
{
    if (!B) return fail(PROCMV_ERR_INVALID_ARG, "null batch");
    if (!X || !Y || reps < 1) return fail(PROCMV_ERR_INVALID_ARG, "bad arguments");
    if (batch_overlap(B, X, Y)) return fail(PROCMV_ERR_INVALID_ARG, "X and Y overlap");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 256;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best = 1e30;
    int bs = B->shape, bg = B->grid, bo = B->order;
    const int mults[4] = {1, 2, 4, 8};
    procmv_status st = PROCMV_OK;
    for (int order = 0; order < 2 && st == PROCMV_OK; ++order)
        for (int shape = 0; shape < 3 && st == PROCMV_OK; ++shape)
            for (int mi = 0; mi < 4 && st == PROCMV_OK; ++mi) {
                st = procmv_batch_configure(B, shape, cus * mults[mi], order);
                if (st != PROCMV_OK) break;
                st = batch_enqueue_apply(B, (const float2*)X, (float2*)Y, s);   // warm-up
                if (st != PROCMV_OK) break;
                if (hipEventRecord(e0, s) != hipSuccess) { st = PROCMV_ERR_HIP; break; }
                for (int r = 0; r < reps && st == PROCMV_OK; ++r)
                    st = batch_enqueue_apply(B, (const float2*)X, (float2*)Y, s);
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    st = fail(PROCMV_ERR_HIP, "autotune timing failed");
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const double t = ms / reps;
                if (t < best) {
                    best = t;
                    bs = shape;
                    bg = cus * mults[mi];
                    bo = order;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PROCMV_OK) return st;
    st = procmv_batch_configure(B, bs, bg, bo);
    if (best_ms) *best_ms = best;
    return st;
}

procmv_status procmv_batch_propagate(procmv_batch_t B, void* psi, double dt, int32_t K,
                                     int32_t nsteps, double spec_c, double spec_R,
                                     int32_t use_graph, double* norms_out, void* stream)
{
    if (!B) return fail(PROCMV_ERR_INVALID_ARG, "null batch");
    if (!psi || nsteps < 0 || !(dt >= 0.0) || !(spec_R > 0.0))
        return fail(PROCMV_ERR_INVALID_ARG, "bad psi/nsteps/dt/R");
    hipStream_t s = (hipStream_t)stream;
    const float alpha = f32_down(1.0 / spec_R);
    const double Reff = 1.0 / (double)alpha;
    if (K <= 0) K = procmv_cheb_order(Reff * dt, 1e-10);
    if (K < 1) return fail(PROCMV_ERR_INVALID_ARG, "Chebyshev order could not be set");
    procmv_status st;
    if (!B->d_q) {
        HIP_TRY(hipMalloc((void**)&B->d_q, (size_t)B->total * sizeof(float2)));
        HIP_TRY(hipMalloc((void**)&B->d_acc, (size_t)B->total * sizeof(double2)));
        HIP_TRY(hipMalloc((void**)&B->d_norm, (size_t)B->n * B->nv * sizeof(double)));
    }
    const std::vector<double> j = bessel_j(Reff * dt, K);
    std::vector<double2> a(K + 1);
    for (int k = 0; k <= K; ++k) {
        const double m = (k == 0 ? 1.0 : 2.0) * j[k];
        const int q = k & 3;
        a[k] = q == 0 ? double2{m, 0.0} : q == 1 ? double2{0.0, -m}
             : q == 2 ? double2{-m, 0.0} : double2{0.0, m};
    }
    const bool same = B->gexec && B->g_psi == psi && B->g_K == K && B->g_key[0] == dt &&
                      B->g_key[1] == spec_c && B->g_key[2] == spec_R;
    if (!same) {
        B->drop_graph();
        std::vector<BatchReduceItem>& ci = B->h_citems;
        ci.assign(B->n, BatchReduceItem{});
        for (int k = 0; k < B->n; ++k) {
            procmv_op* op = B->ops[k];
            ci[k] = BatchReduceItem{};
            ci[k].D = (int32_t)op->D;
            ci[k].n_slots = B->targs[k].n_super + 1;
            ci[k].off = B->off[k];
            ci[k].P = B->targs[k].P;
            ci[k].ldp = op->D;
            ci[k].alpha = alpha;
            const double dconst = op->gen == 1 ? op->d_const : 0.0;
            split_f32((double)alpha * (dconst - spec_c), ci[k].beta_hi, ci[k].beta_lo);
            ci[k].phase = double2{std::cos(spec_c * dt), -std::sin(spec_c * dt)};
        }
        // ordered on the caller's stream after any replay still reading it
        HIP_TRY(hipMemcpyAsync(B->d_citems, ci.data(), B->n * sizeof(BatchReduceItem),
                               hipMemcpyHostToDevice, (hipStream_t)stream));
    }
    // One Chebyshev step over every instance.
    auto enqueue_step = [&](hipStream_t q) -> procmv_status {
        float2* p0 = (float2*)psi;
        procmv_status e = batch_tiles(B, p0, q);
        if (e != PROCMV_OK) return e;
        BatchReduceArgs r = batch_rargs(B, B->d_citems);
        r.X = p0;
        r.Yq1 = B->d_q;
        r.acc = B->d_acc;
        r.a0 = a[0];
        r.a1 = a[1];
        HIP_TRY(launch_reduce_batched(r, Epi::kChebFirst, q));
        float2* cur = B->d_q;
        float2* prev = p0;
        for (int k = 1; k < K; ++k) {
            e = batch_tiles(B, cur, q);
            if (e != PROCMV_OK) return e;
            BatchReduceArgs rs = batch_rargs(B, B->d_citems);
            rs.X = cur;
            rs.Y = prev;
            rs.acc = B->d_acc;
            rs.a0 = a[k + 1];
            HIP_TRY(launch_reduce_batched(rs, Epi::kChebStep, q));
            std::swap(cur, prev);
        }
        HIP_TRY(launch_finish_batched(B->d_citems, B->n, B->nv, B->d_acc, p0, B->d_norm, q));
        return PROCMV_OK;
    };
    if (use_graph) {
        if (!same) {
            if (!B->cap) HIP_TRY(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
            HIP_TRY(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
            st = enqueue_step(B->cap);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(B->cap, &g);
            if (st != PROCMV_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (ec != hipSuccess)
                return fail(PROCMV_ERR_HIP, "graph capture: %s", hipGetErrorString(ec));
            B->graph = g;
            HIP_TRY(hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0));
            B->g_psi = psi;
            B->g_K = K;
            B->g_key[0] = dt;
            B->g_key[1] = spec_c;
            B->g_key[2] = spec_R;
        }
        for (int step = 0; step < nsteps; ++step) HIP_TRY(hipGraphLaunch(B->gexec, s));
    } else {
        for (int step = 0; step < nsteps; ++step) {
            st = enqueue_step(s);
            if (st != PROCMV_OK) return st;
        }
    }
    if (norms_out && nsteps > 0) {
        std::vector<double> n2((size_t)B->n * B->nv);
        HIP_TRY(hipMemcpyAsync(n2.data(), B->d_norm, n2.size() * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (size_t q = 0; q < n2.size(); ++q) norms_out[q] = std::sqrt(n2[q]);
    }
    return PROCMV_OK;
}

procmv_status procmv_set_dvr_kernel(procmv_op_t H, int32_t kind)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (kind < 0 || kind > 3) return fail(PROCMV_ERR_INVALID_ARG, "kernel kind %d", kind);
    H->dvr_kernel = kind;
    return PROCMV_OK;
}

int32_t procmv_tile_shape_fit(int32_t nvec, int32_t shape, int64_t D, int32_t cache_block)
{
    if ((nvec != 1 && nvec != 2 && nvec != 4 && nvec != 8) || shape < 0 || shape > 2 || D < 1 ||
        cache_block < 0 || (cache_block > 0 && cache_block % 64 != 0))
        return -1;
    return fit_tile_shape(nvec, shape, super_edge_tiles(D), cache_block);
}

procmv_status procmv_set_tile_shape(procmv_op_t H, int32_t shape)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (shape < -1 || shape > 2) return fail(PROCMV_ERR_INVALID_ARG, "tile shape %d", shape);
    H->tile_shape = shape;
    return PROCMV_OK;
}

procmv_status procmv_autotune(procmv_op_t H, int32_t nvec, int32_t reps, void* stream,
                              int32_t* shape_out, double* best_ms)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (!H->planned) return fail(PROCMV_ERR_NOT_PLANNED, "autotune before procmv_plan");
    if (nvec < 1 || reps < 1) return fail(PROCMV_ERR_INVALID_ARG, "bad nvec/reps");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)nvec * H->D * sizeof(float2);
    void *X = nullptr, *Y = nullptr;
    HIP_TRY(hipMalloc(&X, bytes));
    if (hipMalloc(&Y, bytes) != hipSuccess) {
        (void)hipFree(X);
        return fail(PROCMV_ERR_OOM, "autotune scratch vectors");
    }
    (void)hipMemsetAsync(X, 0, bytes, s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e30;
    int bshape = H->tile_shape;
    for (int shape = -1; shape < 3 && st == PROCMV_OK; ++shape) {
        H->tile_shape = shape;
        st = procmv_apply(H, X, H->D, Y, H->D, nvec, stream);
        if (st != PROCMV_OK) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == PROCMV_OK; ++r)
            st = procmv_apply(H, X, H->D, Y, H->D, nvec, stream);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
            st = fail(PROCMV_ERR_HIP, "autotune timing failed");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms / reps < best) {
            best = ms / reps;
            bshape = shape;
        }
    }
    H->tile_shape = bshape;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(X);
    (void)hipFree(Y);
    if (st != PROCMV_OK) return st;
    if (shape_out) *shape_out = bshape;
    if (best_ms) *best_ms = best;
    return PROCMV_OK;
}

}  // extern "C"

extern "C" {

procmv_status procmv_measure(procmv_generator gen, uint64_t seed, int64_t D,
                             const void* gen_params, int32_t nvec, int32_t block_size,
                             procmv_strategy strategy, double cache_fraction,
                             procmv_precision precision, int32_t warmup, int32_t reps,
                             void* stream, double* t_fill_ms, double* t_apply_ms)
{
    if (nvec < 1 || warmup < 0 || reps < 1)
        return fail(PROCMV_ERR_INVALID_ARG, "bad nvec/warmup/reps");
    hipStream_t s = (hipStream_t)stream;
    procmv_op_t H = nullptr;
    procmv_status st = procmv_create_operator(gen, seed, D, gen_params, &H);
    if (st != PROCMV_OK) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *X = nullptr, *Y = nullptr;
    const size_t bytes = (size_t)nvec * D * sizeof(float2);
    float ms = 0.f;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (X) (void)hipFree(X);
        if (Y) (void)hipFree(Y);
        procmv_destroy(H);
    };
    {
        hipError_t ee = hipFree(nullptr);   // make sure the device context exists
        if (ee == hipSuccess) ee = hipEventCreate(&e0);
        if (ee == hipSuccess) ee = hipEventCreate(&e1);
        if (ee != hipSuccess) {
            cleanup();
            return fail(PROCMV_ERR_HIP, "event creation failed: %s", hipGetErrorString(ee));
        }
    }
    st = procmv_plan(H, block_size, strategy, cache_fraction, precision, stream);
    if (st != PROCMV_OK) { cleanup(); return st; }
    // fill time: the fill kernels once more on the allocated slots
    if (t_fill_ms) *t_fill_ms = 0.0;
    if (H->p_cache > 0) {
        if (hipEventRecord(e0, s) != hipSuccess) { cleanup(); return fail(PROCMV_ERR_HIP, "event"); }
        const hipError_t fe = launch_cache_fill(H->source(), (int32_t)D, H->d_pairs, H->p_cache,
                                                H->d_slots, s);
        if (fe != hipSuccess) { cleanup(); return fail(PROCMV_ERR_HIP, "fill: %s", hipGetErrorString(fe)); }
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (t_fill_ms) *t_fill_ms = ms;
    }
    if (hipMalloc(&X, bytes) != hipSuccess || hipMalloc(&Y, bytes) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return fail(PROCMV_ERR_OOM, "vectors do not fit");
    }
    (void)hipMemsetAsync(X, 0, bytes, s);
    for (int r = 0; r < warmup; ++r) {
        st = procmv_apply(H, X, D, Y, D, nvec, stream);
        if (st != PROCMV_OK) { cleanup(); return st; }
    }
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) {
        st = procmv_apply(H, X, D, Y, D, nvec, stream);
        if (st != PROCMV_OK) { cleanup(); return st; }
    }
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) { cleanup(); return fail(PROCMV_ERR_HIP, "sync"); }
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (t_apply_ms) *t_apply_ms = (double)ms / reps;
    cleanup();
    return PROCMV_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Planner surrogate: training and inference on the GPU.
// ------------------------------------------------------------------------
namespace {

struct MlpWork {
    float *p = nullptr, *z = nullptr, *t = nullptr, *y = nullptr, *a1 = nullptr, *a2 = nullptr;
    float *gy = nullptr, *ga1 = nullptr, *ga2 = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float* loss = nullptr;
    ~MlpWork()
    {
        for (float* q : {p, z, t, y, a1, a2, gy, ga1, ga2, g, m, v, loss}) if (q) (void)hipFree(q);
    }
};

procmv_status mlp_setup(MlpWork& w, const float* params, const float* z, const float* t, int n)
{
    const size_t P = kMlpParams * sizeof(float), N = (size_t)n * sizeof(float);
    const size_t H = (size_t)n * kMlpHidden * sizeof(float);
    HIP_TRY(hipMalloc((void**)&w.p, P));
    HIP_TRY(hipMalloc((void**)&w.g, P));
    HIP_TRY(hipMalloc((void**)&w.m, P));
    HIP_TRY(hipMalloc((void**)&w.v, P));
    HIP_TRY(hipMalloc((void**)&w.z, N * kMlpIn));
    HIP_TRY(hipMalloc((void**)&w.t, N));
    HIP_TRY(hipMalloc((void**)&w.y, N));
    HIP_TRY(hipMalloc((void**)&w.gy, N));
    HIP_TRY(hipMalloc((void**)&w.a1, H));
    HIP_TRY(hipMalloc((void**)&w.a2, H));
    HIP_TRY(hipMalloc((void**)&w.ga1, H));
    HIP_TRY(hipMalloc((void**)&w.ga2, H));
    HIP_TRY(hipMalloc((void**)&w.loss, sizeof(float)));
    HIP_TRY(hipMemcpy(w.p, params, P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w.z, z, N * kMlpIn, hipMemcpyHostToDevice));
    if (t) HIP_TRY(hipMemcpy(w.t, t, N, hipMemcpyHostToDevice));
    std::vector<float> zero(kMlpParams, 0.f);
    HIP_TRY(hipMemcpy(w.m, zero.data(), P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w.v, zero.data(), P, hipMemcpyHostToDevice));
    return PROCMV_OK;
}

}  // namespace

extern "C" {

int32_t procmv_mlp_param_count(void) { return kMlpParams; }

procmv_status procmv_mlp_grad(const float* params, const float* z, const float* t, int32_t n,
                              float* grad_out, float* loss_out)
{
    if (!params || !z || !t || !grad_out || n < 1)
        return fail(PROCMV_ERR_INVALID_ARG, "bad surrogate arguments");
    MlpWork w;
    procmv_status st = mlp_setup(w, params, z, t, n);
    if (st != PROCMV_OK) return st;
    HIP_TRY(launch_mlp_forward(w.p, w.z, n, w.y, w.a1, w.a2, nullptr));
    HIP_TRY(launch_mlp_loss(w.y, w.t, n, w.loss, nullptr));
    HIP_TRY(launch_mlp_backward(w.p, w.z, w.y, w.t, n, w.a1, w.a2, w.gy, w.ga1, w.ga2, w.g,
                                nullptr));
    HIP_TRY(hipMemcpy(grad_out, w.g, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
    if (loss_out) HIP_TRY(hipMemcpy(loss_out, w.loss, sizeof(float), hipMemcpyDeviceToHost));
    return PROCMV_OK;
}

procmv_status procmv_mlp_train(const float* z, const float* t, int32_t n, int32_t epochs,
                               float lr, float* params_inout, float* loss_hist)
{
    if (!params_inout || !z || !t || n < 1 || epochs < 0 || !(lr > 0.f))
        return fail(PROCMV_ERR_INVALID_ARG, "bad surrogate arguments");
    MlpWork w;
    procmv_status st = mlp_setup(w, params_inout, z, t, n);
    if (st != PROCMV_OK) return st;
    for (int e = 1; e <= epochs; ++e) {
        HIP_TRY(launch_mlp_forward(w.p, w.z, n, w.y, w.a1, w.a2, nullptr));
        if (loss_hist) {
            HIP_TRY(launch_mlp_loss(w.y, w.t, n, w.loss, nullptr));
            HIP_TRY(hipMemcpy(&loss_hist[e - 1], w.loss, sizeof(float), hipMemcpyDeviceToHost));
        }
        HIP_TRY(launch_mlp_backward(w.p, w.z, w.y, w.t, n, w.a1, w.a2, w.gy, w.ga1, w.ga2,
                                    w.g, nullptr));
        HIP_TRY(launch_mlp_adam(w.p, w.g, w.m, w.v, lr, e, nullptr));
    }
    HIP_TRY(hipMemcpy(params_inout, w.p, kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
    return PROCMV_OK;
}

procmv_status procmv_mlp_predict(const float* params, const float* z, int32_t n, float* y_out)
{
    if (!params || !z || !y_out || n < 1)
        return fail(PROCMV_ERR_INVALID_ARG, "bad surrogate arguments");
    MlpWork w;
    procmv_status st = mlp_setup(w, params, z, nullptr, n);
    if (st != PROCMV_OK) return st;
    HIP_TRY(launch_mlp_forward(w.p, w.z, n, w.y, nullptr, nullptr, nullptr));
    HIP_TRY(hipMemcpy(y_out, w.y, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
    return PROCMV_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------
// Execution planner (paper Sec. IV: Algorithm 1 analytic, Algorithm 3
// learned, and the measured exhaustive search that scores both).
// ------------------------------------------------------------------------
namespace {

constexpr int kPlanBlocks[6] = {128, 256, 512, 1024, 2048, 4096};
constexpr int kPlanModes = 5;   // procedural, partial 0.25 / 0.5 / 0.75, full
constexpr double kPlanAlpha = 0.9;

void plan_candidate(int idx, int32_t& b, int32_t& strategy, double& f)
{
    b = kPlanBlocks[idx / kPlanModes];
    const int m = idx % kPlanModes;
    strategy = m == 0 ? PROCMV_PROCEDURAL : m == 4 ? PROCMV_FULL : PROCMV_PARTIAL;
    f = m == 0 ? 0.0 : m == 4 ? 1.0 : 0.25 * m;
}

// Memory of a plan: cache (Eq. planner_partial_cache / planner_full_cache
// over canonical pairs) and workspace (Eq. planner_workspace: partial slots
// plus input, output and, for repeated use, the Chebyshev vectors).
void plan_memory(int64_t D, int32_t nvec, int family, int32_t b, int32_t strategy, double f,
                 int64_t reuse, double& m_op, double& m_work)
{
    const int64_t nb = (D + b - 1) / b;
    const int64_t npair = nb * (nb + 1) / 2;
    int64_t p = 0;
    if (strategy == PROCMV_FULL) p = npair;
    else if (strategy == PROCMV_PARTIAL) p = (int64_t)std::floor(f * (double)npair);
    const double be = family == 0 ? 8.0 : 4.0;
    m_op = (double)p * b * b * be;
    const int64_t ns = (D + 64 * super_edge_tiles(D) - 1) / (64 * super_edge_tiles(D));
    const bool mfma = mfma_path(family, strategy == PROCMV_PROCEDURAL, strategy == PROCMV_FULL,
                                PROCMV_FP32, nvec);
    // vector block of one launch (the matrix-core block is counted at its
    // largest, 16: a bound on the partial buffer for every nvec)
    const int chunk = mfma ? 16 : nvec >= 8 ? 8 : nvec >= 4 ? 4 : nvec >= 2 ? 2 : 1;
    const double slots = (family == 1 && strategy == PROCMV_PROCEDURAL && !mfma)
                             ? (double)((D + 511) / 512) : (double)(ns + 1);
    m_work = slots * chunk * D * 8.0 + 2.0 * nvec * D * 8.0;
    if (reuse > 1) m_work += (double)nvec * D * (8.0 + 16.0);
}

void plan_features(int64_t D, int32_t nvec, double budget, int64_t reuse, int family,
                   int32_t b, int32_t strategy, double f, float* x, double* m_tot)
{
    double mo, mw;
    plan_memory(D, nvec, family, b, strategy, f, reuse, mo, mw);
    x[0] = (float)std::log2((double)D);
    x[1] = (float)std::log2((double)nvec);
    x[2] = (float)std::log2(1.0 + mo / 1e6);          // cache size (MB): fill work
    x[3] = (float)std::log2((double)reuse);
    x[4] = (float)family;
    x[5] = (float)std::log2((double)b);
    x[6] = (float)(strategy == PROCMV_PROCEDURAL ? 0.0 : strategy == PROCMV_FULL ? 1.0 : f);
    x[7] = (float)((mo + mw) / budget);
    if (m_tot) *m_tot = mo + mw;
}

}  // namespace

extern "C" {

int32_t procmv_plan_candidate_count(void)
{
    return (int32_t)(sizeof(kPlanBlocks) / sizeof(kPlanBlocks[0])) * kPlanModes;
}

procmv_status procmv_plan_candidate(int32_t idx, int32_t* block_size, int32_t* strategy,
                                    double* cache_fraction)
{
    if (idx < 0 || idx >= procmv_plan_candidate_count() || !block_size || !strategy ||
        !cache_fraction)
        return fail(PROCMV_ERR_INVALID_ARG, "bad candidate index");
    plan_candidate(idx, *block_size, *strategy, *cache_fraction);
    return PROCMV_OK;
}

procmv_status procmv_plan_features(int64_t D, int32_t nvec, double budget_bytes, int64_t reuse,
                                   int32_t family, int32_t block_size, int32_t strategy,
                                   double cache_fraction, float* x_out, double* m_tot_out,
                                   int32_t* feasible_out)
{
    if (D < 1 || nvec < 1 || !(budget_bytes > 0) || reuse < 1 || !x_out)
        return fail(PROCMV_ERR_INVALID_ARG, "bad planning problem");
    double mt = 0.0;
    plan_features(D, nvec, budget_bytes, reuse, family, block_size, strategy, cache_fraction,
                  x_out, &mt);
    if (m_tot_out) *m_tot_out = mt;
    if (feasible_out) *feasible_out = mt <= kPlanAlpha * budget_bytes ? 1 : 0;
    return PROCMV_OK;
}

procmv_status procmv_plan_model_time(const procmv_machine_model* mm, int64_t D, int32_t nvec,
                                     int32_t family, int32_t block_size, int32_t strategy,
                                     double cache_fraction, int64_t reuse, double* t_fill_s,
                                     double* t_apply_s)
{
    if (!mm || D < 1 || nvec < 1 || reuse < 1)
        return fail(PROCMV_ERR_INVALID_ARG, "bad planning problem");
    double mo, mw;
    plan_memory(D, nvec, family, block_size, strategy, cache_fraction, reuse, mo, mw);
    const double be = family == 0 ? 8.0 : 4.0;
    const double cached_entries = mo / be;
    const double canon = 0.5 * (double)D * (double)(D + 1);
    const double gen_entries = std::max(0.0, canon - cached_entries);
    const bool mfma = mfma_path(family, strategy == PROCMV_PROCEDURAL, strategy == PROCMV_FULL,
                                PROCMV_FP32, nvec);
    int chunks = 0;                 // launches: blocks of 16 (MFMA) or 8/4/2/1 (VALU)
    for (int r = nvec; r > 0; ++chunks)
        r -= mfma ? std::min(r, 16) : r >= 8 ? 8 : r >= 4 ? 4 : r >= 2 ? 2 : 1;
    double t_src;
    if (family == 1 && strategy == PROCMV_PROCEDURAL && !mfma)
        t_src = (double)D * D * nvec / mm->dvr_rate;   // Toeplitz kernel, per vector
    else
        t_src = chunks * (gen_entries / mm->gen_rate[family] + mo / mm->cache_bw);
    const double t_flop = 8.0 * (double)D * D * nvec / mm->flop_rate;
    const double ta = mm->launch_s + std::max(t_src, t_flop);
    const double tf = cached_entries / mm->gen_rate[family] + mo / mm->cache_bw;
    if (t_fill_s) *t_fill_s = tf;
    if (t_apply_s) *t_apply_s = ta;
    return PROCMV_OK;
}

procmv_status procmv_plan_rank(int32_t planner, const procmv_machine_model* mm,
                               const float* mlp_params, const float* mlp_norm, int64_t D,
                               int32_t nvec, double budget_bytes, int64_t reuse,
                               int32_t family, int32_t* order_out, double* score_out,
                               int32_t* n_out)
{
    if (D < 1 || nvec < 1 || reuse < 1 || !(budget_bytes > 0.0) || (family != 0 && family != 1))
        return fail(PROCMV_ERR_INVALID_ARG, "bad planning problem");
    const int nc = procmv_plan_candidate_count();
    std::vector<float> feats;
    std::vector<int> ids;
    for (int q = 0; q < nc; ++q) {
        int32_t b, st;
        double f;
        plan_candidate(q, b, st, f);
        if (b > D && b != kPlanBlocks[0]) continue;
        float x[kMlpIn];
        double mt;
        plan_features(D, nvec, budget_bytes, reuse, family, b, st, f, x, &mt);
        if (mt > kPlanAlpha * budget_bytes) continue;   // Eq. planner_memory_constraint
        ids.push_back(q);
        feats.insert(feats.end(), x, x + kMlpIn);
    }
    if (ids.empty()) return fail(PROCMV_ERR_INFEASIBLE_PLAN, "no plan fits the memory budget");
    std::vector<double> score(ids.size());
    if (planner == 0) {
        if (!mm) return fail(PROCMV_ERR_INVALID_ARG, "analytic planner needs a machine model");
        for (size_t k = 0; k < ids.size(); ++k) {
            int32_t b, st;
            double f, tf, ta;
            plan_candidate(ids[k], b, st, f);
            procmv_status e = procmv_plan_model_time(mm, D, nvec, family, b, st, f, reuse, &tf, &ta);
            if (e != PROCMV_OK) return e;
            score[k] = tf + (double)reuse * ta;
        }
    } else if (planner == 1) {
        if (!mlp_params || !mlp_norm)
            return fail(PROCMV_ERR_INVALID_ARG, "learned planner needs trained parameters");
        for (size_t k = 0; k < ids.size(); ++k)
            for (int i = 0; i < kMlpIn; ++i) {
                float& v = feats[k * kMlpIn + i];
                v = (v - mlp_norm[i]) / mlp_norm[kMlpIn + i];
            }
        std::vector<float> y(ids.size());
        procmv_status e = procmv_mlp_predict(mlp_params, feats.data(), (int32_t)ids.size(), y.data());
        if (e != PROCMV_OK) return e;
        for (size_t k = 0; k < ids.size(); ++k) score[k] = std::exp((double)y[k]);
    } else {
        return fail(PROCMV_ERR_INVALID_ARG, "ranking planner must be 0 (analytic) or 1 (learned)");
    }
    // ascending score; equal scores keep candidate order
    std::vector<size_t> ord(ids.size());
    for (size_t k = 0; k < ord.size(); ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](size_t a, size_t b) { return score[a] < score[b]; });
    for (size_t k = 0; k < ord.size(); ++k) {
        if (order_out) order_out[k] = ids[ord[k]];
        if (score_out) score_out[k] = score[ord[k]];
    }
    if (n_out) *n_out = (int32_t)ord.size();
    return PROCMV_OK;
}

procmv_status procmv_plan_choose(int32_t planner, const procmv_machine_model* mm,
                                 const float* mlp_params, const float* mlp_norm, int64_t D,
                                 int32_t nvec, double budget_bytes, int64_t reuse,
                                 int32_t family, int32_t* best_idx, double* best_score)
{
    if (planner == 2 || planner == 3)
        return fail(PROCMV_ERR_INVALID_ARG,
                    "measured selection (planner %d) times plans of an operator: "
                    "use procmv_plan_auto", planner);
    int32_t order[64];
    double score[64];
    int32_t n = 0;
    procmv_status st = procmv_plan_rank(planner, mm, mlp_params, mlp_norm, D, nvec, budget_bytes,
                                        reuse, family, order, score, &n);
    if (st != PROCMV_OK) return st;
    if (best_idx) *best_idx = order[0];
    if (best_score) *best_score = score[0];
    return PROCMV_OK;
}

procmv_status procmv_plan_auto(procmv_op_t H, int32_t nvec, double budget_bytes,
                               int64_t reuse, int32_t planner, const procmv_machine_model* mm,
                               const float* mlp_params, const float* mlp_norm, void* stream,
                               int32_t* chosen_idx)
{
    procmv_status st = check_op(H);
    if (st != PROCMV_OK) return st;
    if (planner < 0 || planner > 3)
        return fail(PROCMV_ERR_INVALID_ARG, "planner must be 0, 1, 2 or 3");
    // Algorithms 1 / 3 (direct): the best-ranked candidate.  Algorithm 2
    // (planner 2) and the hybrid of Algorithm 3 (planner 3): the analytic or
    // learned ranking keeps its K_bench best, each is timed on this
    // operator's generator, and the smallest measured t_fill + reuse t_apply
    // wins (Eq. bench_argmin with one task: W = 1).
    int32_t order[64];
    double score[64];
    int32_t n = 0;
    st = procmv_plan_rank(planner == 2 ? 0 : planner == 3 ? 1 : planner, mm, mlp_params,
                          mlp_norm, H->D, nvec, budget_bytes, reuse, H->gen, order, score, &n);
    if (st != PROCMV_OK) return st;
    int32_t idx = order[0];
    if (planner >= 2) {
        const int kb = std::min<int32_t>(n, PROCMV_PLAN_K_BENCH);
        double best = INFINITY;
        const void* gp = H->gen == PROCMV_GEN_SINC_DVR ? (const void*)&H->dvr : nullptr;
        for (int k = 0; k < kb; ++k) {
            int32_t b, s;
            double f, tf = 0.0, ta = 0.0;
            plan_candidate(order[k], b, s, f);
            st = procmv_measure((procmv_generator)H->gen, H->seed, H->D, gp, nvec, b,
                                (procmv_strategy)s, f, PROCMV_FP32, 1, 3, stream, &tf, &ta);
            if (st == PROCMV_ERR_OOM) continue;          // does not fit after all
            if (st != PROCMV_OK) return st;
            const double t = tf + (double)reuse * ta;
            if (t < best) {
                best = t;
                idx = order[k];
            }
        }
        if (!(best < INFINITY))
            return fail(PROCMV_ERR_INFEASIBLE_PLAN, "no ranked plan could be measured");
    }
    int32_t b, s;
    double f;
    plan_candidate(idx, b, s, f);
    st = procmv_plan(H, b, (procmv_strategy)s, f, PROCMV_FP32, stream);
    if (st == PROCMV_OK && chosen_idx) *chosen_idx = idx;
    return st;
}

}  // extern "C"

