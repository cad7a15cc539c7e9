/*
 * Plain CPU oracle for the block-procedural matrix-free product phi = H psi.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load.  The GPU library never links, includes or calls it, and it
 * shares no code, header or constant table with the GPU library.
 *
 * What it computes (paper: Sec. II, Eqs. blockmatvec / blockmatvecindex):
 * the ordinary dense product y_i = sum_j H_ij x_j, written out row by row in
 * binary64, with the matrix entries produced on the fly by the generators
 * below.  There is no blocking, tiling or Hermitian reuse here: every entry of
 * every requested row is generated and multiplied once.
 *
 * Generators (paper: Sec. III "Seeded generation" and "Analytic generation";
 * partition invariance: Sec. II, entries keyed on global row/column indices):
 *
 *  - Philox-GUE.  Counter-based Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *    "Parallel random numbers: as easy as 1, 2, 3", SC'11) keyed on the seed,
 *    counter (min(i,j), max(i,j), 0, 0).  Words x0, x1 become two uniforms
 *    u = (2*(x>>9)+1) * 2^-24 and a Box-Muller pair (z0, z1).  The upper
 *    entry is H_ij = s_off*(z0 + i z1) for i<j, H_ji = conj(H_ij), and the
 *    diagonal is H_ii = s_diag*z0.  The FP32 evaluation order below is the
 *    generator's definition: a fixed sequence of IEEE binary32 operations
 *    (own ln and sin/cos polynomials, correctly rounded division and sqrt),
 *    so that any faithful implementation reproduces it bit for bit.
 *
 *  - Sinc-DVR (Colbert-Miller) harmonic oscillator.  Off-diagonal kinetic
 *    entries T_k = (-1)^k / (m dx^2 k^2), k = i-j != 0, diagonal kinetic
 *    constant pi^2/(6 m dx^2), potential V_i = m w^2 x_i^2 / 2.  The FP32
 *    entries are the binary64 values rounded once; the constant diagonal is
 *    kept in binary64 (see the DVR table routine).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math (no contraction,
 * so that every fmaf below is the only fused operation).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11 definition: multipliers, Weyl key increments).       */
/* ------------------------------------------------------------------------ */
#define PHX_M0 0xD2511F53u
#define PHX_M1 0xCD9E8D57u
#define PHX_W0 0x9E3779B9u
#define PHX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHX_W0; k1 += PHX_W1; }
        uint64_t p0 = (uint64_t)PHX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* FP32 building blocks of the Gaussian transform.                           */
/* ------------------------------------------------------------------------ */
static inline uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static inline float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* 24-bit odd numerator over 2^24: strictly inside (0,1), exact in binary32. */
float orc_u01(uint32_t x)
{
    return (float)((x >> 9) * 2u + 1u) * 5.9604644775390625e-8f; /* 2^-24 */
}

/* Natural log for u in (0,1): u = 2^e m, m in [sqrt(1/2), sqrt(2)],
 * ln m = 2 atanh(s), s = (m-1)/(m+1), odd series 2s + 2s^3/3 + ... + 2s^9/9. */
float orc_logf32(float u)
{
    uint32_t b = f2u(u);
    int e = (int)(b >> 23) - 127;
    float m = u2f((b & 0x007FFFFFu) | 0x3F800000u);
    if (m > 1.41421356237309504880f) { m = m * 0.5f; e = e + 1; }
    float f = m - 1.0f;
    float s = f / (2.0f + f);
    float s2 = s * s;
    float p = fmaf(s2, (float)(2.0 / 9.0), (float)(2.0 / 7.0));
    p = fmaf(s2, p, (float)(2.0 / 5.0));
    p = fmaf(s2, p, (float)(2.0 / 3.0));
    float lm = fmaf(s * s2, p, 2.0f * s);
    float ef = (float)e;
    /* ln 2 split into its binary32 rounding and the rounding residual. */
    const float LN2_HI = 0.693147180559945309417f;
    const float LN2_LO = (float)(0.693147180559945309417232121458 -
                                 (double)0.693147180559945309417f);
    return fmaf(ef, LN2_HI, fmaf(ef, LN2_LO, lm));
}

/* sin(2 pi u), cos(2 pi u) for u in (0,1) a multiple of 2^-24.
 * Quarter-turn reduction u = n/4 + r, |r| <= 1/8 (exact), then Taylor
 * polynomials of sin(2 pi r) (to r^9) and cos(2 pi r) (to r^10). */
void orc_sincos2pi_f32(float u, float* s_out, float* c_out)
{
    float n = rintf(4.0f * u);
    float r = fmaf(n, -0.25f, u);
    float r2 = r * r;
    /* Taylor coefficients (2 pi)^k / k!, alternating signs. */
    const float S1 = 6.28318530717958647692f;
    const float S3 = -41.3417022403997602340f;
    const float S5 = 81.6052492760750542034f;
    const float S7 = -76.7058597530613858416f;
    const float S9 = 42.0586939448976531450f;
    const float C2 = -19.7392088021787172377f;
    const float C4 = 64.9393940226682914910f;
    const float C6 = -85.4568172066937277360f;
    const float C8 = 60.2446413718766603627f;
    const float C10 = -26.4262567833743974529f;
    float ps = fmaf(r2, S9, S7);
    ps = fmaf(r2, ps, S5);
    ps = fmaf(r2, ps, S3);
    ps = fmaf(r2, ps, S1);
    float sr = r * ps;
    float pc = fmaf(r2, C10, C8);
    pc = fmaf(r2, pc, C6);
    pc = fmaf(r2, pc, C4);
    pc = fmaf(r2, pc, C2);
    float cr = fmaf(r2, pc, 1.0f);
    int q = ((int)n) & 3;
    float sv, cv;
    if (q == 0)      { sv = sr;  cv = cr;  }
    else if (q == 1) { sv = cr;  cv = -sr; }
    else if (q == 2) { sv = -sr; cv = -cr; }
    else             { sv = -cr; cv = sr;  }
    *s_out = sv; *c_out = cv;
}

/* Box-Muller on two raw words: z0 = r cos(theta), z1 = r sin(theta),
 * r = sqrt(-2 ln u0), theta = 2 pi u1. */
void orc_box_muller_f32(uint32_t x0, uint32_t x1, float* z0, float* z1)
{
    float u0 = orc_u01(x0), u1 = orc_u01(x1);
    float l = orc_logf32(u0);
    float r = sqrtf(-2.0f * l);
    float sv, cv;
    orc_sincos2pi_f32(u1, &sv, &cv);
    *z0 = r * cv;
    *z1 = r * sv;
}

/* One canonical GUE entry (i <= j): returns re, im of H_ij. */
static inline void gue_canon(uint32_t k0, uint32_t k1, uint32_t i, uint32_t j,
                             float s_off, float s_diag, float* re, float* im)
{
    uint32_t ctr[4] = {i, j, 0u, 0u}, key[2] = {k0, k1}, x[4];
    orc_philox4x32_10(ctr, key, x);
    float z0, z1;
    orc_box_muller_f32(x[0], x[1], &z0, &z1);
    if (i == j) { *re = s_diag * z0; *im = 0.0f; }
    else        { *re = s_off * z0;  *im = s_off * z1; }
}

/* Entry H_ij for any (i, j): canonical draw, conjugated below the diagonal. */
void orc_gue_entry_f32(uint64_t seed, int64_t i, int64_t j, float s_off,
                       float s_diag, float* re, float* im)
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (i <= j) {
        gue_canon(k0, k1, (uint32_t)i, (uint32_t)j, s_off, s_diag, re, im);
    } else {
        gue_canon(k0, k1, (uint32_t)j, (uint32_t)i, s_off, s_diag, re, im);
        *im = -*im;
    }
}

/* Dense window of entries: out[(a*nc + b)*2 + {0,1}] = H_{r0+a, c0+b}. */
void orc_gue_entries_f32(uint64_t seed, int64_t r0, int64_t c0, int32_t nr,
                         int32_t nc, float s_off, float s_diag, float* out)
{
#pragma omp parallel for schedule(static)
    for (int32_t a = 0; a < nr; ++a)
        for (int32_t b = 0; b < nc; ++b) {
            float re, im;
            orc_gue_entry_f32(seed, r0 + a, c0 + b, s_off, s_diag, &re, &im);
            out[((int64_t)a * nc + b) * 2 + 0] = re;
            out[((int64_t)a * nc + b) * 2 + 1] = im;
        }
}

/* y_i = sum_j H_ij x_j in binary64 for the listed rows, every vector v.
 * X: complex128 interleaved, vector v at X + 2*v*ldx (ldx >= D).
 * Y: complex128 interleaved, Y[(v*nrows + r)*2 + {0,1}]. */
void orc_gue_apply_rows_f64(uint64_t seed, int64_t D, float s_off,
                            float s_diag, const double* X, int64_t ldx,
                            int32_t R, const int64_t* rows, int64_t nrows,
                            double* Y)
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        double acc[2 * 64];
        double* accp = acc;
        double* heap = NULL;
        if (R > 64) { heap = (double*)calloc((size_t)2 * R, sizeof(double)); accp = heap; }
        else memset(acc, 0, sizeof(acc));
        for (int64_t j = 0; j < D; ++j) {
            float re, im;
            if (i <= j) gue_canon(k0, k1, (uint32_t)i, (uint32_t)j, s_off, s_diag, &re, &im);
            else { gue_canon(k0, k1, (uint32_t)j, (uint32_t)i, s_off, s_diag, &re, &im); im = -im; }
            double hr = (double)re, hi = (double)im;
            for (int32_t v = 0; v < R; ++v) {
                double xr = X[2 * (v * ldx + j)], xi = X[2 * (v * ldx + j) + 1];
                accp[2 * v]     += hr * xr - hi * xi;
                accp[2 * v + 1] += hr * xi + hi * xr;
            }
        }
        for (int32_t v = 0; v < R; ++v) {
            Y[2 * (v * nrows + r)]     = accp[2 * v];
            Y[2 * (v * nrows + r) + 1] = accp[2 * v + 1];
        }
        free(heap);
    }
}

/* ------------------------------------------------------------------------ */
/* Sinc-DVR harmonic oscillator.                                             */
/* ------------------------------------------------------------------------ */

/* Tables of the operator H = T_off + diag(V) + d I on the grid
 * x_i = x_min + i dx, dx = (x_max - x_min)/(D-1):
 *   tk64[k] = (-1)^k / (m dx^2 k^2)  (k = 1..D-1; tk64[0] = 0)
 *   v64[i]  = (m w^2 / 2) x_i^2
 *   d0      = pi^2 / (6 m dx^2)       (kinetic diagonal constant)
 * and their binary32 roundings tk32, v32.  With `compensate`, the binary64
 * diagonal constant also absorbs the rounding error of the binary32
 * off-diagonals, d32 = d0 - 2 sum_k (tk32[k] - tk64[k]), so the rounded
 * operator keeps the exact zero row sum of the kinetic stencil on smooth
 * vectors (the FP32 table alone shifts the low energies by a constant).
 * d_out[0] = exact constant d0, d_out[1] = constant paired with tk32/v32. */
void orc_dvr_tables(int64_t D, double x_min, double x_max, double mass,
                    double omega, int32_t compensate, double* tk64,
                    double* v64, float* tk32, float* v32, double* d_out,
                    double* dx_out)
{
    double dx = (x_max - x_min) / (double)(D - 1);
    double inv_mdx2 = 1.0 / (mass * dx * dx);
    double kpot = 0.5 * mass * omega * omega;
    tk64[0] = 0.0; tk32[0] = 0.0f;
    double err = 0.0;
    for (int64_t k = 1; k < D; ++k) {
        double kk = (double)k * (double)k;
        double t = ((k & 1) ? -inv_mdx2 : inv_mdx2) / kk;
        tk64[k] = t;
        tk32[k] = (float)t;
        err += (double)tk32[k] - t;
    }
    for (int64_t i = 0; i < D; ++i) {
        double x = x_min + (double)i * dx;
        v64[i] = kpot * (x * x);
        v32[i] = (float)v64[i];
    }
    double d0 = (M_PI * M_PI / 6.0) * inv_mdx2;
    d_out[0] = d0;
    d_out[1] = compensate ? d0 - 2.0 * err : d0;
    *dx_out = dx;
}

/* y_i = sum_{j != i} tk[|i-j|] x_j + (v[i] + d) x_i in binary64 for the
 * listed rows (tk, v given in binary64: pass the rounded binary32 tables
 * promoted, or the exact ones). */
void orc_dvr_apply_rows_f64(const double* tk, const double* v, double d,
                            int64_t D, const double* X, int64_t ldx,
                            int32_t R, const int64_t* rows, int64_t nrows,
                            double* Y)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        for (int32_t v_ = 0; v_ < R; ++v_) {
            const double* x = X + 2 * v_ * ldx;
            double ar = 0.0, ai = 0.0;
            for (int64_t j = 0; j < D; ++j) {
                double h = (j == i) ? v[i] + d : tk[j > i ? j - i : i - j];
                ar += h * x[2 * j];
                ai += h * x[2 * j + 1];
            }
            Y[2 * (v_ * nrows + r)] = ar;
            Y[2 * (v_ * nrows + r) + 1] = ai;
        }
    }
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Elementwise forms of the FP32 building blocks, for exhaustive checks. */
void orc_logf32_vec(const float* u, int64_t n, float* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) out[k] = orc_logf32(u[k]);
}

void orc_sincos2pi_vec(const float* u, int64_t n, float* s, float* c)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) orc_sincos2pi_f32(u[k], &s[k], &c[k]);
}

void orc_box_muller_vec(const uint32_t* x0, const uint32_t* x1, int64_t n,
                        float* z0, float* z1)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) orc_box_muller_f32(x0[k], x1[k], &z0[k], &z1[k]);
}

/* Raw Philox words for a list of counters (n x 4) under one key. */
void orc_philox_vec(const uint32_t* ctr, int64_t n, uint32_t k0, uint32_t k1,
                    uint32_t* out)
{
    uint32_t key[2] = {k0, k1};
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) orc_philox4x32_10(ctr + 4 * k, key, out + 4 * k);
}
