/*
 * Oracle B in plain C: the improved-QFT recursion in FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  It exists to give the CPU baseline a compiled
 * implementation of the same eight functions as oracle/qft.py (Pasquini,
 * Sec. 5.2: cdft, rdft, dct, dst, dct_ot, dst_ot, dct_oo, dst_oo; Sec. 3 for
 * the basic elaborations).  It is never linked into the GPU library.
 *
 * Conventions (Table 1, tab:notation): every function receives the stored time
 * samples in increasing n and writes the stored frequency samples in
 * increasing k.  N is the periodization of the call and theta = 2*pi/N
 * (eq. qft_0D).  Build with -ffp-contract=off so that no multiply is fused
 * with an add.  Temporaries come from a per-thread workspace of 12N doubles
 * (a bump allocator; the deepest call chain needs about 7N), so the recursion
 * never calls malloc.  The secants 1/(2 cos(theta n)) of every periodization
 * are evaluated once per call of an entry point into a table (the same
 * expression, so the same FP64 values as evaluating them in place), slice P
 * (odd n = 2j+1 < P/4, j < P/8) at offset P/8 - 2 for P >= 16.
 *
 * Readings of the paper (same as the Python oracle): eq. qft_38B is applied
 * as DCT[s_dc_oo](N/4-1) = DCT[s_dc_oe](N/4-2); dst_oo's special case is at
 * k = 1; the secant is 1/(2 cos(theta n)) on odd n only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double* base;
    size_t top;
    const double* sec; /* secant table, see above */
    double c8, s8;     /* cos(2 pi/8), sin(2 pi/8): the N = 8 base cases */
} arena;

/* Secant table for periodizations 16 .. Nmax: slice P at offset P/8 - 2,
 * entry j = 1/(2 cos(2 pi (2j+1) / P)) (eq. qft_38A); Nmax/4 - 2 entries. */
static double* secant_table(int Nmax) {
    size_t n = Nmax >= 16 ? (size_t)Nmax / 4 - 2 : 1;
    double* t = (double*)malloc(sizeof(double) * n);
    if (!t) return NULL;
    for (int P = 16; P <= Nmax; P *= 2) {
        double* sl = t + P / 8 - 2;
        for (int j = 0; j < P / 8; ++j) {
            double n = 2.0 * j + 1.0;
            sl[j] = 1.0 / (2.0 * cos(2.0 * M_PI * n / P));
        }
    }
    return t;
}

static double* take(arena* a, size_t n) {
    double* p = a->base + a->top;
    a->top += n;
    return p;
}

static void dct_ot(const double* s, int N, double* S, arena* a);
static void dst_ot(const double* s, int N, double* S, arena* a);

/* dct_oo: s_dc_oo (odd n = 1..N/4-1, N/8 samples) -> odd k = 1..N/4-1. */
static void dct_oo(const double* s, int N, double* S, arena* a) {
    int m = N / 8;
    if (N == 8) { /* definition: cos(2 pi / 8) */
        S[0] = s[0] * a->c8;
        return;
    }
    size_t mark = a->top;
    double* t = take(a, m);
    double* T = take(a, m);
    const double* h = a->sec + N / 8 - 2;
    for (int j = 0; j < m; ++j) t[j] = s[j] * h[j]; /* eq. qft_38A on odd n = 2j+1 */
    /* even-harmonic halving: s_A_dc_ot of periodization N/2 (Sec. 3.3) */
    dct_ot(t, N / 2, T, a);
    /* eq. qft_38C for odd k = 2j+1 <= N/4-3, corrected eq. qft_38B at N/4-1 */
    for (int j = 0; j < m - 1; ++j) S[j] = T[j] + T[j + 1];
    S[m - 1] = T[m - 1];
    a->top = mark;
}

/* dct_ot: s_dc_ot (odd n = 1..N/2-1, N/4 samples) -> k = 0..N/4-1. */
static void dct_ot(const double* s, int N, double* S, arena* a) {
    int q = N / 4;
    if (N == 4) { S[0] = s[0]; return; }
    int m = N / 8;
    size_t mark = a->top;
    double* se = take(a, m);
    double* so = take(a, m);
    double* A = take(a, m);
    double* B = take(a, m);
    /* harmonic separation (Sec. 3.2, eqs. qft_1/qft_2): s(n) +- s(N/2-n) */
    for (int j = 0; j < m; ++j) {
        se[j] = s[j] + s[q - 1 - j];
        so[j] = s[j] - s[q - 1 - j];
    }
    dct_ot(se, N / 2, A, a); /* even k = 2 k_A (Sec. 3.3) */
    dct_oo(so, N, B, a);     /* odd k */
    for (int j = 0; j < m; ++j) { /* interleave, eq. qft_4B */
        S[2 * j] = A[j];
        S[2 * j + 1] = B[j];
    }
    a->top = mark;
}

/* dct: s_dc_tt (n = 0..N/2) -> DCT-0 (eq. qft_0B), k = 0..N/2. */
static void dct(const double* s, int N, double* S, arena* a) {
    if (N == 2) {
        S[0] = s[0] + s[1];
        S[1] = s[0] - s[1];
        return;
    }
    int q = N / 4;
    size_t mark = a->top;
    double* se = take(a, q + 1);
    double* so = take(a, q);
    double* E = take(a, q + 1);
    double* O = take(a, q);
    for (int j = 0; j <= q; ++j) se[j] = s[2 * j];     /* even n, halved */
    for (int j = 0; j < q; ++j) so[j] = s[2 * j + 1];  /* odd n */
    dct(se, N / 2, E, a);
    dct_ot(so, N, O, a);
    for (int k = 0; k < q; ++k) { /* eqs. qft_5C/5D */
        S[k] = E[k] + O[k];
        S[N / 2 - k] = E[k] - O[k];
    }
    S[q] = E[q]; /* eq. qft_6 */
    a->top = mark;
}

/* dst_oo: s_ds_oo (odd n = 1..N/4-1) -> odd k = 1..N/4-1. */
static void dst_oo(const double* s, int N, double* S, arena* a) {
    int m = N / 8;
    if (N == 8) {
        S[0] = s[0] * a->s8;
        return;
    }
    size_t mark = a->top;
    double* t = take(a, m);
    double* T = take(a, m);
    const double* h = a->sec + N / 8 - 2;
    for (int j = 0; j < m; ++j) t[j] = s[j] * h[j];
    dst_ot(t, N / 2, T, a); /* T[j] = DST[s_oe](2(j+1)) */
    S[0] = T[0];            /* k = 1: DST[s_oe](0) = 0 */
    for (int j = 1; j < m; ++j) S[j] = T[j - 1] + T[j];
    a->top = mark;
}

/* dst_ot: s_ds_ot (odd n = 1..N/2-1) -> k = 1..N/4 (stored at k-1). */
static void dst_ot(const double* s, int N, double* S, arena* a) {
    int q = N / 4;
    if (N == 4) { S[0] = s[0]; return; }
    int m = N / 8;
    size_t mark = a->top;
    double* se = take(a, m);
    double* so = take(a, m);
    double* A = take(a, m);
    double* B = take(a, m);
    for (int j = 0; j < m; ++j) { /* DST role swap of Sec. 3.2 */
        se[j] = s[j] - s[q - 1 - j];
        so[j] = s[j] + s[q - 1 - j];
    }
    dst_ot(se, N / 2, A, a); /* even k */
    dst_oo(so, N, B, a);     /* odd k */
    for (int j = 0; j < m; ++j) {
        S[2 * j] = B[j];     /* k = 2j+1 */
        S[2 * j + 1] = A[j]; /* k = 2j+2 */
    }
    a->top = mark;
}

/* dst: s_ds_tt (n = 1..N/2-1, stored at n-1) -> k = 1..N/2-1. */
static void dst(const double* s, int N, double* S, arena* a) {
    if (N == 4) { S[0] = s[0]; return; }
    int q = N / 4;
    size_t mark = a->top;
    double* se = take(a, q - 1);
    double* so = take(a, q);
    double* E = take(a, q - 1);
    double* O = take(a, q);
    for (int j = 0; j < q - 1; ++j) se[j] = s[2 * j + 1]; /* n = 2, 4, .. */
    for (int j = 0; j < q; ++j) so[j] = s[2 * j];         /* n = 1, 3, .. */
    dst(se, N / 2, E, a);
    dst_ot(so, N, O, a);
    for (int k = 1; k < q; ++k) { /* eqs. 5C/5D with the DST role swap */
        S[k - 1] = O[k - 1] + E[k - 1];
        S[N / 2 - k - 1] = O[k - 1] - E[k - 1];
    }
    S[q - 1] = O[q - 1]; /* eq. qft_6, DST case */
    a->top = mark;
}

/* rdft: real n = 0..N-1 -> re[k], k = 0..N/2 and im[k-1], k = 1..N/2-1. */
static void rdft(const double* s, int N, double* re, double* im, arena* a) {
    if (N == 2) {
        re[0] = s[0] + s[1];
        re[1] = s[0] - s[1];
        return;
    }
    int h = N / 2;
    size_t mark = a->top;
    double* c = take(a, h + 1);
    double* d = take(a, h - 1);
    double* D = take(a, h - 1);
    c[0] = s[0];
    c[h] = s[h];
    for (int n = 1; n < h; ++n) {
        c[n] = s[n] + s[N - n];
        d[n - 1] = s[n] - s[N - n];
    }
    dct(c, N, re, a);
    dst(d, N, D, a);
    for (int k = 0; k < h - 1; ++k) im[k] = -D[k];
    a->top = mark;
}

/* cdft on split storage: (xr, xi) -> (Xr, Xi), all length N. */
static void cdft(const double* xr, const double* xi, int N, double* Xr, double* Xi,
                 arena* a) {
    if (N == 2) {
        Xr[0] = xr[0] + xr[1]; Xi[0] = xi[0] + xi[1];
        Xr[1] = xr[0] - xr[1]; Xi[1] = xi[0] - xi[1];
        return;
    }
    int h = N / 2;
    size_t mark = a->top;
    double* r1 = take(a, h + 1);
    double* i1 = take(a, h);
    double* r2 = take(a, h + 1);
    double* i2 = take(a, h);
    rdft(xr, N, r1, i1, a);
    rdft(xi, N, r2, i2, a);
    Xr[0] = r1[0]; Xi[0] = r2[0];
    Xr[h] = r1[h]; Xi[h] = r2[h];
    for (int k = 1; k < h; ++k) { /* Sec. 4.1 combine */
        Xr[k] = r1[k] - i2[k - 1];
        Xi[k] = i1[k - 1] + r2[k];
        Xr[N - k] = r1[k] + i2[k - 1];
        Xi[N - k] = r2[k] - i1[k - 1];
    }
    a->top = mark;
}

/* Batched forward CDFT of `batch` signals of length N = 2^log2n, interleaved
 * complex (re, im) doubles, transform-major.  Signals are distributed over
 * OpenMP threads when built with -fopenmp.  Returns 0 on success, -1 on a bad
 * size, -2 when the workspace cannot be allocated. */
int qft_ref_cdft(const double* x, double* X, int log2n, int64_t batch) {
    if (log2n < 1 || log2n > 26 || batch < 0) return -1;
    const int N = 1 << log2n;
    double* sec = secant_table(N);
    if (!sec) return -2;
    const double c8 = cos(2.0 * M_PI / 8.0), s8 = sin(2.0 * M_PI / 8.0);
    int status = 0;
#pragma omp parallel
    {
        double* buf = (double*)malloc(sizeof(double) * (size_t)N * 16);
        if (!buf) {
#pragma omp atomic write
            status = -2;
        } else {
            double* xr = buf;
            double* xi = buf + N;
            double* Xr = buf + 2 * (size_t)N;
            double* Xi = buf + 3 * (size_t)N;
            arena a = {buf + 4 * (size_t)N, 0, sec, c8, s8};
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < batch; ++b) {
                const double* xb = x + 2 * (size_t)N * b;
                double* Xb = X + 2 * (size_t)N * b;
                for (int n = 0; n < N; ++n) { xr[n] = xb[2 * n]; xi[n] = xb[2 * n + 1]; }
                a.top = 0;
                cdft(xr, xi, N, Xr, Xi, &a);
                for (int k = 0; k < N; ++k) { Xb[2 * k] = Xr[k]; Xb[2 * k + 1] = Xi[k]; }
            }
            free(buf);
        }
    }
    free(sec);
    return status;
}

/* Batched DCT-0 (dct on s_dc_tt, N/2+1 samples -> N/2+1 frequencies) when
 * dst == 0, or DST-0 (dst on s_ds_tt, N/2-1 -> N/2-1) when dst != 0, of
 * `batch` real signals of periodization N = 2^log2n, contiguous per signal
 * (Sec. 5.2, eqs. qft_0B/qft_0C).  DST-0 needs N >= 4.  Returns as
 * qft_ref_cdft. */
int qft_ref_dct_dst(const double* s, double* S, int log2n, int64_t batch, int dst_side) {
    if (log2n < 1 || log2n > 26 || batch < 0 || (dst_side && log2n < 2)) return -1;
    const int N = 1 << log2n;
    const int len = dst_side ? N / 2 - 1 : N / 2 + 1;
    double* sec = secant_table(N);
    if (!sec) return -2;
    const double c8 = cos(2.0 * M_PI / 8.0), s8 = sin(2.0 * M_PI / 8.0);
    int status = 0;
#pragma omp parallel
    {
        double* buf = (double*)malloc(sizeof(double) * (size_t)N * 16);
        if (!buf) {
#pragma omp atomic write
            status = -2;
        } else {
            arena a = {buf, 0, sec, c8, s8};
#pragma omp for schedule(dynamic, 1)
            for (int64_t b = 0; b < batch; ++b) {
                a.top = 0;
                if (dst_side) dst(s + (size_t)len * b, N, S + (size_t)len * b, &a);
                else dct(s + (size_t)len * b, N, S + (size_t)len * b, &a);
            }
            free(buf);
        }
    }
    free(sec);
    return status;
}

/* Sets the number of OpenMP threads of later calls (the single-thread CPU
 * baseline uses 1). */
void qft_ref_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of threads the parallel region above uses. */
int qft_ref_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
