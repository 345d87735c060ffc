/*
 * Oracle for Low(A * phi(A)) over a prime field and over F_{p^2}.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or table with the GPU library.
 *
 * What it computes is the plain definition the paper's Algorithm 1 reaches
 * exactly (Theorem "complexitybound", proof of correctness, Section 3):
 *   C_ij = sum_t A_it * phi(A)_tj  reduced mod p, for 0 <= j <= i < n
 * with Low() as in the Low/Up definition of Section 2 (diagonal included).
 * phi = transpose gives C_ij = sum_t A_it A_jt.  phi = conjugate transpose
 * over F_p[i]/(i^2+1) (Section 2, examples of antihomomorphisms; Section 4.4
 * for the field) gives C_ij = sum_t A_it conj(A_jt) with conj(x+iy) = x-iy.
 *
 * Field helpers (Section 4): Legendre symbol by Euler's criterion, modular
 * square root by Tonelli-Shanks, and the sum-of-two-squares construction of
 * Algorithm 2 ("SoS").
 *
 * Accumulation is exact: int64 when k*(p-1)^2 < 2^63, __int128 otherwise,
 * one reduction per entry.  Rows are spread cyclically over OpenMP threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_EPRIME -2
#define ORC_ERANGE -3

typedef __int128 i128;

static int64_t canon128(i128 x, int64_t p)
{
    int64_t r = (int64_t)(x % (i128)p);
    return r < 0 ? r + p : r;
}

static int64_t canon64(int64_t x, int64_t p)
{
    int64_t r = x % p;
    return r < 0 ? r + p : r;
}

/* ---------------- field helpers (Section 4) ---------------- */

int oracle_is_prime(int64_t p)
{
    if (p < 2) return 0;
    if (p % 2 == 0) return p == 2;
    for (int64_t d = 3; d * d <= p; d += 2)
        if (p % d == 0) return 0;
    return 1;
}

int64_t oracle_powmod(int64_t b, int64_t e, int64_t p)
{
    int64_t r = 1 % p;
    b = canon64(b, p);
    while (e > 0) {
        if (e & 1) r = (int64_t)(((i128)r * b) % p);
        b = (int64_t)(((i128)b * b) % p);
        e >>= 1;
    }
    return r;
}

/* Legendre symbol (a/p) for an odd prime p via Euler's criterion: 0, 1 or -1. */
int oracle_legendre(int64_t a, int64_t p)
{
    a = canon64(a, p);
    if (a == 0) return 0;
    int64_t e = oracle_powmod(a, (p - 1) / 2, p);
    return e == 1 ? 1 : -1;
}

int64_t oracle_inverse(int64_t a, int64_t p)
{
    return oracle_powmod(a, p - 2, p); /* Fermat, p prime */
}

/* Square root of a quadratic residue a mod odd prime p by Tonelli-Shanks.
 * Returns the smaller of the two roots, or -1 if a is not a residue. */
int64_t oracle_sqrt_mod(int64_t a, int64_t p)
{
    a = canon64(a, p);
    if (a == 0) return 0;
    if (oracle_legendre(a, p) != 1) return -1;
    int64_t q = p - 1, s = 0;
    while ((q & 1) == 0) { q >>= 1; ++s; }
    int64_t z = 2;
    while (oracle_legendre(z, p) != -1) ++z;
    int64_t m = s;
    int64_t c = oracle_powmod(z, q, p);
    int64_t t = oracle_powmod(a, q, p);
    int64_t r = oracle_powmod(a, (q + 1) / 2, p);
    while (t != 1) {
        int64_t i = 0, tt = t;
        while (tt != 1) { tt = (int64_t)(((i128)tt * tt) % p); ++i; }
        int64_t b = c;
        for (int64_t j = 0; j < m - i - 1; ++j) b = (int64_t)(((i128)b * b) % p);
        m = i;
        c = (int64_t)(((i128)b * b) % p);
        t = (int64_t)(((i128)t * c) % p);
        r = (int64_t)(((i128)r * b) % p);
    }
    return r <= p - r ? r : p - r;
}

/* Algorithm 2 (SoS): (a, b) with a^2 + b^2 = k mod p.  When k is a square the
 * answer is (sqrt(k), 0).  Otherwise s is the least quadratic non-residue,
 * c = sqrt(s-1), r = k/s, a = sqrt(r), b = a*c.  Every sqrt takes the smaller
 * root.  Also reports the non-residue used (0 when k is a square). */
int oracle_sos(int64_t p, int64_t k, int64_t* a, int64_t* b, int64_t* s_used)
{
    if (p < 3 || !oracle_is_prime(p)) return ORC_EPRIME;
    k = canon64(k, p);
    if (oracle_legendre(k, p) >= 0) { /* k is a square (or zero) */
        *a = oracle_sqrt_mod(k, p);
        *b = 0;
        if (s_used) *s_used = 0;
        return ORC_OK;
    }
    int64_t s = 2;
    while (oracle_legendre(s, p) == 1) ++s;
    int64_t c = oracle_sqrt_mod(s - 1, p);
    int64_t r = (int64_t)(((i128)k * oracle_inverse(s, p)) % p);
    int64_t aa = oracle_sqrt_mod(r, p);
    *a = aa;
    *b = (int64_t)(((i128)aa * c) % p);
    if (s_used) *s_used = s;
    return ORC_OK;
}

/* ---------------- the product, transpose case ---------------- */

static int check_args(int64_t n, int64_t k, int64_t p, int64_t lda, int64_t ldc)
{
    if (n < 0 || k < 0) return ORC_EINVAL;
    if (p < 3 || !oracle_is_prime(p)) return ORC_EPRIME;
    if (n > 0 && k > 0 && lda < k) return ORC_EINVAL;
    if (n > 0 && ldc < n) return ORC_EINVAL;
    return ORC_OK;
}

static int range_ok(int64_t n, int64_t k, int64_t p, const int64_t* A, int64_t lda)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t t = 0; t < k; ++t)
            if (A[i * lda + t] < 0 || A[i * lda + t] >= p) return 0;
    return 1;
}

/* C_ij = (sum_t A_it A_jt) mod p for j <= i (full != 0: every j).
 * A: n x k canonical residues, row-major with stride lda.  C: row-major, ldc. */
int oracle_syrk_modp(int64_t n, int64_t k, int64_t p, const int64_t* A, int64_t lda,
                     int64_t* C, int64_t ldc, int full)
{
    int st = check_args(n, k, p, lda, ldc);
    if (st) return st;
    if (!range_ok(n, k, p, A, lda)) return ORC_ERANGE;
    const int wide = (i128)k * (p - 1) * (p - 1) >= ((i128)1 << 62);
#pragma omp parallel for schedule(static, 1)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t jmax = full ? n - 1 : i;
        const int64_t* ai = A + i * lda;
        for (int64_t j = 0; j <= jmax; ++j) {
            const int64_t* aj = A + j * lda;
            if (wide) {
                i128 s = 0;
                for (int64_t t = 0; t < k; ++t) s += (i128)ai[t] * aj[t];
                C[i * ldc + j] = canon128(s, p);
            } else {
                int64_t s = 0;
                for (int64_t t = 0; t < k; ++t) s += ai[t] * aj[t];
                C[i * ldc + j] = canon64(s, p);
            }
        }
    }
    return ORC_OK;
}

/* Selected entries (rows[e], cols[e]) of A*A^T mod p, any (i, j). */
int oracle_syrk_entries(int64_t n, int64_t k, int64_t p, const int64_t* A, int64_t lda,
                        int64_t count, const int64_t* rows, const int64_t* cols, int64_t* out)
{
    int st = check_args(n, k, p, lda, n > 0 ? n : 1);
    if (st) return st;
    for (int64_t e = 0; e < count; ++e)
        if (rows[e] < 0 || rows[e] >= n || cols[e] < 0 || cols[e] >= n) return ORC_EINVAL;
#pragma omp parallel for schedule(static, 1)
    for (int64_t e = 0; e < count; ++e) {
        const int64_t* ai = A + rows[e] * lda;
        const int64_t* aj = A + cols[e] * lda;
        i128 s = 0;
        for (int64_t t = 0; t < k; ++t) s += (i128)ai[t] * aj[t];
        out[e] = canon128(s, p);
    }
    return ORC_OK;
}

/* ---------------- the product, conjugate-transpose case over F_p[i]/(i^2+1) ---------------- */

/* For j <= i (full: every j):
 *   Re C_ij = sum_t (xr_it xr_jt + xi_it xi_jt)
 *   Im C_ij = sum_t (xi_it xr_jt - xr_it xi_jt)         each mod p. */
int oracle_herk_modp2(int64_t n, int64_t k, int64_t p, const int64_t* Ar, const int64_t* Ai,
                      int64_t lda, int64_t* Cr, int64_t* Ci, int64_t ldc, int full)
{
    int st = check_args(n, k, p, lda, ldc);
    if (st) return st;
    if (p % 4 != 3) return ORC_EINVAL; /* i^2+1 must be irreducible */
    if (!range_ok(n, k, p, Ar, lda) || !range_ok(n, k, p, Ai, lda)) return ORC_ERANGE;
#pragma omp parallel for schedule(static, 1)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t jmax = full ? n - 1 : i;
        for (int64_t j = 0; j <= jmax; ++j) {
            i128 re = 0, im = 0;
            for (int64_t t = 0; t < k; ++t) {
                const int64_t xr = Ar[i * lda + t], xi = Ai[i * lda + t];
                const int64_t yr = Ar[j * lda + t], yi = Ai[j * lda + t];
                re += (i128)xr * yr + (i128)xi * yi;
                im += (i128)xi * yr - (i128)xr * yi;
            }
            Cr[i * ldc + j] = canon128(re, p);
            Ci[i * ldc + j] = canon128(im, p);
        }
    }
    return ORC_OK;
}

int oracle_herk_entries(int64_t n, int64_t k, int64_t p, const int64_t* Ar, const int64_t* Ai,
                        int64_t lda, int64_t count, const int64_t* rows, const int64_t* cols,
                        int64_t* out_re, int64_t* out_im)
{
    int st = check_args(n, k, p, lda, n > 0 ? n : 1);
    if (st) return st;
    for (int64_t e = 0; e < count; ++e)
        if (rows[e] < 0 || rows[e] >= n || cols[e] < 0 || cols[e] >= n) return ORC_EINVAL;
#pragma omp parallel for schedule(static, 1)
    for (int64_t e = 0; e < count; ++e) {
        const int64_t i = rows[e], j = cols[e];
        i128 re = 0, im = 0;
        for (int64_t t = 0; t < k; ++t) {
            const int64_t xr = Ar[i * lda + t], xi = Ai[i * lda + t];
            const int64_t yr = Ar[j * lda + t], yi = Ai[j * lda + t];
            re += (i128)xr * yr + (i128)xi * yi;
            im += (i128)xi * yr - (i128)xr * yi;
        }
        out_re[e] = canon128(re, p);
        out_im[e] = canon128(im, p);
    }
    return ORC_OK;
}

/* ---------------- Freivalds check ---------------- */

/* y_c = S x with S the symmetric matrix whose lower triangle is C, and
 * y_a = A (A^T x), both mod p.  For a correct C the two agree for every x;
 * for a wrong C they differ with probability >= 1 - 1/p per random x. */
int oracle_freivalds_syrk(int64_t n, int64_t k, int64_t p, const int64_t* A, int64_t lda,
                          const int64_t* C, int64_t ldc, const int64_t* x,
                          int64_t* y_c, int64_t* y_a)
{
    int st = check_args(n, k, p, lda, ldc);
    if (st) return st;
    int64_t* w = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
    if (!w) return ORC_EINVAL;
    for (int64_t t = 0; t < k; ++t) {
        i128 s = 0;
        for (int64_t i = 0; i < n; ++i) s += (i128)A[i * lda + t] * x[i];
        w[t] = canon128(s, p);
    }
#pragma omp parallel for schedule(static, 16)
    for (int64_t i = 0; i < n; ++i) {
        i128 s = 0;
        for (int64_t t = 0; t < k; ++t) s += (i128)A[i * lda + t] * w[t];
        y_a[i] = canon128(s, p);
        i128 u = 0;
        for (int64_t j = 0; j <= i; ++j) u += (i128)C[i * ldc + j] * x[j];
        for (int64_t j = i + 1; j < n; ++j) u += (i128)C[j * ldc + i] * x[j];
        y_c[i] = canon128(u, p);
    }
    free(w);
    return ORC_OK;
}

/* Hermitian Freivalds over F_p[i]: with S the Hermitian matrix whose lower
 * triangle is C (S_ij = C_ij for j <= i, S_ij = conj(C_ji) above) and a
 * complex x, y_c = S x and y_a = A (A^H x), both mod p, planar re/im. */
int oracle_freivalds_herk(int64_t n, int64_t k, int64_t p, const int64_t* Ar, const int64_t* Ai,
                          int64_t lda, const int64_t* Cr, const int64_t* Ci, int64_t ldc,
                          const int64_t* xr, const int64_t* xi, int64_t* ycr, int64_t* yci,
                          int64_t* yar, int64_t* yai)
{
    int st = check_args(n, k, p, lda, ldc);
    if (st) return st;
    int64_t* wr = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
    int64_t* wi = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
    if (!wr || !wi) { free(wr); free(wi); return ORC_EINVAL; }
    /* w = A^H x: w_t = sum_i conj(A_it) x_i */
    for (int64_t t = 0; t < k; ++t) {
        i128 sr = 0, si = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t ar = Ar[i * lda + t], ai = Ai[i * lda + t];
            sr += (i128)ar * xr[i] + (i128)ai * xi[i];
            si += (i128)ar * xi[i] - (i128)ai * xr[i];
        }
        wr[t] = canon128(sr, p);
        wi[t] = canon128(si, p);
    }
#pragma omp parallel for schedule(static, 16)
    for (int64_t i = 0; i < n; ++i) {
        i128 sr = 0, si = 0;
        for (int64_t t = 0; t < k; ++t) {
            const int64_t ar = Ar[i * lda + t], ai = Ai[i * lda + t];
            sr += (i128)ar * wr[t] - (i128)ai * wi[t];
            si += (i128)ar * wi[t] + (i128)ai * wr[t];
        }
        yar[i] = canon128(sr, p);
        yai[i] = canon128(si, p);
        i128 ur = 0, ui = 0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t cr, ci;
            if (j <= i) { cr = Cr[i * ldc + j]; ci = Ci[i * ldc + j]; }
            else { cr = Cr[j * ldc + i]; ci = -Ci[j * ldc + i]; }
            ur += (i128)cr * xr[j] - (i128)ci * xi[j];
            ui += (i128)cr * xi[j] + (i128)ci * xr[j];
        }
        ycr[i] = canon128(ur, p);
        yci[i] = canon128(ui, p);
    }
    free(wr);
    free(wi);
    return ORC_OK;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
