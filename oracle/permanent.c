/*
 * Oracle for the SLOS strong-simulation hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke check and the CPU-baseline leg of bench.py may load
 * this library.  It shares no code with the HIP path.
 *
 * What it computes (paper, Section 4.2.1, Eq. eqperm): for input Fock state
 * T = (t_1..t_m) and output S = (s_1..s_m) of an m-mode unitary U, build the
 * n x n matrix U_{T,S} whose rows are the rows of U repeated s_j times and
 * whose columns are the columns of U repeated t_i times; the amplitude is
 *     a(S) = Perm(U_{T,S}) / sqrt(s_1!..s_m! t_1!..t_m!)
 * and P(S) = |a(S)|^2.  U[j][i] is the amplitude from input mode i to output
 * mode j (row = output).
 *
 * Permanents (paper, Section 3.2.3, Naive back-end, which names Ryser's and
 * Glynn's formulas):
 *   - brute force: the definition, sum over all n! permutations;
 *   - Ryser:  Perm(A) = (-1)^n sum_{X subset [n]} (-1)^{|X|} prod_r sum_{c in X} A[r][c],
 *             subsets visited in Gray-code order;
 *   - Glynn:  Perm(A) = 2^{-(n-1)} sum_{d in {+-1}^n, d_1=+1} (prod_k d_k)
 *                         prod_c sum_r d_r A[r][c], sign vectors in Gray-code order.
 * Arithmetic is IEEE binary64 at the interfaces; sums and products inside a
 * permanent are carried in x87 extended precision (long double) so that the
 * oracle stays well below the 1e-12 relative bar at n <= 12.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double _Complex lcplx;

#define ORACLE_MAX_N 30

enum { ORACLE_RYSER = 0, ORACLE_GLYNN = 1, ORACLE_BRUTE = 2 };

/* ---- permanents of an n x n matrix held as lcplx a[r*n + c] ---------------- */

static lcplx perm_brute_rec(const lcplx *a, int n, int row, uint32_t used)
{
    if (row == n) return 1.0L;
    lcplx s = 0.0L;
    for (int c = 0; c < n; ++c) {
        if (used & (1u << c)) continue;
        lcplx v = a[row * n + c];
        if (v == 0.0L) continue;
        s += v * perm_brute_rec(a, n, row + 1, used | (1u << c));
    }
    return s;
}

static lcplx perm_brute(const lcplx *a, int n)
{
    return perm_brute_rec(a, n, 0, 0u);
}

static lcplx perm_ryser(const lcplx *a, int n)
{
    if (n == 0) return 1.0L;
    lcplx rowsum[ORACLE_MAX_N];
    for (int r = 0; r < n; ++r) rowsum[r] = 0.0L;
    lcplx total = 0.0L;
    uint64_t nsub = (uint64_t)1 << n;
    uint64_t gray_prev = 0;
    for (uint64_t k = 1; k < nsub; ++k) {
        uint64_t gray = k ^ (k >> 1);
        uint64_t diff = gray ^ gray_prev;
        int c = __builtin_ctzll(diff);
        if (gray & diff) {
            for (int r = 0; r < n; ++r) rowsum[r] += a[r * n + c];
        } else {
            for (int r = 0; r < n; ++r) rowsum[r] -= a[r * n + c];
        }
        gray_prev = gray;
        lcplx prod = 1.0L;
        for (int r = 0; r < n; ++r) prod *= rowsum[r];
        int size = __builtin_popcountll(gray);
        if (size & 1) total -= prod; else total += prod;
    }
    return (n & 1) ? -total : total;
}

static lcplx perm_glynn(const lcplx *a, int n)
{
    if (n == 0) return 1.0L;
    /* colsum[c] = sum_r d_r a[r][c]; start with all d_r = +1 */
    lcplx colsum[ORACLE_MAX_N];
    int d[ORACLE_MAX_N];
    for (int r = 0; r < n; ++r) d[r] = 1;
    for (int c = 0; c < n; ++c) {
        lcplx s = 0.0L;
        for (int r = 0; r < n; ++r) s += a[r * n + c];
        colsum[c] = s;
    }
    lcplx total = 0.0L;
    int sign = 1;
    uint64_t nvec = (uint64_t)1 << (n - 1);
    for (uint64_t k = 0; k < nvec; ++k) {
        if (k > 0) {
            /* flip sign variable d_{1+ctz(k)} (d_0 stays +1) */
            int r = 1 + __builtin_ctzll(k);
            long double f = d[r] > 0 ? -2.0L : 2.0L;
            for (int c = 0; c < n; ++c) colsum[c] += f * a[r * n + c];
            d[r] = -d[r];
            sign = -sign;
        }
        lcplx prod = 1.0L;
        for (int c = 0; c < n; ++c) prod *= colsum[c];
        if (sign > 0) total += prod; else total -= prod;
    }
    return total / ldexpl(1.0L, n - 1);
}

static lcplx perm_dispatch(const lcplx *a, int n, int method)
{
    switch (method) {
    case ORACLE_GLYNN: return perm_glynn(a, n);
    case ORACLE_BRUTE: return perm_brute(a, n);
    default: return perm_ryser(a, n);
    }
}

/* Permanent of a row-major complex128 n x n matrix (interleaved re, im). */
int oracle_perm(int n, const double *A, int method, double *out)
{
    if (n < 0 || n > ORACLE_MAX_N || (method == ORACLE_BRUTE && n > 12)) return -1;
    lcplx a[ORACLE_MAX_N * ORACLE_MAX_N];
    for (int i = 0; i < n * n; ++i) a[i] = (long double)A[2 * i] + I * (long double)A[2 * i + 1];
    lcplx p = perm_dispatch(a, n, method);
    out[0] = (double)creall(p);
    out[1] = (double)cimagl(p);
    return 0;
}

static long double factorial_l(int k)
{
    long double f = 1.0L;
    for (int i = 2; i <= k; ++i) f *= (long double)i;
    return f;
}

/* Build U_{T,S} (Eq. eqperm): row r is output mode rows[r], column c is
 * input mode cols[c].  Returns the normalisation sqrt(prod s! prod t!). */
static long double build_sub(int m, const double *U, const int32_t *T, const int32_t *S,
                             int n, lcplx *sub, int *rows, int *cols)
{
    int nr = 0, nc = 0;
    long double fac = 1.0L;
    for (int j = 0; j < m; ++j) {
        for (int k = 0; k < S[j]; ++k) rows[nr++] = j;
        fac *= factorial_l(S[j]);
    }
    for (int i = 0; i < m; ++i) {
        for (int k = 0; k < T[i]; ++k) cols[nc++] = i;
        fac *= factorial_l(T[i]);
    }
    (void)nc;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            const double *u = U + 2 * ((size_t)rows[r] * m + cols[c]);
            sub[r * n + c] = (long double)u[0] + I * (long double)u[1];
        }
    return sqrtl(fac);
}

static int check_state(int m, int n, const int32_t *s)
{
    int tot = 0;
    for (int j = 0; j < m; ++j) {
        if (s[j] < 0) return -1;
        tot += s[j];
    }
    return tot == n ? 0 : -1;
}

/*
 * Amplitudes a(S) for `count` output states S (row-major count x m int32)
 * of input T through U (row-major m x m complex128, U[j*m+i] = out j, in i).
 * out: count complex128 (interleaved).  nthreads <= 0 uses the OpenMP default.
 */
int oracle_amplitudes(int m, int n, const double *U, const int32_t *T, int64_t count,
                      const int32_t *S, int method, int nthreads, double *out)
{
    if (m < 1 || n < 0 || n > ORACLE_MAX_N || count < 0) return -1;
    if (check_state(m, n, T)) return -2;
    for (int64_t q = 0; q < count; ++q)
        if (check_state(m, n, S + q * m)) return -3;
    int nt = 1;  /* threads of this call only: the process-wide default is left alone */
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    (void)nt;
#endif
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int64_t q = 0; q < count; ++q) {
        lcplx sub[ORACLE_MAX_N * ORACLE_MAX_N];
        int rows[ORACLE_MAX_N], cols[ORACLE_MAX_N];
        long double norm = build_sub(m, U, T, S + q * m, n, sub, rows, cols);
        lcplx p = perm_dispatch(sub, n, method) / norm;
        out[2 * q] = (double)creall(p);
        out[2 * q + 1] = (double)cimagl(p);
    }
    return 0;
}

/* Number of threads an OpenMP parallel region uses here. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
    return t;
#else
    return 1;
#endif
}

/*
 * Gradient of sum_S Re(conj(w_S) a(S)) style losses, in the PyTorch complex
 * convention: given w_S = dL/d conj(a(S)) (times 2, as torch stores it),
 * returns G[j][i] = sum_S w_S * conj(d a(S) / d U[j][i]).
 * Because d Perm(A)/d A[r][c] = Perm(A with row r and column c removed),
 *   d a(S)/d U[j][i] = sum_{r: rows[r]=j} sum_{c: cols[c]=i} Perm(minor_rc) / norm.
 * G: m x m complex128, overwritten.
 */
int oracle_grad_U(int m, int n, const double *U, const int32_t *T, int64_t count,
                  const int32_t *S, const double *w, int nthreads, double *G)
{
    if (m < 1 || n < 1 || n > ORACLE_MAX_N || count < 0) return -1;
    if (check_state(m, n, T)) return -2;
    for (int64_t q = 0; q < count; ++q)
        if (check_state(m, n, S + q * m)) return -3;
    int nt = 1;  /* threads of this call only: the process-wide default is left alone */
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    (void)nt;
#endif
    size_t mm = (size_t)m * m;
    lcplx *acc = (lcplx *)calloc(mm, sizeof(lcplx));
    if (!acc) return -4;
    int alloc_failed = 0;
#pragma omp parallel num_threads(nt)
    {
        lcplx *loc = (lcplx *)calloc(mm, sizeof(lcplx));
        if (!loc) {
#pragma omp atomic write
            alloc_failed = 1;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < count; ++q) {
            lcplx sub[ORACLE_MAX_N * ORACLE_MAX_N];
            lcplx minor[ORACLE_MAX_N * ORACLE_MAX_N];
            int rows[ORACLE_MAX_N], cols[ORACLE_MAX_N];
            long double norm = build_sub(m, U, T, S + q * m, n, sub, rows, cols);
            lcplx wq = (long double)w[2 * q] + I * (long double)w[2 * q + 1];
            for (int r = 0; r < n; ++r)
                for (int c = 0; c < n; ++c) {
                    int k = 0;
                    for (int rr = 0; rr < n; ++rr) {
                        if (rr == r) continue;
                        for (int cc = 0; cc < n; ++cc) {
                            if (cc == c) continue;
                            minor[k++] = sub[rr * n + cc];
                        }
                    }
                    lcplx d = perm_ryser(minor, n - 1) / norm;
                    if (loc) loc[(size_t)rows[r] * m + cols[c]] += wq * conjl(d);
                }
        }
#pragma omp critical
        {
            if (loc)
                for (size_t e = 0; e < mm; ++e) acc[e] += loc[e];
        }
        free(loc);
    }
    if (alloc_failed) {
        free(acc);
        return -4;
    }
    for (size_t e = 0; e < mm; ++e) {
        G[2 * e] = (double)creall(acc[e]);
        G[2 * e + 1] = (double)cimagl(acc[e]);
    }
    free(acc);
    return 0;
}
