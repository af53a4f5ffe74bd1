/*
 * The paper's own method, written plainly for the CPU -- TEST INFRASTRUCTURE
 * AND BASELINE ONLY.
 *
 * Only tests/, the smoke check and the CPU-baseline leg of bench.py may load
 * this library.  It shares no code with the HIP path.
 *
 * What it computes (paper, Section 3.2.3, the SLOS back-end paragraph: the full
 * output distribution by unfolding the computation path in memory, time and
 * memory O(n C(m+n-1, n))): photons are added one at a time, the k-th one
 * entering mode i_k (input modes in ascending order, each repeated t_i times;
 * creation operators commute, so the order does not change the result):
 *     A_0 = [1],  A_k[t] = sum over modes j with t_j > 0 of U[j][i_k] A_{k-1}[t - e_j],
 * over all k-photon states t, and the amplitude of output S is
 *     a(S) = A_n[S] sqrt(s_1!..s_m!) / sqrt(t_1!..t_m!),
 * the same number as the permanent formula of Eq. eqperm.
 *
 * States of k photons are ranked in colex order: with the photon modes sorted,
 * d_1 <= .. <= d_k, and c_r = d_r + r - 1 (a strictly increasing sequence),
 * rank(t) = sum_r C(c_r, r).  Removing one photon of mode j (the last position
 * r0 holding j) keeps c_r for r < r0 and turns c_r into c_r - 1 at position
 * r - 1 for r > r0, so rank(t - e_j) = sum_{r<r0} C(c_r, r) + sum_{r>r0} C(c_r - 1, r - 1).
 * Each layer walks its states in colex order with the next-combination step,
 * one contiguous rank range per OpenMP thread.
 *
 * Arithmetic: IEEE binary64 throughout (complex products and sums in double),
 * the normalisation from a table of sqrt(k!), and the sum of P in a fixed order
 * (per-range partials added in range order).  A second entry point runs the
 * same steps in long double (x87 extended precision) for many-photon cases
 * whose sums cancel heavily.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SR_MAX_N 40
#define SR_MAX_M 256

/* C(a, b) for 0 <= a < rows, 0 <= b < W, at C[a * W + b] */
static int binom_table(int rows, int W, uint64_t **out)
{
    uint64_t *C = (uint64_t *)calloc((size_t)rows * W, sizeof(uint64_t));
    if (!C) return -3;
    for (int a = 0; a < rows; ++a) {
        C[(size_t)a * W] = 1;
        for (int b = 1; b < W && b <= a; ++b) {
            const uint64_t x = C[(size_t)(a - 1) * W + b - 1];
            const uint64_t y = C[(size_t)(a - 1) * W + b];
            if (x > UINT64_MAX - y) {
                free(C);
                return -2;
            }
            C[(size_t)a * W + b] = x + y;
        }
    }
    *out = C;
    return 0;
}

/* The combination c_1 < .. < c_k of colex rank `rank` (greedy from the top). */
static void unrank(const uint64_t *C, int W, int m, int k, uint64_t rank, int *c)
{
    int hi = m + k - 2;
    for (int r = k; r >= 1; --r) {
        int v = hi;
        while (C[(size_t)v * W + r] > rank) --v;
        c[r] = v;
        rank -= C[(size_t)v * W + r];
        hi = v - 1;
    }
}

/* The next combination in colex order: raise the lowest entry that can rise,
   reset the entries below it to 0, 1, 2, .. */
static void next_comb(int k, int *c)
{
    int r = 1;
    while (r < k && c[r] + 1 == c[r + 1]) ++r;
    c[r] += 1;
    for (int q = 1; q < r; ++q) c[q] = q - 1;
}

/*
 * Computes A_1 .. A_n and writes the normalised amplitudes a(S), S of n photons
 * in colex order, to out (interleaved re, im; C(m+n-1, n) complex values, owned
 * by the caller).  U is the m x m matrix as U[2 (j m + i)] = Re U[j][i],
 * U[2 (j m + i) + 1] = Im (row = output mode).  T holds the m input
 * occupations.  *sum_p receives sum_S |a(S)|^2.  threads <= 0: OpenMP's
 * default.  Returns 0, or -1 for invalid arguments, -2 when a count overflows,
 * -3 when memory runs out.  REAL is the type of the layers and of every sum:
 * double (oracle_slos_all), or long double (oracle_slos_all_ext: x87 extended
 * precision, a reference for cases with heavy cancellation over many photons).
 */
#define SR_DEFINE(NAME, REAL, SQRT)                                                                          \
    int NAME(int m, const double *U, const int32_t *T, double *out, double *sum_p, int threads)              \
    {                                                                                                        \
        if (m < 1 || m > SR_MAX_M || !U || !T || !out) return -1;                                            \
        int n = 0;                                                                                           \
        for (int i = 0; i < m; ++i) {                                                                        \
            if (T[i] < 0) return -1;                                                                         \
            n += T[i];                                                                                       \
        }                                                                                                    \
        if (n > SR_MAX_N) return -1;                                                                         \
        uint64_t *C = NULL;                                                                                  \
        const int W = n + 1;                                                                                 \
        {                                                                                                    \
            const int e = binom_table(m + n + 1, W, &C);                                                     \
            if (e) return e;                                                                                 \
        }                                                                                                    \
        if (sum_p) *sum_p = 0.0;                                                                             \
        /* photon list i_1 <= .. <= i_n and sqrt(k!) */                                                     \
        int photon[SR_MAX_N + 1];                                                                            \
        REAL sqrt_fact[SR_MAX_N + 1];                                                                        \
        REAL tfac = 1;                                                                                       \
        {                                                                                                    \
            int k = 0;                                                                                       \
            for (int i = 0; i < m; ++i)                                                                      \
                for (int c = 0; c < T[i]; ++c) photon[++k] = i;                                              \
            REAL f = 1;                                                                                      \
            sqrt_fact[0] = 1;                                                                                \
            for (int q = 1; q <= n; ++q) {                                                                   \
                f *= q;                                                                                      \
                sqrt_fact[q] = SQRT(f);                                                                      \
            }                                                                                                \
            for (int i = 0; i < m; ++i) tfac *= sqrt_fact[T[i]];                                             \
        }                                                                                                    \
        if (n == 0) {                                                                                        \
            out[0] = 1.0;                                                                                    \
            out[1] = 0.0;                                                                                    \
            if (sum_p) *sum_p = 1.0;                                                                         \
            free(C);                                                                                         \
            return 0;                                                                                        \
        }                                                                                                    \
        /* two buffers as large as the largest layer below n */                                             \
        uint64_t big = 1;                                                                                    \
        for (int k = 1; k < n; ++k)                                                                          \
            if (C[(size_t)(m + k - 1) * W + k] > big) big = C[(size_t)(m + k - 1) * W + k];                  \
        REAL *buf[2] = {NULL, NULL};                                                                         \
        if (n > 1) {                                                                                         \
            buf[0] = (REAL *)malloc(2 * sizeof(REAL) * big);                                                 \
            buf[1] = (REAL *)malloc(2 * sizeof(REAL) * big);                                                 \
            if (!buf[0] || !buf[1]) {                                                                        \
                free(buf[0]);                                                                                \
                free(buf[1]);                                                                                \
                free(C);                                                                                     \
                return -3;                                                                                   \
            }                                                                                                \
        }                                                                                                    \
        const REAL one[2] = {1, 0};                                                                          \
        const REAL *prev = one;                                                                              \
        int nthr = 1;                                                                                        \
        SR_THREADS(nthr, threads);                                                                           \
        const int64_t nparts = (int64_t)nthr * 8;                                                            \
        REAL *partial = (REAL *)calloc((size_t)nparts, sizeof(REAL));                                        \
        if (!partial) {                                                                                      \
            free(buf[0]);                                                                                    \
            free(buf[1]);                                                                                    \
            free(C);                                                                                         \
            return -3;                                                                                       \
        }                                                                                                    \
        for (int k = 1; k <= n; ++k) {                                                                       \
            const uint64_t Nk = C[(size_t)(m + k - 1) * W + k];                                              \
            const int last = k == n;                                                                         \
            REAL *cur = last ? NULL : buf[k & 1];                                                            \
            const int col = photon[k];                                                                       \
            SR_PARALLEL_FOR(nthr)                                                                            \
            for (int64_t part = 0; part < nparts; ++part) {                                                  \
                const uint64_t lo = Nk * (uint64_t)part / (uint64_t)nparts;                                  \
                const uint64_t hi = Nk * (uint64_t)(part + 1) / (uint64_t)nparts;                            \
                if (lo >= hi) continue;                                                                      \
                int c[SR_MAX_N + 2];                                                                         \
                uint64_t keep[SR_MAX_N + 2], drop[SR_MAX_N + 2];                                             \
                unrank(C, W, m, k, lo, c);                                                                   \
                REAL psum = 0;                                                                               \
                for (uint64_t t = lo; t < hi; ++t) {                                                         \
                    if (t > lo) next_comb(k, c);                                                             \
                    /* keep[r] = sum_{q<=r} C(c_q, q); drop[r] = sum_{q>=r} C(c_q - 1, q - 1) */            \
                    keep[0] = 0;                                                                             \
                    for (int r = 1; r <= k; ++r) keep[r] = keep[r - 1] + C[(size_t)c[r] * W + r];            \
                    drop[k + 1] = 0;                                                                         \
                    for (int r = k; r >= 1; --r)                                                             \
                        drop[r] = drop[r + 1] + (c[r] >= 1 ? C[(size_t)(c[r] - 1) * W + r - 1] : 0);         \
                    REAL re = 0, im = 0, sfac = 1;                                                           \
                    int run = 0;                                                                             \
                    for (int r = 1; r <= k; ++r) {                                                           \
                        const int d = c[r] - (r - 1);                                                        \
                        ++run;                                                                               \
                        const int d_next = r < k ? c[r + 1] - r : -1;                                        \
                        if (d_next == d) continue; /* mode d has another photon above r */                   \
                        const uint64_t pr = keep[r - 1] + drop[r + 1];                                       \
                        const REAL ur = U[2 * ((size_t)d * m + col)], ui = U[2 * ((size_t)d * m + col) + 1]; \
                        const REAL xr = prev[2 * pr], xi = prev[2 * pr + 1];                                 \
                        re += ur * xr - ui * xi;                                                             \
                        im += ur * xi + ui * xr;                                                             \
                        if (last) sfac *= sqrt_fact[run];                                                    \
                        run = 0;                                                                             \
                    }                                                                                        \
                    if (last) {                                                                              \
                        const REAL f = sfac / tfac;                                                          \
                        re *= f;                                                                             \
                        im *= f;                                                                             \
                        psum += re * re + im * im;                                                           \
                        out[2 * t] = (double)re;                                                             \
                        out[2 * t + 1] = (double)im;                                                         \
                    } else {                                                                                 \
                        cur[2 * t] = re;                                                                     \
                        cur[2 * t + 1] = im;                                                                 \
                    }                                                                                        \
                }                                                                                            \
                if (last) partial[part] = psum;                                                              \
            }                                                                                                \
            prev = cur;                                                                                      \
        }                                                                                                    \
        if (sum_p) {                                                                                         \
            REAL s = 0;                                                                                      \
            for (int64_t part = 0; part < nparts; ++part) s += partial[part];                                \
            *sum_p = (double)s;                                                                              \
        }                                                                                                    \
        free(partial);                                                                                       \
        free(buf[0]);                                                                                        \
        free(buf[1]);                                                                                        \
        free(C);                                                                                             \
        return 0;                                                                                            \
    }

#ifdef _OPENMP
#define SR_THREADS(nthr, threads) (nthr) = (threads) > 0 ? (threads) : omp_get_max_threads()
#define SR_PRAGMA(x) _Pragma(#x)
#define SR_PARALLEL_FOR(nthr) SR_PRAGMA(omp parallel for schedule(dynamic, 1) num_threads(nthr))
#else
#define SR_THREADS(nthr, threads) (void)(threads)
#define SR_PARALLEL_FOR(nthr)
#endif

SR_DEFINE(oracle_slos_all, double, sqrt)
SR_DEFINE(oracle_slos_all_ext, long double, sqrtl)
