/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously correct CPU
 * brute force for the exhaustive Ising low-spectrum search of
 * "Brute-forcing spin-glass problems with CUDA" (arXiv:1904.03621).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this file.  It shares no code, header or table with the GPU library.
 *
 * Conventions (readings of the paper, listed with their reasons in the
 * design notes):
 *   - Spin i (0-based) is bit i of a state mask; bit set <=> s_i = +1
 *     (Sec. 2, Fig. 1 caption: red = +1, blue = -1 / q = 0; q = (s+1)/2).
 *   - J is a dense row-major N x N array; the sum over adjacent sites of
 *     Eq. (1) takes each unordered pair once, read from the strict upper
 *     triangle J[i*N+j], i<j.  Diagonal and lower triangle are ignored.
 *   - The answer of the search is the first S pairs (E(m), m) of all 2^N
 *     states sorted lexicographically ascending (ties broken by the mask).
 *
 * Precision: float instances are evaluated in double (their float values
 * convert exactly), integer instances in int64, summing in the fixed i<j
 * order given by Eq. (1).
 *
 * Pins (see tests/test_oracle_pins.py): the QUBO identity of Eqs. (2)-(3)
 * with its offset, closed forms (ferromagnet, Mattis, free spins with
 * fields 2^i, open chain transfer matrix, J = 0 partition function),
 * invariants (global flip, gauge), brute force by full sort at small N, and
 * central finite differences of log Z for the moments.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- energies */

/* Eq. (1): H(s) = - sum_{i<j} J_ij s_i s_j - sum_i h_i s_i. */
double oracle_energy_f64(int N, const double *J, const double *h, uint64_t mask)
{
    double e = 0.0;
    for (int i = 0; i < N; ++i) {
        double si = ((mask >> i) & 1u) ? 1.0 : -1.0;
        for (int j = i + 1; j < N; ++j) {
            double sj = ((mask >> j) & 1u) ? 1.0 : -1.0;
            e -= J[(size_t)i * N + j] * si * sj;
        }
    }
    for (int i = 0; i < N; ++i) {
        double si = ((mask >> i) & 1u) ? 1.0 : -1.0;
        e -= h[i] * si;
    }
    return e;
}

int64_t oracle_energy_i64(int N, const int64_t *J, const int64_t *h, uint64_t mask)
{
    int64_t e = 0;
    for (int i = 0; i < N; ++i) {
        int64_t si = ((mask >> i) & 1u) ? 1 : -1;
        for (int j = i + 1; j < N; ++j) {
            int64_t sj = ((mask >> j) & 1u) ? 1 : -1;
            e -= J[(size_t)i * N + j] * si * sj;
        }
    }
    for (int i = 0; i < N; ++i) {
        int64_t si = ((mask >> i) & 1u) ? 1 : -1;
        e -= h[i] * si;
    }
    return e;
}

/* Eq. (3): a_ij = 4 J_ij, b_i = 2 h_i - 2 sum_{j adjacent to i} J_ij, and the
 * offset H - F = sum_i h_i - sum_<ij> J_ij.  a is written on the strict upper
 * triangle (dense N x N, zeros elsewhere). */
void oracle_qubo_from_ising(int N, const double *J, const double *h,
                            double *a, double *b, double *offset)
{
    double sumJ = 0.0, sumh = 0.0;
    for (int i = 0; i < N * N; ++i) a[i] = 0.0;
    for (int i = 0; i < N; ++i) {
        double nb = 0.0;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            int lo = i < j ? i : j, hi = i < j ? j : i;
            nb += J[(size_t)lo * N + hi];
        }
        b[i] = 2.0 * h[i] - 2.0 * nb;
        sumh += h[i];
        for (int j = i + 1; j < N; ++j) {
            a[(size_t)i * N + j] = 4.0 * J[(size_t)i * N + j];
            sumJ += J[(size_t)i * N + j];
        }
    }
    *offset = sumh - sumJ;
}

/* Eq. (2): F(q) = - sum_{i<j} a_ij q_i q_j - sum_i b_i q_i, q_i = bit i. */
double oracle_qubo_energy_f64(int N, const double *a, const double *b, uint64_t mask)
{
    double f = 0.0;
    for (int i = 0; i < N; ++i) {
        double qi = (double)((mask >> i) & 1u);
        for (int j = i + 1; j < N; ++j) {
            double qj = (double)((mask >> j) & 1u);
            f -= a[(size_t)i * N + j] * qi * qj;
        }
        f -= b[i] * qi;
    }
    return f;
}

/* --------------------------------------------- bounded selection (S lowest) */

/* Key order: (E, mask) lexicographic ascending.  A max-heap of at most S
 * entries keeps the S smallest keys seen so far. */
typedef struct { double e; uint64_t m; } kd_t;
typedef struct { int64_t e; uint64_t m; } ki_t;

static int kd_less(kd_t x, kd_t y) { return x.e < y.e || (x.e == y.e && x.m < y.m); }
static int ki_less(ki_t x, ki_t y) { return x.e < y.e || (x.e == y.e && x.m < y.m); }

#define DEFINE_HEAP(T, LESS)                                                   \
static void T##_sift_down(T *hp, int n, int i) {                               \
    for (;;) {                                                                 \
        int l = 2 * i + 1, r = l + 1, big = i;                                 \
        if (l < n && LESS(hp[big], hp[l])) big = l;                            \
        if (r < n && LESS(hp[big], hp[r])) big = r;                            \
        if (big == i) return;                                                  \
        T t = hp[i]; hp[i] = hp[big]; hp[big] = t; i = big;                    \
    }                                                                          \
}                                                                              \
static void T##_sift_up(T *hp, int i) {                                        \
    while (i > 0) {                                                            \
        int p = (i - 1) / 2;                                                   \
        if (!LESS(hp[p], hp[i])) return;                                       \
        T t = hp[i]; hp[i] = hp[p]; hp[p] = t; i = p;                          \
    }                                                                          \
}                                                                              \
/* offer x to a heap of capacity S holding *n entries */                      \
static void T##_offer(T *hp, int *n, int S, T x) {                             \
    if (*n < S) { hp[*n] = x; T##_sift_up(hp, *n); ++*n; return; }             \
    if (LESS(x, hp[0])) { hp[0] = x; T##_sift_down(hp, *n, 0); }               \
}                                                                              \
static int T##_cmp(const void *a, const void *b) {                             \
    T x = *(const T *)a, y = *(const T *)b;                                    \
    return LESS(x, y) ? -1 : (LESS(y, x) ? 1 : 0);                             \
}

DEFINE_HEAP(kd_t, kd_less)
DEFINE_HEAP(ki_t, ki_less)

/* Number of threads the parallel loops use when asked for 0 (all). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int oracle_threads(int req)
{
#ifdef _OPENMP
    return req > 0 ? req : omp_get_max_threads();
#else
    (void)req;
    return 1;
#endif
}

/* The S lowest (E, mask) over masks in [lo, hi), written ascending.
 * Returns the number written: min(S, hi - lo).  Threads split [lo, hi)
 * into contiguous slices, each keeps its own heap, and the union is sorted
 * and cut to S at the end. */
int oracle_low_spectrum_f64(int N, const double *J, const double *h, int S,
                            uint64_t lo, uint64_t hi, uint64_t *masks_out,
                            double *e_out, int nthreads)
{
    if (S <= 0 || hi <= lo) return 0;
    int T = oracle_threads(nthreads);
    kd_t *all = (kd_t *)malloc(sizeof(kd_t) * (size_t)S * T);
    int *cnt = (int *)calloc((size_t)T, sizeof(int));
    uint64_t span = hi - lo;
#pragma omp parallel num_threads(T)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        uint64_t a = lo + span / T * t + (t < (int)(span % T) ? t : span % T);
        uint64_t b = a + span / T + (t < (int)(span % T) ? 1 : 0);
        kd_t *hp = all + (size_t)S * t;
        int n = 0;
        for (uint64_t m = a; m < b; ++m) {
            kd_t x = { oracle_energy_f64(N, J, h, m), m };
            kd_t_offer(hp, &n, S, x);
        }
        cnt[t] = n;
    }
    int tot = 0;
    for (int t = 0; t < T; ++t) {
        memmove(all + tot, all + (size_t)S * t, sizeof(kd_t) * cnt[t]);
        tot += cnt[t];
    }
    qsort(all, (size_t)tot, sizeof(kd_t), kd_t_cmp);
    int out = tot < S ? tot : S;
    for (int i = 0; i < out; ++i) { masks_out[i] = all[i].m; e_out[i] = all[i].e; }
    free(all); free(cnt);
    return out;
}

int oracle_low_spectrum_i64(int N, const int64_t *J, const int64_t *h, int S,
                            uint64_t lo, uint64_t hi, uint64_t *masks_out,
                            int64_t *e_out, int nthreads)
{
    if (S <= 0 || hi <= lo) return 0;
    int T = oracle_threads(nthreads);
    ki_t *all = (ki_t *)malloc(sizeof(ki_t) * (size_t)S * T);
    int *cnt = (int *)calloc((size_t)T, sizeof(int));
    uint64_t span = hi - lo;
#pragma omp parallel num_threads(T)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        uint64_t a = lo + span / T * t + (t < (int)(span % T) ? t : span % T);
        uint64_t b = a + span / T + (t < (int)(span % T) ? 1 : 0);
        ki_t *hp = all + (size_t)S * t;
        int n = 0;
        for (uint64_t m = a; m < b; ++m) {
            ki_t x = { oracle_energy_i64(N, J, h, m), m };
            ki_t_offer(hp, &n, S, x);
        }
        cnt[t] = n;
    }
    int tot = 0;
    for (int t = 0; t < T; ++t) {
        memmove(all + tot, all + (size_t)S * t, sizeof(ki_t) * cnt[t]);
        tot += cnt[t];
    }
    qsort(all, (size_t)tot, sizeof(ki_t), ki_t_cmp);
    int out = tot < S ? tot : S;
    for (int i = 0; i < out; ++i) { masks_out[i] = all[i].m; e_out[i] = all[i].e; }
    free(all); free(cnt);
    return out;
}

/* ------------------------------------------------------- density of states */

/*
 * Density of states of an integer instance: counts[k] = number of masks m in
 * [lo, hi) with E(m) = e_min + k (Eq. 1), k in [0, n_bins).  Every mask is
 * evaluated from scratch; each thread keeps its own histogram.  Returns 0, or
 * -1 if some energy falls outside [e_min, e_min + n_bins).
 */
int oracle_dos_i64(int N, const int64_t *J, const int64_t *h, int64_t e_min, int n_bins,
                   uint64_t lo, uint64_t hi, uint64_t *counts, int nthreads)
{
    if (n_bins <= 0 || hi < lo) return -1;
    int T = oracle_threads(nthreads);
    uint64_t *part = (uint64_t *)calloc((size_t)n_bins * T, sizeof(uint64_t));
    int outside = 0;
    uint64_t span = hi - lo;
#pragma omp parallel num_threads(T) reduction(| : outside)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        uint64_t a = lo + span / T * t + (t < (int)(span % T) ? t : span % T);
        uint64_t b = a + span / T + (t < (int)(span % T) ? 1 : 0);
        uint64_t *c = part + (size_t)n_bins * t;
        for (uint64_t m = a; m < b; ++m) {
            int64_t k = oracle_energy_i64(N, J, h, m) - e_min;
            if (k < 0 || k >= n_bins) outside = 1;
            else c[k] += 1;
        }
    }
    for (int k = 0; k < n_bins; ++k) {
        uint64_t v = 0;
        for (int t = 0; t < T; ++t) v += part[(size_t)n_bins * t + k];
        counts[k] = v;
    }
    free(part);
    return outside ? -1 : 0;
}

/* ------------------------------------------------------- log Z and moments */

/* Neumaier (improved Kahan) compensated summation step. */
static void neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

/* Exact Boltzmann statistics over all 2^N states (the Boltzmann weight at
 * inverse temperature beta is the distribution of Sec. 5.2):
 *   e0            = min_m E(m)
 *   logz[b]       = -beta_b e0 + log sum_m exp(-beta_b (E(m) - e0))
 *   mean_s[b,i]   = <s_i>                       (may be NULL)
 *   mean_ss[b,i,j]= <s_i s_j> for i<j, 0 elsewhere (may be NULL)
 * Pass 1 finds e0; pass 2 accumulates the shifted weights, Z with Neumaier
 * summation, the moments with per-thread double sums added at the end. */
int oracle_logz_f64(int N, const double *J, const double *h, int nb,
                    const double *beta, double *logz, double *e0_out,
                    double *mean_s, double *mean_ss, int nthreads)
{
    if (N < 1 || N > 40 || nb < 1) return -1;
    int T = oracle_threads(nthreads);
    uint64_t M = (uint64_t)1 << N;
    double e0 = INFINITY;
#pragma omp parallel for num_threads(T) reduction(min : e0) schedule(static)
    for (long long mm = 0; mm < (long long)M; ++mm) {
        double e = oracle_energy_f64(N, J, h, (uint64_t)mm);
        if (e < e0) e0 = e;
    }
    *e0_out = e0;

    int want_s = mean_s != NULL, want_ss = mean_ss != NULL;
    size_t per = (size_t)nb * (2 + (want_s ? N : 0) + (want_ss ? (size_t)N * N : 0));
    double *acc = (double *)calloc(per * T, sizeof(double));
#pragma omp parallel num_threads(T)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double *my = acc + per * t;
        double *z = my;                  /* [nb] sums     */
        double *zc = my + nb;            /* [nb] compens. */
        double *ms = my + 2 * nb;        /* [nb][N]       */
        double *mss = ms + (want_s ? (size_t)nb * N : 0); /* [nb][N][N] */
        double s[64];
#pragma omp for schedule(static)
        for (long long mm = 0; mm < (long long)M; ++mm) {
            uint64_t m = (uint64_t)mm;
            double e = oracle_energy_f64(N, J, h, m);
            for (int i = 0; i < N; ++i) s[i] = ((m >> i) & 1u) ? 1.0 : -1.0;
            for (int b = 0; b < nb; ++b) {
                double w = exp(-beta[b] * (e - e0));
                neumaier_add(&z[b], &zc[b], w);
                if (want_s)
                    for (int i = 0; i < N; ++i) ms[(size_t)b * N + i] += w * s[i];
                if (want_ss)
                    for (int i = 0; i < N; ++i)
                        for (int j = i + 1; j < N; ++j)
                            mss[((size_t)b * N + i) * N + j] += w * s[i] * s[j];
            }
        }
    }
    for (int b = 0; b < nb; ++b) {
        double zs = 0.0, zcs = 0.0;
        for (int t = 0; t < T; ++t) {
            double *my = acc + per * t;
            neumaier_add(&zs, &zcs, my[b]);
            neumaier_add(&zs, &zcs, my[nb + b]);
        }
        double Z = zs + zcs;
        logz[b] = -beta[b] * e0 + log(Z);
        if (want_s)
            for (int i = 0; i < N; ++i) {
                double v = 0.0;
                for (int t = 0; t < T; ++t) v += (acc + per * t + 2 * nb)[(size_t)b * N + i];
                mean_s[(size_t)b * N + i] = v / Z;
            }
        if (want_ss)
            for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j) {
                    double v = 0.0;
                    if (j > i)
                        for (int t = 0; t < T; ++t)
                            v += (acc + per * t + 2 * nb + (want_s ? (size_t)nb * N : 0))
                                     [((size_t)b * N + i) * N + j];
                    mean_ss[((size_t)b * N + i) * N + j] = v / Z;
                }
    }
    free(acc);
    return 0;
}

/* Gradients of log Z(beta): d logZ / d J_ij = beta <s_i s_j> (i<j, zero
 * elsewhere) and d logZ / d h_i = beta <s_i>, each scaled by the upstream
 * gradient g[b] and summed over the betas. */
int oracle_logz_grad_f64(int N, const double *J, const double *h, int nb,
                         const double *beta, const double *g, double *grad_J,
                         double *grad_h, int nthreads)
{
    double *logz = (double *)malloc(sizeof(double) * nb);
    double *ms = (double *)malloc(sizeof(double) * nb * N);
    double *mss = (double *)malloc(sizeof(double) * (size_t)nb * N * N);
    double e0;
    int rc = oracle_logz_f64(N, J, h, nb, beta, logz, &e0, ms, mss, nthreads);
    if (rc == 0) {
        for (int i = 0; i < N * N; ++i) grad_J[i] = 0.0;
        for (int i = 0; i < N; ++i) grad_h[i] = 0.0;
        for (int b = 0; b < nb; ++b) {
            for (int i = 0; i < N; ++i) grad_h[i] += g[b] * beta[b] * ms[(size_t)b * N + i];
            for (int i = 0; i < N; ++i)
                for (int j = i + 1; j < N; ++j)
                    grad_J[(size_t)i * N + j] += g[b] * beta[b] * mss[((size_t)b * N + i) * N + j];
        }
    }
    free(logz); free(ms); free(mss);
    return rc;
}
