/*
 * oed_oracle.c -- CPU oracle for greedy D-optimal sensor selection.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links, calls or falls back to it.  It shares no code with the HIP sources.
 *
 * What it computes (paper: Sec. III-C "Computable D-optimal objective",
 * Sec. III-D "Greedy algorithm", Sec. III-E complexity, and the "naive
 * formulation" of Sec. IV-A):
 *
 *   f(S)  = 1/2 logdet(sigma^-2 K_SS)   for an ordered list S of sensors,
 *           K_SS = block rows and block columns of K for the sensors in S
 *           (each sensor owns N_t consecutive rows/columns of K).
 *   Greedy step k: for every remaining candidate j, in ascending index order,
 *           g_j = 1/2 [logdet K_{A u j} - logdet K_A] - (N_t/2) ln sigma^2,
 *           where both log-determinants are obtained by factoring the matrix
 *           from scratch with a dense Cholesky (logdet = 2 sum ln L_tt).
 *           A candidate whose factorisation meets a pivot that is not > 0 or
 *           not finite scores -inf.  The pick is the first j with the strictly
 *           largest score, so exact ties go to the lowest index.
 *
 * Only the lower triangle of K (column <= row) is read; element (r, c) with
 * r < c is taken from (c, r).  All arithmetic is IEEE FP64.  Candidates are
 * scored in parallel with OpenMP; every candidate's factorisation is serial,
 * so results do not depend on the thread count.
 *
 * Status codes: 0 ok, 1 bad argument, 2 no candidate with a finite score,
 * 3 out of memory, 4 the factorisation of K_A failed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_OK = 0, ORC_ARG = 1, ORC_NOT_SPD = 2, ORC_OOM = 3, ORC_KA_FAIL = 4 };

/* Element (r, c) of the symmetric K, reading only its lower triangle. */
static double k_lower(const double *K, int64_t ld, int64_t r, int64_t c)
{
    return r >= c ? K[r * ld + c] : K[c * ld + r];
}

/*
 * Cholesky-Banachiewicz factorisation of the n x n symmetric matrix in A
 * (row-major; only the lower triangle is used and it is overwritten by L),
 * followed by logdet = 2 * sum_t ln L_tt.  Returns 0, or -1 when a pivot is
 * not > 0 or not finite (the matrix is not numerically positive definite).
 */
int oedo_chol_logdet(double *A, int64_t n, double *logdet)
{
    double sum_log = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double *Li = A + i * n;
        for (int64_t j = 0; j <= i; ++j) {
            const double *Lj = A + j * n;
            double s = Li[j];
            for (int64_t k = 0; k < j; ++k)
                s -= Li[k] * Lj[k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s))
                    return -1;
                Li[i] = sqrt(s);
                sum_log += log(Li[i]);
            } else {
                Li[j] = s / Lj[j];
            }
        }
    }
    *logdet = 2.0 * sum_log;
    return 0;
}

/* Copy K_SS for the ordered sensor list S (length nS) into M (n x n, n = nS*N_t). */
static void gather_subset(const double *K, int64_t ld, int N_t, const int *S, int nS, double *M)
{
    const int64_t n = (int64_t)nS * N_t;
    for (int a = 0; a < nS; ++a)
        for (int t = 0; t < N_t; ++t) {
            const int64_t r = (int64_t)S[a] * N_t + t;
            double *row = M + ((int64_t)a * N_t + t) * n;
            for (int b = 0; b < nS; ++b)
                for (int u = 0; u < N_t; ++u)
                    row[(int64_t)b * N_t + u] = k_lower(K, ld, r, (int64_t)S[b] * N_t + u);
        }
}

/* logdet(K_SS) by a from-scratch Cholesky.  Returns 0, -1 (not PD) or ORC_OOM. */
int oedo_subset_logdet(const double *K, int64_t ld, int N_t, const int *S, int nS, double *logdet)
{
    if (nS == 0) {
        *logdet = 0.0;
        return 0;
    }
    const int64_t n = (int64_t)nS * N_t;
    double *M = (double *)malloc(sizeof(double) * n * n);
    if (!M)
        return ORC_OOM;
    gather_subset(K, ld, N_t, S, nS, M);
    int rc = oedo_chol_logdet(M, n, logdet);
    free(M);
    return rc;
}

/*
 * Scores of the candidates cand[0..nc) given the ordered prefix A[0..nA):
 * gains[c] = 1/2 [logdet K_{A u cand[c]} - logdet K_A] - h[cand[c]],
 * or -inf when the factorisation of K_{A u cand[c]} fails.  h[j] is 1/2 logdet of sensor j's
 * noise covariance block: with sensors whose noise is independent of each other the noise term of
 * the computable objective (Sec. III-C) is the sum of these over the selected set.  hld == NULL:
 * isotropic noise, h[j] = (N_t/2) ln sigma2 for every sensor.
 */
int oedo_gains(const double *K, int64_t ld, int N_t, double sigma2, const double *hld, const int *A,
               int nA, const int *cand, int nc, double *gains, int nthreads)
{
    if (!K || N_t <= 0 || !(sigma2 > 0.0) || nA < 0 || nc < 0)
        return ORC_ARG;
    double ld_A = 0.0;
    int rc = oedo_subset_logdet(K, ld, N_t, A, nA, &ld_A);
    if (rc == ORC_OOM)
        return ORC_OOM;
    if (rc != 0)
        return ORC_KA_FAIL;
    const double noise = 0.5 * N_t * log(sigma2);
    const int64_t n = (int64_t)(nA + 1) * N_t;
    int oom = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *M = (double *)malloc(sizeof(double) * n * n);
        int *S = (int *)malloc(sizeof(int) * (nA + 1));
        if (!M || !S) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            oom = 1;
        } else {
            if (nA > 0)
                memcpy(S, A, sizeof(int) * nA);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int c = 0; c < nc; ++c) {
                S[nA] = cand[c];
                gather_subset(K, ld, N_t, S, nA + 1, M);
                double ld_Aj;
                if (oedo_chol_logdet(M, n, &ld_Aj) == 0)
                    gains[c] = 0.5 * (ld_Aj - ld_A) - (hld ? hld[cand[c]] : noise);
                else
                    gains[c] = -INFINITY;
            }
        }
        free(M);
        free(S);
    }
    return oom ? ORC_OOM : ORC_OK;
}

/*
 * Greedy selection of B sensors from the candidate list cand[0..nc) (any
 * order; the scan is in ascending sensor index).  The first nprefix picks are
 * forced to prefix[] (resume / replay of another trajectory); their scores are
 * evaluated exactly like free picks.  Outputs, per step k < *n_out:
 *   idx_out[k]  the sensor picked,
 *   gain_out[k] its score g,
 *   gap_out[k]  best score minus second-best score at that step (+inf when
 *               only one candidate has a finite score),
 *   best_out[k], bestgain_out[k]  the candidate the rule would pick at that
 *               step and its score (differs from idx_out[k] only when forced);
 *               either pointer may be NULL.
 */
int oedo_greedy(const double *K, int64_t ld, int N_t, double sigma2, const double *hld, const int *cand,
                int nc, const int *prefix, int nprefix, int B, int *idx_out, double *gain_out,
                double *gap_out, int *best_out, double *bestgain_out, int *n_out, int nthreads)
{
    *n_out = 0;
    if (!K || N_t <= 0 || !(sigma2 > 0.0) || nc <= 0 || B < 1 || B > nc || nprefix < 0 ||
        nprefix > B)
        return ORC_ARG;
    int *pool = (int *)malloc(sizeof(int) * nc); /* remaining candidates, ascending */
    int *A = (int *)malloc(sizeof(int) * B);
    double *g = (double *)malloc(sizeof(double) * nc);
    if (!pool || !A || !g) {
        free(pool);
        free(A);
        free(g);
        return ORC_OOM;
    }
    memcpy(pool, cand, sizeof(int) * nc);
    for (int a = 1; a < nc; ++a) /* insertion sort: ascending scan order */
        for (int b = a; b > 0 && pool[b - 1] > pool[b]; --b) {
            int t = pool[b];
            pool[b] = pool[b - 1];
            pool[b - 1] = t;
        }
    int npool = nc, status = ORC_OK;
    for (int k = 0; k < B; ++k) {
        int rc = oedo_gains(K, ld, N_t, sigma2, hld, A, k, pool, npool, g, nthreads);
        if (rc != ORC_OK) {
            status = rc;
            break;
        }
        int best = 0; /* first candidate with the strictly largest score */
        for (int c = 0; c < npool; ++c) {
            if (isnan(g[c]))
                g[c] = -INFINITY;
            if (g[c] > g[best])
                best = c;
        }
        if (best_out)
            best_out[k] = pool[best];
        if (bestgain_out)
            bestgain_out[k] = g[best];
        if (k < nprefix) {
            best = -1;
            for (int c = 0; c < npool; ++c)
                if (pool[c] == prefix[k])
                    best = c;
            if (best < 0) {
                status = ORC_ARG;
                break;
            }
        }
        if (g[best] == -INFINITY) {
            status = ORC_NOT_SPD;
            break;
        }
        /* gap between the best and runner-up scores among all candidates */
        double top = -INFINITY, run = -INFINITY;
        for (int c = 0; c < npool; ++c) {
            if (g[c] > top) {
                run = top;
                top = g[c];
            } else if (g[c] > run) {
                run = g[c];
            }
        }
        idx_out[k] = pool[best];
        gain_out[k] = g[best];
        gap_out[k] = (run == -INFINITY) ? INFINITY : top - run;
        A[k] = pool[best];
        for (int c = best; c + 1 < npool; ++c)
            pool[c] = pool[c + 1];
        --npool;
        *n_out = k + 1;
    }
    free(pool);
    free(A);
    free(g);
    return status;
}
