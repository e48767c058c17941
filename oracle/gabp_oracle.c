/*
 * FP64 reference ("oracle") for re-weighted, damped Gaussian belief propagation
 * on a general sparse symmetric graph.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into a separate shared
 * object that only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load.  It shares no code, header, table or helper with the
 * GPU library, and the GPU library never calls it.
 *
 * What it computes (paper, Appendix "Background on Message Passing",
 * subsections "Gaussian Setting" and "Re-weighted message updates", and
 * Algorithms 1 and 2):
 *
 *   Graph: nodes i with diagonal precision A_ii (prior diagonal plus
 *   observation precision, Section "Including Observations") and information
 *   b_i; an edge for every off-diagonal A_ij != 0 (Section "Derivation of the
 *   Factor Graph").  Messages are Gaussian in information form,
 *   m_{j->i}(x) = exp(-1/2 Lam x^2 + th x).
 *
 *   One flooding iteration t (every new message from iteration t-1 values):
 *     belief      Lam_i = A_ii + c * sum_k Lam_{k->i},  th_i = b_i + c * sum_k th_{k->i}
 *     cavity      Lam_c = Lam_i - Lam_{j->i},           th_c = th_i - th_{j->i}
 *                 (= A_ii + c sum_{k != j} Lam_{k->i} + (c - 1) Lam_{j->i},
 *                  the re-weighted variable-to-factor parameters)
 *     new message Lam~_{i->j} = -(A_ij / c)^2 / Lam_c
 *                 th~_{i->j}  = -(A_ij / c) * th_c / Lam_c
 *     damping     m^t = (1 - eta) m^{t-1} + eta m~     (Section "Update Damping")
 *   Marginals: mu_i = th_i / Lam_i, var_i = 1 / Lam_i.
 *
 * Reading of the paper: its linear-term update completes the square with the
 * wrong sign, which gives wrong means from a 3-node chain onward; the
 * information form above is the first-principles version (identical to the
 * paper's equations with b -> -b in the message-to-cavity step).  The test
 * suite pins this with exact 2- and 3-node and chain/tree results.
 *
 * Divergence: an iteration whose cavity precision is not strictly positive,
 * or whose new values are not finite, ends the run with status 4; the
 * messages of that iteration are kept.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_E_NOMEM 2
#define ORACLE_E_DIVERGED 4

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Beliefs (marginal natural parameters) of every node from the messages.
 * CSR row i lists the neighbours j of i; slot e = (i, j) holds the message
 * INTO i FROM j.
 */
void oracle_beliefs(int64_t n, const int64_t *row_ptr, const double *adiag,
                    const double *b, double c, const double *lam, const double *th,
                    double *bel_lam, double *bel_th) {
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        double sl = 0.0, st = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            sl += lam[e];
            st += th[e];
        }
        bel_lam[i] = adiag[i] + c * sl;
        bel_th[i] = b[i] + c * st;
    }
}

/*
 * Run `iters` flooding iterations starting from (lam, th) = m^{t0}.
 * On return (lam, th) hold m^{t0 + done}, where done = iters unless the run
 * diverged (then done is the iteration that produced invalid values and the
 * messages of that iteration are returned).
 */
int oracle_gabp_iterate(int64_t n, const int64_t *row_ptr, const int64_t *col,
                        const double *aoff, const int64_t *rev, const double *adiag,
                        const double *b, double c, double eta, int64_t iters,
                        double *lam, double *th, int64_t *iters_done) {
    (void)col;
    int64_t nnz = row_ptr[n];
    double *bl = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *bt = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *nl = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *nt = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!bl || !bt || !nl || !nt) {
        free(bl); free(bt); free(nl); free(nt);
        return ORACLE_E_NOMEM;
    }
    int status = ORACLE_OK;
    int64_t done = 0;
    for (int64_t t = 1; t <= iters; ++t) {
        /* step 1: beliefs from m^{t-1} */
        oracle_beliefs(n, row_ptr, adiag, b, c, lam, th, bl, bt);
        /* step 2: every directed edge i -> j, written at the receiver's slot */
        int bad = 0;
        int64_t i;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (i = 0; i < n; ++i) {
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                /* slot e holds j -> i; the outgoing i -> j lives at rev[e] */
                double lam_c = bl[i] - lam[e];
                double th_c = bt[i] - th[e];
                double q = aoff[e] / c;
                double new_l = -(q * q) / lam_c;
                double new_t = -(q * th_c) / lam_c;
                int64_t r = rev[e];
                double ol = lam[r], ot = th[r];
                double dl = (1.0 - eta) * ol + eta * new_l;
                double dt = (1.0 - eta) * ot + eta * new_t;
                if (!(lam_c > 0.0) || !isfinite(new_l) || !isfinite(new_t) ||
                    !isfinite(dl) || !isfinite(dt))
                    bad |= 1;
                nl[r] = dl;
                nt[r] = dt;
            }
        }
        memcpy(lam, nl, sizeof(double) * (size_t)nnz);
        memcpy(th, nt, sizeof(double) * (size_t)nnz);
        done = t;
        if (bad) {
            status = ORACLE_E_DIVERGED;
            break;
        }
    }
    free(bl); free(bt); free(nl); free(nt);
    *iters_done = done;
    return status;
}

/* Marginal mean and variance of every node (Compute Marginal). */
void oracle_posterior(int64_t n, const int64_t *row_ptr, const double *adiag,
                      const double *b, double c, const double *lam, const double *th,
                      double *mu, double *var) {
    double *bl = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *bt = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    oracle_beliefs(n, row_ptr, adiag, b, c, lam, th, bl, bt);
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        mu[i] = bt[i] / bl[i];
        var[i] = 1.0 / bl[i];
    }
    free(bl);
    free(bt);
}

/*
 * Residual of the posterior-mean equations A mu = b, in FP64:
 * out[0] = ||A mu - b||_2, out[1] = ||b||_2.
 */
void oracle_residual(int64_t n, const int64_t *row_ptr, const int64_t *col,
                     const double *aoff, const double *adiag, const double *b,
                     const double *mu, double *out) {
    double rr = 0.0, bb = 0.0;
    int64_t i;
#pragma omp parallel for schedule(static) reduction(+ : rr, bb)
    for (i = 0; i < n; ++i) {
        double s = adiag[i] * mu[i];
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) s += aoff[e] * mu[col[e]];
        double r = s - b[i];
        rr += r * r;
        bb += b[i] * b[i];
    }
    out[0] = sqrt(rr);
    out[1] = sqrt(bb);
}

/* Sum of |a - b| over both message components (the early-stop statistic's numerator). */
double oracle_abs_change(int64_t nnz, const double *lam_a, const double *th_a,
                         const double *lam_b, const double *th_b) {
    double s = 0.0;
    int64_t e;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (e = 0; e < nnz; ++e) s += fabs(lam_a[e] - lam_b[e]) + fabs(th_a[e] - th_b[e]);
    return s;
}
