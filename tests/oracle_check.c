/*
 * Memory-safety driver for the C oracle (test infrastructure): builds the
 * 5-point lattice graph of a small grid plus one observed node per row in
 * plain C, then runs every oracle entry point -- iterations with and without
 * divergence, beliefs, marginals, residual, message change -- so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer checks every access.
 * Prints "ok" and exits 0 when the run is clean and the results are finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_gabp_iterate(int64_t n, const int64_t *row_ptr, const int64_t *col,
                        const double *aoff, const int64_t *rev, const double *adiag,
                        const double *b, double c, double eta, int64_t iters, double *lam,
                        double *th, int64_t *iters_done);
void oracle_beliefs(int64_t n, const int64_t *row_ptr, const double *adiag, const double *b,
                    double c, const double *lam, const double *th, double *bl, double *bt);
void oracle_posterior(int64_t n, const int64_t *row_ptr, const double *adiag, const double *b,
                      double c, const double *lam, const double *th, double *mu, double *var);
void oracle_residual(int64_t n, const int64_t *row_ptr, const int64_t *col, const double *aoff,
                     const double *adiag, const double *b, const double *mu, double *out);
double oracle_abs_change(int64_t nnz, const double *lam_a, const double *th_a,
                         const double *lam_b, const double *th_b);

enum { NX = 9, NY = 7, N = NX * NY };

int main(void) {
    static int64_t row_ptr[N + 1], col[4 * N], rev[4 * N];
    static double aoff[4 * N], adiag[N], b[N];
    int64_t e = 0;
    for (int i = 0; i < N; ++i) {
        const int x = i % NX, y = i / NX;
        row_ptr[i] = e;
        const int nb[4] = {y > 0 ? i - NX : -1, x > 0 ? i - 1 : -1, x < NX - 1 ? i + 1 : -1,
                           y < NY - 1 ? i + NX : -1};
        int deg = 0;
        for (int k = 0; k < 4; ++k) {
            if (nb[k] < 0) continue;
            col[e] = nb[k];
            aoff[e] = -1.0;
            ++e;
            ++deg;
        }
        adiag[i] = 0.04 + deg + (x == 3 ? 100.0 : 0.0);   /* kappa^2 + degree + observations */
        b[i] = x == 3 ? 100.0 * sin(0.7 * y) : 0.0;
    }
    row_ptr[N] = e;
    for (int64_t s = 0; s < e; ++s) {   /* slot of the reverse edge */
        int64_t i = 0;
        while (row_ptr[i + 1] <= s) ++i;
        const int64_t j = col[s];
        rev[s] = -1;
        for (int64_t r = row_ptr[j]; r < row_ptr[j + 1]; ++r)
            if (col[r] == i) rev[s] = r;
        if (rev[s] < 0) return 2;
    }
    double *lam = calloc((size_t)e, sizeof(double)), *th = calloc((size_t)e, sizeof(double));
    double *lam0 = calloc((size_t)e, sizeof(double)), *th0 = calloc((size_t)e, sizeof(double));
    double bl[N], bt[N], mu[N], var[N], res[2];
    int64_t done = 0;
    if (!lam || !th || !lam0 || !th0) return 3;
    int st = oracle_gabp_iterate(N, row_ptr, col, aoff, rev, adiag, b, 1.0, 0.5, 200, lam, th,
                                 &done);
    if (st != 0 || done != 200) return 4;
    oracle_beliefs(N, row_ptr, adiag, b, 1.0, lam, th, bl, bt);
    oracle_posterior(N, row_ptr, adiag, b, 1.0, lam, th, mu, var);
    oracle_residual(N, row_ptr, col, aoff, adiag, b, mu, res);
    const double ch = oracle_abs_change(e, lam, th, lam0, th0);
    for (int i = 0; i < N; ++i)
        if (!isfinite(mu[i]) || !(var[i] > 0.0) || !isfinite(bl[i]) || !isfinite(bt[i])) return 5;
    if (!(res[0] < 1e-6 * res[1]) || !isfinite(ch)) return 6;
    /* a small re-weighting constant on a weak diagonal drives the cavity
       precisions negative: the run must stop cleanly with status 4 */
    for (int i = 0; i < N; ++i) adiag[i] = 0.01;
    for (int64_t s = 0; s < e; ++s) lam[s] = th[s] = 0.0;
    st = oracle_gabp_iterate(N, row_ptr, col, aoff, rev, adiag, b, 0.3, 1.0, 50, lam, th, &done);
    if (st != 4) return 7;
    free(lam);
    free(th);
    free(lam0);
    free(th0);
    puts("ok");
    return 0;
}
