/*
 * Serial O(N) scan form of the Cox / Fine-Gray coordinate gradient and
 * Hessian.  TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the
 * CPU baseline of the benchmark; never by the product library.
 *
 * Paper: Yang, Schuemie, Ji & Suchard, arXiv 2204.08183.
 *  - Sec. 2.7: with subjects in decreasing order of observed time, the Cox
 *    risk-set sums become prefix sums S_pre (eqs. cox_g, cox_h):
 *        g'  = delta' X_j - delta' G,      g'' = -delta' (H - G*G),
 *        G = S_pre[e x_j] / S_pre[e],      H = S_pre[e x_j^2] / S_pre[e].
 *  - Sec. 2.7: Fine-Gray adds a weighted suffix sum S_suf[e W] over the
 *    competing events that happened earlier in time (eqs. fg_g, fg_h).
 *  - Sec. 2.7, the four steps: (1) transform, (2) scans, (3) element-wise
 *    transform with delta, (4) reductions.  Done here one element at a
 *    time, in that order per element.
 *
 * Readings (where the paper is silent):
 *  - ties: every subject of a tie run is in the risk set of the others
 *    (y_r >= Y_i), so the prefix is taken inclusive up to the run's last
 *    position and weighted by the run's event count (Breslow's form);
 *  - Fine-Gray: R_2(Y_i) needs y_r < Y_i strictly, so the suffix starts
 *    after i's tie run, and each suffix term carries G(Y_i)/G(y_r), the
 *    exact IPCW weight of Sec. 2.2, i.e. W_r = 1/G(y_r) for competing
 *    events and the factor G(Y_i) applied at the evaluation point.
 *
 * All sums are Neumaier-compensated so that the oracle's own rounding stays
 * well below the parity tolerance at N = 1e6 and beyond.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct { double s, c; } csum;

static void cadd(csum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double cval(const csum *a) { return a->s + a->c; }

/*
 * Cox.  Inputs in sorted (decreasing time) order:
 *   y[n] observed times, ev[n] event indicator (0/1), eta[n] linear
 *   predictor, x[n] covariate column j (dense).
 * out[0] = g', out[1] = g'', out[2] = log partial likelihood l,
 * out[3] = sum_k d_k G_k, out[4] = sum_k d_k (H_k - G_k^2),
 * out[5] = sum_k d_k log S0_k.
 * out[6..9] = sum_k d_k |G_k|, sum_k d_k (|H_k| + G_k^2),
 * sum_k d_k |log S0_k| and sum over events of |x_kj|: the magnitudes that
 * scale the parity tolerances (g' and l cancel near an optimum).
 */
int oracle_cox_scan(int64_t n, const double *y, const int64_t *ev,
                    const double *eta, const double *x, double *out)
{
    csum S0 = {0, 0}, S1 = {0, 0}, S2 = {0, 0};
    csum A = {0, 0}, B = {0, 0}, L = {0, 0}, C = {0, 0}, E = {0, 0};
    csum SA = {0, 0}, SB = {0, 0}, SL = {0, 0}, SX = {0, 0};
    int64_t d = 0;
    for (int64_t k = 0; k < n; ++k) {
        double e = exp(eta[k]);              /* step (1) */
        cadd(&S0, e);                        /* step (2) */
        cadd(&S1, e * x[k]);
        cadd(&S2, e * x[k] * x[k]);
        if (ev[k]) {
            cadd(&C, x[k]);                  /* delta' X_j */
            cadd(&E, eta[k]);                /* delta' X beta */
            cadd(&SX, fabs(x[k]));
            d += 1;
        }
        if (k == n - 1 || y[k] != y[k + 1]) {   /* last position of a run */
            if (d > 0) {
                double s0 = cval(&S0), s1 = cval(&S1), s2 = cval(&S2);
                double G = s1 / s0, H = s2 / s0;      /* step (3) */
                cadd(&A, (double)d * G);             /* step (4) */
                cadd(&B, (double)d * (H - G * G));
                cadd(&L, (double)d * log(s0));
                cadd(&SA, (double)d * fabs(G));
                cadd(&SB, (double)d * (fabs(H) + G * G));
                cadd(&SL, (double)d * fabs(log(s0)));
            }
            d = 0;
        }
    }
    out[0] = cval(&C) - cval(&A);
    out[1] = -cval(&B);
    out[2] = cval(&E) - cval(&L);
    out[3] = cval(&A);
    out[4] = cval(&B);
    out[5] = cval(&L);
    out[6] = cval(&SA);
    out[7] = cval(&SB);
    out[8] = cval(&SL);
    out[9] = cval(&SX);
    return 0;
}

/*
 * Fine-Gray.  Inputs in sorted (decreasing time) order:
 *   y[n], status[n] in {0,1,2}, eta[n], x[n] (column j, dense),
 *   gy[n] = G(y_k), the Kaplan-Meier censoring survival at each subject's
 *   own time.
 * Same outputs as oracle_cox_scan; the sums over events run over status 1.
 */
int oracle_fg_scan(int64_t n, const double *y, const int64_t *status,
                   const double *eta, const double *x, const double *gy,
                   double *out)
{
    double *q0 = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *q1 = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *q2 = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!q0 || !q1 || !q2) {
        free(q0); free(q1); free(q2);
        return -1;
    }
    /* backward pass: at each run end k, Q_m = sum over r > k of
     * e_r x_r^m W_r with W_r = I(status_r = 2) / G(y_r) */
    csum Q0 = {0, 0}, Q1 = {0, 0}, Q2 = {0, 0};
    for (int64_t k = n - 1; k >= 0; --k) {
        if (k == n - 1 || y[k] != y[k + 1]) {
            q0[k] = cval(&Q0);
            q1[k] = cval(&Q1);
            q2[k] = cval(&Q2);
        }
        if (status[k] == 2) {
            double ew = exp(eta[k]) / gy[k];
            cadd(&Q0, ew);
            cadd(&Q1, ew * x[k]);
            cadd(&Q2, ew * x[k] * x[k]);
        }
    }
    /* forward pass */
    csum S0 = {0, 0}, S1 = {0, 0}, S2 = {0, 0};
    csum A = {0, 0}, B = {0, 0}, L = {0, 0}, C = {0, 0}, E = {0, 0};
    csum SA = {0, 0}, SB = {0, 0}, SL = {0, 0}, SX = {0, 0};
    int64_t d = 0;
    for (int64_t k = 0; k < n; ++k) {
        double e = exp(eta[k]);
        cadd(&S0, e);
        cadd(&S1, e * x[k]);
        cadd(&S2, e * x[k] * x[k]);
        if (status[k] == 1) {
            cadd(&C, x[k]);
            cadd(&E, eta[k]);
            cadd(&SX, fabs(x[k]));
            d += 1;
        }
        if (k == n - 1 || y[k] != y[k + 1]) {
            if (d > 0) {
                double g = gy[k];
                double s0 = cval(&S0) + g * q0[k];
                double s1 = cval(&S1) + g * q1[k];
                double s2 = cval(&S2) + g * q2[k];
                double G = s1 / s0, H = s2 / s0;
                cadd(&A, (double)d * G);
                cadd(&B, (double)d * (H - G * G));
                cadd(&L, (double)d * log(s0));
                cadd(&SA, (double)d * fabs(G));
                cadd(&SB, (double)d * (fabs(H) + G * G));
                cadd(&SL, (double)d * fabs(log(s0)));
            }
            d = 0;
        }
    }
    out[0] = cval(&C) - cval(&A);
    out[1] = -cval(&B);
    out[2] = cval(&E) - cval(&L);
    out[3] = cval(&A);
    out[4] = cval(&B);
    out[5] = cval(&L);
    out[6] = cval(&SA);
    out[7] = cval(&SB);
    out[8] = cval(&SL);
    out[9] = cval(&SX);
    free(q0); free(q1); free(q2);
    return 0;
}
