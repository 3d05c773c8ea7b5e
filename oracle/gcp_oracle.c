/*
 * gcp_oracle.c -- plain FP64 CPU oracle for generalized canonical
 * purification (hole-particle canonical purification, HPCP).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never links, includes or calls it, and it shares no code with it.
 *
 * Everything is IEEE double, row-major, with plain loops (OpenMP over rows
 * where a loop is embarrassingly parallel).  No BLAS, no blocking, no fusion.
 *
 * Paper: Truflandier, Dianzinga, Bowler, "Generalized canonical purification
 * for density matrix minimization" (arXiv:1512.07236).  Citations below name
 * the paper's equations:
 *   eq. (dmguess)     D0 = beta1*I + beta2*(mu*I - H)
 *   eq. (pmcpguess)   beta1 = theta, beta2 = min(theta/(Hmax-mu), thetabar/(mu-Hmin)),
 *                     mu = Tr(H)/M, bounds from Gershgorin discs
 *   eq. (hpcp3)       D_{n+1} = D_n + 2( D_n^2 Dbar_n - [Tr(D_n^2 Dbar_n)/Tr(D_n Dbar_n)] D_n Dbar_n )
 *                     with the hole matrix Dbar = I - D (eq. closure)
 *   termination       on Tr(D_n Dbar_n) (paper: <= 1e-6), text after eq. (hpcp3)
 *   eq. (mcw1b)       McWeeny functional Omega = Tr((D^2 - D)^2) = ||D^2 - D||_F^2
 *   eq. (mcw4b)       Lagrangian L = Omega - gamma (Tr(3D^2 - 2D^3) - N)
 *   eq. (mcwgama)     gamma = 1/3 - 2/3 c   (d = 0)
 *   eqs. (pm1a),(pm1b) the Palser-Manolopoulos canonical purification (PMCP)
 *                     of the appendix: D' = [(1-2c)D + (1+c)D^2 - D^3]/(1-c)
 *                     for c <= 1/2, D' = [(1+c)D^2 - D^3]/c for c > 1/2, with
 *                     the same c
 *   eq. (hpcpguess)   hole-particle guess D0+ = alpha D0 + (1-alpha)(I - Dbar0),
 *                     Dbar0 from eqs. (dmguess)+(pmcpguess) with
 *                     beta1 = 1-theta, beta2 = -max(beta_tilde, beta_bar)
 *   eq. (hpcpguessalpha) alpha searched in [0,1] so that Tr(D0+^2) hits a
 *                     target (a quadratic in alpha), delta ~ 2/3
 *
 * Where the paper is silent this file takes these readings:
 *   - symmetry of iterates: after each update D <- (D + D^T)/2 (diagonal, and
 *     therefore the trace, unchanged);
 *   - termination is tested before the division that forms c, on the size of
 *     Tr(D Dbar): |Tr(D Dbar)| <= tol_ddbar (eigenvalues may overshoot [0,1]
 *     slightly near convergence, which makes the trace a signed sum), or on
 *     ||D^2 - D||_F <= tol_idem;
 *   - c outside [0,1], or Tr(D Dbar) < -tol_ddbar, before the tolerance is met
 *     is a breakdown (the paper calls these runaway solutions); nothing is
 *     clamped;
 *   - the alpha-search targets (the paper's condition is garbled): Tr D0+^2 =
 *     N - delta N when theta < 1 - delta, N - delta (M - N) when theta > delta,
 *     and alpha = 1/2 in between (each target is reachable only on its side);
 *     a root outside [0,1] is clamped to [0,1];
 *   - if a hole-particle guess gives Tr(D0+ Dbar0+) <= 0 or c_0 outside [0,1]
 *     (the runaway the paper reports for the naive alpha = 1/2 at extreme
 *     fillings), the solve falls back to alpha = 1, the PMCP guess;
 *   - the eigensolver used for the definition D = sum of the lowest-N
 *     eigenprojectors is cyclic Jacobi (Golub & Van Loan, symmetric Schur
 *     rotations), the textbook method, written out here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_NOT_CONVERGED 1
#define ORACLE_BREAKDOWN 2
#define ORACLE_INVALID (-1)

/* Number of doubles per history row written by oracle_purify. */
#define ORACLE_HIST_COLS 9

/* ------------------------------------------------------------------ */
/* Dense building blocks                                                */
/* ------------------------------------------------------------------ */

/* C = A * B for M x M row-major matrices (i-k-j loop order). */
void oracle_matmul(int64_t M, const double *A, const double *B, double *C)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        double *c = C + i * M;
        for (int64_t j = 0; j < M; ++j) c[j] = 0.0;
        for (int64_t k = 0; k < M; ++k) {
            const double a = A[i * M + k];
            const double *b = B + k * M;
            for (int64_t j = 0; j < M; ++j) c[j] += a * b[j];
        }
    }
}

/* Rows [r0, r1) of C = A * B (same loop as oracle_matmul; used to time a
 * bounded sample of the full product). C is (r1-r0) x M. */
void oracle_matmul_rows(int64_t M, int64_t r0, int64_t r1, const double *A,
                        const double *B, double *C)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = r0; i < r1; ++i) {
        double *c = C + (i - r0) * M;
        for (int64_t j = 0; j < M; ++j) c[j] = 0.0;
        for (int64_t k = 0; k < M; ++k) {
            const double a = A[i * M + k];
            const double *b = B + k * M;
            for (int64_t j = 0; j < M; ++j) c[j] += a * b[j];
        }
    }
}

static double trace(int64_t M, const double *A)
{
    double t = 0.0;
    for (int64_t i = 0; i < M; ++i) t += A[i * M + i];
    return t;
}

/* ------------------------------------------------------------------ */
/* Spectral bounds and the initial guess                                */
/* ------------------------------------------------------------------ */

/* Gershgorin discs: every eigenvalue lies in some [H_ii - r_i, H_ii + r_i]
 * with r_i = sum_{j != i} |H_ij|; the union's ends bound the spectrum. */
void oracle_gershgorin(int64_t M, const double *H, double *emin, double *emax)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < M; ++i) {
        double r = 0.0;
        for (int64_t j = 0; j < M; ++j)
            if (j != i) r += fabs(H[i * M + j]);
        const double d = H[i * M + i];
        if (d - r < lo) lo = d - r;
        if (d + r > hi) hi = d + r;
    }
    *emin = lo;
    *emax = hi;
}

/* Canonical (Palser-Manolopoulos) initial guess, eqs. (dmguess)+(pmcpguess):
 *   theta = N/M, mu = Tr(H)/M,
 *   beta_tilde = theta/(emax - mu), beta_bar = (1-theta)/(mu - emin),
 *   beta = min(beta_tilde, beta_bar),  D0 = theta*I + beta*(mu*I - H).
 * Returns ORACLE_INVALID when the bounds do not bracket mu (0 < N < M).
 * For N = 0 or N = M, beta = 0 and D0 is 0 or I. */
int oracle_initial_guess(int64_t M, int64_t N, const double *H, double emin,
                         double emax, double *D0, double *mu_out,
                         double *beta_out)
{
    if (M <= 0 || N < 0 || N > M) return ORACLE_INVALID;
    const double theta = (double)N / (double)M;
    const double mu = trace(M, H) / (double)M;
    double beta = 0.0;
    if (N > 0 && N < M) {
        if (!(emin < mu && mu < emax)) return ORACLE_INVALID;
        const double beta_tilde = theta / (emax - mu);
        const double beta_bar = (1.0 - theta) / (mu - emin);
        beta = beta_tilde < beta_bar ? beta_tilde : beta_bar;
    }
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < M; ++j)
            D0[i * M + j] = (i == j ? theta + beta * mu : 0.0) - beta * H[i * M + j];
    if (mu_out) *mu_out = mu;
    if (beta_out) *beta_out = beta;
    return ORACLE_OK;
}

/* Hole-particle guess, eq. (hpcpguess): the particle guess D0 (beta =
 * min), the hole guess Dbar0 = (1-theta) I - max(beta_tilde, beta_bar)
 * (mu I - H), and D0+ = alpha D0 + (1 - alpha)(I - Dbar0), formed as matrices.
 * mode 1: alpha as given.  mode 2: alpha from the search of eq.
 * (hpcpguessalpha): Tr(D0+(alpha)^2) is a quadratic in alpha, evaluated at
 * alpha = 0, 1/2, 1 and solved for the target (readings above).
 * scal (may be NULL) receives mu, the effective slope
 * alpha*beta_min + (1-alpha)*beta_max, and alpha. */
static void hp_mix(int64_t M, const double *P, const double *Hb, double alpha, double *out)
{
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < M; ++j) {
            const double id = (i == j) ? 1.0 : 0.0;
            out[i * M + j] = alpha * P[i * M + j] + (1.0 - alpha) * (id - Hb[i * M + j]);
        }
}

static double frob2(int64_t M, const double *A)
{
    double s = 0.0;
    for (int64_t e = 0; e < M * M; ++e) s += A[e] * A[e];
    return s;
}

int oracle_initial_guess_hp(int64_t M, int64_t N, const double *H, double emin,
                            double emax, int mode, double alpha, double delta,
                            double *D0, double *scal)
{
    if (M <= 0 || N < 0 || N > M || (mode != 1 && mode != 2)) return ORACLE_INVALID;
    const double theta = (double)N / (double)M;
    const double mu = trace(M, H) / (double)M;
    if (N == 0 || N == M) {   /* beta = 0: D0 = theta I whatever alpha */
        for (int64_t e = 0; e < M * M; ++e) D0[e] = 0.0;
        for (int64_t i = 0; i < M; ++i) D0[i * M + i] = theta;
        if (scal) { scal[0] = mu; scal[1] = 0.0; scal[2] = 1.0; }
        return ORACLE_OK;
    }
    if (!(emin < mu && mu < emax)) return ORACLE_INVALID;
    const double bt = theta / (emax - mu), bb = (1.0 - theta) / (mu - emin);
    const double bmin = bt < bb ? bt : bb, bmax = bt < bb ? bb : bt;
    double *P = (double *)malloc(sizeof(double) * M * M);
    double *Hb = (double *)malloc(sizeof(double) * M * M);
    if (!P || !Hb) { free(P); free(Hb); return ORACLE_INVALID; }
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < M; ++j) {
            const double g = (i == j ? mu : 0.0) - H[i * M + j];   /* (mu I - H)_ij */
            P[i * M + j] = (i == j ? theta : 0.0) + bmin * g;
            Hb[i * M + j] = (i == j ? 1.0 - theta : 0.0) - bmax * g;
        }
    if (mode == 2) {
        double target = NAN;
        if (theta < 1.0 - delta) target = (double)N - delta * (double)N;
        else if (theta > delta) target = (double)N - delta * (double)(M - N);
        if (isnan(target)) {
            alpha = 0.5;
        } else {
            hp_mix(M, P, Hb, 0.0, D0);
            const double f0 = frob2(M, D0);
            hp_mix(M, P, Hb, 0.5, D0);
            const double fh = frob2(M, D0);
            hp_mix(M, P, Hb, 1.0, D0);
            const double f1 = frob2(M, D0);
            /* q(alpha) = qa alpha^2 + qb alpha + f0 */
            const double qa = 2.0 * f1 - 4.0 * fh + 2.0 * f0;
            const double qb = f1 - f0 - qa;
            const double qc = f0 - target;
            double a = NAN;
            if (fabs(qa) > 0.0) {
                const double disc = qb * qb - 4.0 * qa * qc;
                if (disc >= 0.0) {
                    const double r1 = (-qb - sqrt(disc)) / (2.0 * qa);
                    const double r2 = (-qb + sqrt(disc)) / (2.0 * qa);
                    /* Tr D0+^2 falls on [0,1] (the slope falls from beta_max
                       to beta_min): the root there, else the nearer one */
                    if (r1 >= 0.0 && r1 <= 1.0) a = r1;
                    else if (r2 >= 0.0 && r2 <= 1.0) a = r2;
                    else a = fabs(r1 - 0.5) < fabs(r2 - 0.5) ? r1 : r2;
                }
            }
            if (isnan(a)) a = (f1 > target) ? 1.0 : 0.0;   /* no real root: the nearer end */
            alpha = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
        }
    }
    hp_mix(M, P, Hb, alpha, D0);
    if (scal) { scal[0] = mu; scal[1] = alpha * bmin + (1.0 - alpha) * bmax; scal[2] = alpha; }
    free(P); free(Hb);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* The recursion, eq. (hpcp3)                                           */
/* ------------------------------------------------------------------ */

/*
 * Purify D in place, starting from the given D0 (M x M, symmetric).
 *
 * Per iteration n:
 *   X2 = D D,  DDbar = D - X2 (= D Dbar),  Tr(D Dbar) = Tr D - Tr X2
 *   Omega = ||X2 - D||_F^2
 *   stop if |Tr(D Dbar)| <= tol_ddbar or sqrt(Omega) <= tol_idem
 *   X3 = X2 D,  D2Dbar = X2 - X3 (= D^2 Dbar)
 *   c = Tr(D^2 Dbar) / Tr(D Dbar)
 *   D <- D + 2 (D2Dbar - c DDbar), then D <- (D + D^T)/2
 *
 * hist (may be NULL) receives ORACLE_HIST_COLS doubles per evaluated
 * iterate n = 0..iters (so iters+1 rows; room for max_iter+1 rows):
 *   [n, Tr D, Tr D^2, Tr D^3, c, Omega, gamma, L, ||D_{n+1}-D_n||_F]
 * (Tr D^3, c, gamma, L and the step norm are NaN on the final row).
 * *iters = number of updates applied.  Returns ORACLE_OK,
 * ORACLE_NOT_CONVERGED or ORACLE_BREAKDOWN.
 */
int oracle_purify_from_m(int64_t M, int64_t N, double *D, int method, double tol_ddbar,
                         double tol_idem, int max_iter, double *hist, int *iters)
{
    const int64_t MM = M * M;
    double *X2 = (double *)malloc(sizeof(double) * MM);
    double *X3 = (double *)malloc(sizeof(double) * MM);
    double *T = (double *)malloc(sizeof(double) * MM);
    if (!X2 || !X3 || !T) {
        free(X2); free(X3); free(T);
        return ORACLE_INVALID;
    }
    int status = ORACLE_NOT_CONVERGED;
    int n = 0;
    for (;; ++n) {
        oracle_matmul(M, D, D, X2);
        const double t1 = trace(M, D);
        const double t2 = trace(M, X2);
        double omega = 0.0;
        for (int64_t e = 0; e < MM; ++e) {
            const double r = X2[e] - D[e];
            omega += r * r;
        }
        const double tr_ddbar = t1 - t2;
        double *row = hist ? hist + (int64_t)n * ORACLE_HIST_COLS : NULL;
        if (row) {
            row[0] = n; row[1] = t1; row[2] = t2; row[5] = omega;
            row[3] = row[4] = row[6] = row[7] = row[8] = NAN;
        }
        if (!isfinite(t1) || !isfinite(t2) || !isfinite(omega)) {
            status = ORACLE_BREAKDOWN;
            break;
        }
        if (fabs(tr_ddbar) <= tol_ddbar || sqrt(omega) <= tol_idem) {
            status = ORACLE_OK;
            break;
        }
        if (n >= max_iter) {
            status = ORACLE_NOT_CONVERGED;
            break;
        }
        if (tr_ddbar <= 0.0) {
            status = ORACLE_BREAKDOWN;
            break;
        }
        oracle_matmul(M, X2, D, X3);
        const double t3 = trace(M, X3);
        const double tr_d2dbar = t2 - t3;
        const double c = tr_d2dbar / tr_ddbar;
        const double gamma = 1.0 / 3.0 - 2.0 / 3.0 * c;
        if (row) {
            row[3] = t3; row[4] = c; row[6] = gamma;
            row[7] = omega - gamma * (3.0 * t2 - 2.0 * t3 - (double)N);
        }
        if (!isfinite(c) || c < 0.0 || c > 1.0) {
            status = ORACLE_BREAKDOWN;
            break;
        }
        if (method == 0) {
            /* eq. (hpcp3): D' = D + 2 (D^2 Dbar - c D Dbar) */
            for (int64_t e = 0; e < MM; ++e) {
                const double d2dbar = X2[e] - X3[e];
                const double ddbar = D[e] - X2[e];
                T[e] = D[e] + 2.0 * (d2dbar - c * ddbar);
            }
        } else if (c <= 0.5) {
            /* eq. (pm1a) */
            for (int64_t e = 0; e < MM; ++e)
                T[e] = ((1.0 - 2.0 * c) * D[e] + (1.0 + c) * X2[e] - X3[e]) / (1.0 - c);
        } else {
            /* eq. (pm1b) */
            for (int64_t e = 0; e < MM; ++e)
                T[e] = ((1.0 + c) * X2[e] - X3[e]) / c;
        }
        double step = 0.0;
        for (int64_t i = 0; i < M; ++i)
            for (int64_t j = 0; j < M; ++j) {
                const double s = 0.5 * (T[i * M + j] + T[j * M + i]);
                const double dd = s - D[i * M + j];
                step += dd * dd;
                X3[i * M + j] = s;
            }
        if (row) row[8] = sqrt(step);
        memcpy(D, X3, sizeof(double) * MM);
    }
    *iters = n;
    free(X2); free(X3); free(T);
    return status;
}

/*
 * One update of the recursion from a symmetric D at a GIVEN coefficient c:
 * method 0 applies eq. (hpcp3), D' = D + 2 (D^2 Dbar - c D Dbar); method 1
 * eq. (pm1a) for c <= 1/2 and eq. (pm1b) for c > 1/2.  The result is
 * symmetrised, out = (T + T^T)/2.  tr[0..3] receives Tr D, Tr D^2, Tr D^3 of
 * the products formed here and the coefficient Tr(D^2 Dbar)/Tr(D Dbar) that
 * eq. (hpcp3) itself would use; c = NaN applies that coefficient.  This is
 * the single step of oracle_purify_from_m with c supplied from outside, so a
 * recursion computed elsewhere can be checked one update at a time from its
 * own iterate and its own c.  Returns ORACLE_OK or ORACLE_INVALID (no memory).
 */
int oracle_update_at(int64_t M, const double *D, double c, int method, double *out, double *tr)
{
    const int64_t MM = M * M;
    double *X2 = (double *)malloc(sizeof(double) * MM);
    double *X3 = (double *)malloc(sizeof(double) * MM);
    if (!X2 || !X3) {
        free(X2); free(X3);
        return ORACLE_INVALID;
    }
    oracle_matmul(M, D, D, X2);
    oracle_matmul(M, X2, D, X3);
    const double t1 = trace(M, D), t2 = trace(M, X2), t3 = trace(M, X3);
    const double c_own = (t2 - t3) / (t1 - t2);
    if (tr) { tr[0] = t1; tr[1] = t2; tr[2] = t3; tr[3] = c_own; }
    if (isnan(c)) c = c_own;
    for (int64_t e = 0; e < MM; ++e) {
        double t;
        if (method == 0) {
            const double d2dbar = X2[e] - X3[e];   /* (D^2 Dbar)_e */
            const double ddbar = D[e] - X2[e];     /* (D Dbar)_e */
            t = D[e] + 2.0 * (d2dbar - c * ddbar);
        } else if (c <= 0.5) {
            t = ((1.0 - 2.0 * c) * D[e] + (1.0 + c) * X2[e] - X3[e]) / (1.0 - c);
        } else {
            t = ((1.0 + c) * X2[e] - X3[e]) / c;
        }
        X3[e] = t;   /* X3[e] is not read again */
    }
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < M; ++j) out[i * M + j] = 0.5 * (X3[i * M + j] + X3[j * M + i]);
    free(X2); free(X3);
    return ORACLE_OK;
}

int oracle_purify_from(int64_t M, int64_t N, double *D, double tol_ddbar,
                       double tol_idem, int max_iter, double *hist, int *iters)
{
    return oracle_purify_from_m(M, N, D, 0, tol_ddbar, tol_idem, max_iter, hist, iters);
}

/* c_0 of a guess: (Tr D^2 - Tr D^3) / (Tr D - Tr D^2), NaN unless
 * Tr(D Dbar) > 0 (the recursion would stop or break down at n = 0). */
static double first_c(int64_t M, const double *D)
{
    double *X2 = (double *)malloc(sizeof(double) * M * M);
    double *X3 = (double *)malloc(sizeof(double) * M * M);
    if (!X2 || !X3) { free(X2); free(X3); return NAN; }
    oracle_matmul(M, D, D, X2);
    oracle_matmul(M, X2, D, X3);
    const double t1 = trace(M, D), t2 = trace(M, X2), t3 = trace(M, X3);
    free(X2); free(X3);
    return (t1 - t2) > 0.0 ? (t2 - t3) / (t1 - t2) : NAN;
}

/* Full solve with a method (0 HPCP, 1 PMCP) and an initial guess (0 PMCP
 * guess, 1 hole-particle mix with alpha, 2 alpha search with delta).  A
 * hole-particle guess whose c_0 lies outside [0,1] is replaced by the PMCP
 * guess.  hole = 1 purifies Dbar = I - D instead (the alternative the paper
 * gives before eq. (hpcpguess)); the history is then that of Dbar.
 * scal[0..4]: mu, slope beta, emin, emax, alpha used. */
int oracle_purify_ex(int64_t M, int64_t N, const double *H, double emin, double emax,
                     int method, int init_mode, double alpha, double delta, int hole,
                     double tol_ddbar, double tol_idem, int max_iter, double *D, double *hist,
                     int *iters, double *scal)
{
    if (isnan(emin) || isnan(emax)) oracle_gershgorin(M, H, &emin, &emax);
    double sc[3] = {0.0, 0.0, 1.0};
    int st;
    if (init_mode == 0) {
        st = oracle_initial_guess(M, N, H, emin, emax, D, &sc[0], &sc[1]);
    } else {
        st = oracle_initial_guess_hp(M, N, H, emin, emax, init_mode, alpha, delta, D, sc);
        if (st == ORACLE_OK && N > 0 && N < M) {
            const double c0 = first_c(M, D);
            if (!(c0 >= 0.0 && c0 <= 1.0)) {
                st = oracle_initial_guess(M, N, H, emin, emax, D, &sc[0], &sc[1]);
                sc[2] = 1.0;
            }
        }
    }
    if (scal) { scal[0] = sc[0]; scal[1] = sc[1]; scal[2] = emin; scal[3] = emax; scal[4] = sc[2]; }
    if (st != ORACLE_OK) { *iters = 0; return st; }
    if (!hole)
        return oracle_purify_from_m(M, N, D, method, tol_ddbar, tol_idem, max_iter, hist, iters);
    /* purify the hole matrix Dbar = I - D (trace M - N) and return I - Dbar */
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < M; ++j) D[i * M + j] = (i == j ? 1.0 : 0.0) - D[i * M + j];
    st = oracle_purify_from_m(M, M - N, D, method, tol_ddbar, tol_idem, max_iter, hist, iters);
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < M; ++j) D[i * M + j] = (i == j ? 1.0 : 0.0) - D[i * M + j];
    return st;
}

/* Initial guess from (H, N, bounds) followed by the recursion.  NaN bounds
 * select the Gershgorin bounds.  mu/beta/emin/emax are reported in
 * scal[0..3] when scal is not NULL. */
int oracle_purify(int64_t M, int64_t N, const double *H, double emin,
                  double emax, double tol_ddbar, double tol_idem, int max_iter,
                  double *D, double *hist, int *iters, double *scal)
{
    if (isnan(emin) || isnan(emax)) oracle_gershgorin(M, H, &emin, &emax);
    double mu = 0.0, beta = 0.0;
    const int st = oracle_initial_guess(M, N, H, emin, emax, D, &mu, &beta);
    if (scal) { scal[0] = mu; scal[1] = beta; scal[2] = emin; scal[3] = emax; }
    if (st != ORACLE_OK) { *iters = 0; return st; }
    return oracle_purify_from(M, N, D, tol_ddbar, tol_idem, max_iter, hist, iters);
}

/* ------------------------------------------------------------------ */
/* Definition: projector onto the lowest-N eigenvectors (Jacobi)        */
/* ------------------------------------------------------------------ */

/*
 * Cyclic Jacobi eigensolver for a symmetric M x M matrix A (not modified).
 * w receives the eigenvalues in ascending order and V (row-major) the
 * matching eigenvectors as columns: A = V diag(w) V^T.
 * Sweeps stop when the off-diagonal Frobenius norm falls below
 * tol * ||A||_F or after max_sweeps.  Returns the number of sweeps, or -1.
 */
int oracle_jacobi_eigh(int64_t M, const double *A_in, double *w, double *V,
                       double tol, int max_sweeps)
{
    double *A = (double *)malloc(sizeof(double) * M * M);
    if (!A) return -1;
    memcpy(A, A_in, sizeof(double) * M * M);
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < M; ++j) V[i * M + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int64_t e = 0; e < M * M; ++e) fro += A[e] * A[e];
    fro = sqrt(fro);
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        double off = 0.0;
        for (int64_t p = 0; p < M; ++p)
            for (int64_t q = 0; q < M; ++q)
                if (p != q) off += A[p * M + q] * A[p * M + q];
        if (sqrt(off) <= tol * fro) break;
        for (int64_t p = 0; p < M - 1; ++p) {
            for (int64_t q = p + 1; q < M; ++q) {
                const double apq = A[p * M + q];
                if (apq == 0.0) continue;
                /* Symmetric Schur decomposition of the 2x2 block (p, q). */
                const double tau = (A[q * M + q] - A[p * M + p]) / (2.0 * apq);
                const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                              : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                /* A <- J^T A J with J = [[c, s], [-s, c]] in the (p, q) plane. */
                for (int64_t k = 0; k < M; ++k) {   /* columns p, q */
                    const double akp = A[k * M + p], akq = A[k * M + q];
                    A[k * M + p] = c * akp - s * akq;
                    A[k * M + q] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < M; ++k) {   /* rows p, q */
                    const double apk = A[p * M + k], aqk = A[q * M + k];
                    A[p * M + k] = c * apk - s * aqk;
                    A[q * M + k] = s * apk + c * aqk;
                }
                A[p * M + q] = A[q * M + p] = 0.0;
                for (int64_t k = 0; k < M; ++k) {   /* V <- V J */
                    const double vkp = V[k * M + p], vkq = V[k * M + q];
                    V[k * M + p] = c * vkp - s * vkq;
                    V[k * M + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    /* Sort ascending (selection sort on the diagonal, swapping V columns). */
    for (int64_t i = 0; i < M; ++i) w[i] = A[i * M + i];
    for (int64_t i = 0; i < M; ++i) {
        int64_t m = i;
        for (int64_t j = i + 1; j < M; ++j)
            if (w[j] < w[m]) m = j;
        if (m != i) {
            const double tw = w[i]; w[i] = w[m]; w[m] = tw;
            for (int64_t k = 0; k < M; ++k) {
                const double tv = V[k * M + i];
                V[k * M + i] = V[k * M + m];
                V[k * M + m] = tv;
            }
        }
    }
    free(A);
    return sweep;
}

/* P = sum_{i < N} v_i v_i^T  (columns of V, eigenvalues sorted ascending):
 * the N-representable ground-state density matrix when e_N < e_{N+1}. */
void oracle_projector(int64_t M, int64_t N, const double *V, double *P)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < M; ++j) {
            double s = 0.0;
            for (int64_t k = 0; k < N; ++k) s += V[i * M + k] * V[j * M + k];
            P[i * M + j] = s;
        }
}
