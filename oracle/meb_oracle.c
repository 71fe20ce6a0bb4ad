/*
 * meb_oracle.c -- plain FP64 CPU oracle for the minimum enclosing ball (MEB)
 * of m balls in R^d, solved by ripALM with a semismooth-Newton inner solver
 * (Liang & Yang, "Mixed-Precision GPU Acceleration for Large-Scale Minimum
 * Enclosing Ball Problems").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code with the GPU path.
 *
 * Style: every quantity is written the way the paper defines it, one ball at
 * a time, in IEEE double precision.  Sums over balls are accumulated in
 * `long double` in ball order (no blocking, no reordering) so that the
 * oracle's own rounding stays far below the tolerances it is used to check.
 * Per-ball generalized Jacobians are formed as explicit (d+1)x(d+1) matrices.
 *
 * Conventions
 *   x = (r, c) in R^{d+1}, r at index 0 (the SOCP form, Section 2).
 *   C is m x d row-major, R has m entries (NULL means points, r_i = 0).
 *   U has m entries, V is m x d row-major: the conic multipliers (u_i, v_i).
 *
 * Readings of points the paper leaves open (each is also listed in the
 * design notes): the scale L, the starting point, the parameter schedule,
 * the Armijo constants, the two rounding safeguards of the inner loop and
 * the final radius fix-up.  They are marked "reading" below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double acc_t;

/* reading: relative margin of the starting radius above L (see orc_ripalm) */
#define ORC_START_MARGIN 0x1p-10

/* ------------------------------------------------------------------------ */
/* Second-order cone primitives (Section 2, closed-form projection).        */
/* ------------------------------------------------------------------------ */

static double norm2(const double* s, int d) {
    acc_t a = 0;
    for (int k = 0; k < d; ++k) a += (acc_t)s[k] * s[k];
    return sqrt((double)a);
}

/* Projection of (t, s) onto Q_{d+1} = {(t, s) : ||s|| <= t}.
 * Returns the case: 0 = interior (||s|| <= t), 1 = polar (||s|| <= -t),
 * 2 = otherwise.  Ties are taken in that order, so (0, 0) is "interior". */
int orc_soc_project(int d, double t, const double* s, double* pt, double* ps) {
    double n = norm2(s, d);
    if (n <= t) {
        *pt = t;
        for (int k = 0; k < d; ++k) ps[k] = s[k];
        return 0;
    }
    if (n <= -t) {
        *pt = 0.0;
        for (int k = 0; k < d; ++k) ps[k] = 0.0;
        return 1;
    }
    double a = 0.5 * (t + n);
    *pt = a;
    for (int k = 0; k < d; ++k) ps[k] = a * s[k] / n;
    return 2;
}

/* One element of the Clarke generalized Jacobian of the projection at
 * (t, s), written as a full (d+1)x(d+1) row-major matrix P:
 *   interior -> identity, polar -> zero, otherwise the derivative of
 *   ((t+n)/2) (1, s/n), i.e. 1/2 [[1, w^T], [w, (1 + t/n) I - (t/n) w w^T]]
 *   with n = ||s||, w = s/n.  (Section 4, generalized Hessian.) */
int orc_soc_jacobian(int d, double t, const double* s, double* P) {
    int n1 = d + 1;
    double n = norm2(s, d);
    memset(P, 0, sizeof(double) * (size_t)n1 * n1);
    if (n <= t) {
        for (int k = 0; k < n1; ++k) P[k * n1 + k] = 1.0;
        return 0;
    }
    if (n <= -t) return 1;
    double q = t / n;
    P[0] = 0.5;
    for (int k = 0; k < d; ++k) {
        double wk = s[k] / n;
        P[0 * n1 + (k + 1)] = 0.5 * wk;
        P[(k + 1) * n1 + 0] = 0.5 * wk;
        for (int l = 0; l < d; ++l) {
            double wl = s[l] / n;
            double v = -q * wk * wl;
            if (k == l) v += 1.0 + q;
            P[(k + 1) * n1 + (l + 1)] = 0.5 * v;
        }
    }
    return 2;
}

/* Euclidean distance from (t, s) to Q_{d+1}.  It is the norm of
 * (t, s) - Proj(t, s), evaluated from the same three cases. */
static double soc_dist_tn(double t, double n) {
    if (n <= t) return 0.0;
    if (n <= -t) return sqrt(t * t + n * n);
    return (n - t) / sqrt(2.0);
}

double orc_soc_dist(int d, double t, const double* s) { return soc_dist_tn(t, norm2(s, d)); }

/* ------------------------------------------------------------------------ */
/* Proximal augmented Lagrangian evaluation (Sections 2-4).                 */
/* ------------------------------------------------------------------------ */

/* For fixed multipliers (U, V), penalty sigma, proximal weight tau and
 * proximal center xbar, evaluates at x = (r, c):
 *   Psi(x)   = r + sigma/2 sum_i ||Proj(z_i)||^2 - 1/(2 sigma) sum_i ||(u_i, v_i)||^2
 *              + tau/(2 sigma) ||x - xbar||^2,
 *   z_i      = (r_i - r, c_i - c) + (u_i, v_i) / sigma,
 *   g        = (1, 0) - sigma sum_i Proj(z_i) + tau/sigma (x - xbar),
 *   H        = tau/sigma I + sigma sum_i P_i,  P_i a Jacobian element at z_i,
 *   (u_i+, v_i+) = sigma Proj(z_i)  (the multiplier update),
 *   dmult    = sum_i ||(u_i+ - u_i, v_i+ - v_i)||^2.
 * Any output pointer may be NULL.  U or V NULL means zero multipliers.
 * counts (nullable) receives {#interior, #polar, #other}; rscale (nullable)
 * receives sum over non-polar balls of |t_i| + ||s_i||, the magnitude of the
 * terms that cancel in g (used for the rounding floor of the inner loop). */
int orc_al_eval(int64_t m, int d, const double* C, const double* R, const double* U, const double* V,
                const double* x, const double* xbar, double sigma, double tau,
                double* psi, double* g, double* H, double* Unew, double* Vnew, double* dmult,
                int64_t* counts, double* rscale) {
    int n1 = d + 1;
    double* s = (double*)malloc(sizeof(double) * d);
    double* ps = (double*)malloc(sizeof(double) * d);
    double* P = H ? (double*)malloc(sizeof(double) * (size_t)n1 * n1) : NULL;
    acc_t* hacc = H ? (acc_t*)calloc((size_t)n1 * n1, sizeof(acc_t)) : NULL;
    acc_t* gacc = (acc_t*)calloc((size_t)n1, sizeof(acc_t));
    acc_t zsum = 0, wsum = 0, dsum = 0, rs = 0;
    int64_t cnt[3] = {0, 0, 0};
    for (int64_t i = 0; i < m; ++i) {
        const double* ci = C + (size_t)i * d;
        double ri = R ? R[i] : 0.0;
        double ui = U ? U[i] : 0.0;
        const double* vi = V ? V + (size_t)i * d : NULL;
        double t = ri - x[0] + ui / sigma;
        for (int k = 0; k < d; ++k) s[k] = ci[k] - x[1 + k] + (vi ? vi[k] / sigma : 0.0);
        double pt;
        int cs = orc_soc_project(d, t, s, &pt, ps);
        cnt[cs]++;
        if (cs != 1) rs += fabs(t) + norm2(s, d);
        /* ||Proj(z_i)||^2 and ||(u_i, v_i)||^2 */
        acc_t pp = (acc_t)pt * pt;
        for (int k = 0; k < d; ++k) pp += (acc_t)ps[k] * ps[k];
        zsum += pp;
        acc_t ww = (acc_t)ui * ui;
        if (vi)
            for (int k = 0; k < d; ++k) ww += (acc_t)vi[k] * vi[k];
        wsum += ww;
        /* sum of Proj(z_i) -> gradient */
        gacc[0] += pt;
        for (int k = 0; k < d; ++k) gacc[1 + k] += ps[k];
        /* multiplier update and its change */
        double up = sigma * pt;
        acc_t dd = ((acc_t)up - ui) * ((acc_t)up - ui);
        for (int k = 0; k < d; ++k) {
            double vp = sigma * ps[k];
            double vo = vi ? vi[k] : 0.0;
            dd += ((acc_t)vp - vo) * ((acc_t)vp - vo);
        }
        dsum += dd;
        if (Unew) Unew[i] = up;
        if (Vnew)
            for (int k = 0; k < d; ++k) Vnew[(size_t)i * d + k] = sigma * ps[k];
        if (H && cs != 1) {
            orc_soc_jacobian(d, t, s, P);
            for (int a = 0; a < n1 * n1; ++a) hacc[a] += P[a];
        }
    }
    acc_t dx2 = 0;
    for (int k = 0; k < n1; ++k) dx2 += ((acc_t)x[k] - xbar[k]) * ((acc_t)x[k] - xbar[k]);
    if (psi)
        *psi = (double)((acc_t)x[0] + (acc_t)sigma / 2 * zsum - wsum / (2 * (acc_t)sigma) +
                        (acc_t)tau / (2 * (acc_t)sigma) * dx2);
    if (g) {
        for (int k = 0; k < n1; ++k) {
            acc_t v = (k == 0 ? 1.0L : 0.0L) - (acc_t)sigma * gacc[k] +
                      (acc_t)tau / sigma * ((acc_t)x[k] - xbar[k]);
            g[k] = (double)v;
        }
    }
    if (H) {
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n1; ++b)
                H[a * n1 + b] = (double)((a == b ? (acc_t)tau / sigma : 0.0L) + (acc_t)sigma * hacc[a * n1 + b]);
    }
    if (dmult) *dmult = (double)dsum;
    if (rscale) *rscale = (double)rs;
    if (counts) {
        counts[0] = cnt[0];
        counts[1] = cnt[1];
        counts[2] = cnt[2];
    }
    free(s);
    free(ps);
    free(P);
    free(hacc);
    free(gacc);
    return 0;
}

/* Maximum KKT residual (Section 5, "maximum KKT residual"):
 *   max{ |1 - sum u_i|, ||sum v_i||, max_i dist((r - r_i, c - c_i), Q),
 *        max_i dist((u_i, v_i), Q), max_i |(r - r_i) u_i + <c - c_i, v_i>| }.
 * parts (nullable) receives the five terms in that order. */
double orc_kkt_max(int64_t m, int d, const double* C, const double* R, const double* U, const double* V,
                   const double* x, double* parts) {
    acc_t su = 0;
    acc_t* sv = (acc_t*)calloc((size_t)d, sizeof(acc_t));
    double* e = (double*)malloc(sizeof(double) * d);
    double dp = 0, dd = 0, cp = 0;
    for (int64_t i = 0; i < m; ++i) {
        const double* ci = C + (size_t)i * d;
        const double* vi = V + (size_t)i * d;
        double ri = R ? R[i] : 0.0;
        su += U[i];
        for (int k = 0; k < d; ++k) sv[k] += vi[k];
        for (int k = 0; k < d; ++k) e[k] = x[1 + k] - ci[k];
        double tp = x[0] - ri;
        double a = orc_soc_dist(d, tp, e);
        if (a > dp) dp = a;
        double b = orc_soc_dist(d, U[i], vi);
        if (b > dd) dd = b;
        acc_t c = (acc_t)tp * U[i];
        for (int k = 0; k < d; ++k) c += (acc_t)e[k] * vi[k];
        double cc = fabs((double)c);
        if (cc > cp) cp = cc;
    }
    acc_t n2 = 0;
    for (int k = 0; k < d; ++k) n2 += sv[k] * sv[k];
    double p[5] = {fabs((double)(1.0L - su)), sqrt((double)n2), dp, dd, cp};
    double mx = 0;
    for (int k = 0; k < 5; ++k) {
        if (parts) parts[k] = p[k];
        if (p[k] > mx) mx = p[k];
    }
    free(sv);
    free(e);
    return mx;
}

/* ------------------------------------------------------------------------ */
/* Screening and the a-posteriori feasibility check (Section 4.2).          */
/* ------------------------------------------------------------------------ */

/* slack_i = rhat - r_i - ||chat - c_i||; keeps {i : slack_i <= tol_red} in
 * ascending order.  Returns the number kept; slack (nullable) gets all m. */
int64_t orc_screen(int64_t m, int d, const double* C, const double* R, double rhat, const double* chat,
                   double tol_red, int64_t* keep, double* slack) {
    double* e = (double*)malloc(sizeof(double) * d);
    int64_t n = 0;
    for (int64_t i = 0; i < m; ++i) {
        for (int k = 0; k < d; ++k) e[k] = chat[k] - C[(size_t)i * d + k];
        double si = rhat - (R ? R[i] : 0.0) - norm2(e, d);
        if (slack) slack[i] = si;
        if (si <= tol_red) {
            if (keep) keep[n] = i;
            n++;
        }
    }
    free(e);
    return n;
}

/* Delta_max = max_i (r_i + ||c - c_i|| - r) and the violated set
 * {i : r_i + ||c - c_i|| - r > eps} in ascending order (at most cap stored).
 * argmax gets the smallest index attaining the maximum. */
double orc_check_feasible(int64_t m, int d, const double* C, const double* R, double r, const double* c,
                          double eps, int64_t* argmax, int64_t* viol, int64_t cap, int64_t* nviol) {
    double* e = (double*)malloc(sizeof(double) * d);
    double best = -INFINITY;
    int64_t bi = -1, n = 0;
    for (int64_t i = 0; i < m; ++i) {
        for (int k = 0; k < d; ++k) e[k] = c[k] - C[(size_t)i * d + k];
        double v = (R ? R[i] : 0.0) + norm2(e, d) - r;
        if (v > best) {
            best = v;
            bi = i;
        }
        if (v > eps) {
            if (viol && n < cap) viol[n] = i;
            n++;
        }
    }
    if (argmax) *argmax = bi;
    if (nviol) *nviol = n;
    free(e);
    return best;
}

/* ------------------------------------------------------------------------ */
/* Dense Cholesky solve for the Newton system (Section 4.1).                */
/* ------------------------------------------------------------------------ */

/* Solves A x = b for symmetric positive definite A (n x n, row-major) with
 * A = L L^T.  A and b are not modified.  Returns 0, or -1 if a pivot is not
 * positive. */
int orc_chol_solve(int n, const double* A, const double* b, double* x) {
    double* Lm = (double*)calloc((size_t)n * n, sizeof(double));
    for (int j = 0; j < n; ++j) {
        acc_t s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= (acc_t)Lm[j * n + k] * Lm[j * n + k];
        if (!(s > 0)) {
            free(Lm);
            return -1;
        }
        double ljj = sqrt((double)s);
        Lm[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            acc_t t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= (acc_t)Lm[i * n + k] * Lm[j * n + k];
            Lm[i * n + j] = (double)(t / ljj);
        }
    }
    double* y = (double*)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) {
        acc_t t = b[i];
        for (int k = 0; k < i; ++k) t -= (acc_t)Lm[i * n + k] * y[k];
        y[i] = (double)(t / Lm[i * n + i]);
    }
    for (int i = n - 1; i >= 0; --i) {
        acc_t t = y[i];
        for (int k = i + 1; k < n; ++k) t -= (acc_t)Lm[k * n + i] * x[k];
        x[i] = (double)(t / Lm[i * n + i]);
    }
    free(y);
    free(Lm);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* ripALM (Algorithm 1) with the semismooth Newton inner solver (Alg. 2).   */
/* ------------------------------------------------------------------------ */

typedef struct {
    double rho;          /* relative-error weight, in [0, 1)                       */
    double sigma0;       /* first penalty, normalized units (reading: 1)           */
    double sigma_growth; /* sigma_{k+1} = min(growth * sigma_k, sigma_max)        */
    double sigma_max;    /* reading: 1e5                                           */
    double tau;          /* proximal weight, constant (reading: 1)                 */
    double tol;          /* stop when KKT_max (normalized) <= tol                  */
    int max_outer;
    int max_inner;
    int max_ls;
    int stall_outer;     /* stop after this many outer steps without KKT progress */
} orc_params;

typedef struct {
    int outer;
    int inner;
    int ls_evals;
    double kkt;
    double L;
    double rbar;    /* radius returned by the last outer iterate       */
    double r_fixed; /* max(rbar, max_i r_i + ||c - c_i||): feasible   */
    double kkt_parts[5];
} orc_stats;

void orc_default_params(orc_params* p) {
    p->rho = 0.9;
    p->sigma0 = 1.0;
    p->sigma_growth = 5.0;
    p->sigma_max = 1e5;
    p->tau = 1.0;
    p->tol = 1e-8;
    p->max_outer = 200;
    p->max_inner = 50;
    p->max_ls = 40;
    p->stall_outer = 3;
}

/* Solves (MEB) for the m balls (C, R).
 *
 * Reading (scale): the paper states KKT_max and its parameters without
 * units.  The oracle runs the algorithm on normalized data
 *   c_i' = (c_i - c_1) / L,  r_i' = r_i / L,  L = max_i (||c_i - c_1|| + r_i),
 * where L is the radius of a feasible ball centered at c_1 (so L is between
 * r* and 2 r*), and maps the result back.  Multipliers are unitless and are
 * the same in both coordinates.
 * Reading (start): (r^0, c^0) = (1, 0) in normalized units, i.e. the
 * feasible ball (L, c_1); (alpha^0, beta^0) = (r^0, c^0); multipliers zero,
 * unless x0 / U / V warm starts are given (x0 in original units).
 *
 * Outputs: x_out = (r, c) of the last outer iterate (original units);
 * U, V (nullable, m and m x d) receive the final multipliers.
 * Returns 0 if KKT_max <= tol, 1 otherwise (max_outer or stall). */
int orc_ripalm(int64_t m, int d, const double* C, const double* R, const orc_params* prm,
               const double* x0, const double* U0, const double* V0,
               double* x_out, double* U_out, double* V_out, orc_stats* st) {
    const double eps = 2.220446049250313e-16;
    int n1 = d + 1;
    /* normalization */
    double* e = (double*)malloc(sizeof(double) * d);
    double L = 0;
    for (int64_t i = 0; i < m; ++i) {
        for (int k = 0; k < d; ++k) e[k] = C[(size_t)i * d + k] - C[k];
        double v = norm2(e, d) + (R ? R[i] : 0.0);
        if (v > L) L = v;
    }
    if (!(L > 0)) { /* every ball is the point c_1 */
        x_out[0] = 0.0;
        for (int k = 0; k < d; ++k) x_out[1 + k] = C[k];
        if (U_out) { memset(U_out, 0, sizeof(double) * m); U_out[0] = 1.0; }
        if (V_out) memset(V_out, 0, sizeof(double) * (size_t)m * d);
        if (st) { memset(st, 0, sizeof(*st)); }
        free(e);
        return 0;
    }
    double* Cn = (double*)malloc(sizeof(double) * (size_t)m * d);
    double* Rn = (double*)malloc(sizeof(double) * m);
    for (int64_t i = 0; i < m; ++i) {
        for (int k = 0; k < d; ++k) Cn[(size_t)i * d + k] = (C[(size_t)i * d + k] - C[k]) / L;
        Rn[i] = (R ? R[i] : 0.0) / L;
    }
    double* U = (double*)calloc((size_t)m, sizeof(double));
    double* V = (double*)calloc((size_t)m * d, sizeof(double));
    double* Up = (double*)malloc(sizeof(double) * m);
    double* Vp = (double*)malloc(sizeof(double) * (size_t)m * d);
    if (U0) memcpy(U, U0, sizeof(double) * m);
    if (V0) memcpy(V, V0, sizeof(double) * (size_t)m * d);
    double* x = (double*)malloc(sizeof(double) * n1);
    double* xbar = (double*)malloc(sizeof(double) * n1);
    double* ab = (double*)malloc(sizeof(double) * n1);
    double* xt = (double*)malloc(sizeof(double) * n1);
    double* g = (double*)malloc(sizeof(double) * n1);
    double* dl = (double*)malloc(sizeof(double) * n1);
    double* H = (double*)malloc(sizeof(double) * (size_t)n1 * n1);
    if (x0) {
        x[0] = x0[0] / L;
        for (int k = 0; k < d; ++k) x[1 + k] = (x0[1 + k] - C[k]) / L;
    } else {
        /* Algorithm 1 admits any starting point.  (1, 0) in normalized units
         * would put the ball that attains L exactly on the boundary between
         * the polar and the third projection case, where the generalized
         * Jacobian is set-valued and rounding picks the case; a radius a
         * little above L keeps every ball strictly polar at the start. */
        x[0] = 1.0 + ORC_START_MARGIN;
        for (int k = 0; k < d; ++k) x[1 + k] = 0.0;
    }
    memcpy(ab, x, sizeof(double) * n1);
    double sigma = prm->sigma0, tau = prm->tau;
    double kkt = INFINITY, best = INFINITY, parts[5] = {0, 0, 0, 0, 0};
    int stall = 0, k, tot_inner = 0, tot_ls = 0, status = 1;
    for (k = 0; k < prm->max_outer; ++k) {
        memcpy(xbar, x, sizeof(double) * n1);
        int j;
        for (j = 0; j < prm->max_inner; ++j) {
            double psi, dmult, sabs;
            orc_al_eval(m, d, Cn, Rn, U, V, x, xbar, sigma, tau, &psi, g, H, Up, Vp, &dmult, NULL, &sabs);
            tot_inner++;
            /* relative-type stopping condition (Algorithm 1) at the tentative point */
            acc_t ag = 0, gg = 0, dx2 = 0;
            for (int q = 0; q < n1; ++q) {
                ag += ((acc_t)ab[q] - x[q]) * g[q];
                gg += (acc_t)g[q] * g[q];
                dx2 += ((acc_t)x[q] - xbar[q]) * ((acc_t)x[q] - xbar[q]);
            }
            double lhs = (double)(2 * (acc_t)sigma * fabsl(ag) + (acc_t)sigma * sigma * gg);
            double rhs = prm->rho * (double)((acc_t)dmult + (acc_t)tau * dx2);
            /* reading (rounding floor): the computed gradient cannot be more
             * accurate than about eps * (1 + sigma * sum over non-polar balls
             * of |t_i| + ||s_i||); once ||g|| is there, accept the point. */
            double gfloor = 8 * eps * (1 + sigma * sabs);
            if (lhs <= rhs || sqrt((double)gg) <= gfloor || j == prm->max_inner - 1) break;
            /* Newton direction from H d = -g */
            for (int q = 0; q < n1; ++q) xt[q] = -g[q];
            if (orc_chol_solve(n1, H, xt, dl) != 0) break;
            acc_t gd = 0;
            for (int q = 0; q < n1; ++q) gd += (acc_t)g[q] * dl[q];
            /* Armijo backtracking, eta = 1, 1/2, 1/4, ...  reading: constant
             * 1e-4 plus an allowance of 8 eps |Psi| for rounding in Psi */
            double eta = 1.0;
            for (int ls = 0; ls < prm->max_ls; ++ls) {
                for (int q = 0; q < n1; ++q) xt[q] = x[q] + eta * dl[q];
                double p1;
                orc_al_eval(m, d, Cn, Rn, U, V, xt, xbar, sigma, tau, &p1, NULL, NULL, NULL, NULL, NULL, NULL, NULL);
                tot_ls++;
                if (p1 <= psi + 1e-4 * eta * (double)gd + 8 * eps * (fabs(psi) + 1.0)) break;
                eta *= 0.5;
            }
            for (int q = 0; q < n1; ++q) x[q] += eta * dl[q];
        }
        /* accepted inner point: multipliers and auxiliary sequence */
        memcpy(U, Up, sizeof(double) * m);
        memcpy(V, Vp, sizeof(double) * (size_t)m * d);
        for (int q = 0; q < n1; ++q) ab[q] -= sigma * g[q];
        kkt = orc_kkt_max(m, d, Cn, Rn, U, V, x, parts);
        if (kkt <= prm->tol) {
            status = 0;
            k++;
            break;
        }
        if (kkt < 0.5 * best) {
            best = kkt;
            stall = 0;
        } else if (++stall >= prm->stall_outer) {
            k++;
            break;
        }
        sigma = fmin(sigma * prm->sigma_growth, prm->sigma_max);
    }
    /* back to original units */
    x_out[0] = x[0] * L;
    for (int q = 0; q < d; ++q) x_out[1 + q] = C[q] + x[1 + q] * L;
    if (U_out) memcpy(U_out, U, sizeof(double) * m);
    if (V_out) memcpy(V_out, V, sizeof(double) * (size_t)m * d);
    if (st) {
        st->outer = k;
        st->inner = tot_inner;
        st->ls_evals = tot_ls;
        st->kkt = kkt;
        st->L = L;
        st->rbar = x_out[0];
        for (int q = 0; q < 5; ++q) st->kkt_parts[q] = parts[q];
        /* reading (fix-up): the returned radius is made feasible for every
         * ball by taking the largest r_i + ||c - c_i||. */
        double worst = orc_check_feasible(m, d, C, R, 0.0, x_out + 1, INFINITY, NULL, NULL, 0, NULL);
        st->r_fixed = fmax(x_out[0], worst);
    }
    free(e); free(Cn); free(Rn); free(U); free(V); free(Up); free(Vp);
    free(x); free(xbar); free(ab); free(xt); free(g); free(dl); free(H);
    return status;
}
