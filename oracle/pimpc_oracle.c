/*
 * pimpc_oracle.c -- plain, slow, FP64 CPU oracle of the piMPC ADMM iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP implementation and is not a fallback for it.
 *
 * What it computes (paper: "piMPC: A Parallel-in-horizon and Construction-free
 * NMPC Solver", arXiv 2601.14414):
 *
 *   - the velocity-form data of Theorem 2: xbar_k = col(x_k, u_{k-1}),
 *     Abar_k = [[A_k, B_k], [0, I]], Bbar_k = [[B_k], [I]], ebar_k = col(e_k, 0),
 *     Qbar = blkdiag(Q, R), box Xbar = X x U;
 *   - the stage caches of Algorithm 1 ("cache"): J_k = (Bbar_k' Bbar_k)^-1 Bbar_k'
 *     and H_k = (Qbar + rho I + rho Abar_{k+1}' Abar_{k+1})^-1 (k < N-1),
 *     H_{N-1} = (Qbar + rho I)^-1 (proof of Theorem 2, eqn. (8));
 *   - optionally the input-rate weight W_du of the experiments (Section V:
 *     AFTI-16 and CSTR), a term 1/2 ||du_k||^2_{W_du} added to the cost of
 *     Theorem 2.  It enters only the du sub-problem of eqn. (8), which becomes
 *     argmin 1/2 du' W_du du + rho/2 ||Bbar_k du - v_k + beta_k||^2, so
 *     J_k = (W_du + rho Bbar_k' Bbar_k)^-1 rho Bbar_k' (W_du = 0 gives the
 *     paper's J_k);
 *   - the closed-form iteration of eqn. (8) / Algorithm 1 steps 1-3, the
 *     residual c^{i+1} of step 4, the eps stop of step 5 and (optionally) the
 *     restart acceleration of steps 6-7;
 *   - the primal residual s^{i+1} - s^i and dual residual rho F'G(q^{i+1}-q^i)
 *     of Section IV-B (eqns. (9)-(10)), as infinity norms;
 *   - reverse-mode derivatives of u_0 through the unrolled plain iteration
 *     (not in the paper; the paper lists a differentiable version as future
 *     work in its conclusion).
 *
 * Readings where the paper is ambiguous (each is derived from the augmented
 * Lagrangian of Section IV and eqn. (8)'s constraints):
 *   R1  the x-subproblem of stage k couples to constraint k+1, so h_k uses
 *       Abar_{k+1} and ebar_{k+1} (the paper prints index k in places);
 *   R2  z update = Proj((2(xbar_{k+1}+theta_k) + b_k + c_k)/3) as in the proof
 *       of Theorem 1 and eqn. (8), with b = Bbar du + beta, c = Abar xbar_k +
 *       ebar - lambda, gamma = b - c;
 *   R3  the lambda update uses v_k (constraint k), not v_{k+1};
 *   R8  rho multiplies all six terms of c^{i+1}; the z difference is taken on
 *       z_{k+1};
 *   R11 restart follows Algorithm 1: alpha = 1 and hats = current iterate.
 *   Sets: Xbar = X x U (Theorem 2); each factor is a box or one of the other
 *       closed convex sets the proof of Theorem 1 lists (halfspace, affine
 *       hyperplane, second-order cone, l1 ball), so the projection of the z
 *       update is taken factor by factor.
 *   Terminal stage: Qbar applies to xbar_N as to every other stage.
 *
 * Layouts (all row-major, double):
 *   A [N][n][n], B [N][n][m], e [N][n] (NULL = 0), Q [n][n], R [m][m],
 *   Wdu [m][m] (NULL = 0),
 *   qbar [nb] (NULL = 0), lb/ub [nb] (+-INFINITY allowed), xbar0 [nb],
 *   state [5][N][nb] = (v, z, theta, beta, lambda); z[k] holds z_{k+1}.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX2(i, j, ld) ((size_t)(i) * (size_t)(ld) + (size_t)(j))

/* ------------------------------------------------------------------------- */
/* small dense helpers                                                        */
/* ------------------------------------------------------------------------- */

/* y = M x, M is r x c */
static void matvec(int r, int c, const double *M, const double *x, double *y) {
    for (int i = 0; i < r; ++i) {
        double s = 0.0;
        for (int j = 0; j < c; ++j) s += M[IDX2(i, j, c)] * x[j];
        y[i] = s;
    }
}

/* y = M' x, M is r x c, y has c entries */
static void matTvec(int r, int c, const double *M, const double *x, double *y) {
    for (int j = 0; j < c; ++j) {
        double s = 0.0;
        for (int i = 0; i < r; ++i) s += M[IDX2(i, j, c)] * x[i];
        y[j] = s;
    }
}

/* In-place Cholesky M = L L' (lower triangle of M overwritten by L).
 * Returns 0 on success, -1 if a pivot is not strictly positive. */
static int cholesky(int n, double *M) {
    for (int j = 0; j < n; ++j) {
        double d = M[IDX2(j, j, n)];
        for (int k = 0; k < j; ++k) d -= M[IDX2(j, k, n)] * M[IDX2(j, k, n)];
        if (!(d > 0.0)) return -1;
        double l = sqrt(d);
        M[IDX2(j, j, n)] = l;
        for (int i = j + 1; i < n; ++i) {
            double s = M[IDX2(i, j, n)];
            for (int k = 0; k < j; ++k) s -= M[IDX2(i, k, n)] * M[IDX2(j, k, n)];
            M[IDX2(i, j, n)] = s / l;
        }
    }
    return 0;
}

/* Solve L L' x = b given the Cholesky factor in the lower triangle of L. */
static void chol_solve(int n, const double *L, const double *b, double *x) {
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[IDX2(i, k, n)] * x[k];
        x[i] = s / L[IDX2(i, i, n)];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < n; ++k) s -= L[IDX2(k, i, n)] * x[k];
        x[i] = s / L[IDX2(i, i, n)];
    }
}

/* Inverse of an SPD matrix via Cholesky; out may not alias M. */
static int spd_inverse(int n, const double *M, double *out) {
    double *L = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *b = (double *)malloc(sizeof(double) * (size_t)n);
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(L, M, sizeof(double) * (size_t)n * n);
    int rc = cholesky(n, L);
    if (rc == 0) {
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < n; ++i) b[i] = (i == j) ? 1.0 : 0.0;
            chol_solve(n, L, b, x);
            for (int i = 0; i < n; ++i) out[IDX2(i, j, n)] = x[i];
        }
    }
    free(L); free(b); free(x);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* velocity-form data (Theorem 2)                                             */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n, m, nb, N;
    double *Abar;  /* [N][nb][nb] */
    double *Bbar;  /* [N][nb][m]  */
    double *ebar;  /* [N][nb]     */
    double *Qbar;  /* [nb][nb]    */
    double *qbar;  /* [nb]        */
    double *W;     /* [m][m] input-rate weight (zero if absent) */
    int xkind, ukind;      /* set kinds of the X and U factors (ORC_SET_*) */
    double *xpar, *upar;   /* [n+1], [m+1]: (a, b) or (., r) of the factor set */
    double *H;     /* [N][nb][nb] */
    double *J;     /* [N][m][nb]  */
} vform_t;

static void vform_free(vform_t *V) {
    free(V->Abar); free(V->Bbar); free(V->ebar); free(V->Qbar); free(V->qbar); free(V->W);
    free(V->xpar); free(V->upar);
    free(V->H); free(V->J);
}

static void vform_build(vform_t *V, int n, int m, int N, const double *A, const double *B,
                        const double *e, const double *Q, const double *R, const double *W,
                        const double *qbar) {
    int nb = n + m;
    V->n = n; V->m = m; V->nb = nb; V->N = N;
    V->Abar = (double *)calloc((size_t)N * nb * nb, sizeof(double));
    V->Bbar = (double *)calloc((size_t)N * nb * m, sizeof(double));
    V->ebar = (double *)calloc((size_t)N * nb, sizeof(double));
    V->Qbar = (double *)calloc((size_t)nb * nb, sizeof(double));
    V->qbar = (double *)calloc((size_t)nb, sizeof(double));
    V->W = (double *)calloc((size_t)m * m, sizeof(double));
    if (W) memcpy(V->W, W, sizeof(double) * (size_t)m * m);
    V->xkind = V->ukind = 0;
    V->xpar = (double *)calloc((size_t)n + 1, sizeof(double));
    V->upar = (double *)calloc((size_t)m + 1, sizeof(double));
    V->H = (double *)calloc((size_t)N * nb * nb, sizeof(double));
    V->J = (double *)calloc((size_t)N * m * nb, sizeof(double));
    for (int k = 0; k < N; ++k) {
        double *Ab = V->Abar + (size_t)k * nb * nb;
        double *Bb = V->Bbar + (size_t)k * nb * m;
        const double *Ak = A + (size_t)k * n * n;
        const double *Bk = B + (size_t)k * n * m;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) Ab[IDX2(i, j, nb)] = Ak[IDX2(i, j, n)];
            for (int j = 0; j < m; ++j) Ab[IDX2(i, n + j, nb)] = Bk[IDX2(i, j, m)];
            for (int j = 0; j < m; ++j) Bb[IDX2(i, j, m)] = Bk[IDX2(i, j, m)];
        }
        for (int i = 0; i < m; ++i) {
            Ab[IDX2(n + i, n + i, nb)] = 1.0;
            Bb[IDX2(n + i, i, m)] = 1.0;
        }
        if (e)
            for (int i = 0; i < n; ++i) V->ebar[(size_t)k * nb + i] = e[(size_t)k * n + i];
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V->Qbar[IDX2(i, j, nb)] = Q[IDX2(i, j, n)];
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) V->Qbar[IDX2(n + i, n + j, nb)] = R[IDX2(i, j, m)];
    if (qbar)
        for (int i = 0; i < nb; ++i) V->qbar[i] = qbar[i];
}

/* Algorithm 1 "cache": J_k and H_k.  Returns 0, or -1 if a matrix is not SPD. */
static int vform_factor(vform_t *V, double rho) {
    int nb = V->nb, m = V->m, N = V->N;
    double *M = (double *)malloc(sizeof(double) * (size_t)nb * nb);
    double *G = (double *)malloc(sizeof(double) * (size_t)m * m);
    double *Gi = (double *)malloc(sizeof(double) * (size_t)m * m);
    int rc = 0;
    for (int k = 0; k < N && rc == 0; ++k) {
        /* M_k = Qbar + rho I + rho Abar_{k+1}' Abar_{k+1}  (k < N-1) */
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) {
                double s = V->Qbar[IDX2(i, j, nb)] + (i == j ? rho : 0.0);
                if (k < N - 1) {
                    const double *An = V->Abar + (size_t)(k + 1) * nb * nb;
                    double t = 0.0;
                    for (int r = 0; r < nb; ++r) t += An[IDX2(r, i, nb)] * An[IDX2(r, j, nb)];
                    s += rho * t;
                }
                M[IDX2(i, j, nb)] = s;
            }
        rc = spd_inverse(nb, M, V->H + (size_t)k * nb * nb);
        if (rc) break;
        /* G_k = W_du + rho Bbar_k' Bbar_k,  J_k = G_k^-1 rho Bbar_k' */
        const double *Bb = V->Bbar + (size_t)k * nb * m;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double t = 0.0;
                for (int r = 0; r < nb; ++r) t += Bb[IDX2(r, i, m)] * Bb[IDX2(r, j, m)];
                G[IDX2(i, j, m)] = V->W[IDX2(i, j, m)] + rho * t;
            }
        rc = spd_inverse(m, G, Gi);
        if (rc) break;
        double *Jk = V->J + (size_t)k * m * nb;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < nb; ++j) {
                double t = 0.0;
                for (int r = 0; r < m; ++r) t += Gi[IDX2(i, r, m)] * rho * Bb[IDX2(j, r, m)];
                Jk[IDX2(i, j, nb)] = t;
            }
    }
    free(M); free(G); free(Gi);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Euclidean projections onto the factor sets (proof of Theorem 1; formulas   */
/* of Parikh and Boyd, "Proximal Algorithms", Ch. 6)                          */
/* ------------------------------------------------------------------------- */

#define ORC_SET_BOX 0        /* lo <= w <= hi                         */
#define ORC_SET_HALFSPACE 1  /* a'w <= b                              */
#define ORC_SET_HYPERPLANE 2 /* a'w = b                               */
#define ORC_SET_SOC 3        /* ||(w_1..w_{n-1})||_2 <= w_n           */
#define ORC_SET_L1BALL 4     /* ||w||_1 <= r  (r = par[n])            */

static int cmp_desc(const void *x, const void *y) {
    double a = *(const double *)x, b = *(const double *)y;
    return (a < b) - (a > b);
}

/* Project w (n entries) onto the set; par = (a_1..a_n, b) or (., r). */
static void project_set(int kind, int n, const double *par, const double *lo, const double *hi, double *w) {
    if (kind == ORC_SET_BOX) {
        for (int i = 0; i < n; ++i) w[i] = w[i] < lo[i] ? lo[i] : (w[i] > hi[i] ? hi[i] : w[i]);
    } else if (kind == ORC_SET_HALFSPACE || kind == ORC_SET_HYPERPLANE) {
        double s = 0.0, aa = 0.0;
        for (int i = 0; i < n; ++i) {
            s += par[i] * w[i];
            aa += par[i] * par[i];
        }
        s -= par[n];
        if (kind == ORC_SET_HYPERPLANE || s > 0.0)
            for (int i = 0; i < n; ++i) w[i] -= s / aa * par[i];
    } else if (kind == ORC_SET_SOC) {
        double t = w[n - 1], nx2 = 0.0;
        for (int i = 0; i < n - 1; ++i) nx2 += w[i] * w[i];
        double nx = sqrt(nx2);
        if (nx <= t) return;
        if (nx <= -t) {
            for (int i = 0; i < n; ++i) w[i] = 0.0;
            return;
        }
        double al = 0.5 * (nx + t);
        for (int i = 0; i < n - 1; ++i) w[i] = al * w[i] / nx;
        w[n - 1] = al;
    } else if (kind == ORC_SET_L1BALL) {
        double r = par[n], l1 = 0.0;
        for (int i = 0; i < n; ++i) l1 += fabs(w[i]);
        if (l1 <= r) return;
        /* soft threshold at theta with sum max(|w_i| - theta, 0) = r:
         * sort |w| descending, theta = (sum of the rho largest - r) / rho with
         * rho the last index whose entry stays above its running threshold */
        double *mu = (double *)malloc(sizeof(double) * (size_t)n);
        for (int i = 0; i < n; ++i) mu[i] = fabs(w[i]);
        qsort(mu, (size_t)n, sizeof(double), cmp_desc);
        double cs = 0.0, theta = 0.0;
        for (int j = 0; j < n; ++j) {
            cs += mu[j];
            double tj = (cs - r) / (double)(j + 1);
            if (mu[j] - tj > 0.0) theta = tj;
        }
        free(mu);
        for (int i = 0; i < n; ++i) {
            double a = fabs(w[i]) - theta;
            w[i] = a > 0.0 ? (w[i] > 0.0 ? a : -a) : 0.0;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* one ADMM iteration (eqn. (8), Algorithm 1 steps 1-3)                       */
/* ------------------------------------------------------------------------- */

/* Reads hats (v,z,th,be,la) = hat[0..4], writes the new iterate to out[0..4],
 * the step-1 results du [N][m] and xs [N][nb] (xs[k] = xbar_{k+1}). */
static void admm_iteration(const vform_t *V, double rho, const double *lb, const double *ub,
                           const double *xbar0, const double *const hat[5], double *const out[5],
                           double *du, double *xs) {
    int nb = V->nb, m = V->m, N = V->N;
    const double *v = hat[0], *z = hat[1], *th = hat[2], *be = hat[3], *la = hat[4];
    double *w = (double *)malloc(sizeof(double) * nb);
    double *g = (double *)malloc(sizeof(double) * nb);
    double *h = (double *)malloc(sizeof(double) * nb);
    double *d = (double *)malloc(sizeof(double) * nb);
    double *b = (double *)malloc(sizeof(double) * nb);
    double *c = (double *)malloc(sizeof(double) * nb);
    double *y = (double *)malloc(sizeof(double) * nb);

    /* step 1: du_k = J_k (v_k - beta_k);  xbar_{k+1} = H_k h_k with
     * h_k = qbar + rho (z_{k+1} - theta_k + Abar_{k+1}' (z_{k+2} - v_{k+1} - ebar_{k+1} + lambda_{k+1})) */
    for (int k = 0; k < N; ++k) {
        for (int i = 0; i < nb; ++i) d[i] = v[(size_t)k * nb + i] - be[(size_t)k * nb + i];
        matvec(m, nb, V->J + (size_t)k * m * nb, d, du + (size_t)k * m);
        for (int i = 0; i < nb; ++i)
            h[i] = V->qbar[i] + rho * (z[(size_t)k * nb + i] - th[(size_t)k * nb + i]);
        if (k < N - 1) {
            int j = k + 1;
            for (int i = 0; i < nb; ++i)
                w[i] = z[(size_t)j * nb + i] - v[(size_t)j * nb + i] - V->ebar[(size_t)j * nb + i] +
                       la[(size_t)j * nb + i];
            matTvec(nb, nb, V->Abar + (size_t)j * nb * nb, w, g);
            for (int i = 0; i < nb; ++i) h[i] += rho * g[i];
        }
        matvec(nb, nb, V->H + (size_t)k * nb * nb, h, xs + (size_t)k * nb);
    }

    /* steps 2-3 (Theorem 1 closed form: z = Proj_Xbar((2 (xbar + theta) + b + c) / 3),
     * Xbar = X x U projected factor by factor; then the scaled dual updates) */
    int n = V->n;
    for (int k = 0; k < N; ++k) {
        const double *xp = (k == 0) ? xbar0 : xs + (size_t)(k - 1) * nb;
        const double *xk = xs + (size_t)k * nb;
        matvec(nb, m, V->Bbar + (size_t)k * nb * m, du + (size_t)k * m, b);
        matvec(nb, nb, V->Abar + (size_t)k * nb * nb, xp, c);
        for (int i = 0; i < nb; ++i) {
            size_t o = (size_t)k * nb + i;
            b[i] += be[o];
            c[i] += V->ebar[o] - la[o];
            y[i] = (2.0 * (xk[i] + th[o]) + b[i] + c[i]) / 3.0;
        }
        project_set(V->xkind, n, V->xpar, lb, ub, y);
        project_set(V->ukind, m, V->upar, lb + n, ub + n, y + n);
        for (int i = 0; i < nb; ++i) {
            size_t o = (size_t)k * nb + i;
            double bi = b[i], ci = c[i];
            double gam = bi - ci;
            double zn = y[i];
            double vn = 0.5 * (zn + gam);
            out[0][o] = vn;
            out[1][o] = zn;
            out[2][o] = th[o] + xk[i] - zn;
            out[3][o] = bi - vn;
            out[4][o] = zn - vn - ci;
        }
    }
    free(w); free(g); free(h); free(d); free(b); free(c); free(y);
}

/* c^{i+1} (Algorithm 1 step 4), primal residual ||s^{i+1}-s^i||_inf and dual
 * residual rho ||F'G(q^{i+1}-q^i)||_inf (Section IV-B), with q = (V, Z),
 * s = (Theta, Beta, Lambda) and the differences taken against the hats. */
static void residuals(const vform_t *V, double rho, const double *const hat[5],
                      const double *const nw[5], double *c_out, double *rp_out, double *rd_out) {
    int nb = V->nb, m = V->m, N = V->N;
    double csum = 0.0, rp = 0.0, rd = 0.0;
    double *t = (double *)malloc(sizeof(double) * nb);
    double *tt = (double *)malloc(sizeof(double) * nb);
    for (int k = 0; k < N; ++k) {
        for (int i = 0; i < nb; ++i) {
            size_t o = (size_t)k * nb + i;
            double dv = nw[0][o] - hat[0][o], dz = nw[1][o] - hat[1][o];
            double dth = nw[2][o] - hat[2][o], dbe = nw[3][o] - hat[3][o];
            double dla = nw[4][o] - hat[4][o];
            csum += dth * dth + dbe * dbe + dla * dla + dz * dz + dv * dv + (dz - dv) * (dz - dv);
            rp = fmax(rp, fmax(fabs(dth), fmax(fabs(dbe), fabs(dla))));
        }
        /* F'G dq, block of du_k: -Bbar_k' dv_k */
        for (int i = 0; i < nb; ++i) t[i] = nw[0][(size_t)k * nb + i] - hat[0][(size_t)k * nb + i];
        double bt[64];
        double *btp = (m <= 64) ? bt : (double *)malloc(sizeof(double) * m);
        matTvec(nb, m, V->Bbar + (size_t)k * nb * m, t, btp);
        for (int i = 0; i < m; ++i) rd = fmax(rd, fabs(btp[i]));
        if (btp != bt) free(btp);
        /* block of xbar_{k+1}: -dz_{k+1} - Abar_{k+1}'(dz_{k+2} - dv_{k+1}) */
        for (int i = 0; i < nb; ++i) tt[i] = 0.0;
        if (k < N - 1) {
            int j = k + 1;
            for (int i = 0; i < nb; ++i) {
                size_t o = (size_t)j * nb + i;
                t[i] = (nw[1][o] - hat[1][o]) - (nw[0][o] - hat[0][o]);
            }
            matTvec(nb, nb, V->Abar + (size_t)j * nb * nb, t, tt);
        }
        for (int i = 0; i < nb; ++i) {
            size_t o = (size_t)k * nb + i;
            rd = fmax(rd, fabs((nw[1][o] - hat[1][o]) + tt[i]));
        }
    }
    free(t); free(tt);
    *c_out = rho * csum;
    *rp_out = rp;
    *rd_out = rho * rd;
}

/* ------------------------------------------------------------------------- */
/* exported API                                                               */
/* ------------------------------------------------------------------------- */

/* Stage caches only: H [N][nb][nb], J [N][m][nb].  0 or -1 (not SPD). */
int orc_factor(int n, int m, int N, const double *A, const double *B, const double *Q,
               const double *R, const double *Wdu, double rho, double *H, double *J) {
    vform_t V;
    vform_build(&V, n, m, N, A, B, NULL, Q, R, Wdu, NULL);
    int rc = vform_factor(&V, rho);
    if (rc == 0) {
        memcpy(H, V.H, sizeof(double) * (size_t)N * V.nb * V.nb);
        memcpy(J, V.J, sizeof(double) * (size_t)N * m * V.nb);
    }
    vform_free(&V);
    return rc;
}

/*
 * Run Algorithm 1 for at most K iterations from `state` (in: initial iterate,
 * out: final iterate).  The X and U factors of the constraint set are of kind
 * xkind / ukind (ORC_SET_*) with parameters xpar [n+1] / upar [m+1] (NULL =
 * zeros); box factors use lb / ub.  eps <= 0 disables the stop of step 5.  accel = 0 runs
 * plain ADMM (hats = previous iterate); accel = 1 adds steps 6-7 with the
 * given eta.  Outputs (any may be NULL except state):
 *   du [N][m], xs [N][nb]  step-1 results of the last iteration run
 *   hist [K][4]            c^{i+1}, r_prim, r_dual, restart flag per iteration
 *   iters                  number of iterations run
 * Returns 0, -1 if a stage matrix is not SPD, -2 on bad arguments.
 */
int orc_solve(int n, int m, int N, const double *A, const double *B, const double *e,
              const double *Q, const double *R, const double *Wdu, const double *qbar,
              const double *lb, const double *ub, int xkind, const double *xpar, int ukind,
              const double *upar, const double *xbar0, double rho, int K, double eps,
              int accel, double eta, double *state, double *du, double *xs, double *hist,
              int *iters) {
    if (n <= 0 || m <= 0 || N <= 0 || K < 0 || !(rho > 0.0)) return -2;
    if (xkind < 0 || xkind > 4 || ukind < 0 || ukind > 4) return -2;
    if ((xkind == ORC_SET_SOC && n < 2) || (ukind == ORC_SET_SOC && m < 2)) return -2;
    int nb = n + m;
    size_t S = (size_t)N * nb;
    vform_t V;
    vform_build(&V, n, m, N, A, B, e, Q, R, Wdu, qbar);
    V.xkind = xkind;
    V.ukind = ukind;
    if (xpar) memcpy(V.xpar, xpar, sizeof(double) * ((size_t)n + 1));
    if (upar) memcpy(V.upar, upar, sizeof(double) * ((size_t)m + 1));
    int rc = vform_factor(&V, rho);
    if (rc) { vform_free(&V); return -1; }

    double *cur = (double *)malloc(sizeof(double) * 5 * S);   /* previous actual iterate */
    double *hat = (double *)malloc(sizeof(double) * 5 * S);   /* hats read by step 1 */
    double *nw = (double *)malloc(sizeof(double) * 5 * S);    /* new iterate */
    double *du_l = (double *)malloc(sizeof(double) * (size_t)N * m);
    double *xs_l = (double *)malloc(sizeof(double) * S);
    memcpy(cur, state, sizeof(double) * 5 * S);
    memcpy(hat, state, sizeof(double) * 5 * S);
    const double *hp[5];
    double *np_[5];
    for (int q = 0; q < 5; ++q) { hp[q] = hat + q * S; np_[q] = nw + q * S; }

    double alpha = 1.0, c_prev = 1.0;
    int it = 0;
    for (int i = 0; i < K; ++i) {
        admm_iteration(&V, rho, lb, ub, xbar0, hp, np_, du_l, xs_l);
        double c, rp, rd;
        residuals(&V, rho, hp, (const double *const *)np_, &c, &rp, &rd);
        it = i + 1;
        int restart = 0;
        int stop = (eps > 0.0 && c <= eps);
        if (!stop) {
            if (accel) {
                if (c <= eta * c_prev) {
                    double a1 = 0.5 + 0.5 * sqrt(1.0 + 4.0 * alpha * alpha);
                    double coef = (alpha - 1.0) / a1;
                    for (size_t t = 0; t < 5 * S; ++t) hat[t] = nw[t] + coef * (nw[t] - cur[t]);
                    alpha = a1;
                } else {
                    alpha = 1.0;
                    memcpy(hat, nw, sizeof(double) * 5 * S);
                    restart = 1;
                }
                c_prev = c;
            } else {
                memcpy(hat, nw, sizeof(double) * 5 * S);
            }
        }
        memcpy(cur, nw, sizeof(double) * 5 * S);
        if (hist) {
            hist[4 * (size_t)i + 0] = c;
            hist[4 * (size_t)i + 1] = rp;
            hist[4 * (size_t)i + 2] = rd;
            hist[4 * (size_t)i + 3] = restart;
        }
        if (stop) break;
    }
    memcpy(state, cur, sizeof(double) * 5 * S);
    if (du) memcpy(du, du_l, sizeof(double) * (size_t)N * m);
    if (xs) memcpy(xs, xs_l, sizeof(double) * S);
    if (iters) *iters = it;
    free(cur); free(hat); free(nw); free(du_l); free(xs_l);
    vform_free(&V);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* reverse mode through the unrolled plain iteration                          */
/* ------------------------------------------------------------------------- */

/*
 * Loss gradient for a time-invariant instance with diagonal weights, e = 0,
 * qbar = 0, u_prev = 0 and a cold start; Wdu [m][m] (NULL = 0) is a fixed,
 * non-differentiated input-rate weight.  The output u_0 = du_0 of the K-th
 * step 1 (Algorithm 1 output) is a function of (x0, diag Q, diag R, A, B);
 * given ubar = dL/du_0 this returns the vector-Jacobian products.
 *   A [n][n], B [n][m], Qd [n], Rd [m], lb/ub [nb], x0 [n], ubar [m]
 *   out: u0 [m], dA [n][n], dB [n][m], dQd [n], dRd [m], dx0 [n]
 * The whole tape (K states) is kept in memory.  Returns 0, -1 (not SPD), -2.
 */
int orc_grad(int n, int m, int N, const double *A, const double *B, const double *Qd,
             const double *Rd, const double *Wdu, const double *lb, const double *ub, const double *x0, double rho,
             int K, const double *ubar, double *u0, double *dA, double *dB, double *dQd,
             double *dRd, double *dx0) {
    if (n <= 0 || m <= 0 || N <= 0 || K < 1 || !(rho > 0.0)) return -2;
    int nb = n + m;
    size_t S = (size_t)N * nb;
    double *Aall = (double *)malloc(sizeof(double) * (size_t)N * n * n);
    double *Ball = (double *)malloc(sizeof(double) * (size_t)N * n * m);
    double *Q = (double *)calloc((size_t)n * n, sizeof(double));
    double *R = (double *)calloc((size_t)m * m, sizeof(double));
    for (int k = 0; k < N; ++k) {
        memcpy(Aall + (size_t)k * n * n, A, sizeof(double) * n * n);
        memcpy(Ball + (size_t)k * n * m, B, sizeof(double) * n * m);
    }
    for (int i = 0; i < n; ++i) Q[IDX2(i, i, n)] = Qd[i];
    for (int i = 0; i < m; ++i) R[IDX2(i, i, m)] = Rd[i];
    vform_t V;
    vform_build(&V, n, m, N, Aall, Ball, NULL, Q, R, Wdu, NULL);
    if (vform_factor(&V, rho)) {
        vform_free(&V); free(Aall); free(Ball); free(Q); free(R);
        return -1;
    }
    double *xbar0 = (double *)calloc(nb, sizeof(double));
    for (int i = 0; i < n; ++i) xbar0[i] = x0[i];

    /* forward: tape[i] = state entering iteration i, i = 0..K-1 */
    double *tape = (double *)calloc((size_t)K * 5 * S, sizeof(double));
    double *du = (double *)malloc(sizeof(double) * (size_t)N * m);
    double *xs = (double *)malloc(sizeof(double) * S);
    for (int i = 0; i + 1 < K; ++i) {
        const double *hp[5];
        double *op[5];
        for (int q = 0; q < 5; ++q) {
            hp[q] = tape + (size_t)i * 5 * S + q * S;
            op[q] = tape + (size_t)(i + 1) * 5 * S + q * S;
        }
        admm_iteration(&V, rho, lb, ub, xbar0, hp, op, du, xs);
    }
    /* output of the last step 1: du_0 = J_0 (v_0 - beta_0) of state K-1 */
    const double *sK = tape + (size_t)(K - 1) * 5 * S;
    double *dlast = (double *)malloc(sizeof(double) * nb);
    for (int i = 0; i < nb; ++i) dlast[i] = sK[0 * S + i] - sK[3 * S + i];
    matvec(m, nb, V.J, dlast, u0);

    /* parameter adjoints of the velocity-form data */
    double *Jb = (double *)calloc((size_t)m * nb, sizeof(double));
    double *Hab = (double *)calloc((size_t)nb * nb, sizeof(double)); /* H_k, k < N-1 */
    double *Hbb = (double *)calloc((size_t)nb * nb, sizeof(double)); /* H_{N-1} */
    double *Abb = (double *)calloc((size_t)nb * nb, sizeof(double)); /* Abar */
    double *Bbb = (double *)calloc((size_t)nb * m, sizeof(double));  /* Bbar */
    double *x0b = (double *)calloc(nb, sizeof(double));
    double *sb = (double *)calloc(5 * S, sizeof(double));  /* adjoint of state s^{i+1} */
    double *sa = (double *)calloc(5 * S, sizeof(double));  /* adjoint of state s^i */

    /* seed: u0 = J (v_0 - beta_0) at state K-1 */
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < nb; ++j) Jb[IDX2(i, j, nb)] += ubar[i] * dlast[j];
    for (int j = 0; j < nb; ++j) {
        double t = 0.0;
        for (int i = 0; i < m; ++i) t += V.J[IDX2(i, j, nb)] * ubar[i];
        sb[0 * S + j] += t;
        sb[3 * S + j] -= t;
    }

    double *xsb = (double *)malloc(sizeof(double) * S);
    double *gb = (double *)malloc(sizeof(double) * S);
    double *dub = (double *)malloc(sizeof(double) * (size_t)N * m);
    double *hv = (double *)malloc(sizeof(double) * S);
    double *bv = (double *)malloc(sizeof(double) * nb);
    double *cv = (double *)malloc(sizeof(double) * nb);
    double *cb = (double *)malloc(sizeof(double) * nb);
    double *bb = (double *)malloc(sizeof(double) * nb);
    double *tmp = (double *)malloc(sizeof(double) * nb);
    double *tmp2 = (double *)malloc(sizeof(double) * nb);

    for (int it = K - 2; it >= 0; --it) {
        const double *s = tape + (size_t)it * 5 * S;
        const double *v = s, *z = s + S, *th = s + 2 * S, *be = s + 3 * S, *la = s + 4 * S;
        const double *vbo = sb, *zbo = sb + S, *thbo = sb + 2 * S, *bebo = sb + 3 * S,
                     *labo = sb + 4 * S;
        double *vb = sa, *zb = sa + S, *thb = sa + 2 * S, *beb = sa + 3 * S, *lab = sa + 4 * S;
        memset(sa, 0, sizeof(double) * 5 * S);
        memset(xsb, 0, sizeof(double) * S);
        memset(gb, 0, sizeof(double) * S);

        /* recompute step 1 of this iteration: du, h, xs */
        for (int k = 0; k < N; ++k) {
            for (int i = 0; i < nb; ++i) tmp[i] = v[(size_t)k * nb + i] - be[(size_t)k * nb + i];
            matvec(m, nb, V.J, tmp, du + (size_t)k * m);
            for (int i = 0; i < nb; ++i) hv[(size_t)k * nb + i] = rho * (z[(size_t)k * nb + i] - th[(size_t)k * nb + i]);
            if (k < N - 1) {
                int j = k + 1;
                for (int i = 0; i < nb; ++i)
                    tmp[i] = z[(size_t)j * nb + i] - v[(size_t)j * nb + i] + la[(size_t)j * nb + i];
                matTvec(nb, nb, V.Abar, tmp, tmp2);
                for (int i = 0; i < nb; ++i) hv[(size_t)k * nb + i] += rho * tmp2[i];
            }
            matvec(nb, nb, V.H + (size_t)k * nb * nb, hv + (size_t)k * nb, xs + (size_t)k * nb);
        }
        /* reverse of steps 2-3, stage by stage */
        for (int k = 0; k < N; ++k) {
            const double *xp = (k == 0) ? xbar0 : xs + (size_t)(k - 1) * nb;
            matvec(nb, m, V.Bbar, du + (size_t)k * m, bv);
            matvec(nb, nb, V.Abar, xp, cv);
            for (int i = 0; i < nb; ++i) {
                size_t o = (size_t)k * nb + i;
                double bi = bv[i] + be[o];
                double ci = cv[i] - la[o];
                double y = (2.0 * (xs[o] + th[o]) + bi + ci) / 3.0;
                double mask = (y > lb[i] && y < ub[i]) ? 1.0 : 0.0;
                /* theta' = theta + xs - z' */
                double znb = zbo[o] - thbo[o];
                thb[o] += thbo[o];
                xsb[o] += thbo[o];
                /* beta' = b - v' */
                double bbi = bebo[o];
                double vnb = vbo[o] - bebo[o];
                /* lambda' = z' - v' - c */
                znb += labo[o];
                vnb -= labo[o];
                double cbi = -labo[o];
                /* v' = (z' + gamma)/2 */
                znb += 0.5 * vnb;
                double gamb = 0.5 * vnb;
                /* z' = clamp(y) */
                double yb = mask * znb;
                /* y = (2(xs + theta) + b + c)/3 */
                xsb[o] += (2.0 / 3.0) * yb;
                thb[o] += (2.0 / 3.0) * yb;
                bbi += yb / 3.0;
                cbi += yb / 3.0;
                /* gamma = b - c */
                bbi += gamb;
                cbi -= gamb;
                bb[i] = bbi;
                cb[i] = cbi;
            }
            /* c = Abar xp + ebar - lambda */
            for (int i = 0; i < nb; ++i) lab[(size_t)k * nb + i] -= cb[i];
            matTvec(nb, nb, V.Abar, cb, tmp);
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < nb; ++j) Abb[IDX2(i, j, nb)] += cb[i] * xp[j];
            if (k == 0)
                for (int i = 0; i < nb; ++i) x0b[i] += tmp[i];
            else
                for (int i = 0; i < nb; ++i) xsb[(size_t)(k - 1) * nb + i] += tmp[i];
            /* b = Bbar du + beta */
            for (int i = 0; i < nb; ++i) beb[(size_t)k * nb + i] += bb[i];
            matTvec(nb, m, V.Bbar, bb, dub + (size_t)k * m);
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < m; ++j) Bbb[IDX2(i, j, m)] += bb[i] * du[(size_t)k * m + j];
        }
        /* reverse of step 1 */
        for (int k = 0; k < N; ++k) {
            const double *Hk = V.H + (size_t)k * nb * nb;
            double *Hkb = (k < N - 1) ? Hab : Hbb;
            /* xs = H h */
            matTvec(nb, nb, Hk, xsb + (size_t)k * nb, tmp);
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < nb; ++j)
                    Hkb[IDX2(i, j, nb)] += xsb[(size_t)k * nb + i] * hv[(size_t)k * nb + j];
            /* h = rho (z - theta) + rho g_{k+1} */
            for (int i = 0; i < nb; ++i) {
                zb[(size_t)k * nb + i] += rho * tmp[i];
                thb[(size_t)k * nb + i] -= rho * tmp[i];
                if (k < N - 1) gb[(size_t)(k + 1) * nb + i] += rho * tmp[i];
            }
        }
        for (int j = 1; j < N; ++j) {
            /* g_j = Abar' w_j, w_j = z_j - v_j + lambda_j */
            for (int i = 0; i < nb; ++i)
                tmp2[i] = z[(size_t)j * nb + i] - v[(size_t)j * nb + i] + la[(size_t)j * nb + i];
            matvec(nb, nb, V.Abar, gb + (size_t)j * nb, tmp);
            for (int i = 0; i < nb; ++i)
                for (int r = 0; r < nb; ++r) Abb[IDX2(i, r, nb)] += tmp2[i] * gb[(size_t)j * nb + r];
            for (int i = 0; i < nb; ++i) {
                zb[(size_t)j * nb + i] += tmp[i];
                vb[(size_t)j * nb + i] -= tmp[i];
                lab[(size_t)j * nb + i] += tmp[i];
            }
        }
        for (int k = 0; k < N; ++k) {
            /* du = J (v - beta) */
            for (int i = 0; i < nb; ++i) tmp2[i] = v[(size_t)k * nb + i] - be[(size_t)k * nb + i];
            matTvec(m, nb, V.J, dub + (size_t)k * m, tmp);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < nb; ++j) Jb[IDX2(i, j, nb)] += dub[(size_t)k * m + i] * tmp2[j];
            for (int i = 0; i < nb; ++i) {
                vb[(size_t)k * nb + i] += tmp[i];
                beb[(size_t)k * nb + i] -= tmp[i];
            }
        }
        /* the adjoint of s^it becomes the incoming adjoint for it-1 */
        double *sw = sb; sb = sa; sa = sw;
    }

    /* chain through the caches to (A, B, diag Q, diag R) */
    double *Mb = (double *)malloc(sizeof(double) * (size_t)nb * nb);
    double *T1 = (double *)malloc(sizeof(double) * (size_t)nb * nb);
    double *qbd = (double *)calloc(nb, sizeof(double));
    for (int pass = 0; pass < 2; ++pass) {
        const double *Hm = (pass == 0) ? V.H : V.H + (size_t)(N - 1) * nb * nb;
        const double *Hb = (pass == 0) ? Hab : Hbb;
        if (pass == 0 && N == 1) continue;
        /* Mbar = -H' Hbar H' (H symmetric) */
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) {
                double t = 0.0;
                for (int r = 0; r < nb; ++r) t += Hm[IDX2(i, r, nb)] * Hb[IDX2(r, j, nb)];
                T1[IDX2(i, j, nb)] = t;
            }
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) {
                double t = 0.0;
                for (int r = 0; r < nb; ++r) t += T1[IDX2(i, r, nb)] * Hm[IDX2(r, j, nb)];
                Mb[IDX2(i, j, nb)] = -t;
            }
        for (int i = 0; i < nb; ++i) qbd[i] += Mb[IDX2(i, i, nb)];
        if (pass == 0) {
            /* M = Qbar + rho I + rho Abar' Abar  ->  Abar_bar += rho Abar (Mb + Mb') */
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < nb; ++j) {
                    double t = 0.0;
                    for (int r = 0; r < nb; ++r)
                        t += V.Abar[IDX2(i, r, nb)] * (Mb[IDX2(r, j, nb)] + Mb[IDX2(j, r, nb)]);
                    Abb[IDX2(i, j, nb)] += rho * t;
                }
        }
    }
    /* J = G^-1 rho Bbar', G = W_du + rho Bbar' Bbar:  Gbar = -G^-1 Jbar J',
     * Bbar_bar += rho Jbar' G^-1 + rho Bbar (Gbar + Gbar') */
    {
        double *G = (double *)malloc(sizeof(double) * (size_t)m * m);
        double *Gi = (double *)malloc(sizeof(double) * (size_t)m * m);
        double *Gb = (double *)malloc(sizeof(double) * (size_t)m * m);
        double *GiJb = (double *)malloc(sizeof(double) * (size_t)m * nb);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double t = 0.0;
                for (int r = 0; r < nb; ++r) t += V.Bbar[IDX2(r, i, m)] * V.Bbar[IDX2(r, j, m)];
                G[IDX2(i, j, m)] = V.W[IDX2(i, j, m)] + rho * t;
            }
        spd_inverse(m, G, Gi);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < nb; ++j) {
                double t = 0.0;
                for (int r = 0; r < m; ++r) t += Gi[IDX2(i, r, m)] * Jb[IDX2(r, j, nb)];
                GiJb[IDX2(i, j, nb)] = t;
            }
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double t = 0.0;
                for (int r = 0; r < nb; ++r) t += GiJb[IDX2(i, r, nb)] * V.J[IDX2(j, r, nb)];
                Gb[IDX2(i, j, m)] = -t;
            }
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < m; ++j) {
                double t = GiJb[IDX2(j, i, nb)];
                for (int r = 0; r < m; ++r)
                    t += V.Bbar[IDX2(i, r, m)] * (Gb[IDX2(r, j, m)] + Gb[IDX2(j, r, m)]);
                Bbb[IDX2(i, j, m)] += rho * t;
            }
        free(G); free(Gi); free(Gb); free(GiJb);
    }
    /* read back the primitive blocks */
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) dA[IDX2(i, j, n)] = Abb[IDX2(i, j, nb)];
        for (int j = 0; j < m; ++j) dB[IDX2(i, j, m)] = Abb[IDX2(i, n + j, nb)] + Bbb[IDX2(i, j, m)];
        dQd[i] = qbd[i];
        dx0[i] = x0b[i];
    }
    for (int i = 0; i < m; ++i) dRd[i] = qbd[n + i];

    free(Mb); free(T1); free(qbd);
    free(xsb); free(gb); free(dub); free(hv); free(bv); free(cv); free(cb); free(bb); free(tmp); free(tmp2);
    free(Jb); free(Hab); free(Hbb); free(Abb); free(Bbb); free(x0b); free(sb); free(sa);
    free(tape); free(du); free(xs); free(dlast); free(xbar0);
    vform_free(&V); free(Aall); free(Ball); free(Q); free(R);
    return 0;
}

/* Projection of w (n entries) onto one factor set (exported for the pins). */
void orc_project(int kind, int n, const double *par, const double *lo, const double *hi, double *w) {
    static const double zero[1] = {0.0};
    project_set(kind, n, par ? par : zero, lo, hi, w);
}
