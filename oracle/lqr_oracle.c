/*
 * lqr_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load or call this file's library. It shares no code with the
 * GPU path.
 *
 * A plain, serial, double-precision CPU solver for the finite-horizon,
 * time-varying, discrete-time LQR problem of Laine & Tomlin, "The
 * Parallelization of Riccati Recursion" (arXiv:1809.06360), Sec. II, problem
 * (opt:globalwords) with the stage and terminal costs of eq. (costtform):
 *
 *   minimise  sum_{t<T} [ 1/2 x_t'Q_t x_t + u_t'S_t x_t + 1/2 u_t'R_t u_t
 *                          + q_t'x_t + r_t'u_t ]  +  1/2 x_T'Q_T x_T + q_T'x_T
 *   s.t.      x_{t+1} = A_t x_t + B_t u_t + c_t   (eq. dynamicsform),
 *             x_0 = x0.
 *
 * Paper symbols -> names here: Q_xx -> Q, Q_ux -> S, Q_uu -> R, q_x1 -> q,
 * q_u1 -> r, F_x -> A, F_u -> B, f_1 -> c, V_xx -> P, v_x1 -> p,
 * K_x -> K, k_1 -> k.
 *
 * Why the serial recursion is the oracle: the split/solve/link construction of
 * Sec. II-A reproduces the global optimum exactly (the link equation pins
 * x_link to the global optimum, and Sec. III-A states that the trajectories of
 * the serial and parallel methods are identical). The global optimum has a
 * plain definition -- the unique solution of the KKT system (eq. KKT), unique
 * because problem (opt:globalwords) is strictly convex under the assumptions
 * stated right after eq. (dynamicsform). Its plain serial computation is the
 * dynamic-programming (Riccati) recursion named in Sec. I, which is the
 * unconstrained special case of the recursion of Sec. II-B: with no constraint
 * to go, P_y is empty and Z_w = I (the degenerate case after eq.
 * (controlwupdate)), so the policy is eq. (Kx)/(k1) with only the M_uu terms
 * and the value update is eq. (update:Vxx)/(update:vx).
 *
 * Reading of the paper used here (the printed m_x1, m_u1 omit the affine
 * offset f_1): the linear terms of the per-stage problem are
 *   m_x1 = q + A'(P_{t+1} c + p_{t+1}),   m_u1 = r + B'(P_{t+1} c + p_{t+1}),
 * which is what substituting x_{t+1} = A x + B u + c into the quadratic
 * cost-to-go gives.
 *
 * Layout: row-major, time-major contiguous arrays:
 *   A[T][n][n] B[T][n][m] c[T][n] Q[T+1][n][n] q[T+1][n] R[T][m][m] r[T][m]
 *   S[T][m][n] (may be NULL = zero) x0[n]
 *   K[T][m][n] k[T][m] P[T+1][n][n] p[T+1][n] x[T+1][n] u[T][m] lam[T+1][n]
 * lam_t = P_t x_t + p_t is the costate; it equals minus the paper's lambda_t
 * (eq. mults1/multsT1 are written with +lambda_t on the x_t row).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((size_t)(i) * (size_t)(ld) + (size_t)(j))

/* In-place Cholesky H = L L' of an m x m symmetric matrix (lower triangle
 * written; the strict upper triangle is left untouched). Returns 0 on success,
 * 1 if a pivot is not positive or not finite. */
static int cholesky_lower(int m, double *H)
{
    for (int j = 0; j < m; ++j) {
        double d = H[IDX(j, j, m)];
        for (int l = 0; l < j; ++l)
            d -= H[IDX(j, l, m)] * H[IDX(j, l, m)];
        if (!(d > 0.0) || !isfinite(d))
            return 1;
        double ljj = sqrt(d);
        H[IDX(j, j, m)] = ljj;
        for (int i = j + 1; i < m; ++i) {
            double s = H[IDX(i, j, m)];
            for (int l = 0; l < j; ++l)
                s -= H[IDX(i, l, m)] * H[IDX(j, l, m)];
            H[IDX(i, j, m)] = s / ljj;
        }
    }
    return 0;
}

/* Solve (L L') X = Y in place for an m x ncol right-hand side Y (row-major,
 * leading dimension ncol), L lower triangular from cholesky_lower. */
static void cholesky_solve(int m, const double *L, int ncol, double *Y)
{
    for (int col = 0; col < ncol; ++col) {
        for (int i = 0; i < m; ++i) {            /* L z = y */
            double s = Y[IDX(i, col, ncol)];
            for (int l = 0; l < i; ++l)
                s -= L[IDX(i, l, m)] * Y[IDX(l, col, ncol)];
            Y[IDX(i, col, ncol)] = s / L[IDX(i, i, m)];
        }
        for (int i = m - 1; i >= 0; --i) {       /* L' x = z */
            double s = Y[IDX(i, col, ncol)];
            for (int l = i + 1; l < m; ++l)
                s -= L[IDX(l, i, m)] * Y[IDX(l, col, ncol)];
            Y[IDX(i, col, ncol)] = s / L[IDX(i, i, m)];
        }
    }
}

/*
 * Serial Riccati recursion and forward simulation.
 *
 * Backward, t = T-1 .. 0, with P_T = Q_T, p_T = q_T (the terminal cost-to-go):
 *   v    = P_{t+1} c_t + p_{t+1}
 *   M_xx = Q_t + A'P_{t+1}A       M_ux = S_t + B'P_{t+1}A    M_uu = R_t + B'P_{t+1}B
 *   m_x1 = q_t + A'v              m_u1 = r_t + B'v
 *   K_t  = -M_uu^{-1} M_ux        k_t  = -M_uu^{-1} m_u1          (eq. Kx, k1)
 *   P_t  = M_xx + M_ux'K_t        (eq. update:Vxx: M_xx + 2M_ux'K + K'M_uu K
 *                                  collapses to this at the minimiser)
 *   p_t  = m_x1 + M_ux'k_t        (eq. update:vx, likewise)
 * then P_t <- (P_t + P_t')/2 (the exact P_t is symmetric).
 * Forward (Sec. II-B, "Trajectory"): x_0 = x0, u_t = K_t x_t + k_t,
 * x_{t+1} = A_t x_t + B_t u_t + c_t.
 *
 * Returns 0 on success, t+1 if M_uu at stage t is not positive definite (the
 * recursion stops there; outputs are then incomplete), -1 on bad arguments or
 * allocation failure.
 */
int lqr_oracle_solve(int n, int m, int T,
                     const double *A, const double *B, const double *c,
                     const double *Q, const double *q,
                     const double *R, const double *r, const double *S,
                     const double *x0,
                     double *K, double *k, double *P, double *p,
                     double *x, double *u, double *lam)
{
    if (n < 1 || m < 1 || T < 1 || !A || !B || !c || !Q || !q || !R || !r || !x0 ||
        !K || !k || !P || !p || !x || !u)
        return -1;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m, mm = (size_t)m * m;
    double *PA = malloc(sizeof(double) * nn);
    double *PB = malloc(sizeof(double) * nm);
    double *v = malloc(sizeof(double) * n);
    double *Muu = malloc(sizeof(double) * mm);
    /* right-hand side [M_ux | m_u1], m x (n+1) */
    double *rhs = malloc(sizeof(double) * (size_t)m * (n + 1));
    double *sol = malloc(sizeof(double) * (size_t)m * (n + 1));
    if (!PA || !PB || !v || !Muu || !rhs || !sol) {
        free(PA); free(PB); free(v); free(Muu); free(rhs); free(sol);
        return -1;
    }

    memcpy(P + (size_t)T * nn, Q + (size_t)T * nn, sizeof(double) * nn);
    memcpy(p + (size_t)T * n, q + (size_t)T * n, sizeof(double) * n);

    int info = 0;
    for (int t = T - 1; t >= 0 && info == 0; --t) {
        const double *At = A + (size_t)t * nn, *Bt = B + (size_t)t * nm, *ct = c + (size_t)t * n;
        const double *Qt = Q + (size_t)t * nn, *qt = q + (size_t)t * n;
        const double *Rt = R + (size_t)t * mm, *rt = r + (size_t)t * m;
        const double *St = S ? S + (size_t)t * nm : NULL;
        const double *Pn = P + (size_t)(t + 1) * nn, *pn = p + (size_t)(t + 1) * n;
        double *Pt = P + (size_t)t * nn, *pt = p + (size_t)t * n;
        double *Kt = K + (size_t)t * nm, *kt = k + (size_t)t * m;

        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += Pn[IDX(i, l, n)] * At[IDX(l, j, n)];
                PA[IDX(i, j, n)] = s;
            }
            for (int j = 0; j < m; ++j) {
                double s = 0.0;
                for (int l = 0; l < n; ++l) s += Pn[IDX(i, l, n)] * Bt[IDX(l, j, m)];
                PB[IDX(i, j, m)] = s;
            }
            double s = pn[i];
            for (int l = 0; l < n; ++l) s += Pn[IDX(i, l, n)] * ct[l];
            v[i] = s;
        }
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) {
                double s = Rt[IDX(i, j, m)];
                for (int l = 0; l < n; ++l) s += Bt[IDX(l, i, m)] * PB[IDX(l, j, m)];
                Muu[IDX(i, j, m)] = s;
            }
            for (int j = 0; j < n; ++j) {
                double s = St ? St[IDX(i, j, n)] : 0.0;
                for (int l = 0; l < n; ++l) s += Bt[IDX(l, i, m)] * PA[IDX(l, j, n)];
                rhs[IDX(i, j, n + 1)] = s;
            }
            double s = rt[i];
            for (int l = 0; l < n; ++l) s += Bt[IDX(l, i, m)] * v[l];
            rhs[IDX(i, n, n + 1)] = s;
        }
        if (cholesky_lower(m, Muu)) {
            info = t + 1;
            break;
        }
        /* rhs <- M_uu^{-1} [M_ux | m_u1]; K = -that, k = -that */
        memcpy(sol, rhs, sizeof(double) * (size_t)m * (n + 1));
        cholesky_solve(m, Muu, n + 1, sol);
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < n; ++j) Kt[IDX(i, j, n)] = -sol[IDX(i, j, n + 1)];
            kt[i] = -sol[IDX(i, n, n + 1)];
        }
        /* P_t = Q + A'PA + M_ux'K,  p_t = q + A'v + M_ux'k */
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                double s = Qt[IDX(i, j, n)];
                for (int l = 0; l < n; ++l) s += At[IDX(l, i, n)] * PA[IDX(l, j, n)];
                for (int l = 0; l < m; ++l) s += rhs[IDX(l, i, n + 1)] * Kt[IDX(l, j, n)];
                Pt[IDX(i, j, n)] = s;
            }
            double s = qt[i];
            for (int l = 0; l < n; ++l) s += At[IDX(l, i, n)] * v[l];
            for (int l = 0; l < m; ++l) s += rhs[IDX(l, i, n + 1)] * kt[l];
            pt[i] = s;
        }
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                double s = 0.5 * (Pt[IDX(i, j, n)] + Pt[IDX(j, i, n)]);
                Pt[IDX(i, j, n)] = s;
                Pt[IDX(j, i, n)] = s;
            }
    }
    free(PA); free(PB); free(v); free(Muu); free(rhs); free(sol);
    if (info != 0)
        return info;

    memcpy(x, x0, sizeof(double) * n);
    for (int t = 0; t < T; ++t) {
        const double *At = A + (size_t)t * nn, *Bt = B + (size_t)t * nm, *ct = c + (size_t)t * n;
        const double *Kt = K + (size_t)t * nm, *kt = k + (size_t)t * m;
        const double *xt = x + (size_t)t * n;
        double *ut = u + (size_t)t * m, *xn = x + (size_t)(t + 1) * n;
        for (int i = 0; i < m; ++i) {
            double s = kt[i];
            for (int l = 0; l < n; ++l) s += Kt[IDX(i, l, n)] * xt[l];
            ut[i] = s;
        }
        for (int i = 0; i < n; ++i) {
            double s = ct[i];
            for (int l = 0; l < n; ++l) s += At[IDX(i, l, n)] * xt[l];
            for (int l = 0; l < m; ++l) s += Bt[IDX(i, l, m)] * ut[l];
            xn[i] = s;
        }
    }
    if (lam) {
        for (int t = 0; t <= T; ++t) {
            const double *Pt = P + (size_t)t * nn, *pt = p + (size_t)t * n, *xt = x + (size_t)t * n;
            double *lt = lam + (size_t)t * n;
            for (int i = 0; i < n; ++i) {
                double s = pt[i];
                for (int l = 0; l < n; ++l) s += Pt[IDX(i, l, n)] * xt[l];
                lt[i] = s;
            }
        }
    }
    return 0;
}

/*
 * Gradient of a scalar loss l(x, u) of the optimal trajectory with respect to
 * every problem datum, by implicit differentiation of the KKT system (eq. KKT).
 *
 * The optimal (x, u, lam) is the stationary point of the Lagrangian
 *   L = cost(x, u) + sum_t lam_{t+1}'(A_t x_t + B_t u_t + c_t - x_{t+1})
 *                  + lam_0'(x0 - x_0),
 * whose KKT matrix is symmetric and bilinear in the data. Differentiating
 * "KKT matrix * z = -data" gives dl/dtheta = -zhat' (dKKT/dtheta z + ddata/dtheta),
 * where zhat solves the same KKT matrix against the right-hand side dl/dz.
 * That is the same LQR problem with linear terms qhat_t = -dl/dx_t,
 * rhat_t = -dl/du_t, offsets chat_t = 0 and initial state xhat_0 = 0, solved
 * here by the same serial recursion. With (xhat, uhat, lamhat) its solution:
 *   dl/dq_t = -xhat_t                 dl/dr_t = -uhat_t
 *   dl/dc_t = -lamhat_{t+1}           dl/dx0  = -lamhat_0
 *   dl/dQ_t = -(xhat_t x_t' + x_t xhat_t')/2     (t = 0..T)
 *   dl/dR_t = -(uhat_t u_t' + u_t uhat_t')/2
 *   dl/dS_t = -(uhat_t x_t' + u_t xhat_t')
 *   dl/dA_t = -(lamhat_{t+1} x_t' + lam_{t+1} xhat_t')
 *   dl/dB_t = -(lamhat_{t+1} u_t' + lam_{t+1} uhat_t')
 * Gradients for the symmetric Q_t and R_t are given in symmetric form.
 *
 * x, u, lam are the forward solution (lam_t = P_t x_t + p_t). dl_dx[T+1][n],
 * dl_du[T][m]. Any output pointer may be NULL (skipped). Returns as
 * lqr_oracle_solve.
 */
int lqr_oracle_backward(int n, int m, int T,
                        const double *A, const double *B,
                        const double *Q, const double *R, const double *S,
                        const double *x, const double *u, const double *lam,
                        const double *dl_dx, const double *dl_du,
                        double *dA, double *dB, double *dc,
                        double *dQ, double *dq, double *dR, double *dr,
                        double *dS, double *dx0)
{
    if (n < 1 || m < 1 || T < 1 || !A || !B || !Q || !R || !x || !u || !lam || !dl_dx || !dl_du)
        return -1;
    const size_t nn = (size_t)n * n, nm = (size_t)n * m, mm = (size_t)m * m;
    double *qh = malloc(sizeof(double) * (size_t)(T + 1) * n);
    double *rh = malloc(sizeof(double) * (size_t)T * m);
    double *ch = calloc((size_t)T * n, sizeof(double));
    double *x0h = calloc((size_t)n, sizeof(double));
    double *Kh = malloc(sizeof(double) * (size_t)T * nm);
    double *kh = malloc(sizeof(double) * (size_t)T * m);
    double *Ph = malloc(sizeof(double) * (size_t)(T + 1) * nn);
    double *ph = malloc(sizeof(double) * (size_t)(T + 1) * n);
    double *xh = malloc(sizeof(double) * (size_t)(T + 1) * n);
    double *uh = malloc(sizeof(double) * (size_t)T * m);
    double *lh = malloc(sizeof(double) * (size_t)(T + 1) * n);
    int info = -1;
    if (qh && rh && ch && x0h && Kh && kh && Ph && ph && xh && uh && lh) {
        for (size_t i = 0; i < (size_t)(T + 1) * n; ++i) qh[i] = -dl_dx[i];
        for (size_t i = 0; i < (size_t)T * m; ++i) rh[i] = -dl_du[i];
        info = lqr_oracle_solve(n, m, T, A, B, ch, Q, qh, R, rh, S, x0h,
                                Kh, kh, Ph, ph, xh, uh, lh);
    }
    if (info == 0) {
        for (int t = 0; t <= T; ++t) {
            const double *xt = x + (size_t)t * n, *xht = xh + (size_t)t * n;
            if (dq)
                for (int i = 0; i < n; ++i) dq[(size_t)t * n + i] = -xht[i];
            if (dQ)
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j)
                        dQ[(size_t)t * nn + IDX(i, j, n)] = -0.5 * (xht[i] * xt[j] + xt[i] * xht[j]);
        }
        for (int t = 0; t < T; ++t) {
            const double *xt = x + (size_t)t * n, *xht = xh + (size_t)t * n;
            const double *ut = u + (size_t)t * m, *uht = uh + (size_t)t * m;
            const double *l1 = lam + (size_t)(t + 1) * n, *lh1 = lh + (size_t)(t + 1) * n;
            if (dr)
                for (int i = 0; i < m; ++i) dr[(size_t)t * m + i] = -uht[i];
            if (dc)
                for (int i = 0; i < n; ++i) dc[(size_t)t * n + i] = -lh1[i];
            if (dR)
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < m; ++j)
                        dR[(size_t)t * mm + IDX(i, j, m)] = -0.5 * (uht[i] * ut[j] + ut[i] * uht[j]);
            if (dS)
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < n; ++j)
                        dS[(size_t)t * nm + IDX(i, j, n)] = -(uht[i] * xt[j] + ut[i] * xht[j]);
            if (dA)
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j)
                        dA[(size_t)t * nn + IDX(i, j, n)] = -(lh1[i] * xt[j] + l1[i] * xht[j]);
            if (dB)
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < m; ++j)
                        dB[(size_t)t * nm + IDX(i, j, m)] = -(lh1[i] * ut[j] + l1[i] * uht[j]);
        }
        if (dx0)
            for (int i = 0; i < n; ++i) dx0[i] = -lh[i];
    }
    free(qh); free(rh); free(ch); free(x0h); free(Kh); free(kh);
    free(Ph); free(ph); free(xh); free(uh); free(lh);
    return info;
}
