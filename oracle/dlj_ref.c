/*
 * dlj_ref.c -- plain FP64 CPU reference of the double-layer Jacobi method for
 * finite-difference PDE-constrained NMPC (Deng & Ohtsuka, arXiv 2004.02484).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle: it is compiled and called
 * by the tests, by the smoke check and by the benchmark's CPU-baseline leg, and
 * by nothing else. It shares no code with the HIP library.
 *
 * Everything is written as plain loops over explicit matrix rows so that it can
 * be checked against the paper by eye:
 *   - problem:   N-stage backward-Euler NMPC (Sec. 3, eq. nlp), stage cost
 *                l = 0.5 q |x - xref|^2 + 0.5 r |u|^2; with tau > 0 the input
 *                box u_lo <= u <= u_hi enters as the log barrier
 *                Phi = -tau sum_j (ln(u_j - u_lo) + ln(u_hi - u_j)) of the
 *                relaxed problem (eq. nlp_relaxed) and the Jacobi step is cut
 *                by the fraction-to-the-boundary rule (eq. eq_alphamax);
 *                tau = 0: no inequality constraints, alpha = 1;
 *   - dynamics:  f(u, x) = k(x) .* (L x) + B u, k(w) = k0 (1 + k1 w), L the
 *                central-difference Laplacian with zero Dirichlet values
 *                (class of eq. pde, discretization of Sec. 2.1);
 *   - KKT:       K_i(x_{i-1}, s_i, lambda_{i+1}) of Sec. 3.2 (eq. KKT);
 *   - upper:     S^{k+1} = S^k - (D^k)^{-1} K^k, stage blocks independent
 *                (eq. 1st_jacobi, Sec. 4.2);
 *   - lower:     reordered stage system (eq. sublinsys_cpx / sublinsys_simple),
 *                Schur elimination onto v3 (eq. step12) solved by the fixed-count
 *                iteration with diagonal A_uu of Sec. 5.2, each saddle solve by
 *                F_x v5 = b4 then F_x^T v4 = b5 - A_xx v5 (eq. coff), and every
 *                F_x / F_x^T solve by point Jacobi from a zero initial guess
 *                (Lemma lemma_jaco, Sec. 4.3).
 *
 * Layout: node p = iy * nsx + ix; X, LAM are [N][n], U is [N][m]; B is dense
 * [n][m] row-major (the caller builds it).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops below (timing of the oracle on n cores). */
void ref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

typedef struct {
    int dim, nsx, nsy, N, m;
    const double *B;                 /* [n][m] */
    double h, k0, k1, q, r, gamma;
    double tau, u_lo, u_hi;          /* input box by log barrier; tau = 0: none */
} ref_problem;

static int ref_n(const ref_problem *P) { return P->nsx * P->nsy; }

/* Barrier Phi(u) = -tau sum_j (ln(u_j - u_lo) + ln(u_hi - u_j)) of the
 * input box (eq. nlp_relaxed with G = (u - u_lo, u_hi - u)): its gradient and
 * the diagonal of its Hessian for one input; 0 without a box. */
static double bar_grad(const ref_problem *P, double u)
{
    if (P->tau <= 0.0) return 0.0;
    return -P->tau / (u - P->u_lo) + P->tau / (P->u_hi - u);
}
static double bar_hess(const ref_problem *P, double u)
{
    if (P->tau <= 0.0) return 0.0;
    double a = u - P->u_lo, b = P->u_hi - u;
    return P->tau / (a * a) + P->tau / (b * b);
}

/* Conductivity k(w) = k0 (1 + k1 w) and its derivative k' = k0 k1. */
static double cond(const ref_problem *P, double w) { return P->k0 * (1.0 + P->k1 * w); }
static double dcond(const ref_problem *P) { return P->k0 * P->k1; }

/* Row p of the Laplacian L: off-diagonal neighbours (index, weight) and the
 * diagonal weight. Off-grid neighbours carry the value 0 (Dirichlet). */
static int lap_row(const ref_problem *P, int p, int *qi, double *qw, double *diag)
{
    int ix = p % P->nsx, iy = p / P->nsx, c = 0;
    double ax = (double)(P->nsx + 1) * (double)(P->nsx + 1);   /* 1/dx^2 */
    double ay = (double)(P->nsy + 1) * (double)(P->nsy + 1);   /* 1/dy^2 */
    *diag = -2.0 * ax;
    if (ix > 0)           { qi[c] = p - 1; qw[c++] = ax; }
    if (ix < P->nsx - 1)  { qi[c] = p + 1; qw[c++] = ax; }
    if (P->dim == 2) {
        *diag += -2.0 * ay;
        if (iy > 0)          { qi[c] = p - P->nsx; qw[c++] = ay; }
        if (iy < P->nsy - 1) { qi[c] = p + P->nsx; qw[c++] = ay; }
    }
    return c;
}

static void lap_apply(const ref_problem *P, const double *v, double *out)
{
    int n = ref_n(P);
    for (int p = 0; p < n; ++p) {
        int qi[4]; double qw[4], d;
        int c = lap_row(P, p, qi, qw, &d);
        double s = d * v[p];
        for (int j = 0; j < c; ++j) s += qw[j] * v[qi[j]];
        out[p] = s;
    }
}

/* f(u, x) = k(x) .* (L x) + B u  (dynamics of the discretized PDE). */
static void dyn_f(const ref_problem *P, const double *x, const double *u, double *f)
{
    int n = ref_n(P), m = P->m;
    double *Lx = (double *)malloc(sizeof(double) * n);
    lap_apply(P, x, Lx);
    for (int p = 0; p < n; ++p) {
        double bu = 0.0;
        for (int j = 0; j < m; ++j) bu += P->B[(size_t)p * m + j] * u[j];
        f[p] = cond(P, x[p]) * Lx[p] + bu;
    }
    free(Lx);
}

/* (grad_x f)^T lam: scatter of the rows of grad_x f, whose entries are
 * (grad_x f)_{pq} = k(x_p) L_{pq} + [p == q] k' (L x)_p. */
static void dfx_T_apply(const ref_problem *P, const double *x, const double *lam, double *out)
{
    int n = ref_n(P);
    double *Lx = (double *)malloc(sizeof(double) * n);
    lap_apply(P, x, Lx);
    for (int q = 0; q < n; ++q) out[q] = 0.0;
    for (int p = 0; p < n; ++p) {
        int qi[4]; double qw[4], d;
        int c = lap_row(P, p, qi, qw, &d);
        double kp = cond(P, x[p]);
        out[p] += (kp * d + dcond(P) * Lx[p]) * lam[p];
        for (int j = 0; j < c; ++j) out[qi[j]] += kp * qw[j] * lam[p];
    }
    free(Lx);
}

/*
 * KKT function K_i of Sec. 3.2 for all stages, with x_0 = x0 and
 * lambda_{N+1} = 0:
 *   KX_i = x_{i-1} - x_i + h f(u_i, x_i)
 *   KU_i = h (r u_i + grad Phi(u_i) + B^T lam_i) + gamma (u_i - ut_i)
 *   KL_i = lam_{i+1} - lam_i + h (q (x_i - xref_i) + (grad_x f_i)^T lam_i)
 * xref has xref_stride = 0 (one reference for all stages) or n (per stage).
 * ut (the regularization reference) may be NULL, meaning ut = u.
 */
static void stage_kkt(const ref_problem *P, int i, const double *x0, const double *xref,
                      int xref_stride, const double *X, const double *U, const double *LAM,
                      const double *UT, double *kx, double *ku, double *kl)
{
    int n = ref_n(P), m = P->m, N = P->N;
    const double *xprev = (i == 0) ? x0 : X + (size_t)(i - 1) * n;
    const double *x = X + (size_t)i * n, *u = U + (size_t)i * m, *lam = LAM + (size_t)i * n;
    const double *xr = xref + (size_t)i * xref_stride;
    double *f = (double *)malloc(sizeof(double) * n);
    double *g = (double *)malloc(sizeof(double) * n);
    dyn_f(P, x, u, f);
    for (int p = 0; p < n; ++p) kx[p] = xprev[p] - x[p] + P->h * f[p];
    for (int j = 0; j < m; ++j) {
        double btl = 0.0;
        for (int p = 0; p < n; ++p) btl += P->B[(size_t)p * m + j] * lam[p];
        double reg = UT ? P->gamma * (u[j] - UT[(size_t)i * m + j]) : 0.0;
        ku[j] = P->h * (P->r * u[j] + bar_grad(P, u[j]) + btl) + reg;
    }
    dfx_T_apply(P, x, lam, g);
    for (int p = 0; p < n; ++p) {
        double lnext = (i == N - 1) ? 0.0 : LAM[(size_t)(i + 1) * n + p];
        kl[p] = lnext - lam[p] + P->h * (P->q * (x[p] - xr[p]) + g[p]);
    }
    free(f); free(g);
}

void ref_kkt(const ref_problem *P, const double *x0, const double *xref, int xref_stride,
             const double *X, const double *U, const double *LAM, const double *UT,
             double *KX, double *KU, double *KL)
{
    int n = ref_n(P), m = P->m, N = P->N;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        stage_kkt(P, i, x0, xref, xref_stride, X, U, LAM, UT, KX + (size_t)i * n,
                  KU + (size_t)i * m, KL + (size_t)i * n);
}

/* Residual norms: r_paper = |K|_inf; r_scaled divides the input rows by h r
 * and the costate rows by h (units of u and of q (x - xref)). */
void ref_norms(const ref_problem *P, const double *KX, const double *KU, const double *KL,
               double *r_scaled, double *r_paper)
{
    size_t nN = (size_t)ref_n(P) * P->N, mN = (size_t)P->m * P->N;
    double ax = 0.0, au = 0.0, al = 0.0;
    int bad = 0;
    for (size_t t = 0; t < nN; ++t) {
        if (!isfinite(KX[t]) || !isfinite(KL[t])) bad = 1;
        if (fabs(KX[t]) > ax) ax = fabs(KX[t]);
        if (fabs(KL[t]) > al) al = fabs(KL[t]);
    }
    for (size_t t = 0; t < mN; ++t) {
        if (!isfinite(KU[t])) bad = 1;
        if (fabs(KU[t]) > au) au = fabs(KU[t]);
    }
    double rp = ax > au ? ax : au; rp = rp > al ? rp : al;
    double rs = ax, su = au / (P->h * P->r), sl = al / P->h;
    rs = rs > su ? rs : su; rs = rs > sl ? rs : sl;
    if (bad) { rp = NAN; rs = NAN; }
    if (r_paper) *r_paper = rp;
    if (r_scaled) *r_scaled = rs;
}

/* ---------------------------------------------------------------- lower layer */

typedef struct {
    const ref_problem *P;
    const double *x, *lam;   /* stage iterate */
    double *kx, *Lx, *Fd;    /* k(x), L x, diagonal of F_x */
} stage_ctx;

/* F_x = h grad_x f - I: diagonal h (k(x_p) L_pp + k' (Lx)_p) - 1,
 * off-diagonal (p, q) = h k(x_p) L_pq. */
static void stage_setup(stage_ctx *S)
{
    const ref_problem *P = S->P;
    int n = ref_n(P);
    lap_apply(P, S->x, S->Lx);
    for (int p = 0; p < n; ++p) {
        int qi[4]; double qw[4], d;
        lap_row(P, p, qi, qw, &d);
        S->kx[p] = cond(P, S->x[p]);
        S->Fd[p] = P->h * (S->kx[p] * d + dcond(P) * S->Lx[p]) - 1.0;
    }
}

/* n_sw point-Jacobi sweeps for F_x y = c from y = 0. */
static void jacobi_F(const stage_ctx *S, int n_sw, const double *c, double *y, double *tmp)
{
    const ref_problem *P = S->P;
    int n = ref_n(P);
    for (int p = 0; p < n; ++p) y[p] = 0.0;
    for (int it = 0; it < n_sw; ++it) {
        for (int p = 0; p < n; ++p) {
            int qi[4]; double qw[4], d;
            int cnt = lap_row(P, p, qi, qw, &d);
            double off = 0.0;
            for (int j = 0; j < cnt; ++j) off += P->h * S->kx[p] * qw[j] * y[qi[j]];
            tmp[p] = (c[p] - off) / S->Fd[p];
        }
        memcpy(y, tmp, sizeof(double) * n);
    }
}

/* n_sw point-Jacobi sweeps for F_x^T y = c from y = 0; (F_x^T)_{pq} = (F_x)_{qp}. */
static void jacobi_FT(const stage_ctx *S, int n_sw, const double *c, double *y, double *tmp)
{
    const ref_problem *P = S->P;
    int n = ref_n(P);
    for (int p = 0; p < n; ++p) y[p] = 0.0;
    for (int it = 0; it < n_sw; ++it) {
        for (int p = 0; p < n; ++p) {
            int qi[4]; double qw[4], d;
            int cnt = lap_row(P, p, qi, qw, &d);
            double off = 0.0;
            /* L is symmetric, so L_qp = L_pq = qw[j]. */
            for (int j = 0; j < cnt; ++j) off += P->h * S->kx[qi[j]] * qw[j] * y[qi[j]];
            tmp[p] = (c[p] - off) / S->Fd[p];
        }
        memcpy(y, tmp, sizeof(double) * n);
    }
}

/* A_xx y = h grad_xx^2 H y with (grad_xx^2 H)_{ps} = q [p == s] + k' L_ps (lam_p + lam_s),
 * the second derivative of q/2 |x - xref|^2 + lam^T f in x (k'' = 0). */
static void axx_apply(const stage_ctx *S, const double *y, double *out)
{
    const ref_problem *P = S->P;
    int n = ref_n(P);
    double kp = dcond(P);
    for (int p = 0; p < n; ++p) {
        int qi[4]; double qw[4], d;
        int cnt = lap_row(P, p, qi, qw, &d);
        double s = P->q * y[p] + kp * d * (2.0 * S->lam[p]) * y[p];
        for (int j = 0; j < cnt; ++j) s += kp * qw[j] * (S->lam[p] + S->lam[qi[j]]) * y[qi[j]];
        out[p] = P->h * s;
    }
}

static void B_apply(const ref_problem *P, const double *v, double *out)
{
    int n = ref_n(P), m = P->m;
    for (int p = 0; p < n; ++p) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += P->B[(size_t)p * m + j] * v[j];
        out[p] = s;
    }
}

static void BT_apply(const ref_problem *P, const double *y, double *out)
{
    int n = ref_n(P), m = P->m;
    for (int j = 0; j < m; ++j) {
        double s = 0.0;
        for (int p = 0; p < n; ++p) s += P->B[(size_t)p * m + j] * y[p];
        out[j] = s;
    }
}

/*
 * Lower layer for one stage: approximately solve D_i ds = K_i.
 * Reordered unknowns v1 = d lambda, v2 = d x, v3 = d u and right-hand sides
 * b1 = KX_i, b2 = KL_i, b3 = KU_i. Blocks: F_x = h grad_x f - I, F_u = h B,
 * A_xx = h grad_xx^2 H, A_xu = A_ux = 0 (f is affine in u, l separable),
 * A_uu = h (r + Phi''(u)) + gamma, diagonal (u: the stage's inputs; may be
 * NULL without a box).
 *  Schur iteration (n_schur times from v3 = 0):
 *     v5 = F_x^{-1} (F_u v3 - b1)
 *     v4 = F_x^{-T} (-b2 - A_xx v5)
 *     v3 = (b3 + F_u^T v4) / A_uu
 *  then eq. step2:  v2 = F_x^{-1} (b1 - F_u v3),  v1 = F_x^{-T} (b2 - A_xx v2),
 *  with every F_x^{-1} / F_x^{-T} replaced by n_sw point-Jacobi sweeps.
 */
void ref_stage_solve(const ref_problem *P, const double *x, const double *lam, const double *u,
                     const double *b1, const double *b2, const double *b3,
                     int n_sw, int n_schur, double *dx, double *du, double *dlam)
{
    int n = ref_n(P), m = P->m;
    double *w = (double *)malloc(sizeof(double) * (size_t)(9 * n + 2 * m));
    stage_ctx S = {P, x, lam, w, w + n, w + 2 * n};
    double *c = w + 3 * n, *v5 = w + 4 * n, *v4 = w + 5 * n, *tmp = w + 6 * n;
    double *Bv = w + 7 * n, *Ay = w + 8 * n;
    double *v3 = w + 9 * n, *btv = w + 9 * n + m;
    double Auu = P->h * P->r + P->gamma;
    stage_setup(&S);

    for (int j = 0; j < m; ++j) v3[j] = 0.0;
    for (int it = 0; it < n_schur; ++it) {
        B_apply(P, v3, Bv);
        for (int p = 0; p < n; ++p) c[p] = P->h * Bv[p] - b1[p];
        jacobi_F(&S, n_sw, c, v5, tmp);
        axx_apply(&S, v5, Ay);
        for (int p = 0; p < n; ++p) c[p] = -b2[p] - Ay[p];
        jacobi_FT(&S, n_sw, c, v4, tmp);
        BT_apply(P, v4, btv);
        for (int j = 0; j < m; ++j)
            v3[j] = (b3[j] + P->h * btv[j]) / (Auu + (u ? P->h * bar_hess(P, u[j]) : 0.0));
    }
    B_apply(P, v3, Bv);
    for (int p = 0; p < n; ++p) c[p] = b1[p] - P->h * Bv[p];
    jacobi_F(&S, n_sw, c, v5, tmp);              /* v2 */
    axx_apply(&S, v5, Ay);
    for (int p = 0; p < n; ++p) c[p] = b2[p] - Ay[p];
    jacobi_FT(&S, n_sw, c, v4, tmp);             /* v1 */
    for (int p = 0; p < n; ++p) { dx[p] = v5[p]; dlam[p] = v4[p]; }
    for (int j = 0; j < m; ++j) du[j] = v3[j];
    free(w);
}

/* ---------------------------------------------------------------- upper layer */

/*
 * Fraction-to-the-boundary rule (eq. eq_alphamax) for the input box: the
 * largest alpha in (0, 1] with G(u - alpha du) >= 0.005 G(u) for every input
 * of every stage, i.e. alpha <= 0.995 (u - u_lo) / du where du > 0 and
 * alpha <= 0.995 (u_hi - u) / (-du) where du < 0. 1 without a box.
 */
double ref_alpha_max(const ref_problem *P, const double *U, const double *DU)
{
    if (P->tau <= 0.0) return 1.0;
    double a = 1.0;
    size_t mN = (size_t)P->N * P->m;
    for (size_t t = 0; t < mN; ++t) {
        double u = U[t], d = DU[t], lim = 1.0;
        if (d > 0.0) lim = 0.995 * (u - P->u_lo) / d;
        else if (d < 0.0) lim = 0.995 * (P->u_hi - u) / (-d);
        if (lim < a) a = lim;
    }
    return a;
}

/*
 * One upper-layer Jacobi iteration (eq. 1st_jacobi with the regularization
 * reference ut = u^k): evaluates K^k, its norms, and writes
 * S^{k+1} = S^k - alpha (D^k)^{-1} K^k into (Xn, Un, LAMn), alpha from the
 * fraction-to-the-boundary rule (1 without a box). All stage blocks are
 * solved independently from S^k.
 */
void ref_iterate(const ref_problem *P, const double *x0, const double *xref, int xref_stride,
                 const double *X, const double *U, const double *LAM,
                 double *Xn, double *Un, double *LAMn, int n_sw, int n_schur,
                 double *r_scaled, double *r_paper)
{
    int n = ref_n(P), m = P->m, N = P->N;
    double *KX = (double *)malloc(sizeof(double) * (size_t)N * n);
    double *KL = (double *)malloc(sizeof(double) * (size_t)N * n);
    double *KU = (double *)malloc(sizeof(double) * (size_t)N * m);
    ref_kkt(P, x0, xref, xref_stride, X, U, LAM, U, KX, KU, KL);
    ref_norms(P, KX, KU, KL, r_scaled, r_paper);
    if (Xn) {
        /* the steps of all stages first (into the outputs), then alpha */
        double *DU = (double *)malloc(sizeof(double) * (size_t)N * m);
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < N; ++i)
            ref_stage_solve(P, X + (size_t)i * n, LAM + (size_t)i * n, U + (size_t)i * m,
                            KX + (size_t)i * n, KL + (size_t)i * n, KU + (size_t)i * m,
                            n_sw, n_schur, Xn + (size_t)i * n, DU + (size_t)i * m,
                            LAMn + (size_t)i * n);
        const double alpha = ref_alpha_max(P, U, DU);
        for (size_t t = 0; t < (size_t)N * n; ++t) {
            Xn[t] = X[t] - alpha * Xn[t];
            LAMn[t] = LAM[t] - alpha * LAMn[t];
        }
        for (size_t t = 0; t < (size_t)N * m; ++t) Un[t] = U[t] - alpha * DU[t];
        free(DU);
    }
    free(KX); free(KL); free(KU);
}

/*
 * Iterate from the start held in (X, U, LAM) until r_scaled(S^k) <= tol or
 * k == max_iter. On return (X, U, LAM) hold the last evaluated iterate S^k,
 * *iters = k and the residuals of S^k. rhist (may be NULL) receives r_scaled
 * of S^0..S^k. Returns 0 converged, 1 not converged, 2 non-finite residual.
 */
int ref_solve(const ref_problem *P, const double *x0, const double *xref, int xref_stride,
              double *X, double *U, double *LAM, double tol, int max_iter,
              int n_sw, int n_schur, int *iters, double *r_scaled, double *r_paper,
              double *rhist)
{
    int n = ref_n(P), m = P->m, N = P->N, k = 0, status = 1;
    size_t sz = (size_t)N * (2 * n + m);
    double *buf = (double *)malloc(sizeof(double) * sz);
    double *Xn = buf, *LAMn = buf + (size_t)N * n, *Un = buf + (size_t)2 * N * n;
    double rs = 0.0, rp = 0.0;
    for (;;) {
        int last = (k >= max_iter);
        ref_iterate(P, x0, xref, xref_stride, X, U, LAM, Xn, Un, LAMn, n_sw, n_schur, &rs, &rp);
        if (rhist) rhist[k] = rs;
        if (!isfinite(rs)) { status = 2; break; }
        if (rs <= tol) { status = 0; break; }
        if (last) { status = 1; break; }
        memcpy(X, Xn, sizeof(double) * (size_t)N * n);
        memcpy(LAM, LAMn, sizeof(double) * (size_t)N * n);
        memcpy(U, Un, sizeof(double) * (size_t)N * m);
        ++k;
    }
    free(buf);
    if (iters) *iters = k;
    if (r_scaled) *r_scaled = rs;
    if (r_paper) *r_paper = rp;
    return status;
}

/* ------------------------------------------------ Gauss-Seidel upper layers */

/*
 * One Gauss-Seidel sweep over the stages (Sec. 4.4, Jacobi-type variants),
 * in place: the stages are visited in turn (dir > 0: i = 1..N, forward;
 * dir < 0: i = N..1, backward) and each stage block is solved from the
 * current trajectory, in which the stages visited before already hold their
 * new values. The regularization reference is the stage's current input
 * (u~ = u^k), as in the Jacobi iteration.
 *
 * K_i depends on x_{i-1} and lambda_{i+1} only through the terms x_{i-1} and
 * lambda_{i+1} themselves, and D_i only on s_i, so a forward sweep is exactly
 * S - (D^k + L)^{-1} K^k (eq. fgs) and a backward sweep S - (D^k + U)^{-1} K^k
 * (BGS), with L / U the blocks coupling a stage to the previous / next one.
 * UT (may be NULL) is the regularization reference u~ of every stage: NULL
 * means the stage's input at its visit, which is u^k in a single sweep.
 * omega scales every stage's step (successive over-relaxation, Sec. 4.4): a
 * forward sweep is then S - omega (D^k + omega L)^{-1} K^k, and omega = 1 is
 * the plain sweep.
 */
void ref_gs_sweep(const ref_problem *P, const double *x0, const double *xref, int xref_stride,
                  double *X, double *U, double *LAM, const double *UT, int dir, int n_sw,
                  int n_schur, double omega)
{
    int n = ref_n(P), m = P->m, N = P->N;
    double *w = (double *)malloc(sizeof(double) * (size_t)(4 * n + 2 * m));
    double *kx = w, *kl = w + n, *dx = w + 2 * n, *dl = w + 3 * n;
    double *ku = w + 4 * n, *du = w + 4 * n + m;
    for (int t = 0; t < N; ++t) {
        int i = dir > 0 ? t : N - 1 - t;
        stage_kkt(P, i, x0, xref, xref_stride, X, U, LAM, UT, kx, ku, kl);
        ref_stage_solve(P, X + (size_t)i * n, LAM + (size_t)i * n, U + (size_t)i * m, kx, kl, ku,
                        n_sw, n_schur, dx, du, dl);
        for (int p = 0; p < n; ++p) {
            X[(size_t)i * n + p] -= omega * dx[p];
            LAM[(size_t)i * n + p] -= omega * dl[p];
        }
        for (int j = 0; j < m; ++j) U[(size_t)i * m + j] -= omega * du[j];
    }
    free(w);
}

/*
 * A Gauss-Seidel sweep cut by the fraction-to-the-boundary rule (eq.
 * eq_alphamax) when an input box is set: the sweep's result S_sweep replaces
 * S only as far as S + alpha (S_sweep - S), alpha the largest step that keeps
 * every input's distance to the box above 0.005 of its value at S (the
 * paper states the rule for the Jacobi step; a sweep is read as one such
 * step). Sc: scratch of N (2n + m) doubles.
 */
static void gs_sweep_cut(const ref_problem *P, const double *x0, const double *xref,
                         int xref_stride, double *X, double *U, double *LAM, const double *UT,
                         int dir, int n_sw, int n_schur, double omega, double *Sc)
{
    int n = ref_n(P), m = P->m, N = P->N;
    size_t nx = (size_t)N * n, nu = (size_t)N * m;
    if (P->tau <= 0.0) {
        ref_gs_sweep(P, x0, xref, xref_stride, X, U, LAM, UT, dir, n_sw, n_schur, omega);
        return;
    }
    double *X0 = Sc, *L0 = Sc + nx, *U0 = Sc + 2 * nx;
    memcpy(X0, X, sizeof(double) * nx);
    memcpy(L0, LAM, sizeof(double) * nx);
    memcpy(U0, U, sizeof(double) * nu);
    ref_gs_sweep(P, x0, xref, xref_stride, X, U, LAM, UT, dir, n_sw, n_schur, omega);
    double *DU = (double *)malloc(sizeof(double) * nu);
    for (size_t t = 0; t < nu; ++t) DU[t] = U0[t] - U[t];
    const double a = ref_alpha_max(P, U0, DU);
    free(DU);
    if (a < 1.0) {
        for (size_t t = 0; t < nx; ++t) {
            X[t] = X0[t] + a * (X[t] - X0[t]);
            LAM[t] = L0[t] + a * (LAM[t] - L0[t]);
        }
        for (size_t t = 0; t < nu; ++t) U[t] = U0[t] + a * (U[t] - U0[t]);
    }
}

/*
 * Upper layer by Gauss-Seidel sweeps: upper = 1 FGS (eq. fgs), 2 BGS,
 * 3 SGS (eq. sgs, read as a backward sweep followed by a forward sweep, both
 * with the regularization reference u~ = u^k of the iteration; in the linear
 * case this is eq. sgs exactly). Every iteration first evaluates K(S^k) and
 * its norms for the stopping test, exactly as ref_solve does; the returned
 * trajectory is the last evaluated iterate S^k. omega: the over-relaxation of
 * every sweep (SOR forward, backward; SSOR for SGS). With an input box each
 * sweep is cut by the fraction-to-the-boundary rule (gs_sweep_cut).
 */
int ref_solve_gs(const ref_problem *P, const double *x0, const double *xref, int xref_stride,
                 double *X, double *U, double *LAM, int upper, double tol, int max_iter,
                 int n_sw, int n_schur, int *iters, double *r_scaled, double *r_paper,
                 double *rhist, double omega)
{
    int n = ref_n(P), m = P->m, N = P->N, k = 0, status = 1;
    double *KX = (double *)malloc(sizeof(double) * (size_t)N * n);
    double *KL = (double *)malloc(sizeof(double) * (size_t)N * n);
    double *KU = (double *)malloc(sizeof(double) * (size_t)N * m);
    double *UK = (double *)malloc(sizeof(double) * (size_t)N * m);
    double *Sc = (double *)malloc(sizeof(double) * (size_t)N * (2 * n + m));
    double rs = 0.0, rp = 0.0;
    for (;;) {
        ref_kkt(P, x0, xref, xref_stride, X, U, LAM, U, KX, KU, KL);
        ref_norms(P, KX, KU, KL, &rs, &rp);
        if (rhist) rhist[k] = rs;
        if (!isfinite(rs)) { status = 2; break; }
        if (rs <= tol) { status = 0; break; }
        if (k >= max_iter) { status = 1; break; }
        if (upper == 1) {
            gs_sweep_cut(P, x0, xref, xref_stride, X, U, LAM, NULL, +1, n_sw, n_schur, omega, Sc);
        } else if (upper == 2) {
            gs_sweep_cut(P, x0, xref, xref_stride, X, U, LAM, NULL, -1, n_sw, n_schur, omega, Sc);
        } else {
            memcpy(UK, U, sizeof(double) * (size_t)N * m);
            gs_sweep_cut(P, x0, xref, xref_stride, X, U, LAM, NULL, -1, n_sw, n_schur, omega, Sc);
            gs_sweep_cut(P, x0, xref, xref_stride, X, U, LAM, UK, +1, n_sw, n_schur, omega, Sc);
        }
        ++k;
    }
    free(KX); free(KL); free(KU); free(UK); free(Sc);
    if (iters) *iters = k;
    if (r_scaled) *r_scaled = rs;
    if (r_paper) *r_paper = rp;
    return status;
}
