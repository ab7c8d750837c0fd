/*
 * ch_oracle.c -- plain FP64 CPU oracle for the Cahn-Hilliard ensemble hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity reference that the HIP
 * path is checked against.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.  It
 * shares no code, header, table or constant generator with the HIP library.
 *
 * What it computes (paper: Section 1, eq. (ch) and eq. (dFdt_ch); Section 4.1
 * "Methodology"; eq. (betadef)):
 *
 *   dC/dt = lap(C^3 - C - gamma lap C)  on a periodic grid, D = 2 or 3,
 *
 * stepped by the semi-implicit ADI finite-difference scheme (Section 4.1 and
 * Appendix A say "semi-implicit ADI, periodic, first order"; the scheme below
 * is the reading adopted where the paper is silent):
 *
 *   N^n   = C^n C^n C^n - C^n
 *   RHS   = C^n + dt lap_h N^n - 2 gamma dt sum_{d<e} D_d D_e C^n
 *   w^0   = RHS;  for d = 1..D:  (I + gamma dt D_d^2) w^d = w^{d-1}  on d-lines
 *   C^n+1 = w^D
 *
 * with D_d f = (f_{+1} - 2 f + f_{-1}) / h_d^2 (periodic), lap_h = sum_d D_d.
 * This is theta = 1 of the theta-weighted ADI family
 *
 *   prod_d (I + theta gamma dt D_d^2) C^{n+1}
 *       = prod_d (I - (1-theta) gamma dt D_d^2) C^n + RHS - C^n,
 *
 * whose theta = 1/2 member is the Crank-Nicolson ADI variant: second order in
 * dt where only the pure fourth derivatives act (Appendix A: the scheme for
 * hyper-diffusion alone is second order), first order once the explicit
 * nonlinear and mixed terms enter (orc_step_theta).
 *
 * Diagnostics (eq. (dFdt_ch), eq. (betadef)):
 *   F      = prod(h) sum_sites [ e(C) + gamma/2 sum_d ((C_{+d}-C)/h_d)^2 ]
 *            e(C) = (C^2-1)^2/4 (default) or (C^2-1)^2/2 (as printed)
 *   <C>    = sum C / #sites
 *   G_id   = -prod(h) sum_sites sum_d ((mu_{+d}-mu)/h_d)^2,
 *            mu = C^3 - C - gamma lap_h C     (the dF/dt identity)
 *   G_fd   = (F^{n+1} - F^{n-1}) / (2 dt)  (one-sided at the ends of the run)
 *   beta   = -(t / F) G_fd,  t = n dt
 * Sums are exactly rounded (Shewchuk's non-overlapping partials).
 *
 * The periodic line solve uses the Sherman-Morrison-Woodbury formula on top of
 * a banded LU factorisation of the non-periodic pentadiagonal part (a direct
 * method unrelated to whatever the GPU uses).  The line mean passes through
 * the solve exactly (constants are fixed points of the operator, which is what
 * conserves <C>), and one residual-correction step restores the digits the
 * Woodbury cancellation loses at large gamma dt / h^4.
 *
 * Initial condition: C = c0 + noise (2u - 1), where u is built from the
 * (site+1)-th output of the SplitMix64 generator (Steele, Lea & Flood 2014)
 * seeded with the member's seed: u = (out >> 11) * 2^-53.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): state advances by the  */
/* golden-ratio increment; each output is the state passed through the   */
/* variant-13 finaliser.                                                  */
/* ------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ULL; /* state after k advances */
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

double orc_uniform(uint64_t seed, uint64_t site)
{
    return (double)(orc_splitmix64(seed, site + 1) >> 11) * (1.0 / 9007199254740992.0);
}

static int64_t nsites(int dim, const int32_t *n)
{
    return (int64_t)n[0] * n[1] * (dim == 3 ? n[2] : 1);
}

void orc_init_field(int dim, const int32_t *n, double c0, double noise, uint64_t seed,
                    double *C)
{
    int64_t S = nsites(dim, n);
    for (int64_t s = 0; s < S; s++)
        C[s] = c0 + noise * (2.0 * orc_uniform(seed, (uint64_t)s) - 1.0);
}

/* ------------------------------------------------------------------ */
/* Exactly rounded summation: Shewchuk (1997) non-overlapping partials,  */
/* with the round-half-even fix-up of the final partials that CPython's  */
/* math.fsum applies (R. Hettinger's msum recipe built on Shewchuk).     */
/* ------------------------------------------------------------------ */
typedef struct {
    double p[160];
    int n;
    double naive; /* plain sum, used only when an input is not finite */
    int nonfinite;
} xsum;

static void xsum_init(xsum *s)
{
    s->n = 0;
    s->naive = 0.0;
    s->nonfinite = 0;
}

static void xsum_add(xsum *s, double x)
{
    s->naive += x;
    if (!isfinite(x)) {
        s->nonfinite = 1;
        return;
    }
    int i = 0;
    for (int j = 0; j < s->n; j++) {
        double y = s->p[j];
        if (fabs(x) < fabs(y)) {
            double t = x;
            x = y;
            y = t;
        }
        double hi = x + y;
        double lo = y - (hi - x);
        if (lo != 0.0) s->p[i++] = lo;
        x = hi;
    }
    s->p[i++] = x;
    s->n = i;
    if (!isfinite(x)) s->nonfinite = 1; /* overflow of the running sum */
}

static double xsum_result(const xsum *s)
{
    if (s->nonfinite) return s->naive;
    int n = s->n;
    double hi = 0.0, lo = 0.0;
    if (n > 0) {
        hi = s->p[--n];
        while (n > 0) {
            double x = hi;
            double y = s->p[--n];
            hi = x + y;
            double yr = hi - x;
            lo = y - yr;
            if (lo != 0.0) break;
        }
        if (n > 0 && ((lo < 0.0 && s->p[n - 1] < 0.0) || (lo > 0.0 && s->p[n - 1] > 0.0))) {
            double y = lo * 2.0;
            double x = hi + y;
            double yr = x - hi;
            if (y == yr) hi = x;
        }
    }
    return hi;
}

double orc_exact_sum(const double *x, int64_t m)
{
    xsum s;
    xsum_init(&s);
    for (int64_t i = 0; i < m; i++) xsum_add(&s, x[i]);
    return xsum_result(&s);
}

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int dim;
    int64_t n[3];
    int64_t stride[3];
    double h[3];
    int64_t S;
} grid;

static void grid_make(grid *g, int dim, const int32_t *n, const double *L)
{
    g->dim = dim;
    for (int d = 0; d < 3; d++) {
        g->n[d] = (d < dim) ? n[d] : 1;
        g->h[d] = (d < dim) ? L[d] / (double)n[d] : 1.0;
    }
    g->stride[0] = 1;
    g->stride[1] = g->n[0];
    g->stride[2] = g->n[0] * g->n[1];
    g->S = g->n[0] * g->n[1] * g->n[2];
}

/* index of the site displaced by `off` along axis d (periodic) */
static inline int64_t nb(const grid *g, int64_t s, int d, int off)
{
    int64_t i = (s / g->stride[d]) % g->n[d];
    int64_t j = i + off;
    if (j < 0) j += g->n[d];
    if (j >= g->n[d]) j -= g->n[d];
    return s + (j - i) * g->stride[d];
}

/* second difference along d: D_d f = (f+ - 2f + f-)/h^2 */
static void second_diff(const grid *g, int d, const double *f, double *out)
{
    double ih2 = 1.0 / (g->h[d] * g->h[d]);
    int64_t S = g->S;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; s++)
        out[s] = (f[nb(g, s, d, +1)] - 2.0 * f[s] + f[nb(g, s, d, -1)]) * ih2;
}

/* lap_h f = sum_d D_d f */
void orc_laplacian(int dim, const int32_t *n, const double *L, const double *f, double *out)
{
    grid g;
    grid_make(&g, dim, n, L);
    double *t = (double *)malloc(sizeof(double) * g.S);
    memset(out, 0, sizeof(double) * g.S);
    for (int d = 0; d < dim; d++) {
        second_diff(&g, d, f, t);
        for (int64_t s = 0; s < g.S; s++) out[s] += t[s];
    }
    free(t);
}

/* sum_{d<e} D_d D_e f (the mixed fourth-order terms of lap^2) */
void orc_cross(int dim, const int32_t *n, const double *L, const double *f, double *out)
{
    grid g;
    grid_make(&g, dim, n, L);
    double *a = (double *)malloc(sizeof(double) * g.S);
    double *b = (double *)malloc(sizeof(double) * g.S);
    memset(out, 0, sizeof(double) * g.S);
    for (int e = 1; e < dim; e++) {
        second_diff(&g, e, f, a);
        for (int d = 0; d < e; d++) {
            second_diff(&g, d, a, b);
            for (int64_t s = 0; s < g.S; s++) out[s] += b[s];
        }
    }
    free(a);
    free(b);
}

/* ------------------------------------------------------------------ */
/* Periodic pentadiagonal solve  (I + rho [1,-4,6,-4,1]) y = f           */
/* via Woodbury on the non-periodic band B:  A = B + P K P^T, with        */
/* P = [e_0, e_1, e_{n-2}, e_{n-1}] holding the wrap-around corners.      */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    double rho;
    double *l1, *l2;   /* unit-lower band multipliers (sub-diagonals 1, 2) */
    double *u0, *u1, *u2; /* upper band: diagonal, super-diagonals 1, 2 */
    double *Z;         /* B^{-1} P, n x 4, column-major */
    double Kmat[16];   /* the 4x4 corner coupling K */
    double Smat[16];   /* I + K P^T Z, LU-factorised in place (row-major) */
    int piv[4];
} penta;

static void band_solve(const penta *q, const double *f, double *y)
{
    int64_t n = q->n;
    /* forward: L z = f */
    for (int64_t i = 0; i < n; i++) {
        double z = f[i];
        if (i >= 1) z -= q->l1[i] * y[i - 1];
        if (i >= 2) z -= q->l2[i] * y[i - 2];
        y[i] = z;
    }
    /* backward: U y = z */
    for (int64_t i = n - 1; i >= 0; i--) {
        double z = y[i];
        if (i + 1 < n) z -= q->u1[i] * y[i + 1];
        if (i + 2 < n) z -= q->u2[i] * y[i + 2];
        y[i] = z / q->u0[i];
    }
}

static int penta_setup(penta *q, int64_t n, double rho)
{
    q->n = n;
    q->rho = rho;
    q->l1 = (double *)calloc(n, sizeof(double));
    q->l2 = (double *)calloc(n, sizeof(double));
    q->u0 = (double *)calloc(n, sizeof(double));
    q->u1 = (double *)calloc(n, sizeof(double));
    q->u2 = (double *)calloc(n, sizeof(double));
    q->Z = (double *)calloc(4 * n, sizeof(double));
    if (!q->l1 || !q->l2 || !q->u0 || !q->u1 || !q->u2 || !q->Z) return -1;

    /* Band LU of B (symmetric positive definite, so no pivoting).  Row i of B
     * holds rho, -4rho, 1+6rho, -4rho, rho at columns i-2..i+2. */
    double a0 = 1.0 + 6.0 * rho, a1 = -4.0 * rho, a2 = rho;
    for (int64_t i = 0; i < n; i++) {
        /* entries of row i before elimination */
        double b_im2 = (i >= 2) ? a2 : 0.0; /* column i-2 */
        double b_im1 = (i >= 1) ? a1 : 0.0; /* column i-1 */
        double d = a0, s1 = (i + 1 < n) ? a1 : 0.0, s2 = (i + 2 < n) ? a2 : 0.0;
        /* eliminate column i-2 with pivot row i-2 */
        if (i >= 2) {
            double m = b_im2 / q->u0[i - 2];
            q->l2[i] = m;
            b_im1 -= m * q->u1[i - 2];
            d -= m * q->u2[i - 2];
        }
        /* eliminate column i-1 with pivot row i-1 */
        if (i >= 1) {
            double m = b_im1 / q->u0[i - 1];
            q->l1[i] = m;
            d -= m * q->u1[i - 1];
            s1 -= m * q->u2[i - 1];
        }
        q->u0[i] = d;
        q->u1[i] = s1;
        q->u2[i] = s2;
    }

    /* corners: A[0][n-2]=rho, A[0][n-1]=-4rho, A[1][n-1]=rho and the mirror */
    int64_t idx[4] = {0, 1, n - 2, n - 1};
    memset(q->Kmat, 0, sizeof(q->Kmat));
    q->Kmat[0 * 4 + 2] = rho;
    q->Kmat[0 * 4 + 3] = -4.0 * rho;
    q->Kmat[1 * 4 + 3] = rho;
    q->Kmat[2 * 4 + 0] = rho;
    q->Kmat[3 * 4 + 0] = -4.0 * rho;
    q->Kmat[3 * 4 + 1] = rho;

    double *e = (double *)calloc(n, sizeof(double));
    if (!e) return -1;
    for (int c = 0; c < 4; c++) {
        memset(e, 0, sizeof(double) * n);
        e[idx[c]] = 1.0;
        band_solve(q, e, q->Z + c * n);
    }
    free(e);

    /* S = I + K P^T Z */
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            double acc = (r == c) ? 1.0 : 0.0;
            for (int k = 0; k < 4; k++) acc += q->Kmat[r * 4 + k] * q->Z[c * n + idx[k]];
            q->Smat[r * 4 + c] = acc;
        }
    /* LU with partial pivoting, 4x4 */
    for (int k = 0; k < 4; k++) {
        int p = k;
        for (int r = k + 1; r < 4; r++)
            if (fabs(q->Smat[r * 4 + k]) > fabs(q->Smat[p * 4 + k])) p = r;
        q->piv[k] = p;
        if (p != k)
            for (int c = 0; c < 4; c++) {
                double t = q->Smat[k * 4 + c];
                q->Smat[k * 4 + c] = q->Smat[p * 4 + c];
                q->Smat[p * 4 + c] = t;
            }
        if (q->Smat[k * 4 + k] == 0.0) return -2;
        for (int r = k + 1; r < 4; r++) {
            double m = q->Smat[r * 4 + k] / q->Smat[k * 4 + k];
            q->Smat[r * 4 + k] = m;
            for (int c = k + 1; c < 4; c++) q->Smat[r * 4 + c] -= m * q->Smat[k * 4 + c];
        }
    }
    return 0;
}

static void penta_free(penta *q)
{
    free(q->l1);
    free(q->l2);
    free(q->u0);
    free(q->u1);
    free(q->u2);
    free(q->Z);
}

/* y = A^{-1} f by the Woodbury formula: A = B + P K P^T, so
 * A^{-1} f = B^{-1} f - Z (I + K P^T Z)^{-1} K P^T B^{-1} f with Z = B^{-1} P.
 * tmp has room for n doubles; y must not alias f. */
static void woodbury(const penta *q, const double *f, double *y, double *tmp)
{
    int64_t n = q->n;
    int64_t idx[4] = {0, 1, n - 2, n - 1};
    band_solve(q, f, tmp); /* tmp = B^{-1} f */
    double t[4];
    for (int r = 0; r < 4; r++) {
        double acc = 0.0;
        for (int k = 0; k < 4; k++) acc += q->Kmat[r * 4 + k] * tmp[idx[k]];
        t[r] = acc;
    }
    /* solve S s = t with the stored LU */
    for (int k = 0; k < 4; k++) {
        int p = q->piv[k];
        if (p != k) {
            double x = t[k];
            t[k] = t[p];
            t[p] = x;
        }
    }
    for (int r = 1; r < 4; r++)
        for (int k = 0; k < r; k++) t[r] -= q->Smat[r * 4 + k] * t[k];
    for (int r = 3; r >= 0; r--) {
        for (int k = r + 1; k < 4; k++) t[r] -= q->Smat[r * 4 + k] * t[k];
        t[r] /= q->Smat[r * 4 + r];
    }
    for (int64_t i = 0; i < n; i++)
        y[i] = tmp[i] - (q->Z[0 * n + i] * t[0] + q->Z[1 * n + i] * t[1] + q->Z[2 * n + i] * t[2] +
                         q->Z[3 * n + i] * t[3]);
}

/* y = A^{-1} f, y may alias f; work has room for 3n doubles.
 * A maps constants to themselves (A 1 = 1: the line solve conserves the
 * mean), so the mean of f passes through exactly and only the fluctuation
 * g = f - mean(f) goes through Woodbury, followed by one step of residual
 * correction with the exact stencil (the Woodbury formula on the non-periodic
 * band loses a few digits to cancellation when rho is large). */
static void penta_solve(const penta *q, const double *f, double *y, double *work)
{
    int64_t n = q->n;
    double rho = q->rho;
    double *g = work, *d = work + n, *tmp = work + 2 * n;
    double mean = orc_exact_sum(f, n) / (double)n;
    for (int64_t i = 0; i < n; i++) g[i] = f[i] - mean;
    woodbury(q, g, d, tmp); /* d = A^{-1} g (first pass) */
    for (int64_t i = 0; i < n; i++) {
        int64_t im2 = (i - 2 + n) % n, im1 = (i - 1 + n) % n;
        int64_t ip1 = (i + 1) % n, ip2 = (i + 2) % n;
        double Ad = d[i] + rho * (d[im2] - 4.0 * d[im1] + 6.0 * d[i] - 4.0 * d[ip1] + d[ip2]);
        g[i] = g[i] - Ad; /* residual */
    }
    woodbury(q, g, y, tmp); /* correction */
    for (int64_t i = 0; i < n; i++) y[i] = mean + (d[i] + y[i]);
}

/* Public single-line solve, for the pins. Returns 0 on success. */
int orc_cyclic_penta_solve(int64_t n, double rho, const double *f, double *y)
{
    if (n < 5) return -1;
    penta q;
    if (penta_setup(&q, n, rho) != 0) {
        penta_free(&q);
        return -2;
    }
    double *work = (double *)malloc(sizeof(double) * 3 * n);
    penta_solve(&q, f, y, work);
    free(work);
    penta_free(&q);
    return 0;
}

/* solve (I + theta gamma dt D_d^2) on every d-line of u, in place */
static int sweep(const grid *g, int d, double gamma, double dt, double theta, double *u)
{
    double h2 = g->h[d] * g->h[d];
    double rho = theta * gamma * dt / (h2 * h2);
    penta q;
    if (penta_setup(&q, g->n[d], rho) != 0) {
        penta_free(&q);
        return -2;
    }
    int64_t n = g->n[d], st = g->stride[d];
    int64_t nlines = g->S / n;
    int64_t lo = st, hi = g->n[d] * st; /* line start = (s % lo) + (s / lo) * hi */
#pragma omp parallel
    {
        double *line = (double *)malloc(sizeof(double) * n);
        double *tmp = (double *)malloc(sizeof(double) * 3 * n);
#pragma omp for schedule(static)
        for (int64_t l = 0; l < nlines; l++) {
            int64_t base = (l % lo) + (l / lo) * hi;
            for (int64_t i = 0; i < n; i++) line[i] = u[base + i * st];
            penta_solve(&q, line, line, tmp);
            for (int64_t i = 0; i < n; i++) u[base + i * st] = line[i];
        }
        free(line);
        free(tmp);
    }
    penta_free(&q);
    return 0;
}

/* u <- (I - c gamma dt D_d^2) u along axis d (explicit half of the
   Crank-Nicolson factor), D_d^2 = [1, -4, 6, -4, 1] / h^4 */
static void apply_explicit(const grid *g, int d, double c, double gamma, double dt, double *u)
{
    double h2 = g->h[d] * g->h[d];
    double r = c * gamma * dt / (h2 * h2);
    double *v = (double *)malloc(sizeof(double) * g->S);
    memcpy(v, u, sizeof(double) * g->S);
    for (int64_t s = 0; s < g->S; s++) {
        double d4 = v[nb(g, s, d, -2)] - 4.0 * v[nb(g, s, d, -1)] + 6.0 * v[s] - 4.0 * v[nb(g, s, d, 1)] +
                    v[nb(g, s, d, 2)];
        u[s] = v[s] - r * d4;
    }
    free(v);
}

/* ------------------------------------------------------------------ */
/* One member's state and the time step                                 */
/* ------------------------------------------------------------------ */
/* RHS = C + dt lap_h(C^3 - C) - 2 gamma dt sum_{d<e} D_d D_e C */
void orc_rhs(int dim, const int32_t *n, const double *L, double gamma, double dt,
             const double *C, double *out)
{
    grid g;
    grid_make(&g, dim, n, L);
    double *N = (double *)malloc(sizeof(double) * g.S);
    double *lapN = (double *)malloc(sizeof(double) * g.S);
    double *X = (double *)malloc(sizeof(double) * g.S);
    for (int64_t s = 0; s < g.S; s++) N[s] = C[s] * C[s] * C[s] - C[s];
    orc_laplacian(dim, n, L, N, lapN);
    orc_cross(dim, n, L, C, X);
    for (int64_t s = 0; s < g.S; s++) out[s] = C[s] + dt * lapN[s] - 2.0 * gamma * dt * X[s];
    free(N);
    free(lapN);
    free(X);
}

/* advance C by nsteps steps of the theta-weighted ADI scheme
 *   prod_d (I + theta gamma dt D_d^2) C^{n+1}
 *       = prod_d (I - (1-theta) gamma dt D_d^2) C^n + dt lap_h(C^3 - C) - 2 gamma dt sum_{d<e} D_d D_e C^n
 * theta = 1: the implicit (backward Euler) ADI step; theta = 1/2: the
 * Crank-Nicolson ADI step.  Returns 0 on success. */
int orc_step_theta(int dim, const int32_t *n, const double *L, double gamma, double dt, double theta,
                   double *C, int64_t nsteps)
{
    grid g;
    grid_make(&g, dim, n, L);
    double *w = (double *)malloc(sizeof(double) * g.S);
    double *e = (double *)malloc(sizeof(double) * g.S);
    if (!w || !e) {
        free(w);
        free(e);
        return -1;
    }
    for (int64_t k = 0; k < nsteps; k++) {
        orc_rhs(dim, n, L, gamma, dt, C, w); /* C + explicit terms */
        if (theta != 1.0) {
            /* replace the leading C by prod_d (I - (1-theta) gamma dt D_d^2) C */
            memcpy(e, C, sizeof(double) * g.S);
            for (int d = 0; d < dim; d++) apply_explicit(&g, d, 1.0 - theta, gamma, dt, e);
            for (int64_t s = 0; s < g.S; s++) w[s] = e[s] + (w[s] - C[s]);
        }
        for (int d = 0; d < dim; d++)
            if (sweep(&g, d, gamma, dt, theta, w) != 0) {
                free(w);
                free(e);
                return -2;
            }
        memcpy(C, w, sizeof(double) * g.S);
    }
    free(w);
    free(e);
    return 0;
}

/* advance C by nsteps steps of the implicit ADI scheme (theta = 1) */
int orc_step(int dim, const int32_t *n, const double *L, double gamma, double dt, double *C,
             int64_t nsteps)
{
    return orc_step_theta(dim, n, L, gamma, dt, 1.0, C, nsteps);
}

/* ------------------------------------------------------------------ */
/* Diagnostics                                                          */
/* ------------------------------------------------------------------ */
/* conv = 0: bulk energy (C^2-1)^2/4 ; conv = 1: (C^2-1)^2/2 as printed */
double orc_energy(int dim, const int32_t *n, const double *L, double gamma, int conv,
                  const double *C)
{
    grid g;
    grid_make(&g, dim, n, L);
    double cb = conv ? 0.5 : 0.25;
    xsum acc;
    xsum_init(&acc);
    for (int64_t s = 0; s < g.S; s++) {
        double q = C[s] * C[s] - 1.0;
        double grad2 = 0.0;
        for (int d = 0; d < dim; d++) {
            double gd = (C[nb(&g, s, d, +1)] - C[s]) / g.h[d];
            grad2 += gd * gd;
        }
        xsum_add(&acc, cb * q * q + 0.5 * gamma * grad2);
    }
    double vol = g.h[0] * g.h[1] * g.h[2];
    return vol * xsum_result(&acc);
}

double orc_mean(int dim, const int32_t *n, const double *C)
{
    int64_t S = nsites(dim, n);
    return orc_exact_sum(C, S) / (double)S;
}

/* identity dF/dt = -prod(h) sum |grad+ mu|^2, mu = C^3 - C - gamma lap_h C */
double orc_dFdt_identity(int dim, const int32_t *n, const double *L, double gamma,
                         const double *C)
{
    grid g;
    grid_make(&g, dim, n, L);
    double *lap = (double *)malloc(sizeof(double) * g.S);
    double *mu = (double *)malloc(sizeof(double) * g.S);
    orc_laplacian(dim, n, L, C, lap);
    for (int64_t s = 0; s < g.S; s++) mu[s] = C[s] * C[s] * C[s] - C[s] - gamma * lap[s];
    xsum acc;
    xsum_init(&acc);
    for (int64_t s = 0; s < g.S; s++) {
        double q = 0.0;
        for (int d = 0; d < dim; d++) {
            double gd = (mu[nb(&g, s, d, +1)] - mu[s]) / g.h[d];
            q += gd * gd;
        }
        xsum_add(&acc, q);
    }
    free(lap);
    free(mu);
    double vol = g.h[0] * g.h[1] * g.h[2];
    return -vol * xsum_result(&acc);
}

/* ------------------------------------------------------------------ */
/* A whole run with the beta series.                                    */
/* Samples are taken at n = jK, j = 0..floor(nsteps/K).  Each sample row  */
/* holds: t, F, G_fd, G_id, beta, <C>.  G_fd is the central difference   */
/* (F^{n+1} - F^{n-1}) / (2 dt); forward at n = 0, backward at n = nsteps.*/
/* C is advanced in place.  Returns the number of samples written, or    */
/* a negative value on error.                                           */
/* ------------------------------------------------------------------ */
int64_t orc_run_series_theta(int dim, const int32_t *n, const double *L, double gamma, double dt,
                             double theta, int conv, int32_t K, int64_t nsteps, double *C, double *out,
                             int64_t cap)
{
    if (K < 1 || nsteps < 0) return -1;
    int64_t J = nsteps / K + 1;
    if (J > cap) return -1;
    double *Fm = (double *)malloc(sizeof(double) * J);
    double *F0 = (double *)malloc(sizeof(double) * J);
    double *Fp = (double *)malloc(sizeof(double) * J);
    for (int64_t j = 0; j < J; j++) Fm[j] = F0[j] = Fp[j] = NAN;
    for (int64_t k = 0; k <= nsteps; k++) {
        /* diagnostics of the state C^k */
        int need = 0;
        if (k % K == 0) need = 1;
        if (k >= 1 && (k - 1) % K == 0) need = 1;
        if ((k + 1) % K == 0) need = 1;
        if (need) {
            double F = orc_energy(dim, n, L, gamma, conv, C);
            if (k % K == 0) {
                int64_t j = k / K;
                F0[j] = F;
                out[j * 6 + 0] = (double)k * dt;
                out[j * 6 + 3] = orc_dFdt_identity(dim, n, L, gamma, C);
                out[j * 6 + 5] = orc_mean(dim, n, C);
            }
            if (k >= 1 && (k - 1) % K == 0) Fp[(k - 1) / K] = F;
            if ((k + 1) % K == 0 && (k + 1) / K < J) Fm[(k + 1) / K] = F;
        }
        if (k < nsteps && orc_step_theta(dim, n, L, gamma, dt, theta, C, 1) != 0) {
            free(Fm);
            free(F0);
            free(Fp);
            return -2;
        }
    }
    for (int64_t j = 0; j < J; j++) {
        int64_t k = j * K;
        double G;
        if (k == 0 && nsteps == 0)
            G = NAN;
        else if (k == 0)
            G = (Fp[j] - F0[j]) / dt;
        else if (k == nsteps)
            G = (F0[j] - Fm[j]) / dt;
        else
            G = (Fp[j] - Fm[j]) / (2.0 * dt);
        out[j * 6 + 1] = F0[j];
        out[j * 6 + 2] = G;
        out[j * 6 + 4] = (k == 0) ? 0.0 : -((double)k * dt) * G / F0[j];
    }
    free(Fm);
    free(F0);
    free(Fp);
    return J;
}

int64_t orc_run_series(int dim, const int32_t *n, const double *L, double gamma, double dt,
                       int conv, int32_t K, int64_t nsteps, double *C, double *out,
                       int64_t cap)
{
    return orc_run_series_theta(dim, n, L, gamma, dt, 1.0, conv, K, nsteps, C, out, cap);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (n >= 1); returns the previous count. */
int orc_set_num_threads(int n)
{
    const int prev = orc_num_threads();
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return prev;
}
