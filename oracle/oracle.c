/*
 * UNO-CG oracle: a plain, slow, FP64 CPU implementation of what the solver
 * computes, written from the paper (Herb & Fritzen, "Accelerating Conjugate
 * Gradient Solvers for Homogenization Problems with Unitary Neural
 * Operators", arXiv 2508.02681).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * Conventions (the paper's discrete field, Sec. 2.1 "Notation"):
 *   - a d-dimensional periodic grid of N_1 x ... x N_d voxels; with periodic
 *     boundary conditions there are n = N_1 ... N_d free nodes (Sec. 3.1);
 *   - fields are stored in C order, last axis contiguous;
 *   - node (i_1,...,i_d) is the lower corner of voxel (i_1,...,i_d); voxel e
 *     owns the nodes e + s (mod N) for s in {0,1}^d;
 *   - voxel edge lengths h_b = L0 / N_b on the domain [-L0/2, L0/2]^d (Sec. 5).
 *
 * Every routine follows the plain definition: element-by-element assembly
 * with 2-point Gauss quadrature per axis (exact for multilinear elements),
 * a recursive mixed-radix DFT, Algorithm 1 of Sec. 3.2 written out, and so
 * on.  No blocking, fusion or reordering beyond the definitions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>

#define ORC_PI 3.14159265358979323846264338327950288

typedef double complex cplx;

#define ORC_MAXD 3

typedef struct {
    int dim;
    int n[ORC_MAXD];
    double h[ORC_MAXD];
} orc_grid;

static orc_grid mk_grid(int dim, const int32_t *n, const double *h)
{
    orc_grid g;
    memset(&g, 0, sizeof g);
    g.dim = dim;
    for (int b = 0; b < ORC_MAXD; ++b) {
        g.n[b] = (b < dim) ? n[b] : 1;
        g.h[b] = (b < dim) ? h[b] : 1.0;
    }
    return g;
}

static int64_t grid_size(const orc_grid *g)
{
    int64_t s = 1;
    for (int b = 0; b < g->dim; ++b) s *= g->n[b];
    return s;
}

/* multi-index -> linear index (C order) */
static int64_t lin(const orc_grid *g, const int *idx)
{
    int64_t l = 0;
    for (int b = 0; b < g->dim; ++b) l = l * g->n[b] + idx[b];
    return l;
}

static void unlin(const orc_grid *g, int64_t l, int *idx)
{
    for (int b = g->dim - 1; b >= 0; --b) {
        idx[b] = (int)(l % g->n[b]);
        l /= g->n[b];
    }
}

static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* ---------------------------------------------------------------------
 * Linear finite elements on a voxel (Sec. 3.1, Sec. 5.1).
 * Local node a <-> s in {0,1}^d with a = sum_b s_b 2^(d-1-b).
 * Shape function N_s(xi) = prod_b (s_b ? xi_b : 1 - xi_b), xi in [0,1]^d.
 * ------------------------------------------------------------------- */

static int local_bit(int dim, int a, int b) { return (a >> (dim - 1 - b)) & 1; }

/* gradient of shape function a at local coordinates xi, physical units */
static void shape_grad(const orc_grid *g, int a, const double *xi, double *grad)
{
    for (int b = 0; b < g->dim; ++b) {
        double v = local_bit(g->dim, a, b) ? 1.0 / g->h[b] : -1.0 / g->h[b];
        for (int c = 0; c < g->dim; ++c) {
            if (c == b) continue;
            v *= local_bit(g->dim, a, c) ? xi[c] : 1.0 - xi[c];
        }
        grad[b] = v;
    }
}

/* 2-point Gauss rule on [0,1]: exact for polynomials of degree <= 3 per axis */
static const double GAUSS_X[2] = {0.5 - 0.28867513459481288225, 0.5 + 0.28867513459481288225};

static int n_gauss(const orc_grid *g) { return 1 << g->dim; }

static double gauss_point(const orc_grid *g, int q, double *xi)
{
    double w = 1.0;
    for (int b = 0; b < g->dim; ++b) {
        xi[b] = GAUSS_X[(q >> b) & 1];
        w *= 0.5 * g->h[b];
    }
    return w;
}

/* unit-conductivity element stiffness K_ab = int_e grad N_a . grad N_b */
void orc_element_matrix(int dim, const int32_t *n, const double *h, double *K)
{
    orc_grid g = mk_grid(dim, n, h);
    int na = 1 << dim;
    memset(K, 0, sizeof(double) * na * na);
    for (int q = 0; q < n_gauss(&g); ++q) {
        double xi[ORC_MAXD], w = gauss_point(&g, q, xi);
        double ga[ORC_MAXD], gb[ORC_MAXD];
        for (int a = 0; a < na; ++a) {
            shape_grad(&g, a, xi, ga);
            for (int bb = 0; bb < na; ++bb) {
                shape_grad(&g, bb, xi, gb);
                double dot = 0.0;
                for (int c = 0; c < dim; ++c) dot += ga[c] * gb[c];
                K[a * na + bb] += w * dot;
            }
        }
    }
}

/* global node index of local node a of voxel e */
static int64_t elem_node(const orc_grid *g, const int *e, int a)
{
    int idx[ORC_MAXD];
    for (int b = 0; b < g->dim; ++b) idx[b] = wrap(e[b] + local_bit(g->dim, a, b), g->n[b]);
    return lin(g, idx);
}

/* y = A(kappa) u by an element loop: gather, multiply, scatter-add (Sec. 3.1,
 * the stiffness matrix of the linear system; matrix-free). */
void orc_fe_apply(int dim, const int32_t *n, const double *h, const double *kappa,
                  const double *u, double *y)
{
    orc_grid g = mk_grid(dim, n, h);
    int na = 1 << dim;
    double K[64];
    orc_element_matrix(dim, n, h, K);
    int64_t nn = grid_size(&g);
    memset(y, 0, sizeof(double) * nn);
    for (int64_t le = 0; le < nn; ++le) {
        int e[ORC_MAXD];
        unlin(&g, le, e);
        int64_t gi[8];
        double ue[8];
        for (int a = 0; a < na; ++a) {
            gi[a] = elem_node(&g, e, a);
            ue[a] = u[gi[a]];
        }
        for (int a = 0; a < na; ++a) {
            double acc = 0.0;
            for (int bb = 0; bb < na; ++bb) acc += K[a * na + bb] * ue[bb];
            y[gi[a]] += kappa[le] * acc;
        }
    }
}

/* diagonal A_ii of the assembled matrix (Jacobi preconditioner, Sec. 3.2),
 * assembled element-wise: every element entry K_ab whose two local nodes are
 * the same global node contributes (on an axis with a single voxel both
 * node layers of an element are one node). */
void orc_jacobi_diag(int dim, const int32_t *n, const double *h, const double *kappa, double *diag)
{
    orc_grid g = mk_grid(dim, n, h);
    int na = 1 << dim;
    double K[64];
    orc_element_matrix(dim, n, h, K);
    int64_t nn = grid_size(&g);
    memset(diag, 0, sizeof(double) * nn);
    for (int64_t le = 0; le < nn; ++le) {
        int e[ORC_MAXD];
        unlin(&g, le, e);
        for (int a = 0; a < na; ++a)
            for (int bb = 0; bb < na; ++bb) {
                int64_t ga = elem_node(&g, e, a);
                if (ga == elem_node(&g, e, bb)) diag[ga] += kappa[le] * K[a * na + bb];
            }
    }
}

/* right-hand side of the fluctuation problem for a macroscopic temperature
 * gradient gbar (decomposition theta = T0 + gbar.x + theta~, Sec. 5.1):
 *   f_a = - int kappa grad N_a . gbar  (Gauss quadrature per element). */
void orc_rhs(int dim, const int32_t *n, const double *h, const double *kappa,
             const double *gbar, double *f)
{
    orc_grid g = mk_grid(dim, n, h);
    int na = 1 << dim;
    int64_t nn = grid_size(&g);
    memset(f, 0, sizeof(double) * nn);
    for (int64_t le = 0; le < nn; ++le) {
        int e[ORC_MAXD];
        unlin(&g, le, e);
        for (int q = 0; q < n_gauss(&g); ++q) {
            double xi[ORC_MAXD], w = gauss_point(&g, q, xi);
            for (int a = 0; a < na; ++a) {
                double ga[ORC_MAXD];
                shape_grad(&g, a, xi, ga);
                double dot = 0.0;
                for (int c = 0; c < dim; ++c) dot += ga[c] * gbar[c];
                f[elem_node(&g, e, a)] -= w * kappa[le] * dot;
            }
        }
    }
}

/* volume averages over the domain of the flux-like quantity
 *   q_i = kappa (gbar + grad theta~)_i          (flux form)
 * returned in out[0..dim-1]; Gauss quadrature per element. */
void orc_flux_average(int dim, const int32_t *n, const double *h, const double *kappa,
                      const double *gbar, const double *theta, double *out)
{
    orc_grid g = mk_grid(dim, n, h);
    int na = 1 << dim;
    int64_t nn = grid_size(&g);
    double vol = 1.0;
    for (int b = 0; b < dim; ++b) vol *= g.n[b] * g.h[b];
    for (int c = 0; c < dim; ++c) out[c] = 0.0;
    for (int64_t le = 0; le < nn; ++le) {
        int e[ORC_MAXD];
        unlin(&g, le, e);
        for (int q = 0; q < n_gauss(&g); ++q) {
            double xi[ORC_MAXD], w = gauss_point(&g, q, xi);
            double grad[ORC_MAXD] = {0, 0, 0};
            for (int a = 0; a < na; ++a) {
                double ga[ORC_MAXD];
                shape_grad(&g, a, xi, ga);
                double ua = theta[elem_node(&g, e, a)];
                for (int c = 0; c < dim; ++c) grad[c] += ga[c] * ua;
            }
            for (int c = 0; c < dim; ++c) out[c] += w * kappa[le] * (gbar[c] + grad[c]);
        }
    }
    for (int c = 0; c < dim; ++c) out[c] /= vol;
}

/* energy form (1/|Omega|) int kappa (g1 + grad t1).(g2 + grad t2) */
double orc_energy_average(int dim, const int32_t *n, const double *h, const double *kappa,
                          const double *g1, const double *t1, const double *g2, const double *t2)
{
    orc_grid g = mk_grid(dim, n, h);
    int na = 1 << dim;
    int64_t nn = grid_size(&g);
    double vol = 1.0, acc = 0.0;
    for (int b = 0; b < dim; ++b) vol *= g.n[b] * g.h[b];
    for (int64_t le = 0; le < nn; ++le) {
        int e[ORC_MAXD];
        unlin(&g, le, e);
        for (int q = 0; q < n_gauss(&g); ++q) {
            double xi[ORC_MAXD], w = gauss_point(&g, q, xi);
            double a1[ORC_MAXD], a2[ORC_MAXD];
            for (int c = 0; c < dim; ++c) { a1[c] = g1[c]; a2[c] = g2[c]; }
            for (int a = 0; a < na; ++a) {
                double ga[ORC_MAXD];
                shape_grad(&g, a, xi, ga);
                int64_t gn = elem_node(&g, e, a);
                for (int c = 0; c < dim; ++c) { a1[c] += ga[c] * t1[gn]; a2[c] += ga[c] * t2[gn]; }
            }
            double dot = 0.0;
            for (int c = 0; c < dim; ++c) dot += a1[c] * a2[c];
            acc += w * kappa[le] * dot;
        }
    }
    return acc / vol;
}

/* Per-element energy density of two load cases,
 *   out[e] = (1/|Omega|) int_e (g1 + grad t1).(g2 + grad t2) dx,
 * i.e. the derivative of the energy form (1/|Omega|) sum_e kappa_e
 * int_e (...).(...) with respect to kappa_e at fixed fields.  At the discrete
 * solutions of the periodic cell problem this is also the total derivative
 * d(g1 . kappa_bar g2)/d kappa_e: the problem is self-adjoint, the solution
 * of load 1 is the adjoint state of load 2, and the terms with the field
 * sensitivities vanish by the Galerkin equations (Sec. 3.1 weak form).
 * Gauss quadrature as in orc_energy_average. */
void orc_energy_density(int dim, const int32_t *n, const double *h, const double *g1, const double *t1,
                        const double *g2, const double *t2, double *out)
{
    orc_grid g = mk_grid(dim, n, h);
    int na = 1 << dim;
    int64_t nn = grid_size(&g);
    double vol = 1.0;
    for (int b = 0; b < dim; ++b) vol *= g.n[b] * g.h[b];
    for (int64_t le = 0; le < nn; ++le) {
        int e[ORC_MAXD];
        unlin(&g, le, e);
        double acc = 0.0;
        for (int q = 0; q < n_gauss(&g); ++q) {
            double xi[ORC_MAXD], w = gauss_point(&g, q, xi);
            double a1[ORC_MAXD], a2[ORC_MAXD];
            for (int c = 0; c < dim; ++c) { a1[c] = g1[c]; a2[c] = g2[c]; }
            for (int a = 0; a < na; ++a) {
                double ga[ORC_MAXD];
                shape_grad(&g, a, xi, ga);
                int64_t gn = elem_node(&g, e, a);
                for (int c = 0; c < dim; ++c) { a1[c] += ga[c] * t1[gn]; a2[c] += ga[c] * t2[gn]; }
            }
            double dot = 0.0;
            for (int c = 0; c < dim; ++c) dot += a1[c] * a2[c];
            acc += w * dot;
        }
        out[le] = acc / vol;
    }
}

/* ---------------------------------------------------------------------
 * Unitary discrete Fourier transform (the unitary transform T of Sec. 4.2.1
 * for periodic boundary conditions).  Recursive mixed-radix decimation in
 * time over the smallest prime factor; a prime length falls back to the
 * O(N^2) definition.  sign = -1 forward, +1 inverse (unnormalised here).
 * ------------------------------------------------------------------- */

static cplx unit_root(int64_t num, int64_t den, int sign)
{
    /* exp(sign * 2 pi i num/den) with exact reduction of num mod den */
    int64_t r = ((num % den) + den) % den;
    double ang = 2.0 * ORC_PI * (double)r / (double)den;
    return cos(ang) + sign * I * sin(ang);
}

static void dft_rec(const cplx *x, int64_t stride, int64_t len, cplx *out, int sign)
{
    if (len == 1) { out[0] = x[0]; return; }
    int64_t p = 0;
    for (int64_t q = 2; q * q <= len; ++q) if (len % q == 0) { p = q; break; }
    if (p == 0) { /* prime length: direct sum */
        for (int64_t k = 0; k < len; ++k) {
            cplx acc = 0;
            for (int64_t j = 0; j < len; ++j) acc += x[j * stride] * unit_root(j * k, len, sign);
            out[k] = acc;
        }
        return;
    }
    int64_t m = len / p;
    cplx *sub = (cplx *)malloc(sizeof(cplx) * len);
    /* sub-transform r holds DFT_m of x[r], x[r+p], x[r+2p], ... */
    for (int64_t r = 0; r < p; ++r) dft_rec(x + r * stride, stride * p, m, sub + r * m, sign);
    for (int64_t k = 0; k < len; ++k) {
        cplx acc = 0;
        for (int64_t r = 0; r < p; ++r) acc += unit_root(r * k, len, sign) * sub[r * m + (k % m)];
        out[k] = acc;
    }
    free(sub);
}

/* in-place unitary DFT along every axis of a complex C-order array */
void orc_fft_nd(int dim, const int32_t *n, double *data_ri, int sign)
{
    cplx *a = (cplx *)data_ri;
    orc_grid g = mk_grid(dim, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    for (int ax = 0; ax < dim; ++ax) {
        int64_t len = g.n[ax], stride = 1;
        for (int b = ax + 1; b < dim; ++b) stride *= g.n[b];
        cplx *line = (cplx *)malloc(sizeof(cplx) * len);
        cplx *res = (cplx *)malloc(sizeof(cplx) * len);
        double scale = 1.0 / sqrt((double)len);
        for (int64_t l = 0; l < nn; ++l) {
            int idx[ORC_MAXD];
            unlin(&g, l, idx);
            if (idx[ax] != 0) continue; /* one line per start point */
            for (int64_t j = 0; j < len; ++j) line[j] = a[l + j * stride];
            dft_rec(line, 1, len, res, sign);
            for (int64_t j = 0; j < len; ++j) a[l + j * stride] = res[j] * scale;
        }
        free(line);
        free(res);
    }
}

/* ---------------------------------------------------------------------
 * UNO preconditioner for periodic problems, c = 1 (Sec. 4.2.1-4.2.3,
 * mode table for periodic BC).
 *   theta[0]            bypass weight  (W = psi(theta^0) = theta0^2)
 *   theta[1..k_max]     weights of the learned modes
 *                       K = [-M..M]^(d-1) x [0..M] \ {0}
 * in lexicographic order of (k_1, ..., k_d) with the zero mode skipped.
 * Readings of the text, stated here because the paper leaves them open:
 *   - the conjugate set is taken as the point reflection -K, so that the
 *     preconditioned residual is real; on the plane k_d = 0 both k and -k
 *     are learned, and the table uses the mean of their two entries (this
 *     is what taking the real part of the inverse transform amounts to);
 *   - the zero mode, which the learned set excludes, carries the value 0,
 *     so the preconditioner shares the constant null space of A.
 * ------------------------------------------------------------------- */

static int centred(int i, int n) { return (2 * i <= n) ? i : i - n; }

int64_t orc_uno_num_weights(int dim, int M)
{
    int64_t w = M + 1;
    for (int b = 0; b < dim - 1; ++b) w *= 2 * M + 1;
    return w; /* (2M+1)^(d-1) (M+1) = 1 + k_max */
}

/* slot of mode k (1..k_max) if k in K, else 0 */
static int64_t learned_slot(int dim, int M, const int *k)
{
    for (int b = 0; b < dim - 1; ++b) if (k[b] < -M || k[b] > M) return 0;
    if (k[dim - 1] < 0 || k[dim - 1] > M) return 0;
    int allzero = 1;
    for (int b = 0; b < dim; ++b) if (k[b] != 0) allzero = 0;
    if (allzero) return 0;
    int64_t L = 0, L0 = 0;
    for (int b = 0; b < dim - 1; ++b) {
        L = L * (2 * M + 1) + (k[b] + M);
        L0 = L0 * (2 * M + 1) + M;
    }
    L = L * (M + 1) + k[dim - 1];
    L0 = L0 * (M + 1);
    return (L < L0) ? L + 1 : L;
}

/* Phi(k) of the paper's parametrization before symmetrization */
static double phi_raw(int dim, int M, const double *theta, const int *k)
{
    int allzero = 1;
    for (int b = 0; b < dim; ++b) if (k[b] != 0) allzero = 0;
    if (allzero) return 0.0;
    double W = theta[0] * theta[0];
    int64_t s = learned_slot(dim, M, k);
    if (s > 0) return W + theta[s] * theta[s];
    int mk[ORC_MAXD];
    for (int b = 0; b < dim; ++b) mk[b] = -k[b];
    s = (k[dim - 1] < 0) ? learned_slot(dim, M, mk) : 0; /* conjugate set */
    if (s > 0) return W + theta[s] * theta[s];
    return W;
}

/* full-spectrum table Phi(k) on the n index points of the DFT grid */
void orc_uno_table(int dim, const int32_t *n, int M, const double *theta, double *table)
{
    orc_grid g = mk_grid(dim, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    for (int64_t l = 0; l < nn; ++l) {
        int idx[ORC_MAXD], k[ORC_MAXD], mk[ORC_MAXD];
        unlin(&g, l, idx);
        for (int b = 0; b < dim; ++b) { k[b] = centred(idx[b], g.n[b]); mk[b] = -k[b]; }
        table[l] = 0.5 * (phi_raw(dim, M, theta, k) + phi_raw(dim, M, theta, mk));
    }
}

/* s = T^H diag(table) T r ; returns max |Im| of the result before discarding */
double orc_table_apply(int dim, const int32_t *n, const double *table, const double *r, double *s)
{
    orc_grid g = mk_grid(dim, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    cplx *a = (cplx *)malloc(sizeof(cplx) * nn);
    for (int64_t l = 0; l < nn; ++l) a[l] = r[l];
    orc_fft_nd(dim, n, (double *)a, -1);
    for (int64_t l = 0; l < nn; ++l) a[l] *= table[l];
    orc_fft_nd(dim, n, (double *)a, +1);
    double im = 0.0;
    for (int64_t l = 0; l < nn; ++l) {
        s[l] = creal(a[l]);
        if (fabs(cimag(a[l])) > im) im = fabs(cimag(a[l]));
    }
    free(a);
    return im;
}

/* FANS preconditioner (Sec. 3.3.4): inverse of the homogeneous reference
 * operator A_ref = kappa_ref A(1) on the Fourier grid, zero on the null
 * space.  The symbol is the DFT of the impulse response A(1) e_0 (A(1) is
 * circulant on the periodic grid). */
void orc_fans_table(int dim, const int32_t *n, const double *h, double kappa_ref, double *table)
{
    orc_grid g = mk_grid(dim, n, h);
    int64_t nn = grid_size(&g);
    double *one = (double *)malloc(sizeof(double) * nn);
    double *e0 = (double *)calloc(nn, sizeof(double));
    double *col = (double *)malloc(sizeof(double) * nn);
    for (int64_t l = 0; l < nn; ++l) one[l] = 1.0;
    e0[0] = 1.0;
    orc_fe_apply(dim, n, h, one, e0, col);
    cplx *a = (cplx *)malloc(sizeof(cplx) * nn);
    for (int64_t l = 0; l < nn; ++l) a[l] = col[l];
    orc_fft_nd(dim, n, (double *)a, -1);
    double sq = sqrt((double)nn);
    for (int64_t l = 0; l < nn; ++l) {
        double lam = creal(a[l]) * sq;
        table[l] = (l == 0) ? 0.0 : 1.0 / (kappa_ref * lam);
    }
    free(one); free(e0); free(col); free(a);
}

/* ---------------------------------------------------------------------
 * Preconditioned conjugate gradients, Algorithm 1 (Sec. 3.2), with the
 * UNO preconditioner as in Algorithm 2 (Sec. 4.2.4).
 *   kind 0: P = I;  1: Jacobi;  2: spectral table (UNO or FANS).
 * The loop runs while ||r||_inf > rtol ||r0||_inf (the relative residual of
 * the experiments, Sec. 6.1); iters counts loop passes.  On exit the mean is
 * removed from u (the fluctuation field has zero mean, Sec. 5.1).
 * res_hist (nullable, max_iter + 1 entries) receives ||r||_inf per pass.
 * ------------------------------------------------------------------- */

static double norm_inf(const double *v, int64_t nn)
{
    double m = 0.0;
    for (int64_t l = 0; l < nn; ++l) if (fabs(v[l]) > m) m = fabs(v[l]);
    return m;
}

static double dot(const double *a, const double *b, int64_t nn)
{
    double s = 0.0;
    for (int64_t l = 0; l < nn; ++l) s += a[l] * b[l];
    return s;
}

int orc_pcg(int dim, const int32_t *n, const double *h, const double *kappa, const double *f,
            double *u, int kind, const double *table, double rtol, int max_iter,
            double *res_hist, double *final_rel)
{
    orc_grid g = mk_grid(dim, n, h);
    int64_t nn = grid_size(&g);
    double *r = (double *)malloc(sizeof(double) * nn);
    double *s = (double *)malloc(sizeof(double) * nn);
    double *d = (double *)calloc(nn, sizeof(double));
    double *p = (double *)malloc(sizeof(double) * nn);
    double *diag = NULL;
    if (kind == 1) {
        diag = (double *)malloc(sizeof(double) * nn);
        orc_jacobi_diag(dim, n, h, kappa, diag);
    }
    /* r = f - A u0 */
    orc_fe_apply(dim, n, h, kappa, u, p);
    for (int64_t l = 0; l < nn; ++l) r[l] = f[l] - p[l];
    double gamma1 = 1.0, gamma0;
    double r0 = norm_inf(r, nn), rn = r0;
    double tol = rtol * r0;
    int it = 0;
    if (res_hist) res_hist[0] = r0;
    while (rn > tol && it < max_iter) {
        if (kind == 0) memcpy(s, r, sizeof(double) * nn);
        else if (kind == 1) for (int64_t l = 0; l < nn; ++l) s[l] = r[l] / diag[l];
        else orc_table_apply(dim, n, table, r, s);
        gamma0 = gamma1;
        gamma1 = dot(r, s, nn);
        for (int64_t l = 0; l < nn; ++l) d[l] = s[l] + (gamma1 / gamma0) * d[l];
        orc_fe_apply(dim, n, h, kappa, d, p);
        double alpha = gamma1 / dot(d, p, nn);
        for (int64_t l = 0; l < nn; ++l) r[l] -= alpha * p[l];
        for (int64_t l = 0; l < nn; ++l) u[l] += alpha * d[l];
        ++it;
        rn = norm_inf(r, nn);
        if (res_hist) res_hist[it] = rn;
    }
    double mean = 0.0;
    for (int64_t l = 0; l < nn; ++l) mean += u[l];
    mean /= (double)nn;
    for (int64_t l = 0; l < nn; ++l) u[l] -= mean;
    if (final_rel) *final_rel = (r0 > 0.0) ? rn / r0 : 0.0;
    free(r); free(s); free(d); free(p); free(diag);
    return it;
}

/* ---------------------------------------------------------------------
 * Second-order training, c = 1 (Sec. 4.4, features of the one-DOF case).
 * Features over the full Fourier grid (hats = unitary T):
 *   alpha_k = (1/Ns) sum_j |f^_j(k)|^2,
 *   beta_k  = (2/Ns) sum_j Re(conj(f^_j(k)) u^_j(k)),
 *   delta   = (1/Ns) sum_j ||u_j||^2.
 * ------------------------------------------------------------------- */
void orc_train_features(int dim, const int32_t *n, int ns, const double *f, const double *u,
                        double *alpha, double *beta, double *delta)
{
    orc_grid g = mk_grid(dim, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    cplx *fh = (cplx *)malloc(sizeof(cplx) * nn);
    cplx *uh = (cplx *)malloc(sizeof(cplx) * nn);
    memset(alpha, 0, sizeof(double) * nn);
    memset(beta, 0, sizeof(double) * nn);
    *delta = 0.0;
    for (int j = 0; j < ns; ++j) {
        for (int64_t l = 0; l < nn; ++l) { fh[l] = f[j * nn + l]; uh[l] = u[j * nn + l]; }
        orc_fft_nd(dim, n, (double *)fh, -1);
        orc_fft_nd(dim, n, (double *)uh, -1);
        for (int64_t l = 0; l < nn; ++l) {
            alpha[l] += creal(conj(fh[l]) * fh[l]) / ns;
            beta[l] += 2.0 * creal(conj(fh[l]) * uh[l]) / ns;
        }
        for (int64_t l = 0; l < nn; ++l) *delta += u[j * nn + l] * u[j * nn + l] / ns;
    }
    free(fh);
    free(uh);
}

/* loss L(theta) = alpha . (Phi o Phi) - beta . Phi + delta */
double orc_train_loss(int dim, const int32_t *n, int M, const double *theta,
                      const double *alpha, const double *beta, double delta)
{
    orc_grid g = mk_grid(dim, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    double *tab = (double *)malloc(sizeof(double) * nn);
    orc_uno_table(dim, n, M, theta, tab);
    double L = delta;
    for (int64_t l = 0; l < nn; ++l) L += alpha[l] * tab[l] * tab[l] - beta[l] * tab[l];
    free(tab);
    return L;
}

/* Exact minimiser of the loss over theta (c = 1).  With a = theta0^2 and
 * b = theta_m^2 >= 0 the table is Phi_k = a + b_g(k) on each group g of modes
 * sharing one learned value (k and -k; on the plane k_d = 0 the two slots of
 * k and -k move together), and Phi_k = a on the remaining modes k != 0.
 * The loss is a sum of convex quadratics in Phi, so per group the optimum is
 * b_g = max(0, c_g - a), c_g = B_g / (2 A_g), and a minimises the convex
 * piecewise quadratic
 *   g(a) = A_u a^2 - B_u a + sum_g [A_g max(a,c_g)^2 - B_g max(a,c_g)],
 * found by scanning the sorted breakpoints.  Returns theta (both slots of a
 * k_d = 0 pair get the same value). */
typedef struct { double c, A, B; } orc_grp;

static int cmp_grp(const void *x, const void *y)
{
    double a = ((const orc_grp *)x)->c, b = ((const orc_grp *)y)->c;
    return (a < b) ? -1 : (a > b) ? 1 : 0;
}

void orc_train_closed_form(int dim, const int32_t *n, int M, const double *alpha,
                           const double *beta, double *theta)
{
    orc_grid g = mk_grid(dim, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    int64_t nw = orc_uno_num_weights(dim, M);
    /* accumulate A, B per slot; a k_d = 0 pair is keyed by its smaller slot */
    double *As = (double *)calloc(nw, sizeof(double));
    double *Bs = (double *)calloc(nw, sizeof(double));
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * nw);
    for (int64_t s = 0; s < nw; ++s) key[s] = s;
    double Au = 0.0, Bu = 0.0;
    for (int64_t l = 1; l < nn; ++l) {
        int idx[ORC_MAXD], k[ORC_MAXD], mk[ORC_MAXD];
        unlin(&g, l, idx);
        for (int b = 0; b < dim; ++b) { k[b] = centred(idx[b], g.n[b]); mk[b] = -k[b]; }
        int64_t s1 = learned_slot(dim, M, k), s2 = learned_slot(dim, M, mk);
        if (s1 == 0 && k[dim - 1] < 0) s1 = s2; /* conjugate mode */
        if (s2 == 0 && mk[dim - 1] < 0) s2 = s1;
        if (s1 == 0 && s2 == 0) { Au += alpha[l]; Bu += beta[l]; continue; }
        int64_t gkey = (s1 < s2) ? s1 : s2;
        key[s1] = gkey;
        key[s2] = gkey;
        As[gkey] += alpha[l];
        Bs[gkey] += beta[l];
    }
    int64_t ng = 0;
    orc_grp *grp = (orc_grp *)malloc(sizeof(orc_grp) * nw);
    for (int64_t s = 1; s < nw; ++s) {
        if (key[s] != s) continue;
        grp[ng].A = As[s];
        grp[ng].B = Bs[s];
        grp[ng].c = (As[s] > 0.0) ? Bs[s] / (2.0 * As[s]) : -INFINITY;
        ++ng;
    }
    qsort(grp, ng, sizeof(orc_grp), cmp_grp);
    /* g'(a) = 2 (Au + sum_{c_g < a} A_g) a - (Bu + sum_{c_g < a} B_g) */
    double SA = Au, SB = Bu, a = 0.0;
    int64_t i = 0;
    while (i < ng && grp[i].c <= 0.0) { SA += grp[i].A; SB += grp[i].B; ++i; }
    for (;;) {
        double cand = (SA > 0.0) ? SB / (2.0 * SA) : 0.0;
        if (cand < 0.0) cand = 0.0;
        double hi = (i < ng) ? grp[i].c : INFINITY;
        if (cand <= hi) { a = cand; break; }
        SA += grp[i].A;
        SB += grp[i].B;
        ++i;
    }
    theta[0] = sqrt(a);
    for (int64_t s = 1; s < nw; ++s) {
        int64_t gk = key[s];
        double c = (As[gk] > 0.0) ? Bs[gk] / (2.0 * As[gk]) : -INFINITY;
        double b = c - a;
        theta[s] = (b > 0.0) ? sqrt(b) : 0.0;
    }
    free(As); free(Bs); free(key); free(grp);
}

/* =====================================================================
 * Linear elasticity, d = 3, c = 3 (Sec. 5.2): displacement fluctuation u
 * with three components stored planar (u[c * n + node]); strain and stress
 * in the Mandel basis (App. A: e1 e1, e2 e2, e3 e3, sqrt2 sym(e1 e2),
 * sqrt2 sym(e1 e3), sqrt2 sym(e2 e3)); isotropic stiffness
 * D = 3 lambda P1 + 2 mu I_sym, i.e. in Mandel form lambda 1 1^T on the
 * normal block plus 2 mu I6.  Trilinear hex8 elements, 2-point Gauss rule
 * per axis (exact), periodic grid.
 * ===================================================================== */

static const double ORC_SQ2 = 1.41421356237309504880;

/* Mandel strain rows of the B matrix for corner a at point xi: strain =
 * sum_a B_a u_a, B_a[k][c] (k Mandel index, c displacement component) */
static void el_bmat(const orc_grid *g, int a, const double *xi, double B[6][3])
{
    double gr[3];
    shape_grad(g, a, xi, gr);
    memset(B, 0, sizeof(double) * 18);
    B[0][0] = gr[0];
    B[1][1] = gr[1];
    B[2][2] = gr[2];
    B[3][0] = gr[1] / ORC_SQ2; B[3][1] = gr[0] / ORC_SQ2;
    B[4][0] = gr[2] / ORC_SQ2; B[4][2] = gr[0] / ORC_SQ2;
    B[5][1] = gr[2] / ORC_SQ2; B[5][2] = gr[1] / ORC_SQ2;
}

static void el_dmat(double lam, double mu, double D[6][6])
{
    memset(D, 0, sizeof(double) * 36);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) D[i][j] = lam;
    for (int i = 0; i < 6; ++i) D[i][i] += 2.0 * mu;
}

/* element stiffness K[(a,c)][(b,e)] = int B_a^T D B_b, 24 x 24, index a*3+c */
void orc_el_element_matrix(const int32_t *n, const double *h, double lam, double mu, double *K)
{
    orc_grid g = mk_grid(3, n, h);
    double D[6][6];
    el_dmat(lam, mu, D);
    memset(K, 0, sizeof(double) * 576);
    for (int q = 0; q < n_gauss(&g); ++q) {
        double xi[3], w = gauss_point(&g, q, xi);
        double B[8][6][3];
        for (int a = 0; a < 8; ++a) el_bmat(&g, a, xi, B[a]);
        for (int a = 0; a < 8; ++a)
            for (int c = 0; c < 3; ++c)
                for (int b = 0; b < 8; ++b)
                    for (int e = 0; e < 3; ++e) {
                        double v = 0.0;
                        for (int k = 0; k < 6; ++k)
                            for (int l = 0; l < 6; ++l) v += B[a][k][c] * D[k][l] * B[b][l][e];
                        K[(a * 3 + c) * 24 + b * 3 + e] += w * v;
                    }
    }
}

/* y = A(lambda, mu) u by the element loop */
void orc_el_apply(const int32_t *n, const double *h, const double *lam, const double *mu, const double *u,
                  double *y)
{
    orc_grid g = mk_grid(3, n, h);
    int64_t nn = grid_size(&g);
    double K1[576], K2[576];
    orc_el_element_matrix(n, h, 1.0, 0.0, K1); /* lambda part */
    orc_el_element_matrix(n, h, 0.0, 1.0, K2); /* mu part */
    memset(y, 0, sizeof(double) * 3 * nn);
    for (int64_t le = 0; le < nn; ++le) {
        int e[3];
        unlin(&g, le, e);
        int64_t nd[8];
        for (int a = 0; a < 8; ++a) nd[a] = elem_node(&g, e, a);
        for (int a = 0; a < 8; ++a)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int b = 0; b < 8; ++b)
                    for (int f = 0; f < 3; ++f) {
                        int ij = (a * 3 + c) * 24 + b * 3 + f;
                        acc += (lam[le] * K1[ij] + mu[le] * K2[ij]) * u[f * nn + nd[b]];
                    }
                y[c * nn + nd[a]] += acc;
            }
    }
}

/* assembled diagonal (3 per node) */
void orc_el_diag(const int32_t *n, const double *h, const double *lam, const double *mu, double *dg)
{
    orc_grid g = mk_grid(3, n, h);
    int64_t nn = grid_size(&g);
    double K1[576], K2[576];
    orc_el_element_matrix(n, h, 1.0, 0.0, K1);
    orc_el_element_matrix(n, h, 0.0, 1.0, K2);
    memset(dg, 0, sizeof(double) * 3 * nn);
    for (int64_t le = 0; le < nn; ++le) {
        int e[3];
        unlin(&g, le, e);
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) {
                if (elem_node(&g, e, a) != elem_node(&g, e, b)) continue; /* coinciding nodes on 1-voxel axes */
                for (int c = 0; c < 3; ++c) {
                    int ij = (a * 3 + c) * 24 + b * 3 + c;
                    dg[c * nn + elem_node(&g, e, a)] += lam[le] * K1[ij] + mu[le] * K2[ij];
                }
            }
    }
}

/* f = -sum_e int B^T D eps_bar (macroscopic Mandel strain eps_bar) */
void orc_el_rhs(const int32_t *n, const double *h, const double *lam, const double *mu, const double *eps,
                double *f)
{
    orc_grid g = mk_grid(3, n, h);
    int64_t nn = grid_size(&g);
    memset(f, 0, sizeof(double) * 3 * nn);
    for (int64_t le = 0; le < nn; ++le) {
        int e[3];
        unlin(&g, le, e);
        double D[6][6], sig[6];
        el_dmat(lam[le], mu[le], D);
        for (int k = 0; k < 6; ++k) {
            sig[k] = 0.0;
            for (int l = 0; l < 6; ++l) sig[k] += D[k][l] * eps[l];
        }
        for (int q = 0; q < n_gauss(&g); ++q) {
            double xi[3], w = gauss_point(&g, q, xi);
            for (int a = 0; a < 8; ++a) {
                double B[6][3];
                el_bmat(&g, a, xi, B);
                for (int c = 0; c < 3; ++c) {
                    double v = 0.0;
                    for (int k = 0; k < 6; ++k) v += B[k][c] * sig[k];
                    f[c * nn + elem_node(&g, e, a)] -= w * v;
                }
            }
        }
    }
}

/* volume average of the Mandel stress D (eps_bar + B u) */
void orc_el_stress_average(const int32_t *n, const double *h, const double *lam, const double *mu,
                           const double *eps, const double *u, double *out)
{
    orc_grid g = mk_grid(3, n, h);
    int64_t nn = grid_size(&g);
    double vol = 1.0;
    for (int b = 0; b < 3; ++b) vol *= g.n[b] * g.h[b];
    for (int k = 0; k < 6; ++k) out[k] = 0.0;
    for (int64_t le = 0; le < nn; ++le) {
        int e[3];
        unlin(&g, le, e);
        double D[6][6];
        el_dmat(lam[le], mu[le], D);
        for (int q = 0; q < n_gauss(&g); ++q) {
            double xi[3], w = gauss_point(&g, q, xi);
            double st[6];
            for (int k = 0; k < 6; ++k) st[k] = eps[k];
            for (int a = 0; a < 8; ++a) {
                double B[6][3];
                el_bmat(&g, a, xi, B);
                int64_t nd = elem_node(&g, e, a);
                for (int k = 0; k < 6; ++k)
                    for (int c = 0; c < 3; ++c) st[k] += B[k][c] * u[c * nn + nd];
            }
            for (int k = 0; k < 6; ++k) {
                double v = 0.0;
                for (int l = 0; l < 6; ++l) v += D[k][l] * st[l];
                out[k] += w * v;
            }
        }
    }
    for (int k = 0; k < 6; ++k) out[k] /= vol;
}

/* Algorithm 1 for the elastic operator: P = none (kind 0) or Jacobi (1);
 * relative infinity-norm stop as in orc_pcg; componentwise mean removal at
 * the end.  Returns the loop passes. */
double orc_uno3_apply(const int32_t *n, const double *table, const double *r, double *s);

/* kind: 0 none, 1 Jacobi, 2 UNO table of orc_uno3_table */
int orc_el_pcg(const int32_t *n, const double *h, const double *lam, const double *mu, const double *f, double *u,
               int kind, const double *table, double rtol, int max_iter)
{
    orc_grid g = mk_grid(3, n, h);
    int64_t nn = grid_size(&g), N = 3 * nn;
    double *r = (double *)malloc(sizeof(double) * N), *s = (double *)malloc(sizeof(double) * N);
    double *d = (double *)calloc(N, sizeof(double)), *p = (double *)malloc(sizeof(double) * N);
    double *dg = (double *)malloc(sizeof(double) * N);
    orc_el_diag(n, h, lam, mu, dg);
    orc_el_apply(n, h, lam, mu, u, p);
    for (int64_t i = 0; i < N; ++i) r[i] = f[i] - p[i];
    double r0 = 0.0;
    for (int64_t i = 0; i < N; ++i) r0 = fmax(r0, fabs(r[i]));
    double g1 = 1.0;
    int k = 0;
    for (;;) {
        double rm = 0.0;
        for (int64_t i = 0; i < N; ++i) rm = fmax(rm, fabs(r[i]));
        if (!(rm > rtol * r0) || k >= max_iter) break;
        if (kind == 2) orc_uno3_apply(n, table, r, s);
        else
            for (int64_t i = 0; i < N; ++i) s[i] = kind == 1 ? r[i] / dg[i] : r[i];
        double g0 = g1;
        g1 = 0.0;
        for (int64_t i = 0; i < N; ++i) g1 += r[i] * s[i];
        double beta = (k == 0) ? 0.0 : g1 / g0;
        for (int64_t i = 0; i < N; ++i) d[i] = s[i] + beta * d[i];
        orc_el_apply(n, h, lam, mu, d, p);
        double dp = 0.0;
        for (int64_t i = 0; i < N; ++i) dp += d[i] * p[i];
        double alpha = g1 / dp;
        for (int64_t i = 0; i < N; ++i) {
            r[i] -= alpha * p[i];
            u[i] += alpha * d[i];
        }
        ++k;
    }
    for (int c = 0; c < 3; ++c) {
        double m = 0.0;
        for (int64_t i = 0; i < nn; ++i) m += u[c * nn + i];
        m /= (double)nn;
        for (int64_t i = 0; i < nn; ++i) u[c * nn + i] -= m;
    }
    free(r); free(s); free(d); free(p); free(dg);
    return k;
}

/* =====================================================================
 * UNO preconditioner, c = 3 (Sec. 4.2.2: eqs. fnocg-parametrization and
 * fnocg-op-fundsol; App. B: eq. local-param-3 and the band matrix Q).
 *   theta[6 s + m]: weights w_1..w_6 of slot s (s = 0 the bypass, s >= 1
 *   the learned modes K in the order of the c = 1 table).
 *   psi(w) = L L^T with L lower triangular, L_11 = w_1, L_22 = w_2,
 *   L_21 = w_3, L_33 = w_4, L_32 = w_5, L_31 = w_6.
 *   Phi(k) = psi(w^0) + psi(w^s) on a learned mode k (or its conjugate -k)
 *   and psi(w^0) elsewhere; the same readings as for c = 1 (mean over k
 *   and -k, zero mode 0).
 * The table holds the unique blocks of Q per mode, in the paper's order
 *   q1 = Phi_11, q2 = Phi_22, q3 = Phi_12, q4 = Phi_33, q5 = Phi_23,
 *   q6 = Phi_13,
 * planar: table[e n + l] for e = 0..5 (q_(e+1)), l the mode's C-order index.
 * Displacement-like vectors are planar too: component c at [c n + node].
 * ===================================================================== */

static void psi3(const double *w, double q[6])
{
    double L[3][3] = {{w[0], 0.0, 0.0}, {w[2], w[1], 0.0}, {w[5], w[4], w[3]}};
    double P[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            P[i][j] = 0.0;
            for (int k = 0; k < 3; ++k) P[i][j] += L[i][k] * L[j][k];
        }
    q[0] = P[0][0]; q[1] = P[1][1]; q[2] = P[0][1];
    q[3] = P[2][2]; q[4] = P[1][2]; q[5] = P[0][2];
}

void orc_psi3(const double *w, double *q) { psi3(w, q); }

static void phi3_raw(int M, const double *theta, const int *k, double q[6])
{
    for (int e = 0; e < 6; ++e) q[e] = 0.0;
    if (k[0] == 0 && k[1] == 0 && k[2] == 0) return;
    psi3(theta, q);
    int64_t s = learned_slot(3, M, k);
    if (s == 0 && k[2] < 0) {
        int mk[3] = {-k[0], -k[1], -k[2]};
        s = learned_slot(3, M, mk);
    }
    if (s > 0) {
        double t[6];
        psi3(theta + 6 * s, t);
        for (int e = 0; e < 6; ++e) q[e] += t[e];
    }
}

void orc_uno3_table(const int32_t *n, int M, const double *theta, double *table)
{
    orc_grid g = mk_grid(3, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    for (int64_t l = 0; l < nn; ++l) {
        int idx[3], k[3], mk[3];
        unlin(&g, l, idx);
        for (int b = 0; b < 3; ++b) { k[b] = centred(idx[b], g.n[b]); mk[b] = -k[b]; }
        double a[6], b6[6];
        phi3_raw(M, theta, k, a);
        phi3_raw(M, theta, mk, b6);
        for (int e = 0; e < 6; ++e) table[e * nn + l] = 0.5 * (a[e] + b6[e]);
    }
}

/* s_i = T^H (sum_j Phi_ij o T r_j) (eq. fnocg-op-fundsol), T the unitary
 * DFT of each component; returns max |Im| before it is discarded */
double orc_uno3_apply(const int32_t *n, const double *table, const double *r, double *s)
{
    orc_grid g = mk_grid(3, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    cplx *a = (cplx *)malloc(sizeof(cplx) * 3 * nn);
    cplx *b = (cplx *)malloc(sizeof(cplx) * 3 * nn);
    for (int64_t i = 0; i < 3 * nn; ++i) a[i] = r[i];
    for (int c = 0; c < 3; ++c) orc_fft_nd(3, n, (double *)(a + c * nn), -1);
    static const int qi[3][3] = {{0, 2, 5}, {2, 1, 4}, {5, 4, 3}};
    for (int64_t l = 0; l < nn; ++l)
        for (int i = 0; i < 3; ++i) {
            cplx v = 0.0;
            for (int j = 0; j < 3; ++j) v += table[qi[i][j] * nn + l] * a[j * nn + l];
            b[i * nn + l] = v;
        }
    for (int c = 0; c < 3; ++c) orc_fft_nd(3, n, (double *)(b + c * nn), +1);
    double im = 0.0;
    for (int64_t i = 0; i < 3 * nn; ++i) {
        s[i] = creal(b[i]);
        if (fabs(cimag(b[i])) > im) im = fabs(cimag(b[i]));
    }
    free(a);
    free(b);
    return im;
}

/* ---------------------------------------------------------------------
 * Second-order training, c = 3 (Sec. 4.4 with App. B).  Features over the
 * full Fourier grid (hats = unitary T, x/y/z = components 1/2/3):
 *   alpha_1 = <|f^_x|^2>, alpha_2 = <|f^_y|^2>, alpha_4 = <|f^_z|^2>,
 *   alpha_3 = <2 Re(conj f^_x f^_y)>, alpha_5 = <2 Re(conj f^_y f^_z)>,
 *   alpha_6 = <2 Re(conj f^_x f^_z)>,
 *   beta_1 = <2 Re(conj f^_x u^_x)>, beta_2 = <2 Re(conj f^_y u^_y)>,
 *   beta_4 = <2 Re(conj f^_z u^_z)>,
 *   beta_3 = <2 Re(conj f^_x u^_y + conj f^_y u^_x)>,
 *   beta_5 = <2 Re(conj f^_y u^_z + conj f^_z u^_y)>,
 *   beta_6 = <2 Re(conj f^_x u^_z + conj f^_z u^_x)>,
 *   delta = <||u||^2>,  <.> the mean over the ns samples.
 * (For real f the products conj(f^_x) f^_y + conj(f^_y) f^_x are real.)
 * alpha, beta planar: [e n + l], e = 0..5 for index e + 1.
 * ------------------------------------------------------------------- */
void orc_train3_features(const int32_t *n, int ns, const double *f, const double *u, double *alpha, double *beta,
                         double *delta)
{
    orc_grid g = mk_grid(3, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    cplx *fh = (cplx *)malloc(sizeof(cplx) * 3 * nn);
    cplx *uh = (cplx *)malloc(sizeof(cplx) * 3 * nn);
    memset(alpha, 0, sizeof(double) * 6 * nn);
    memset(beta, 0, sizeof(double) * 6 * nn);
    *delta = 0.0;
    for (int j = 0; j < ns; ++j) {
        const double *fj = f + (int64_t)j * 3 * nn, *uj = u + (int64_t)j * 3 * nn;
        for (int64_t i = 0; i < 3 * nn; ++i) { fh[i] = fj[i]; uh[i] = uj[i]; }
        for (int c = 0; c < 3; ++c) {
            orc_fft_nd(3, n, (double *)(fh + c * nn), -1);
            orc_fft_nd(3, n, (double *)(uh + c * nn), -1);
        }
        for (int64_t l = 0; l < nn; ++l) {
            cplx fx = fh[l], fy = fh[nn + l], fz = fh[2 * nn + l];
            cplx ux = uh[l], uy = uh[nn + l], uz = uh[2 * nn + l];
            alpha[0 * nn + l] += creal(conj(fx) * fx) / ns;
            alpha[1 * nn + l] += creal(conj(fy) * fy) / ns;
            alpha[2 * nn + l] += 2.0 * creal(conj(fx) * fy) / ns;
            alpha[3 * nn + l] += creal(conj(fz) * fz) / ns;
            alpha[4 * nn + l] += 2.0 * creal(conj(fy) * fz) / ns;
            alpha[5 * nn + l] += 2.0 * creal(conj(fx) * fz) / ns;
            beta[0 * nn + l] += 2.0 * creal(conj(fx) * ux) / ns;
            beta[1 * nn + l] += 2.0 * creal(conj(fy) * uy) / ns;
            beta[2 * nn + l] += 2.0 * creal(conj(fx) * uy + conj(fy) * ux) / ns;
            beta[3 * nn + l] += 2.0 * creal(conj(fz) * uz) / ns;
            beta[4 * nn + l] += 2.0 * creal(conj(fy) * uz + conj(fz) * uy) / ns;
            beta[5 * nn + l] += 2.0 * creal(conj(fx) * uz + conj(fz) * ux) / ns;
        }
        for (int64_t i = 0; i < 3 * nn; ++i) *delta += uj[i] * uj[i] / ns;
    }
    free(fh);
    free(uh);
}

/* loss per mode from the table entries q (App. B), without delta */
static double loss3_mode(const double *q, const double *a, const double *b)
{
    const double q1 = q[0], q2 = q[1], q3 = q[2], q4 = q[3], q5 = q[4], q6 = q[5];
    return a[0] * (q1 * q1 + q3 * q3 + q6 * q6) + a[1] * (q2 * q2 + q3 * q3 + q5 * q5) +
           a[2] * (q1 * q3 + q2 * q3 + q5 * q6) + a[3] * (q4 * q4 + q5 * q5 + q6 * q6) +
           a[4] * (q2 * q5 + q3 * q6 + q4 * q5) + a[5] * (q1 * q6 + q3 * q5 + q4 * q6) -
           (b[0] * q1 + b[1] * q2 + b[2] * q3 + b[3] * q4 + b[4] * q5 + b[5] * q6);
}

/* dL/dq per mode (App. B) */
static void grad3_mode(const double *q, const double *a, const double *b, double g[6])
{
    const double q1 = q[0], q2 = q[1], q3 = q[2], q4 = q[3], q5 = q[4], q6 = q[5];
    g[0] = 2 * a[0] * q1 + a[2] * q3 + a[5] * q6 - b[0];
    g[1] = 2 * a[1] * q2 + a[2] * q3 + a[4] * q5 - b[1];
    g[2] = 2 * a[0] * q3 + 2 * a[1] * q3 + a[2] * (q1 + q2) + a[4] * q6 + a[5] * q5 - b[2];
    g[3] = 2 * a[3] * q4 + a[4] * q5 + a[5] * q6 - b[3];
    g[4] = 2 * a[1] * q5 + a[2] * q6 + 2 * a[3] * q5 + a[4] * (q2 + q4) + a[5] * q3 - b[4];
    g[5] = 2 * a[0] * q6 + a[2] * q5 + 2 * a[3] * q6 + a[4] * q3 + a[5] * (q1 + q4) - b[5];
}

/* d^2 L / dq dq per mode (App. B), 6 x 6 row-major */
static void hess3_mode(const double *a, double H[36])
{
    memset(H, 0, sizeof(double) * 36);
#define HQ(i, j, v) (H[(i - 1) * 6 + (j - 1)] = (v))
    HQ(1, 1, 2 * a[0]); HQ(1, 3, a[2]); HQ(1, 6, a[5]);
    HQ(2, 2, 2 * a[1]); HQ(2, 3, a[2]); HQ(2, 5, a[4]);
    HQ(3, 1, a[2]); HQ(3, 2, a[2]); HQ(3, 3, 2 * (a[0] + a[1])); HQ(3, 5, a[5]); HQ(3, 6, a[4]);
    HQ(4, 4, 2 * a[3]); HQ(4, 5, a[4]); HQ(4, 6, a[5]);
    HQ(5, 2, a[4]); HQ(5, 3, a[5]); HQ(5, 4, a[4]); HQ(5, 5, 2 * (a[1] + a[3])); HQ(5, 6, a[2]);
    HQ(6, 1, a[5]); HQ(6, 3, a[4]); HQ(6, 4, a[5]); HQ(6, 5, a[2]); HQ(6, 6, 2 * (a[0] + a[3]));
#undef HQ
}

/* dpsi/dw: J[e][m] = d q_e / d w_m; d2psi/dw dw: D2[e][m][p] (constant) */
static void psi3_jac(const double *w, double J[6][6])
{
    double Lw[6][3][3];  /* dL/dw_m */
    memset(Lw, 0, sizeof(Lw));
    Lw[0][0][0] = 1; Lw[1][1][1] = 1; Lw[2][1][0] = 1; Lw[3][2][2] = 1; Lw[4][2][1] = 1; Lw[5][2][0] = 1;
    double L[3][3] = {{w[0], 0.0, 0.0}, {w[2], w[1], 0.0}, {w[5], w[4], w[3]}};
    static const int pi[6] = {0, 1, 0, 2, 1, 0}, pj[6] = {0, 1, 1, 2, 2, 2};
    for (int m = 0; m < 6; ++m)
        for (int e = 0; e < 6; ++e) {
            const int i = pi[e], j = pj[e];
            double v = 0.0;  /* d (L L^T)_ij = dL_i . L_j + L_i . dL_j */
            for (int k = 0; k < 3; ++k) v += Lw[m][i][k] * L[j][k] + L[i][k] * Lw[m][j][k];
            J[e][m] = v;
        }
}

static void psi3_hess(double D2[6][6][6])
{
    double Lw[6][3][3];
    memset(Lw, 0, sizeof(Lw));
    Lw[0][0][0] = 1; Lw[1][1][1] = 1; Lw[2][1][0] = 1; Lw[3][2][2] = 1; Lw[4][2][1] = 1; Lw[5][2][0] = 1;
    static const int pi[6] = {0, 1, 0, 2, 1, 0}, pj[6] = {0, 1, 1, 2, 2, 2};
    for (int e = 0; e < 6; ++e)
        for (int m = 0; m < 6; ++m)
            for (int p = 0; p < 6; ++p) {
                const int i = pi[e], j = pj[e];
                double v = 0.0;
                for (int k = 0; k < 3; ++k) v += Lw[m][i][k] * Lw[p][j][k] + Lw[p][i][k] * Lw[m][j][k];
                D2[e][m][p] = v;
            }
}

/* the parameter slots a mode's table entry depends on, with weights:
 * q(k) = psi(w^0) + 1/2 psi(w^s1) + 1/2 psi(w^s2), s1 = slot of k (or of
 * -k through the conjugate set), s2 = the same for -k (0: none) */
static void mode_slots(int M, const int *k, int64_t *s1, int64_t *s2)
{
    int mk[3] = {-k[0], -k[1], -k[2]};
    *s1 = *s2 = 0;
    if (k[0] == 0 && k[1] == 0 && k[2] == 0) return;
    int64_t a = learned_slot(3, M, k);
    if (a == 0 && k[2] < 0) a = learned_slot(3, M, mk);
    int64_t b = learned_slot(3, M, mk);
    if (b == 0 && mk[2] < 0) b = learned_slot(3, M, k);
    *s1 = a;
    *s2 = b;
}

double orc_train3_loss(const int32_t *n, int M, const double *theta, const double *alpha, const double *beta,
                       double delta)
{
    orc_grid g = mk_grid(3, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    double *tab = (double *)malloc(sizeof(double) * 6 * nn);
    orc_uno3_table(n, M, theta, tab);
    double L = delta;
    for (int64_t l = 0; l < nn; ++l) {
        double q[6], a[6], b[6];
        for (int e = 0; e < 6; ++e) { q[e] = tab[e * nn + l]; a[e] = alpha[e * nn + l]; b[e] = beta[e * nn + l]; }
        L += loss3_mode(q, a, b);
    }
    free(tab);
    return L;
}

/* gradient (nw = 6 (k_max + 1)) and dense Hessian (nw x nw, nullable) of
 * the loss with respect to theta, by the chain rule through the table
 * (Sec. 4.4, Newton-Raphson paragraph) */
void orc_train3_grad_hess(const int32_t *n, int M, const double *theta, const double *alpha, const double *beta,
                          double *grad, double *hess)
{
    orc_grid g = mk_grid(3, n, (const double[3]){1, 1, 1});
    int64_t nn = grid_size(&g);
    int64_t nw = 6 * orc_uno_num_weights(3, M);
    double *tab = (double *)malloc(sizeof(double) * 6 * nn);
    orc_uno3_table(n, M, theta, tab);
    memset(grad, 0, sizeof(double) * nw);
    if (hess) memset(hess, 0, sizeof(double) * nw * nw);
    double D2[6][6][6];
    psi3_hess(D2);
    for (int64_t l = 0; l < nn; ++l) {
        int idx[3], k[3];
        unlin(&g, l, idx);
        for (int b = 0; b < 3; ++b) k[b] = centred(idx[b], g.n[b]);
        if (k[0] == 0 && k[1] == 0 && k[2] == 0) continue; /* the zero mode's entry is fixed to 0 */
        double q[6], a[6], b[6], gq[6], Hq[36];
        for (int e = 0; e < 6; ++e) { q[e] = tab[e * nn + l]; a[e] = alpha[e * nn + l]; b[e] = beta[e * nn + l]; }
        grad3_mode(q, a, b, gq);
        hess3_mode(a, Hq);
        int64_t s1, s2;
        mode_slots(M, k, &s1, &s2);
        /* dq/dtheta as a list of (slot, weight) blocks */
        int64_t sl[3] = {0, s1, s2};
        double wt[3] = {1.0, 0.5, 0.5};
        int nb = (s1 > 0) ? 3 : 1;
        double J[3][6][6];
        for (int t = 0; t < nb; ++t) {
            psi3_jac(theta + 6 * sl[t], J[t]);
            for (int e = 0; e < 6; ++e)
                for (int m = 0; m < 6; ++m) J[t][e][m] *= wt[t];
        }
        for (int t = 0; t < nb; ++t)
            for (int m = 0; m < 6; ++m) {
                double v = 0.0;
                for (int e = 0; e < 6; ++e) v += gq[e] * J[t][e][m];
                grad[6 * sl[t] + m] += v;
            }
        if (!hess) continue;
        for (int t = 0; t < nb; ++t)
            for (int u = 0; u < nb; ++u)
                for (int m = 0; m < 6; ++m)
                    for (int p = 0; p < 6; ++p) {
                        double v = 0.0;
                        for (int e = 0; e < 6; ++e)
                            for (int f = 0; f < 6; ++f) v += J[t][e][m] * Hq[e * 6 + f] * J[u][f][p];
                        hess[(6 * sl[t] + m) * nw + 6 * sl[u] + p] += v;
                    }
        for (int t = 0; t < nb; ++t)
            for (int m = 0; m < 6; ++m)
                for (int p = 0; p < 6; ++p) {
                    double v = 0.0;
                    for (int e = 0; e < 6; ++e) v += gq[e] * wt[t] * D2[e][m][p];
                    hess[(6 * sl[t] + m) * nw + 6 * sl[t] + p] += v;
                }
    }
    free(tab);
}
