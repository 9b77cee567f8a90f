/*
 * unocg.h -- C ABI of the MI355X (gfx950) UNO-CG hot path.
 *
 * Implements the solver of Herb & Fritzen, "Accelerating Conjugate Gradient
 * Solvers for Homogenization Problems with Unitary Neural Operators"
 * (arXiv 2508.02681): the matrix-free linear finite-element operator of a
 * periodic voxel cell with per-voxel conductivities (Sec. 3.1, Sec. 5.1),
 * the Jacobi preconditioner (Sec. 3.2), the UNO preconditioner
 * s = T^H Q T r with a unitary DFT T and per-mode weights (Sec. 4.2,
 * eq. (fnocg-operator), Algorithm 2), preconditioned CG (Algorithm 1) and the
 * effective conductivity of the cell (Sec. 5.1).
 *
 * Conventions shared by every entry point
 *   Grid      d = 2 or 3; n[0..d-1] voxels per axis; domain [-L0/2, L0/2]^d,
 *             voxel edge h_b = L0 / n[b] (Sec. 5).  Periodic boundary
 *             conditions: n = prod n[b] free nodes (Sec. 3.1).
 *   Layout    every field is a dense C-order array of n values, last axis
 *             contiguous.  Node (i_1..i_d) is the lower corner of voxel
 *             (i_1..i_d); voxel e owns the nodes e + s (mod n) for s in {0,1}^d.
 *   Memory    every array argument is a DEVICE pointer owned by the caller,
 *             except where a comment says "host".  The library never frees
 *             caller memory.
 *   Streams   `stream` is a hipStream_t (NULL = the default stream).  Work is
 *             enqueued on it; calls return before it completes unless stated.
 *   Errors    every call returns a uno_status; on failure nothing has been
 *             written to the outputs unless stated.  uno_status_string()
 *             names a status.
 *   Precision UNO_F64 arrays are double, UNO_F32 arrays are float.
 */
#ifndef UNOCG_H
#define UNOCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    UNO_OK = 0,
    UNO_ERR_ARG = -1,       /* null pointer, bad enum, bad tolerance, ... */
    UNO_ERR_SHAPE = -2,     /* unsupported grid, or weight count mismatch */
    UNO_ERR_NOT_SPD = -3,   /* safety check of Sec. 4.2.4 failed */
    UNO_ERR_BREAKDOWN = -4, /* CG scalar non-finite or non-positive */
    UNO_ERR_DEVICE = -5,    /* a HIP runtime call failed */
    UNO_ERR_NOMEM = -6      /* device allocation failed */
} uno_status;

typedef enum { UNO_F64 = 0, UNO_F32 = 1, UNO_BF16 = 2 } uno_dtype;

typedef struct {
    int32_t dim;   /* 2 or 3 */
    int32_t n[3];  /* voxels per axis; n[2] ignored for dim = 2 */
    double L0;     /* edge of the cubic domain, > 0 */
} uno_grid;

/* Per-voxel conductivity kappa (phase-wise constant and isotropic in the
 * paper, Sec. 5.1), n values, each > 0. dtype UNO_F64 or UNO_F32. */
typedef struct {
    const void *kappa;
    uno_dtype dtype;
} uno_material;

/* Name of a status code (library utility, no passage of the paper). */
const char *uno_status_string(uno_status s);

/* y = A(kappa) u: matrix-free stiffness apply of the periodic linear FE
 * discretization (Sec. 3.1, eq. (fem-linear-system); operator of Sec. 5.1).
 * u, y: n values of dtype vec_t (UNO_F64 or UNO_F32), y must not alias u.
 * material->dtype must equal vec_t. */
uno_status fe_apply(const uno_grid *grid, const uno_material *mat, const void *u, void *y,
                    uno_dtype vec_t, void *stream);

/* s = D^-1 r with D = diag A(kappa): the Jacobi preconditioner (Sec. 3.2).
 * The diagonal is formed from kappa on the fly; same dtypes as fe_apply.
 * s may alias r. */
uno_status jac_precond_apply(const uno_grid *grid, const uno_material *mat, const void *r, void *s,
                             uno_dtype vec_t, void *stream);

/* f = right-hand side of the fluctuation problem for the macroscopic
 * temperature gradient gbar (host, d values): f_i = -int kappa grad N_i . gbar
 * (decomposition of Sec. 5.1, eq. (thermal-decomposition)).  f: n values of
 * dtype vec_t.  sum f = 0 up to rounding. */
uno_status uno_macro_rhs(const uno_grid *grid, const uno_material *mat, const double *gbar, void *f,
                         uno_dtype vec_t, void *stream);

/* ---- UNO preconditioner (Sec. 4.2) ---------------------------------- */
typedef struct uno_precond uno_precond; /* opaque; owns its device table and scratch */

/* Builds Q of eq. (prec-sparse-def) for c = 1 from the weights
 * theta (host, ntheta = (2M+1)^(d-1) (M+1) values):
 *   theta[0]   bypass, W = theta[0]^2                          (psi(t) = t^2)
 *   theta[i]   learned mode i of K = [-M..M]^(d-1) x [0..M] \ {0}, modes in
 *              lexicographic order of (k_1..k_d) with the zero mode skipped;
 *   Phi(k) = W + theta[i]^2 on k in K and on its point reflection -k,
 *            W elsewhere, 0 at k = 0 (the preconditioner shares the constant
 *            null space of A, Sec. 4.2.4 remark); on the plane k_d = 0, where
 *            k and -k are both learned, the mean of the two values is used
 *            so that the output is real.
 * Requires 2M+1 <= n[b] on every axis.  The safety check of Sec. 4.2.4 is
 * run on the host: every Phi(k), k != 0, must exceed eps_spd, else
 * UNO_ERR_NOT_SPD.  table_t (UNO_F64, UNO_F32 or UNO_BF16): precision the
 * table values are rounded to (BF16: 8-bit significand, round to nearest
 * even) before the check; applies compute in the vector precision.
 * Allocates device memory on the current device; synchronous. */
uno_status uno_precond_create(const uno_grid *grid, int32_t M, const double *theta, int64_t ntheta,
                              double eps_spd, uno_dtype table_t, uno_precond **out);

/* FANS reference preconditioner (Sec. 3.3.4, eq. (FANS-prec-fields)) as a
 * UNO table: Phi(k) = 1 / (kappa_ref lambda(k)), lambda the symbol of the
 * homogeneous unit-conductivity operator, 0 at k = 0 (the UNO with this
 * table reproduces FANS, Sec. 4.2.2). */
uno_status uno_precond_create_fans(const uno_grid *grid, double kappa_ref, uno_dtype table_t,
                                   uno_precond **out);

/* s = T^H Q T r (Algorithm 2, preconditioner lines) with T the unitary DFT.
 * r, s: n values of dtype vec_t; s may alias r.  Uses the precond's scratch,
 * so concurrent applies of one precond on different streams race. */
uno_status uno_precond_apply(const uno_precond *p, const void *r, void *s, uno_dtype vec_t, void *stream);

/* Selects how FP64 applies of a UNO preconditioner are computed; both give
 * the same operator (Sec. 4.2.2: modes outside the learned set carry only
 * the bypass).  UNO_PATH_AUTO (default) and UNO_PATH_LEARNED use the
 * learned-mode passes when the preconditioner has them (UNO tables whose
 * learned block is small against the grid): since Phi equals the bypass W
 * outside the learned block, s = W r + T^H ((Phi - W) o T r) needs the
 * transform of r on the learned modes only.  UNO_PATH_SPECTRAL always runs the
 * full transform over the half spectrum.  UNO_PATH_FUSED: the learned-mode
 * passes inside FP64 CG with the last one folded into the operator apply (s
 * evaluated on each operator tile and its halo, r.s by Parseval); three
 * kernels per CG pass instead of four, at about 3x the arithmetic of the
 * last pass (UNO_ERR_SHAPE when the block does not fit the tile's LDS). */
enum { UNO_PATH_AUTO = 0, UNO_PATH_SPECTRAL = 1, UNO_PATH_LEARNED = 2, UNO_PATH_FUSED = 3 };
uno_status uno_precond_set_path(uno_precond *p, int32_t path);

/* Copies the half-spectrum table Phi of eq. (fnocg-parametrization)
 * (n[0] x .. x n[d-2] x (n[d-1]/2+1) values, C order, unscaled) to host
 * memory `out` (host). For inspection. */
uno_status uno_precond_table(const uno_precond *p, double *out, int64_t nout);

/* Releases a preconditioner of uno_precond_create, uno_precond_create_fans
 * or el_uno_precond_create (Sec. 4.2) and its device memory. */
uno_status uno_precond_destroy(uno_precond *p);

/* ---- Preconditioned CG (Algorithm 1 / Algorithm 2) ------------------ */
enum { UNO_PREC_NONE = 0, UNO_PREC_JACOBI = 1, UNO_PREC_UNO = 2 };

typedef struct {
    int32_t kind;            /* UNO_PREC_* */
    const uno_precond *uno;  /* required for UNO_PREC_UNO */
    double rtol;             /* stop when ||r||_inf <= rtol ||r_0||_inf */
    int32_t max_iter;        /* > 0 */
    uno_dtype op_t;          /* operator apply: UNO_F64, or UNO_F32 (with prec_t = UNO_F32) */
    uno_dtype prec_t;        /* preconditioner apply: UNO_F64, or UNO_F32 (with op_t = UNO_F32);
                                FP32 mode keeps r, u, all reductions and the stop test in FP64
                                and needs, for UNO, the learned-mode passes (uno_precond_set_path);
                                it replaces r by f - A u (FP64) whenever ||r||_inf has dropped by
                                1e2 since the last replacement (the search direction continues),
                                and reopens a load whose FP64 true residual is above its
                                tolerance when every load has ended.  UNO_BF16 (with
                                op_t = UNO_F32, UNO-CG with the learned-mode passes of a
                                one-DOF preconditioner): the FP32 mode with the passes' table,
                                row-chunk partials and per-mode coefficients stored in BF16
                                (rounded to nearest even; their arithmetic stays FP64) */
    int32_t graph_chunk;     /* iterations per host check; 0 = adaptive */
    int32_t use_graphs;      /* 1: after the first 8 passes, run the passes as replays of a
                                captured hipGraph of 8 passes (FP64, learned-mode or Jacobi /
                                plain CG; kept per workspace, recaptured when a pointer or the
                                preconditioner changes); results equal the eager launches' */
} uno_solve_opts;

typedef struct {
    int32_t iters;        /* loop passes = preconditioner applies = matvecs */
    int32_t converged;    /* 1 if ||r||_inf <= rtol ||r_0||_inf */
    double rel_res;       /* recurrence residual ||r||_inf / ||r_0||_inf */
    double true_rel_res;  /* ||f - A u||_inf / ||f||_inf recomputed in FP64 */
    double r0_norm;       /* ||r_0||_inf */
} uno_solve_info;

/* Solves A(kappa) u = f for the zero-mean periodic fluctuation by
 * preconditioned CG (Algorithm 1; Jacobi: Sec. 3.2, UNO: Algorithm 2).
 * f is uno_macro_rhs(gbar = macro_load) when macro_load (host, d values) is
 * non-NULL, else `rhs` (device, n doubles).  u (device, n doubles) holds the
 * initial guess on entry and the zero-mean solution on exit.
 * Reductions, the residual recurrence and the stopping test are FP64 in
 * every mode.  Non-convergence within max_iter is not an error (converged =
 * 0); a non-finite or non-positive r.s or d.A d gives UNO_ERR_BREAKDOWN.
 * res_hist (host, nullable, max_iter + 1 doubles) receives ||r||_inf per
 * pass.  Synchronous: returns after the solve has finished on `stream`.
 * The workspace is cached per (device, grid, stream) and released by
 * uno_shutdown(); a solve holds its workspace from start to end, so solves
 * on different streams (from different host threads) run concurrently and
 * solves on one stream take turns. */
uno_status pcg_solve(const uno_grid *grid, const uno_material *mat, const double *macro_load,
                     const double *rhs, double *u, const uno_solve_opts *opts, uno_solve_info *info,
                     double *res_hist, void *stream);

/* nrhs independent solves with one preconditioner: the load cases of one
 * microstructure (Sec. 5.1: one cell problem per unit macroscopic gradient)
 * or of many (Sec. 4.5: batched solution of many problems).  mat->kappa is
 * one conductivity field shared by all loads (kappa_per_rhs = 0) or nrhs
 * fields, field j at + n j (kappa_per_rhs = 1).  Load j is
 * uno_macro_rhs(gbar = macro_loads + d j) of its field (host, nrhs x d) when
 * macro_loads is non-NULL, else rhs + n j (device, nrhs x n doubles).
 * u (device, nrhs x n doubles) holds the initial guesses and receives the
 * zero-mean solutions; info (host, nullable) receives nrhs records.
 * Every pass kernel carries all right-hand sides (grid y), each with its own
 * scalars and stopping test: a load that has converged stops updating.
 * Results equal those of pcg_solve on the same load bitwise when the
 * batch's launch shapes are the single solve's (few loads on small grids);
 * larger batches group the per-workgroup partial sums differently, which
 * changes results by rounding only; in the FP32 mode the residual
 * replacements of all loads happen together, so results agree with
 * pcg_solve to the tolerance.  The spectral passes (FP64) are batched too.
 * 1 <= nrhs <= 256.  Returns UNO_ERR_BREAKDOWN if any load broke down (see
 * info).  Synchronous. */
uno_status pcg_solve_batch(const uno_grid *grid, const uno_material *mat, int32_t kappa_per_rhs, int32_t nrhs,
                           const double *macro_loads, const double *rhs, double *u,
                           const uno_solve_opts *opts, uno_solve_info *info, void *stream);

/* Size of the device array behind pcg_solve_noalloc, per device. */
#define UNO_NOALLOC_SCRATCH_BYTES (24u << 20)

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): pcg_solve
 * (Algorithm 1, as above) with its workspace carved from a device array of
 * the library, UNO_NOALLOC_SCRATCH_BYTES per device, held from the first
 * call on a device until the process ends; the entry point itself is a
 * library utility (no passage of the paper).  Same arguments as pcg_solve,
 * one load, results bitwise those of pcg_solve; it calls no allocation
 * routine.  The workspace (7 FP64 vectors of n values, half a vector more
 * in the FP32 mode, partial sums, 2 (max_iter + 1) history values and the
 * preconditioner's transform scratch) must fit: a 64^3 grid with M = 12 in
 * FP64 fits, 96^3 does not; a problem that does not fit returns
 * UNO_ERR_SHAPE before any work.  Calls on one device share the array and
 * keep the last call's contents: the library serializes them (each returns
 * after its solve has finished), so concurrent callers wait rather than
 * race.  Synchronous. */
uno_status pcg_solve_noalloc(const uno_grid *grid, const uno_material *mat, const double *macro_load,
                             const double *rhs, double *u, const uno_solve_opts *opts, uno_solve_info *info,
                             double *res_hist, void *stream);

/* Autotuner of the operator apply inside CG: a library utility, no passage of the paper.
 * It times every candidate shape of the march kernel -- footprint
 * width tz in {16, 32, 64} nodes along the contiguous axis, rows per thread
 * ry in {1, 2} (ry 256 / tz rows; ry = 2 for tz of 32 and 64) and planes
 * per workgroup xb over the even splits of the first axis -- for
 * nrhs right-hand sides of `grid` in precision dtype (UNO_F64 or UNO_F32)
 * with one conductivity field per right-hand side (kappa_per_rhs = 1) or
 * one shared, on synthetic operands it allocates on `stream`, and records
 * the fastest; later solves with that (grid, nrhs, dtype, kappa_per_rhs) on
 * this device use it (results then differ from the rule's shapes only in
 * the rounding of the d.Ad partial sums).  tz, ry, xb, us (host, nullable)
 * receive the shape and its time per launch in microseconds.  Records are
 * kept until uno_shutdown().  Synchronous. */
uno_status uno_autotune_operator(const uno_grid *grid, int32_t nrhs, int32_t kappa_per_rhs, uno_dtype dtype,
                                 void *stream, int32_t *tz, int32_t *ry, int32_t *xb, double *us);

/* Records a march shape for (grid, nrhs, dtype, kappa_per_rhs) on the
 * current device as uno_autotune_operator would (a library utility,
 * no passage of the paper): to reuse a shape measured earlier, or to pin one.
 * tz in {16, 32, 64}, ry in {1, 2} (ry = 2 with tz of 32 or 64), xb >= 1
 * planes per workgroup (clipped to [2, n0] at launch).  UNO_ERR_ARG for a
 * shape that is not built.  Host only, no device work. */
uno_status uno_set_operator_shape(const uno_grid *grid, int32_t nrhs, int32_t kappa_per_rhs, uno_dtype dtype,
                                  int32_t tz, int32_t ry, int32_t xb);

/* Effective conductivity (Sec. 5.1; the homogenized property handed back to
 * the macro scale, Sec. 1): for load j with gradient g_j (host loads,
 * nload x d) and solution u_j (device, nload x n doubles, C order),
 *   q_j = (1/|Omega|) int kappa (g_j + grad u_j) dx,
 * and out (host, d x d, row-major) = Q G^-1 with Q = [q_1..q_d],
 * G = [g_1..g_d]; nload must equal d and G be invertible.  Synchronous. */
uno_status effective_tensor(const uno_grid *grid, const uno_material *mat, int32_t nload,
                            const double *loads, const double *u, double *out, void *stream);

/* effective_tensor for nmat microstructures of one grid in one call (the
 * batched solves of Sec. 4.5): mat->kappa holds nmat fields (field m at
 * + m n, one dtype), loads (host, nload x d, nload = d) apply to every
 * field, u (device) holds solution j of field m at + (m nload + j) n, and
 * out (host, nmat x d x d) receives tensor m at + m d d.  The flux partials
 * of all fields and loads are read back in one copy; each result equals
 * effective_tensor on its field.  nmat >= 1.  Synchronous. */
uno_status effective_tensor_batch(const uno_grid *grid, const uno_material *mat, int32_t nmat, int32_t nload,
                                  const double *loads, const double *u, double *out, void *stream);

/* Gradient of the effective conductivity with respect to every voxel
 * conductivity.  The cell problem is self-adjoint (Sec. 3.1 weak form), so
 * at the discrete solutions the derivative of g_a . kappa_bar g_b with
 * respect to kappa_e is the element energy density (1/|Omega|) int_e
 * (g_a + grad u_a).(g_b + grad u_b): no adjoint solve.  loads (host,
 * nload x d, nload = d, invertible) and u (device, nload x n doubles) as
 * for effective_tensor.  weights == NULL: out (device, d x d x n doubles)
 * receives d kappa_bar_ij / d kappa_e at out[(i d + j) n + e]; otherwise
 * (host, d x d) out (device, n doubles) receives sum_ij weights_ij
 * d kappa_bar_ij / d kappa_e (a vector-Jacobian product).  Asynchronous. */
uno_status effective_tensor_grad(const uno_grid *grid, int32_t nload, const double *loads, const double *u,
                                 const double *weights, double *out, void *stream);

/* ---- Many problems of uneven sizes (the batched solution of Sec. 4.5 for
 * the many-query setting of Sec. 1) ---------------------------------------- */
/* One problem: its own grid, conductivity field and load cases. */
typedef struct {
    uno_grid grid;
    const double *kappa;        /* device, n doubles (FP64) */
    int32_t nload;              /* load cases, 1..3 */
    const double *loads;        /* host, nload x dim macroscopic gradients */
    double *u;                  /* device, nload x n: initial guesses in, zero-mean solutions out */
    const uno_precond *uno;     /* preconditioner of this grid (opts->kind UNO_PREC_UNO), else ignored */
    uno_solve_info *info;       /* host, nload records, nullable */
} uno_problem;

/* Solves the load cases of nprob independent problems (Algorithm 1 or 2;
 * opts->kind, rtol, max_iter, graph_chunk and the precisions apply to all:
 * FP64, or the FP32 mode of pcg_solve with FP64 residuals, reductions and
 * stop test; opts->uno is ignored in favour of each problem's).  Problems with the same grid and
 * preconditioner form a class; the load cases of a class are carried
 * together by every pass kernel (up to 256 per launch, each with its own
 * conductivity field and stopping test); the classes run concurrently,
 * up to 8 at once, each driven by a host thread of the library on a stream
 * of its own (created once per device, default priority), forked from and
 * joined back into `stream` by events.
 * Results are those of the classes solved one after another.  The library
 * gathers each class's fields into device memory it allocates for the
 * call, and caches the CG workspace per (grid, stream) (held until
 * uno_shutdown).  Returns the first error, or UNO_ERR_BREAKDOWN if any
 * load case broke down (its info says which).  Synchronous. */
uno_status pcg_solve_many(int32_t nprob, const uno_problem *probs, const uno_solve_opts *opts, void *stream);

/* ---- Linear elasticity, d = 3, three nodal DOF (Sec. 5.2) ------------ */
/* Periodic voxel grid (grid->dim = 3, every n >= 2), trilinear hex8
 * elements, isotropic stiffness D = 3 lambda P1 + 2 mu I_sym per voxel
 * (lambda, mu: device, n doubles each, voxel e = lower corner node e).
 * Displacements are planar, component c of node i at u[c n + i] (3n
 * doubles); strains and stresses use the Mandel basis of App. A
 * (e1 e1, e2 e2, e3 e3, sqrt2 sym(e1 e2), sqrt2 sym(e1 e3), sqrt2 sym(e2 e3)).
 *
 * y = A(lambda, mu) u, the assembled stiffness applied matrix-free (Sec.
 * 3.1).  u must not alias y.  Asynchronous. */
uno_status el_apply(const uno_grid *grid, const double *lambda, const double *mu, const double *u, double *y,
                    void *stream);
/* f = -sum_e int_e B^T D eps_bar, the load of the fluctuation problem for
 * the macroscopic Mandel strain eps_bar (host, 6 values), eq.
 * (mechanical-decomposition).  Asynchronous. */
uno_status el_macro_rhs(const uno_grid *grid, const double *lambda, const double *mu, const double *strain,
                        double *f, void *stream);
/* nrhs solves for the macroscopic strains (host, nrhs x 6) carried by every
 * CG pass kernel (Algorithm 1 with P = none, the Jacobi diagonal, or the
 * preconditioner of el_uno_precond_create in opts->uno (Algorithm 2)).
 * Precision: FP64 (op_t = prec_t = UNO_F64), or for UNO-CG the FP32 mode of
 * pcg_solve (op_t = prec_t = UNO_F32: operator, preconditioner and the
 * search direction in FP32, r, u, reductions and the stop test in FP64,
 * residual replacement and exit check by the FP64 operator); Jacobi and
 * plain CG in FP32 give UNO_ERR_ARG.  lame_per_rhs = 0: one (lambda, mu) field pair for all loads;
 * 1: nrhs pairs, pair j at + n j.  u (device, nrhs x 3n) holds the initial
 * guesses and receives the zero-mean fluctuations; info (host, nullable)
 * nrhs records.  1 <= nrhs <= 64.  Synchronous. */
uno_status el_pcg_solve(const uno_grid *grid, const double *lambda, const double *mu, int32_t lame_per_rhs,
                        int32_t nrhs, const double *strains, double *u, const uno_solve_opts *opts,
                        uno_solve_info *info, void *stream);
/* UNO preconditioner for the elastic problem (c = 3): Phi(k) = psi(w^0) +
 * psi(w^s) on the learned modes (and conjugates), psi(w^0) elsewhere, 0 at
 * k = 0 (eqs. fnocg-parametrization, fnocg-op-fundsol), with psi(w) = L L^T
 * of eq. (local-param-3), L = [w1 0 0; w3 w2 0; w6 w5 w4].  theta (host,
 * ntheta = 6 (k_max + 1)): w^s at theta + 6 s, s = 0 the bypass and s >= 1
 * the learned modes in the order of uno_precond_create; the table is the
 * mean over k and -k.  Every 3 x 3 block must have its eigenvalues above
 * eps_spd (the safety check of Sec. 4.2.3), else UNO_ERR_NOT_SPD.  Applied
 * by the learned-mode passes (the block [-M..M]^2 x [0..M] must fit the
 * staging, else UNO_ERR_SHAPE), FP64 only: uno_precond_apply with planar
 * 3n-vectors (r must not alias s), and el_pcg_solve with kind UNO_PREC_UNO.
 * Release with uno_precond_destroy.  Synchronous. */
uno_status el_uno_precond_create(const uno_grid *grid, int32_t M, const double *theta, int64_t ntheta,
                                 double eps_spd, uno_precond **out);
/* Effective stiffness (Sec. 5.2; Mandel basis, App. A) (host out, 6 x 6
 * row-major): column j of
 * S = <D (eps_j + eps(u_j))> for the six loads eps_j (host, 6 x 6, rows)
 * with solutions u (device, 6 x 3n), and out = S L^-T with L the loads as
 * columns (invertible).  Synchronous. */
uno_status el_effective_stiffness(const uno_grid *grid, const double *lambda, const double *mu, int32_t nload,
                                  const double *strains, const double *u, double *out, void *stream);

/* ---- Second-order training of the weights (Sec. 4.4, c = 1) ---------- */
/* Accumulates the features of eq. (features-c-1) over ns samples:
 *   alpha(k) += (1/ns_total) |f^(k)|^2, beta(k) += (2/ns_total) Re(conj(f^) u^)
 * with hats = unitary DFT, on the half spectrum (n[0] x .. x (n[d-1]/2+1)
 * doubles each, device, caller-zeroed before the first call).  f, u: device,
 * ns x n doubles.  Asynchronous. */
uno_status uno_train_accumulate(const uno_grid *grid, int32_t ns, const double *f, const double *u,
                                double ns_total, double *alpha, double *beta, void *stream);

/* Exact minimiser (Sec. 4.4) over theta (host, ntheta values) of the loss
 * L = alpha.(Phi o Phi) - beta.Phi with Phi parametrized as in
 * uno_precond_create; alpha, beta: device half-spectrum features.
 * Synchronous. */
uno_status uno_train_fit(const uno_grid *grid, int32_t M, const double *alpha, const double *beta,
                         double *theta, int64_t ntheta, void *stream);

/* Loss and gradient for a first-order training step of the weights
 * (Algorithm 3, c = 1): with the features alpha, beta (device half
 * spectrum, from uno_train_accumulate over a batch of pairs), loss (host)
 * = sum over the full spectrum of alpha Phi^2 - beta Phi, which is the
 * batch's mean ||P_theta f_j - u_j||^2 less its constant (1/Ns) sum
 * ||u_j||^2 (T unitary), and grad (host, ntheta) = dloss/dtheta with Phi
 * parametrized as in uno_precond_create (the hand-written backward through
 * T: the transform is diagonalized away by Parseval).  Synchronous. */
uno_status uno_train_loss_grad(const uno_grid *grid, int32_t M, const double *alpha, const double *beta,
                               const double *theta, int64_t ntheta, double *loss, double *grad, void *stream);

/* ---- Second-order training for three nodal DOF (App. B) -------------- */
/* Accumulates the twelve features of App. B over ns samples (f, u: device,
 * ns x 3n, planar components): with hats the unitary DFT of each component,
 * alpha_1 += |f^_x|^2 / ns_total, alpha_2 (y), alpha_4 (z),
 * alpha_3 += 2 Re(conj f^_x f^_y) / ns_total, alpha_5 (y, z), alpha_6 (x, z),
 * beta_1 += 2 Re(conj f^_x u^_x) / ns_total, beta_2, beta_4 likewise,
 * beta_3 += 2 Re(conj f^_x u^_y + conj f^_y u^_x) / ns_total, beta_5, beta_6.
 * alpha, beta: device, 6 x nspec doubles each (entry e - 1 of feature e at
 * + (e - 1) nspec, nspec = n0 n1 (n2/2 + 1) half-spectrum modes),
 * caller-zeroed before the first call.  Asynchronous. */
uno_status el_uno_train_accumulate(const uno_grid *grid, int32_t ns, const double *f, const double *u,
                                   double ns_total, double *alpha, double *beta, void *stream);
/* Algorithm 4: Newton iterations on the loss of App. B in the weights of
 * el_uno_precond_create (ntheta = 6 (k_max + 1), out in theta), from the
 * features of el_uno_train_accumulate, at most max_epochs steps.  The two
 * slots of a pair k, -k on the plane k_z = 0 share one weight vector.  Each
 * step solves (H + lam I) dw = -g with a Levenberg-Marquardt shift lam that
 * shrinks after a step lowering the loss and grows otherwise; it stops when
 * the gradient has dropped by 1e-10 or two steps no longer lower the loss.
 * loss (host, nullable): the final loss less its constant <||u||^2>.
 * Synchronous. */
uno_status el_uno_train_fit(const uno_grid *grid, int32_t M, const double *alpha, const double *beta,
                            int32_t max_epochs, double *theta, int64_t ntheta, double *loss, void *stream);

/* ---- Timing of one kernel family (for roofline accounting) ----------- */
enum {
    UNO_KT_NONE = 0,
    UNO_KT_MATVEC = 1,   /* operator apply inside CG (direction update + A d + d.Ad) */
    UNO_KT_UPDATE = 2,   /* residual/solution update (+ Jacobi + r.s) */
    UNO_KT_FFT_FWD = 3,  /* first transform pass of the UNO apply */
    UNO_KT_FFT_MID = 4,  /* middle pass: transform, Phi multiply, inverse */
    UNO_KT_FFT_INV = 5,  /* last inverse pass (+ r.s) */
    UNO_KT_APPLY = 6     /* operator apply outside CG (fe_apply, residuals) */
};
/* Measurement utility (no passage of the paper).  Brackets every launch
 * of kernel family `which` with start/stop HIP events
 * of the launch itself (hipExtLaunchKernelGGL) on its stream; UNO_KT_NONE
 * disables.  The events come from a pool and carry no system-scope fence.
 * uno_timing_read synchronizes those events and returns the summed duration
 * (ms) and launch count since enabling.  Host-global; not for concurrent use
 * from several threads with different families. */
uno_status uno_timing_enable(int32_t which);
uno_status uno_timing_read(double *total_ms, int64_t *launches);

/* Library utility (no passage of the paper): releases cached workspaces
 * (all devices) and the timing event pool. */
uno_status uno_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* UNOCG_H */
