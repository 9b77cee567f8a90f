// Preconditioned conjugate gradients (Algorithm 1; Algorithm 2 with the UNO
// preconditioner) with every scalar kept on the device.
//
// One pass of the while loop is a short fixed sequence of kernels:
//   [preconditioner passes (UNO) ->] matvec -> update
// matvec : beta = gamma1 / gamma0 (0 on the first pass), d <- s + beta d,
//          p <- A d, and d.p;
// update : alpha = gamma1 / (d.p), r <- r - alpha p, u <- u + alpha d,
//          ||r||_inf, and for Jacobi / no preconditioner also s <- P r and
//          r.s of the next pass.
// Each kernel first reads the solver state and returns at once when the loop
// has ended (converged, max_iter reached, or breakdown), so the host can
// enqueue passes ahead of the convergence decision and only reads the state
// every few passes.  Reductions are FP64 and combined in a fixed order by
// the last workgroup to finish, which also updates the state.
//
// The search direction is double-buffered (d_old read at the halo, d_new
// written), so the direction update is fused into the operator apply.
#include <cmath>
#include <cstring>

#include "unocg_internal.h"
#include "reduce.h"

namespace unocg {

__device__ __forceinline__ int wrap_i(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ void voxel_kappa(const GridDev& g, const T* __restrict__ kappa, int x, int y, int z,
                                            T k[2][2][2])
{
#pragma unroll
    for (int s0 = 0; s0 < 2; ++s0)
#pragma unroll
        for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                int xx = wrap_i(x - 1 + s0, g.n0), yy = wrap_i(y - 1 + s1, g.n1), zz = wrap_i(z - 1 + s2, g.n2);
                k[s0][s1][s2] = kappa[((int64_t)xx * g.n1 + yy) * g.n2 + zz];
            }
}

// Initial state: ||r0||_inf, and for Jacobi / none s0 = P r0 and r0.s0.
// MODE 0: none (s aliases r), 1: Jacobi, 2: UNO (only the norm).
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_cg_init(GridDev g, const double* __restrict__ kappa, const double* __restrict__ r,
                                                    double* __restrict__ s, double* __restrict__ part_max,
                                                    double* __restrict__ part_dot, CgState* state, double rtol,
                                                    int max_iter, double* hist, int hist_len)
{
    __shared__ double slots[kBlock / 64];
    __shared__ int lastflag;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double m = 0.0, dt = 0.0;
    if (i < g.n) {
        double ri = r[i];
        m = fabs(ri);
        if (MODE == 0) dt = ri * ri;
        if (MODE == 1) {
            int z = (int)(i % g.n2);
            int64_t t = i / g.n2;
            int y = (int)(t % g.n1), x = (int)(t / g.n1);
            double k[2][2][2];
            voxel_kappa(g, kappa, x, y, z, k);
            double ks = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) ks += k[q >> 2][(q >> 1) & 1][q & 1];
            double si = ri / (g.cdiag * ks);
            s[i] = si;
            dt = ri * si;
        }
    }
    double bm = block_reduce<OpMax>(m, slots);
    double bd = block_reduce<OpSum>(dt, slots);
    if (threadIdx.x == 0) {
        part_max[blockIdx.x] = bm;
        part_dot[blockIdx.x] = bd;
    }
    if (arrive_last(&state->counter, &lastflag)) {
        double r0 = combine_partials<OpMax>(part_max, gridDim.x, slots);
        double gsum = combine_partials<OpSum>(part_dot, gridDim.x, slots);
        if (threadIdx.x == 0) {
            state->r0max = r0;
            state->rmax = r0;
            state->tol_abs = rtol * r0;
            state->iters = 0;
            state->max_iter = max_iter;
            state->status = (r0 == r0) ? 0 : 1;
            state->hist_len = hist_len;
            state->dp = 0.0;
            if (MODE == 2) {
                state->gamma0 = 1.0;
                state->gamma1 = 1.0;
            } else {
                state->gamma0 = 1.0;
                state->gamma1 = gsum;
                if (r0 > state->tol_abs && (!(gsum > 0.0) || !isfinite(gsum))) state->status = 1;
            }
            if (hist && hist_len > 0) hist[0] = r0;
            state->counter = 0;
        }
    }
}

// d_new = s + beta d_old, p = A d_new, d_new . p   (one node per thread)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_matvec(GridDev g, const T* __restrict__ kappa, const T* __restrict__ s,
                                                      const T* __restrict__ dold, T* __restrict__ dnew,
                                                      T* __restrict__ p, double* __restrict__ part, CgState* state)
{
    __shared__ double slots[kBlock / 64];
    __shared__ int lastflag;
    if (cg_done(state)) return;
    const bool first = state->iters == 0;
    const T beta = first ? (T)0 : (T)(state->gamma1 / state->gamma0);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dot = 0.0;
    if (i < g.n) {
        int z = (int)(i % g.n2);
        int64_t t = i / g.n2;
        int y = (int)(t % g.n1), x = (int)(t / g.n1);
        T k[2][2][2];
        voxel_kappa(g, kappa, x, y, z, k);
        // compatible-voxel sums per offset
        T A[2][2][3], B[2][3][3], K3[3][3][3];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                A[a][b][0] = k[a][b][0];
                A[a][b][1] = k[a][b][0] + k[a][b][1];
                A[a][b][2] = k[a][b][1];
            }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                B[a][0][c] = A[a][0][c];
                B[a][1][c] = A[a][0][c] + A[a][1][c];
                B[a][2][c] = A[a][1][c];
            }
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                K3[0][b][c] = B[0][b][c];
                K3[1][b][c] = B[0][b][c] + B[1][b][c];
                K3[2][b][c] = B[1][b][c];
            }
        T acc = 0, dself = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int xx = wrap_i(x + a - 1, g.n0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                int yy = wrap_i(y + b - 1, g.n1);
                int64_t row = ((int64_t)xx * g.n1 + yy) * g.n2;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    int zz = wrap_i(z + c - 1, g.n2);
                    T dv = s[row + zz];
                    if (!first) dv += beta * dold[row + zz];
                    int m = ((a != 1) << 2) | ((b != 1) << 1) | (c != 1);
                    acc += (T)g.w[m] * K3[a][b][c] * dv;
                    if (a == 1 && b == 1 && c == 1) dself = dv;
                }
            }
        }
        dnew[i] = dself;
        p[i] = acc;
        dot = (double)dself * (double)acc;
    }
    double bd = block_reduce<OpSum>(dot, slots);
    if (threadIdx.x == 0) part[blockIdx.x] = bd;
    if (arrive_last(&state->counter, &lastflag)) {
        double v = combine_partials<OpSum>(part, gridDim.x, slots);
        if (threadIdx.x == 0) {
            state->dp = v;
            if (!(v > 0.0) || !isfinite(v)) state->status = 1;
            state->counter = 0;
        }
    }
}

// r -= alpha p; u += alpha d; ||r||_inf; MODE 0/1 also s = P r and r.s.
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_cg_update(GridDev g, const T* __restrict__ kappa, double* __restrict__ r,
                                                      double* __restrict__ u, const T* __restrict__ d,
                                                      const T* __restrict__ p, T* __restrict__ s,
                                                      double* __restrict__ part_max, double* __restrict__ part_dot,
                                                      CgState* state, double* hist)
{
    __shared__ double slots[kBlock / 64];
    __shared__ int lastflag;
    if (cg_done(state)) return;
    const double alpha = state->gamma1 / state->dp;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double m = 0.0, dt = 0.0;
    if (i < g.n) {
        double ri = r[i] - alpha * (double)p[i];
        r[i] = ri;
        u[i] += alpha * (double)d[i];
        m = fabs(ri);
        if (MODE == 0) dt = ri * ri;
        if (MODE == 1) {
            int z = (int)(i % g.n2);
            int64_t t = i / g.n2;
            int y = (int)(t % g.n1), x = (int)(t / g.n1);
            T k[2][2][2];
            voxel_kappa(g, kappa, x, y, z, k);
            double ks = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) ks += (double)k[q >> 2][(q >> 1) & 1][q & 1];
            T si = (T)(ri / (g.cdiag * ks));
            s[i] = si;
            dt = ri * (double)si;
        }
        if (MODE == 3) s[i] = (T)ri;  // low-precision copy of r for the preconditioner
    }
    double bm = block_reduce<OpMax>(m, slots);
    double bd = (MODE <= 1) ? block_reduce<OpSum>(dt, slots) : 0.0;
    if (threadIdx.x == 0) {
        part_max[blockIdx.x] = bm;
        if (MODE <= 1) part_dot[blockIdx.x] = bd;
    }
    if (arrive_last(&state->counter, &lastflag)) {
        double rm = combine_partials<OpMax>(part_max, gridDim.x, slots);
        double gs = (MODE <= 1) ? combine_partials<OpSum>(part_dot, gridDim.x, slots) : 0.0;
        if (threadIdx.x == 0) {
            state->rmax = rm;
            int it = state->iters + 1;
            state->iters = it;
            if (hist && it < state->hist_len) hist[it] = rm;
            if (!(rm == rm)) state->status = 1;
            if (MODE <= 1) {
                state->gamma0 = state->gamma1;
                state->gamma1 = gs;
                if (rm > state->tol_abs && (!(gs > 0.0) || !isfinite(gs))) state->status = 1;
            }
            state->counter = 0;
        }
    }
}

// r = f - A u0 (y holds A u0)
__global__ void __launch_bounds__(kBlock) k_sub(int64_t n, const double* __restrict__ f, const double* __restrict__ y,
                                                double* __restrict__ r)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = f[i] - y[i];
}

// mean of u into state->mean (last-block combination)
__global__ void __launch_bounds__(kBlock) k_mean(int64_t n, const double* __restrict__ u, double* __restrict__ part,
                                                 CgState* state)
{
    __shared__ double slots[kBlock / 64];
    __shared__ int lastflag;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = (i < n) ? u[i] : 0.0;
    double b = block_reduce<OpSum>(v, slots);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
    if (arrive_last(&state->counter, &lastflag)) {
        double s = combine_partials<OpSum>(part, gridDim.x, slots);
        if (threadIdx.x == 0) {
            state->mean = s / (double)n;
            state->counter = 0;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_sub_mean(int64_t n, double* __restrict__ u, const CgState* state)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] -= state->mean;
}

// ||f - y||_inf and ||f||_inf into state->dmax / fmax
__global__ void __launch_bounds__(kBlock) k_resid_norms(int64_t n, const double* __restrict__ f,
                                                        const double* __restrict__ y, double* __restrict__ pa,
                                                        double* __restrict__ pb, CgState* state)
{
    __shared__ double slots[kBlock / 64];
    __shared__ int lastflag;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (i < n) {
        a = fabs(f[i] - y[i]);
        b = fabs(f[i]);
    }
    double ba = block_reduce<OpMax>(a, slots);
    double bb = block_reduce<OpMax>(b, slots);
    if (threadIdx.x == 0) {
        pa[blockIdx.x] = ba;
        pb[blockIdx.x] = bb;
    }
    if (arrive_last(&state->counter, &lastflag)) {
        double A = combine_partials<OpMax>(pa, gridDim.x, slots);
        double B = combine_partials<OpMax>(pb, gridDim.x, slots);
        if (threadIdx.x == 0) {
            state->dmax = A;
            state->fmax = B;
            state->counter = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// driver

namespace {

struct Workspace {
    int device = -1;
    int n[3] = {0, 0, 0};
    int64_t total = 0;
    double *f = nullptr, *r = nullptr, *s = nullptr, *d[2] = {nullptr, nullptr}, *p = nullptr;
    double* part = nullptr;   // 2 * nblocks
    double2* spec = nullptr;  // nspec
    int64_t nspec = 0;
    CgState* state = nullptr;
    CgState* host_state = nullptr;  // pinned
    double* hist = nullptr;
    int hist_cap = 0;
};

std::vector<Workspace*> g_ws;

void ws_free(Workspace* w)
{
    (void)hipFree(w->f);
    (void)hipFree(w->r);
    (void)hipFree(w->s);
    (void)hipFree(w->d[0]);
    (void)hipFree(w->d[1]);
    (void)hipFree(w->p);
    (void)hipFree(w->part);
    (void)hipFree(w->spec);
    (void)hipFree(w->state);
    (void)hipHostFree(w->host_state);
    (void)hipFree(w->hist);
    delete w;
}

uno_status ws_get(const Grid& g, int64_t nspec, int hist_need, Workspace** out)
{
    int dev = 0;
    UNO_HIP(hipGetDevice(&dev));
    Workspace* w = nullptr;
    for (Workspace* c : g_ws)
        if (c->device == dev && c->n[0] == g.n[0] && c->n[1] == g.n[1] && c->n[2] == g.n[2]) w = c;
    if (!w) {
        w = new Workspace();
        w->device = dev;
        for (int b = 0; b < 3; ++b) w->n[b] = g.n[b];
        w->total = g.total;
        const size_t vb = sizeof(double) * (size_t)g.total;
        const int64_t nb = (g.total + kBlock - 1) / kBlock;
        bool ok = hipMalloc(&w->f, vb) == hipSuccess && hipMalloc(&w->r, vb) == hipSuccess &&
                  hipMalloc(&w->s, vb) == hipSuccess && hipMalloc(&w->d[0], vb) == hipSuccess &&
                  hipMalloc(&w->d[1], vb) == hipSuccess && hipMalloc(&w->p, vb) == hipSuccess &&
                  hipMalloc(&w->part, sizeof(double) * 3 * nb + 64) == hipSuccess &&
                  hipMalloc(&w->state, sizeof(CgState)) == hipSuccess &&
                  hipHostMalloc(&w->host_state, sizeof(CgState), hipHostMallocDefault) == hipSuccess;
        if (!ok) {
            ws_free(w);
            return UNO_ERR_NOMEM;
        }
        UNO_HIP(hipMemset(w->state, 0, sizeof(CgState)));
        g_ws.push_back(w);
    }
    if (nspec > w->nspec) {
        (void)hipFree(w->spec);
        w->spec = nullptr;
        if (hipMalloc(&w->spec, sizeof(double2) * nspec) != hipSuccess) return UNO_ERR_NOMEM;
        w->nspec = nspec;
    }
    if (hist_need > w->hist_cap) {
        (void)hipFree(w->hist);
        w->hist = nullptr;
        if (hipMalloc(&w->hist, sizeof(double) * hist_need) != hipSuccess) return UNO_ERR_NOMEM;
        w->hist_cap = hist_need;
    }
    *out = w;
    return UNO_OK;
}

}  // namespace

uno_status ws_release_all()
{
    for (Workspace* w : g_ws) ws_free(w);
    g_ws.clear();
    return UNO_OK;
}

static uno_status enqueue_pass(const Grid& g, Workspace* w, int kind, const uno_precond* pc, const double* kappa,
                               double* u, int64_t k, hipStream_t st, int nb)
{
    double* dold = w->d[k & 1];
    double* dnew = w->d[(k + 1) & 1];
    double* part_a = w->part;
    double* part_b = w->part + nb;
    KTimer kt;
    const double* s = (kind == UNO_PREC_NONE) ? w->r : w->s;
    if (kind == UNO_PREC_UNO) {
        RsReduce red{w->r, part_b, w->state};
        uno_status e = uno_apply_passes(g, pc->plan, pc->table, pc->table_t, w->r, w->s, UNO_F64, w->spec, &red,
                                        w->state, st);
        if (e != UNO_OK) return e;
    }
    ktimer_begin(&kt, UNO_KT_MATVEC, st);
    hipLaunchKernelGGL(k_cg_matvec<double>, dim3(nb), dim3(kBlock), 0, st, g.dev, kappa, s, dold, dnew, w->p, part_a,
                       w->state);
    ktimer_end(&kt);
    UNO_HIP(hipGetLastError());
    ktimer_begin(&kt, UNO_KT_UPDATE, st);
    if (kind == UNO_PREC_NONE)
        hipLaunchKernelGGL((k_cg_update<double, 0>), dim3(nb), dim3(kBlock), 0, st, g.dev, kappa, w->r, u, dnew, w->p,
                           w->s, part_a, part_b, w->state, w->hist);
    else if (kind == UNO_PREC_JACOBI)
        hipLaunchKernelGGL((k_cg_update<double, 1>), dim3(nb), dim3(kBlock), 0, st, g.dev, kappa, w->r, u, dnew, w->p,
                           w->s, part_a, part_b, w->state, w->hist);
    else
        hipLaunchKernelGGL((k_cg_update<double, 2>), dim3(nb), dim3(kBlock), 0, st, g.dev, kappa, w->r, u, dnew, w->p,
                           w->s, part_a, part_b, w->state, w->hist);
    ktimer_end(&kt);
    UNO_HIP(hipGetLastError());
    return UNO_OK;
}

uno_status pcg_run(const Grid& g, const double* kappa, const double* macro_load3, const double* rhs, double* u,
                   const uno_solve_opts* o, uno_solve_info* info, double* res_hist, hipStream_t st)
{
    const uno_precond* pc = o->uno;
    Workspace* w = nullptr;
    const int hist_need = o->max_iter + 1;
    uno_status e = ws_get(g, pc ? pc->plan.nspec : 0, hist_need, &w);
    if (e != UNO_OK) return e;
    const int nb = (int)((g.total + kBlock - 1) / kBlock);
    // rhs and initial residual
    if (macro_load3) {
        e = launch_rhs(g, kappa, UNO_F64, macro_load3, w->f, UNO_F64, st);
        if (e != UNO_OK) return e;
    } else {
        UNO_HIP(hipMemcpyAsync(w->f, rhs, sizeof(double) * g.total, hipMemcpyDeviceToDevice, st));
    }
    e = launch_fe_apply(g, kappa, u, w->p, UNO_F64, st);
    if (e != UNO_OK) return e;
    hipLaunchKernelGGL(k_sub, dim3(nb), dim3(kBlock), 0, st, g.total, w->f, w->p, w->r);
    UNO_HIP(hipGetLastError());
    double* part_a = w->part;
    double* part_b = w->part + nb;
    if (o->kind == UNO_PREC_NONE)
        hipLaunchKernelGGL(k_cg_init<0>, dim3(nb), dim3(kBlock), 0, st, g.dev, kappa, w->r, w->s, part_a, part_b,
                           w->state, o->rtol, o->max_iter, w->hist, hist_need);
    else if (o->kind == UNO_PREC_JACOBI)
        hipLaunchKernelGGL(k_cg_init<1>, dim3(nb), dim3(kBlock), 0, st, g.dev, kappa, w->r, w->s, part_a, part_b,
                           w->state, o->rtol, o->max_iter, w->hist, hist_need);
    else
        hipLaunchKernelGGL(k_cg_init<2>, dim3(nb), dim3(kBlock), 0, st, g.dev, kappa, w->r, w->s, part_a, part_b,
                           w->state, o->rtol, o->max_iter, w->hist, hist_need);
    UNO_HIP(hipGetLastError());

    // passes in chunks; the host reads the state between chunks
    int64_t k = 0;
    int chunk = o->graph_chunk > 0 ? o->graph_chunk : 8;
    int prev_it = 0;
    double prev_r = -1.0;
    for (;;) {
        for (int c = 0; c < chunk; ++c, ++k) {
            e = enqueue_pass(g, w, o->kind, pc, kappa, u, k, st, nb);
            if (e != UNO_OK) return e;
        }
        UNO_HIP(hipMemcpyAsync(w->host_state, w->state, sizeof(CgState), hipMemcpyDeviceToHost, st));
        UNO_HIP(hipStreamSynchronize(st));
        const CgState& hs = *w->host_state;
        if (cg_done(&hs)) break;
        if (o->graph_chunk <= 0) {
            // predict the passes still needed from the observed contraction rate
            int next = 16;
            if (prev_r > 0.0 && hs.rmax > 0.0 && hs.iters > prev_it && hs.rmax < prev_r) {
                double rate = std::pow(hs.rmax / prev_r, 1.0 / (hs.iters - prev_it));
                double need = std::log(hs.tol_abs / hs.rmax) / std::log(rate);
                next = (int)std::ceil(need * 1.05) + 1;
            }
            if (next < 4) next = 4;
            if (next > 256) next = 256;
            int left = hs.max_iter - hs.iters;
            if (next > left) next = left;
            chunk = next < 1 ? 1 : next;
        }
        prev_it = hs.iters;
        prev_r = hs.rmax;
    }
    const CgState hs = *w->host_state;
    // zero-mean fluctuation (Sec. 5.1) and the true residual in FP64
    hipLaunchKernelGGL(k_mean, dim3(nb), dim3(kBlock), 0, st, g.total, u, part_a, w->state);
    hipLaunchKernelGGL(k_sub_mean, dim3(nb), dim3(kBlock), 0, st, g.total, u, (const CgState*)w->state);
    e = launch_fe_apply(g, kappa, u, w->p, UNO_F64, st);
    if (e != UNO_OK) return e;
    hipLaunchKernelGGL(k_resid_norms, dim3(nb), dim3(kBlock), 0, st, g.total, w->f, w->p, part_a, part_b, w->state);
    UNO_HIP(hipGetLastError());
    UNO_HIP(hipMemcpyAsync(w->host_state, w->state, sizeof(CgState), hipMemcpyDeviceToHost, st));
    if (res_hist) {
        int nh = hs.iters + 1;
        if (nh > hist_need) nh = hist_need;
        UNO_HIP(hipMemcpyAsync(res_hist, w->hist, sizeof(double) * nh, hipMemcpyDeviceToHost, st));
    }
    UNO_HIP(hipStreamSynchronize(st));
    const CgState& fin = *w->host_state;
    if (info) {
        info->iters = hs.iters;
        info->converged = (hs.status == 0 && hs.rmax <= hs.tol_abs) ? 1 : 0;
        info->rel_res = hs.r0max > 0.0 ? hs.rmax / hs.r0max : 0.0;
        info->true_rel_res = fin.fmax > 0.0 ? fin.dmax / fin.fmax : 0.0;
        info->r0_norm = hs.r0max;
    }
    if (hs.status != 0) return UNO_ERR_BREAKDOWN;
    return UNO_OK;
}

}  // namespace unocg
