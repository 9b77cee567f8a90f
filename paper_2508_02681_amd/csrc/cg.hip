// Preconditioned conjugate gradients (Algorithm 1; Algorithm 2 with the UNO
// preconditioner) with every scalar kept on the device.
//
// One pass k of the while loop is a short fixed sequence of kernels:
//   [UNO passes (the first one tests convergence) ->] matvec -> update
// matvec : gamma_k = r.s (combined from partials), beta = gamma_k /
//          gamma_{k-1} (0 on the first pass), d <- s + beta d, p <- A d,
//          partials of d.p;
// update : alpha = gamma_k / (d.p), r <- r - alpha p, u <- u + alpha d,
//          partials of ||r||_inf, and for Jacobi / no preconditioner also
//          s <- P r and partials of r.s for the next pass.
// The host enqueues passes without waiting; every kernel returns at once when
// the loop has ended (converged or breakdown), so the host reads the state
// only between chunks of passes.  Reductions are FP64, written as one partial
// per workgroup and combined in a fixed order by the kernels that need them.
// The search direction is double-buffered (d_old read around the node,
// d_new written), which fuses the direction update into the operator apply.
#include <climits>
#include <cmath>
#include <cstring>

#include "unocg_internal.h"
#include "reduce.h"
#include "cg_ctl.h"
#include "stencil_tile.h"

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

template <typename T>
__device__ __forceinline__ double diag_at(const GridDev& g, const T* __restrict__ kappa, int64_t i)
{
    int z = (int)(i % g.n2);
    int64_t t = i / g.n2;
    int y = (int)(t % g.n1), x = (int)(t / g.n1);
    T k[2][2][2];
    voxel_kappa(g, kappa, x, y, z, k);
    double ks = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) ks += (double)k[q >> 2][(q >> 1) & 1][q & 1];
    return g.cdiag * ks;
}

// Initial partials: ||r_0||_inf and, for Jacobi / none, s_0 = P r_0 and r_0.s_0.
// MODE 0: none (s is r), 1: Jacobi, 2: UNO (only the norm).
// inverse of the assembled diagonal (Jacobi), formed once per solve
__global__ void __launch_bounds__(kBlock) k_inv_diag(GridDev g, const double* __restrict__ kappa,
                                                     double* __restrict__ dinv)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * blockDim.x)
        dinv[i] = 1.0 / diag_at(g, kappa, i);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_cg_init(GridDev g, const double* __restrict__ dinv,
                                                    const double* __restrict__ r, double* __restrict__ s,
                                                    double* __restrict__ part_rmax, double* __restrict__ part_rs,
                                                    CgState* st)
{
    __shared__ double slots[kBlock / 64];
    double m = 0.0, dt = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = r[i];
        m = OpMax::apply(m, fabs(ri));
        if (MODE == 0) dt += ri * ri;
        if (MODE == 1) {
            const double si = ri * dinv[i];
            s[i] = si;
            dt += ri * si;
        }
    }
    const double bm = block_reduce<OpMax>(m, slots);
    const double bd = block_reduce<OpSum>(dt, slots);
    if (threadIdx.x == 0) {
        part_rmax[blockIdx.x] = bm;
        part_rs[blockIdx.x] = bd;
        if (blockIdx.x == 0) {
            st->done = INT_MAX;
            st->status = 0;
            st->fail_iter = -1;
            st->k_last = -1;
        }
    }
}

// update of pass k.  MODE 0: none, 1: Jacobi (both also form s and r.s for
// pass k + 1), 2: UNO.
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_cg_update(GridDev g, const T* __restrict__ dinv, double* __restrict__ r,
                                                      double* __restrict__ u, const T* __restrict__ d,
                                                      const T* __restrict__ p, T* __restrict__ s, CgIter it,
                                                      const double* __restrict__ part_dp, int np_dp,
                                                      const double* __restrict__ gam, double* __restrict__ part_rmax,
                                                      double* __restrict__ part_rs_next)
{
    __shared__ double slots[kBlock / 64];
    // all loads first: state, d.p partials, gamma_k and the first element's operands
    const StateLoad sl = load_state(it.st);
    const double dp_share = load_share<OpSum>(part_dp, np_dp);
    const double gk = gam[it.k];
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r0 = 0.0, p0 = 0.0, u0 = 0.0, d0 = 0.0;
    if (i0 < g.n) {
        r0 = r[i0];
        p0 = (double)p[i0];
        u0 = u[i0];
        d0 = (double)d[i0];
    }
    if (ended(sl, it.k)) return;
    const double dp = combine_share<OpSum>(dp_share, slots);
    if (!(dp > 0.0) || !isfinite(dp)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { it.st->status = 1; it.st->fail_iter = it.k; }
        return;
    }
    const double alpha = gk / dp;
    double m = 0.0, dt = 0.0;
    for (int64_t i = i0; i < g.n; i += (int64_t)gridDim.x * blockDim.x) {
        if (i != i0) {
            r0 = r[i];
            p0 = (double)p[i];
            u0 = u[i];
            d0 = (double)d[i];
        }
        const double ri = r0 - alpha * p0;
        r[i] = ri;
        u[i] = u0 + alpha * d0;
        m = OpMax::apply(m, fabs(ri));
        if (MODE == 0) dt += ri * ri;
        if (MODE == 1) {
            const T si = (T)(ri * (double)dinv[i]);
            s[i] = si;
            dt += ri * (double)si;
        }
    }
    const double bm = block_reduce<OpMax>(m, slots);
    const double bd = (MODE <= 1) ? block_reduce<OpSum>(dt, slots) : 0.0;
    if (threadIdx.x == 0) {
        part_rmax[blockIdx.x] = bm;
        if (MODE <= 1) part_rs_next[blockIdx.x] = bd;
    }
}

// convergence test after the last pass of a chunk (one workgroup)
__global__ void __launch_bounds__(kBlock) k_cg_check(CgIter it)
{
    __shared__ double slots[kBlock / 64];
    (void)head_check(it, slots);
}

// r = f - y
__global__ void __launch_bounds__(kBlock) k_sub(int64_t n, const double* __restrict__ f, const double* __restrict__ y,
                                                double* __restrict__ r)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        r[i] = f[i] - y[i];
}

// partial sums of u
__global__ void __launch_bounds__(kBlock) k_sum_parts(int64_t n, const double* __restrict__ u,
                                                      double* __restrict__ part)
{
    __shared__ double slots[kBlock / 64];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v += u[i];
    const double b = block_reduce<OpSum>(v, slots);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// u -= mean(u), the mean combined from the partials in every workgroup
__global__ void __launch_bounds__(kBlock) k_sub_mean(int64_t n, double* __restrict__ u, const double* __restrict__ part,
                                                     int np, CgState* st)
{
    __shared__ double slots[kBlock / 64];
    const double mean = reduce_parts<OpSum>(part, np, slots) / (double)n;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->mean = mean;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        u[i] -= mean;
}

// partials of ||f - y||_inf and ||f||_inf
__global__ void __launch_bounds__(kBlock) k_resid_parts(int64_t n, const double* __restrict__ f,
                                                        const double* __restrict__ y, double* __restrict__ pa,
                                                        double* __restrict__ pb)
{
    __shared__ double slots[kBlock / 64];
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a = OpMax::apply(a, fabs(f[i] - y[i]));
        b = OpMax::apply(b, fabs(f[i]));
    }
    const double ra = block_reduce<OpMax>(a, slots);
    const double rb = block_reduce<OpMax>(b, slots);
    if (threadIdx.x == 0) {
        pa[blockIdx.x] = ra;
        pb[blockIdx.x] = rb;
    }
}

__global__ void __launch_bounds__(kBlock) k_resid_final(const double* __restrict__ pa, const double* __restrict__ pb,
                                                        int np, CgState* st)
{
    __shared__ double slots[kBlock / 64];
    const double a = reduce_parts<OpMax>(pa, np, slots);
    const double b = reduce_parts<OpMax>(pb, np, slots);
    if (threadIdx.x == 0) {
        st->dmax = a;
        st->fmax = b;
    }
}

// ---------------------------------------------------------------------------
// driver

namespace {

constexpr int kMaxStreamBlocks = 512;

struct Workspace {
    int device = -1;
    int n[3] = {0, 0, 0};
    int64_t total = 0;
    int nbr = 0;              // workgroups of the streaming CG kernels
    int npart = 0;            // capacity of each partial buffer
    double *f = nullptr, *r = nullptr, *s = nullptr, *d[2] = {nullptr, nullptr}, *p = nullptr;
    double* dinv = nullptr;   // inverse Jacobi diagonal of the current solve
    double* part = nullptr;   // 4 partial buffers: rmax, rs[2], dp
    double2* spec = nullptr;
    int64_t nspec = 0;
    CgState* state = nullptr;
    CgState* host_state = nullptr;  // pinned
    double* hist = nullptr;
    double* gam = nullptr;
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
    (void)hipFree(w->dinv);
    (void)hipFree(w->part);
    (void)hipFree(w->spec);
    (void)hipFree(w->state);
    (void)hipHostFree(w->host_state);
    (void)hipFree(w->hist);
    (void)hipFree(w->gam);
    delete w;
}

uno_status ws_get(const Grid& g, const FftPlan* plan, int extra_parts, int hist_need, Workspace** out)
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
        const int64_t nb = (g.total + kBlock - 1) / kBlock;
        w->nbr = (int)(nb < kMaxStreamBlocks ? nb : kMaxStreamBlocks);
        const size_t vb = sizeof(double) * (size_t)g.total;
        bool ok = hipMalloc(&w->f, vb) == hipSuccess && hipMalloc(&w->r, vb) == hipSuccess &&
                  hipMalloc(&w->s, vb) == hipSuccess && hipMalloc(&w->d[0], vb) == hipSuccess &&
                  hipMalloc(&w->d[1], vb) == hipSuccess && hipMalloc(&w->p, vb) == hipSuccess &&
                  hipMalloc(&w->dinv, vb) == hipSuccess &&
                  hipMalloc(&w->state, sizeof(CgState)) == hipSuccess &&
                  hipHostMalloc(&w->host_state, sizeof(CgState), hipHostMallocDefault) == hipSuccess;
        if (!ok) {
            ws_free(w);
            return UNO_ERR_NOMEM;
        }
        UNO_HIP(hipMemset(w->state, 0, sizeof(CgState)));
        g_ws.push_back(w);
    }
    int need = w->nbr;
    const int ntile = choose_tile(g).blocks;
    if (ntile > need) need = ntile;
    if (extra_parts > need) need = extra_parts;
    if (need > w->npart) {
        (void)hipFree(w->part);
        w->part = nullptr;
        if (hipMalloc(&w->part, sizeof(double) * 4 * (size_t)need) != hipSuccess) return UNO_ERR_NOMEM;
        w->npart = need;
    }
    if (plan && plan->nspec > w->nspec) {
        (void)hipFree(w->spec);
        w->spec = nullptr;
        if (hipMalloc(&w->spec, sizeof(double2) * plan->nspec) != hipSuccess) return UNO_ERR_NOMEM;
        w->nspec = plan->nspec;
    }
    if (hist_need > w->hist_cap) {
        (void)hipFree(w->hist);
        (void)hipFree(w->gam);
        w->hist = w->gam = nullptr;
        if (hipMalloc(&w->hist, sizeof(double) * hist_need) != hipSuccess) return UNO_ERR_NOMEM;
        if (hipMalloc(&w->gam, sizeof(double) * hist_need) != hipSuccess) return UNO_ERR_NOMEM;
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

namespace {

struct Parts {
    double* rmax;
    double* rs[2];
    double* dp;
};

Parts parts_of(Workspace* w)
{
    Parts P;
    P.rmax = w->part;
    P.rs[0] = w->part + w->npart;
    P.rs[1] = w->part + 2 * (size_t)w->npart;
    P.dp = w->part + 3 * (size_t)w->npart;
    return P;
}

// np_update: workgroups of the update kernel (they write the ||r||_inf
// partials read at the head of pass k > 0; pass 0 reads the init kernel's)
CgIter iter_of(Workspace* w, const Parts& P, int k, double rtol, int hist_len, int np_update)
{
    CgIter it;
    memset(&it, 0, sizeof(it));
    it.k = k;
    it.st = w->state;
    it.part_rmax = P.rmax;
    it.np_rmax = (k == 0) ? w->nbr : np_update;
    it.rtol = rtol;
    it.hist = w->hist;
    it.hist_len = hist_len;
    it.r = w->r;
    it.part_rs = P.rs[k & 1];
    return it;
}

}  // namespace

static uno_status enqueue_pass(const Grid& g, Workspace* w, int kind, const uno_precond* pc, const double* kappa,
                               double* u, int k, double rtol, int hist_len, hipStream_t st)
{
    const Parts P = parts_of(w);
    const int nb = w->nbr;
    double* dold = w->d[k & 1];
    double* dnew = w->d[(k + 1) & 1];
    KTimer kt;
    const double* s = (kind == UNO_PREC_NONE) ? w->r : w->s;
    int np_rs = nb;
    if (kind == UNO_PREC_UNO && uno_use_lowrank(pc)) {
        // learned-mode flow: [B (head) + C] -> matvec -> [update + A of pass k+1]
        CgIter it = iter_of(w, P, k, rtol, hist_len, lowrank_update_blocks(pc->lr));
        uno_status e = lowrank_finish(pc->lr, w->r, w->s, &it, &np_rs, st);
        if (e != UNO_OK) return e;
        ktimer_begin(&kt, UNO_KT_MATVEC, st);
        const int np_dp =
            launch_tile<double, true, false>(g, kappa, s, dold, dnew, w->p, P.dp, it, P.rs[k & 1], np_rs, w->gam, st);
        ktimer_end(&kt);
        UNO_HIP(hipGetLastError());
        return lowrank_update_forward(pc->lr, w->r, u, dnew, w->p, it, P.dp, np_dp, w->gam, P.rmax, st);
    }
    CgIter it = iter_of(w, P, k, rtol, hist_len, nb);
    if (kind == UNO_PREC_UNO) {
        uno_status e = uno_apply_passes(g, pc->plan, pc->table, pc->table_t, w->r, w->s, UNO_F64, w->spec, &it,
                                        &np_rs, st);
        if (e != UNO_OK) return e;
    }
    ktimer_begin(&kt, UNO_KT_MATVEC, st);
    int np_dp;
    if (kind == UNO_PREC_UNO)
        np_dp = launch_tile<double, true, false>(g, kappa, s, dold, dnew, w->p, P.dp, it, P.rs[k & 1], np_rs, w->gam, st);
    else
        np_dp = launch_tile<double, true, true>(g, kappa, s, dold, dnew, w->p, P.dp, it, P.rs[k & 1], np_rs, w->gam, st);
    ktimer_end(&kt);
    UNO_HIP(hipGetLastError());
    ktimer_begin(&kt, UNO_KT_UPDATE, st);
    double* rs_next = P.rs[(k + 1) & 1];
    if (kind == UNO_PREC_NONE)
        hipLaunchKernelGGL((k_cg_update<double, 0>), dim3(nb), dim3(kBlock), 0, st, g.dev, (const double*)w->dinv, w->r, u, dnew, w->p,
                           w->s, it, (const double*)P.dp, np_dp, (const double*)w->gam, P.rmax, rs_next);
    else if (kind == UNO_PREC_JACOBI)
        hipLaunchKernelGGL((k_cg_update<double, 1>), dim3(nb), dim3(kBlock), 0, st, g.dev, (const double*)w->dinv, w->r, u, dnew, w->p,
                           w->s, it, (const double*)P.dp, np_dp, (const double*)w->gam, P.rmax, rs_next);
    else
        hipLaunchKernelGGL((k_cg_update<double, 2>), dim3(nb), dim3(kBlock), 0, st, g.dev, (const double*)w->dinv, w->r, u, dnew, w->p,
                           w->s, it, (const double*)P.dp, np_dp, (const double*)w->gam, P.rmax, rs_next);
    ktimer_end(&kt);
    UNO_HIP(hipGetLastError());
    return UNO_OK;
}

uno_status pcg_run(const Grid& g, const double* kappa, const double* macro_load3, const double* rhs, double* u,
                   const uno_solve_opts* o, uno_solve_info* info, double* res_hist, hipStream_t st)
{
    const uno_precond* pc = (o->kind == UNO_PREC_UNO) ? o->uno : nullptr;
    Workspace* w = nullptr;
    const int hist_len = o->max_iter + 1;
    uno_status e = ws_get(g, pc ? &pc->plan : nullptr, pc ? pc->rs_blocks : 0, hist_len, &w);
    if (e != UNO_OK) return e;
    const int nb = w->nbr;
    const Parts P = parts_of(w);
    // rhs and initial residual r_0 = f - A u_0
    if (macro_load3) {
        e = launch_rhs(g, kappa, UNO_F64, macro_load3, w->f, UNO_F64, st);
        if (e != UNO_OK) return e;
    } else {
        UNO_HIP(hipMemcpyAsync(w->f, rhs, sizeof(double) * g.total, hipMemcpyDeviceToDevice, st));
    }
    e = launch_fe_apply(g, kappa, u, w->p, UNO_F64, st);
    if (e != UNO_OK) return e;
    hipLaunchKernelGGL(k_sub, dim3(nb), dim3(kBlock), 0, st, g.total, (const double*)w->f, (const double*)w->p, w->r);
    UNO_HIP(hipGetLastError());
    const double* dinv = w->dinv;
    if (o->kind == UNO_PREC_NONE)
        hipLaunchKernelGGL(k_cg_init<0>, dim3(nb), dim3(kBlock), 0, st, g.dev, dinv, w->r, w->s, P.rmax, P.rs[0],
                           w->state);
    else if (o->kind == UNO_PREC_JACOBI) {
        hipLaunchKernelGGL(k_inv_diag, dim3(nb), dim3(kBlock), 0, st, g.dev, kappa, w->dinv);
        hipLaunchKernelGGL(k_cg_init<1>, dim3(nb), dim3(kBlock), 0, st, g.dev, dinv, w->r, w->s, P.rmax, P.rs[0],
                           w->state);
    } else
        hipLaunchKernelGGL(k_cg_init<2>, dim3(nb), dim3(kBlock), 0, st, g.dev, dinv, w->r, w->s, P.rmax, P.rs[0],
                           w->state);
    UNO_HIP(hipGetLastError());
    const bool lowrank = pc && uno_use_lowrank(pc);
    const int np_update = lowrank ? lowrank_update_blocks(pc->lr) : nb;
    if (lowrank) {
        e = lowrank_forward(pc->lr, w->r, st);  // transform of r_0 for the first pass
        if (e != UNO_OK) return e;
    }

    // passes in chunks; the host reads the state between chunks
    int k = 0;
    int chunk = o->graph_chunk > 0 ? o->graph_chunk : 8;
    int prev_k = -1;
    double prev_r = -1.0;
    for (;;) {
        if (chunk > o->max_iter - k) chunk = o->max_iter - k;
        for (int c = 0; c < chunk; ++c, ++k) {
            e = enqueue_pass(g, w, o->kind, pc, kappa, u, k, o->rtol, hist_len, st);
            if (e != UNO_OK) return e;
        }
        CgIter it = iter_of(w, P, k, o->rtol, hist_len, np_update);
        hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(kBlock), 0, st, it);
        UNO_HIP(hipGetLastError());
        UNO_HIP(hipMemcpyAsync(w->host_state, w->state, sizeof(CgState), hipMemcpyDeviceToHost, st));
        UNO_HIP(hipStreamSynchronize(st));
        const CgState& hs = *w->host_state;
        if (hs.status != 0 || hs.done != INT_MAX || k >= o->max_iter) break;
        if (o->graph_chunk <= 0) {
            // predict the passes still needed from the observed contraction rate
            int next = 16;
            if (prev_r > 0.0 && hs.rmax_last > 0.0 && hs.k_last > prev_k && hs.rmax_last < prev_r) {
                const double rate = std::pow(hs.rmax_last / prev_r, 1.0 / (hs.k_last - prev_k));
                const double need = std::log(hs.tol_abs / hs.rmax_last) / std::log(rate);
                next = (int)std::ceil(need * 1.05) + 1;
            }
            chunk = next < 4 ? 4 : (next > 256 ? 256 : next);
        }
        prev_k = hs.k_last;
        prev_r = hs.rmax_last;
    }
    const CgState hs = *w->host_state;
    // zero-mean fluctuation (Sec. 5.1) and the true residual in FP64
    hipLaunchKernelGGL(k_sum_parts, dim3(nb), dim3(kBlock), 0, st, g.total, (const double*)u, P.dp);
    hipLaunchKernelGGL(k_sub_mean, dim3(nb), dim3(kBlock), 0, st, g.total, u, (const double*)P.dp, nb, w->state);
    e = launch_fe_apply(g, kappa, u, w->p, UNO_F64, st);
    if (e != UNO_OK) return e;
    hipLaunchKernelGGL(k_resid_parts, dim3(nb), dim3(kBlock), 0, st, g.total, (const double*)w->f,
                       (const double*)w->p, P.rs[0], P.rs[1]);
    hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(kBlock), 0, st, (const double*)P.rs[0], (const double*)P.rs[1], nb,
                       w->state);
    UNO_HIP(hipGetLastError());
    UNO_HIP(hipMemcpyAsync(w->host_state, w->state, sizeof(CgState), hipMemcpyDeviceToHost, st));
    const int iters = (hs.done != INT_MAX) ? hs.done : (hs.status != 0 ? hs.fail_iter : k);
    if (res_hist) {
        int nh = iters + 1;
        if (nh > hist_len) nh = hist_len;
        UNO_HIP(hipMemcpyAsync(res_hist, w->hist, sizeof(double) * nh, hipMemcpyDeviceToHost, st));
    }
    UNO_HIP(hipStreamSynchronize(st));
    const CgState& fin = *w->host_state;
    if (info) {
        info->iters = iters;
        info->converged = (hs.status == 0 && hs.done != INT_MAX) ? 1 : 0;
        info->rel_res = hs.r0max > 0.0 ? hs.rmax_last / hs.r0max : 0.0;
        info->true_rel_res = fin.fmax > 0.0 ? fin.dmax / fin.fmax : 0.0;
        info->r0_norm = hs.r0max;
    }
    if (hs.status != 0) return UNO_ERR_BREAKDOWN;
    return UNO_OK;
}

}  // namespace unocg
