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
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

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
template <typename T>
__global__ void __launch_bounds__(kBlock) k_inv_diag(GridDev g, const double* __restrict__ kappa,
                                                     T* __restrict__ dinv)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * blockDim.x)
        dinv[i] = (T)(1.0 / diag_at(g, kappa, i));
}

// vector precision copy (conductivities for the FP32 operator)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_convert(int64_t n, const double* __restrict__ a, T* __restrict__ b)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (T)a[i];
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_cg_init(GridDev g, const T* __restrict__ dinv,
                                                    const double* __restrict__ r, T* __restrict__ s,
                                                    double* __restrict__ part_rmax, double* __restrict__ part_rs,
                                                    double* __restrict__ part_ss, CgState* st, int ps, int64_t ks,
                                                    int reset = 1)
{
    __shared__ double slots[kBlock / 64];
    if (blockIdx.y > 0) {  // right-hand side blockIdx.y of a batch
        const int64_t vo = (int64_t)blockIdx.y * g.n, po = (int64_t)blockIdx.y * ps;
        dinv += (int64_t)blockIdx.y * ks;
        r += vo;
        s += vo;
        part_rmax += po;
        part_rs += po;
        part_ss += po;
        st += blockIdx.y;
    }
    double m = 0.0, dt = 0.0, ss = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = r[i];
        m = OpMax::apply(m, fabs(ri));
        if (MODE == 0) {
            const T si = (T)ri;
            s[i] = si;
            dt += ri * (double)si;
            ss += (double)si;
        }
        if (MODE == 1) {
            const T si = (T)(ri * (double)dinv[i]);
            s[i] = si;
            dt += ri * (double)si;
            ss += (double)si;
        }
    }
    const double bm = block_reduce<OpMax>(m, slots);
    const double bd = block_reduce<OpSum>(dt, slots);
    const double bs = block_reduce<OpSum>(ss, slots);
    if (threadIdx.x == 0) {
        part_rmax[blockIdx.x] = bm;
        part_rs[blockIdx.x] = bd;
        part_ss[blockIdx.x] = bs;
        if (reset && blockIdx.x == 0) {  // (a restart keeps the states: ended loads stay ended)
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
                                                      double* __restrict__ part_rs_next, double* __restrict__ part_ss_next)
{
    resolve_pass(it);
    __shared__ double slots[kBlock / 64];
    if (blockIdx.y > 0) {  // right-hand side blockIdx.y of a batch
        const int64_t vo = (int64_t)blockIdx.y * it.vs, po = (int64_t)blockIdx.y * it.ps;
        dinv += (int64_t)blockIdx.y * it.ks;
        r += vo;
        u += vo;
        d += vo;
        p += vo;
        s += vo;
        part_dp += po;
        gam += (int64_t)blockIdx.y * it.hs;
        part_rmax += po;
        part_rs_next += po;
        part_ss_next += po;
        it = rhs_iter(it);
    }
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
    double m = 0.0, dt = 0.0, ss = 0.0;
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
        if (MODE == 0) {
            const T si = (T)ri;
            s[i] = si;
            dt += ri * (double)si;
            ss += (double)si;
        }
        if (MODE == 1) {
            const T si = (T)(ri * (double)dinv[i]);
            s[i] = si;
            dt += ri * (double)si;
            ss += (double)si;
        }
    }
    const double bm = block_reduce<OpMax>(m, slots);
    const double bd = (MODE <= 1) ? block_reduce<OpSum>(dt, slots) : 0.0;
    const double bs = (MODE <= 1) ? block_reduce<OpSum>(ss, slots) : 0.0;
    if (threadIdx.x == 0) {
        part_rmax[blockIdx.x] = bm;
        if (MODE <= 1) {
            part_rs_next[blockIdx.x] = bd;
            part_ss_next[blockIdx.x] = bs;
        }
    }
}

// convergence test after the last pass of a chunk (one workgroup)
__global__ void __launch_bounds__(kBlock) k_cg_check(CgIter it)
{
    resolve_pass(it);
    __shared__ double slots[kBlock / 64];
    (void)head_check(rhs_iter(it), slots);
}

// device pass index of graph-captured chunks: set before a series of
// replays, advanced by the last node of each replay
__global__ void k_set_pass(int* kdev, int k)
{
    if (threadIdx.x == 0) *kdev = k;
}
__global__ void k_advance_pass(int* kdev, int by)
{
    if (threadIdx.x == 0) *kdev += by;
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

// Right-hand sides of a batch: f_b = rhs of the macroscopic gradient b for
// the conductivity field kappa + b ks (blockIdx.y = b), as k_rhs_node.
constexpr int kLoads3 = 64;
struct Loads3 {
    double g[kLoads3][3];
};

__global__ void __launch_bounds__(kBlock) k_rhs_batch(GridDev g, const double* __restrict__ kappa, int64_t ks,
                                                      Loads3 L, double* __restrict__ f)
{
    const int b = blockIdx.y;
    kappa += (int64_t)b * ks;
    f += (int64_t)b * g.n;
    const double c0 = L.g[b][0] * g.gcoef[0], c1 = L.g[b][1] * g.gcoef[1], c2 = L.g[b][2] * g.gcoef[2];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(i % g.n2);
        const int64_t t = i / g.n2;
        const int y = (int)(t % g.n1), x = (int)(t / g.n1);
        double acc = 0.0;
#pragma unroll
        for (int s0 = 0; s0 < 2; ++s0)
#pragma unroll
            for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    // voxel x - 1 + s: the node is its upper corner along b for s_b = 0
                    const int xe = (x - 1 + s0 < 0) ? x - 1 + s0 + g.n0 : x - 1 + s0;
                    const int ye = (y - 1 + s1 < 0) ? y - 1 + s1 + g.n1 : y - 1 + s1;
                    const int ze = (z - 1 + s2 < 0) ? z - 1 + s2 + g.n2 : z - 1 + s2;
                    const double k = kappa[((int64_t)xe * g.n1 + ye) * g.n2 + ze];
                    acc += k * ((s0 ? -c0 : c0) + (s1 ? -c1 : c1) + (s2 ? -c2 : c2));
                }
        f[i] = -g.hvol * acc;
    }
}

// batched forms (blockIdx.y = right-hand side b: vectors at + b vs, partials
// at + b ps, state b) of the mean removal and the true residual
__global__ void __launch_bounds__(kBlock) k_sum_parts_b(int64_t n, const double* __restrict__ u,
                                                        double* __restrict__ part, int64_t vs, int ps)
{
    __shared__ double slots[kBlock / 64];
    u += (int64_t)blockIdx.y * vs;
    part += (int64_t)blockIdx.y * ps;
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v += u[i];
    const double b = block_reduce<OpSum>(v, slots);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

__global__ void __launch_bounds__(kBlock) k_sub_mean_b(int64_t n, double* __restrict__ u,
                                                       const double* __restrict__ part, int np, CgState* st,
                                                       int64_t vs, int ps)
{
    __shared__ double slots[kBlock / 64];
    u += (int64_t)blockIdx.y * vs;
    part += (int64_t)blockIdx.y * ps;
    st += blockIdx.y;
    const double mean = reduce_parts<OpSum>(part, np, slots) / (double)n;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->mean = mean;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        u[i] -= mean;
}

__global__ void __launch_bounds__(kBlock) k_resid_parts_b(int64_t n, const double* __restrict__ f,
                                                          const double* __restrict__ y, double* __restrict__ pa,
                                                          double* __restrict__ pb, int64_t vs, int ps)
{
    __shared__ double slots[kBlock / 64];
    f += (int64_t)blockIdx.y * vs;
    y += (int64_t)blockIdx.y * vs;
    pa += (int64_t)blockIdx.y * ps;
    pb += (int64_t)blockIdx.y * ps;
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

__global__ void __launch_bounds__(kBlock) k_resid_final_b(const double* __restrict__ pa, const double* __restrict__ pb,
                                                          int np, CgState* st, int ps)
{
    __shared__ double slots[kBlock / 64];
    pa += (int64_t)blockIdx.y * ps;
    pb += (int64_t)blockIdx.y * ps;
    st += blockIdx.y;
    const double a = reduce_parts<OpMax>(pa, np, slots);
    const double b = reduce_parts<OpMax>(pb, np, slots);
    if (threadIdx.x == 0) {
        st->dmax = a;
        st->fmax = b;
    }
}

// ---------------------------------------------------------------------------
// host side: workspace, the CG loop, batch setup and finish

namespace {

constexpr int kMaxStreamBlocks = 512;

// CG workspace of one (device, grid shape, stream).  Vectors, partial
// buffers, loop states and scalar histories are held for up to nrhs_cap
// right-hand sides solved together: vector b at + b n, partial buffer `kind`
// of b at part + (kind nrhs_cap + b) npart, state b at state + b, history b
// at hist + b hist_cap.  A solve holds the workspace's mutex from ws_get to
// its end: solves on different streams use different workspaces and run
// concurrently; solves on one stream from several host threads take turns
// (the device would order their kernels anyway, but they would share the
// vectors, loop states and pinned host copy of the states).
struct Workspace {
    int device = -1;
    hipStream_t stream = nullptr;
    std::mutex mu;
    int n[3] = {0, 0, 0};
    int64_t total = 0;
    int nbr = 0;              // workgroups of the streaming CG kernels
    int npart = 0;            // capacity of each partial buffer (per right-hand side)
    int nrhs_cap = 0;
    double *f = nullptr, *r = nullptr, *s = nullptr, *d[2] = {nullptr, nullptr}, *p = nullptr;
    double* dinv = nullptr;   // inverse Jacobi diagonal(s) of the current solve
    float* kap32 = nullptr;   // FP32 conductivities (mixed precision)
    int kap32_cap = 0;        // fields it holds
    double* part = nullptr;   // 8 partial buffers: rmax, rs[2], dp, ss[2], ds[2]
    double2* spec = nullptr;
    int64_t nspec = 0;  // spectral scratch per right-hand side (double2), for spec_cap of them
    int spec_cap = 0;
    double2* lr_gp = nullptr; // learned-mode scratch per right-hand side
    double2* lr_h = nullptr;
    bool lr_bf = false;       // the current solve stores that scratch in BF16
    int64_t lr_ngp = 0, lr_nh = 0;
    int lr_cap = 0;
    CgState* state = nullptr;
    CgState* host_state = nullptr;  // pinned
    double* hist = nullptr;
    double* gam = nullptr;
    int hist_cap = 0;
    // captured chunks of passes (graph mode): the device pass index they
    // read, the pass index kernels are recorded against while capturing, and
    // the instantiated graphs with the arguments they were captured with
    int* kdev = nullptr;
    const int* capture_kdev = nullptr;
    hipStream_t capture_stream = nullptr;
    struct Graph {
        std::vector<int64_t> key;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
};

// kernel arguments recorded in a workspace's graphs are stale once a buffer
// of the workspace has been reallocated
void ws_drop_graphs(Workspace* w)
{
    for (auto& gr : w->graphs) (void)hipGraphExecDestroy(gr.exec);
    w->graphs.clear();
}

std::vector<Workspace*> g_ws;
std::mutex g_ws_mu;

void ws_free_vectors(Workspace* w)
{
    (void)hipFree(w->f);
    (void)hipFree(w->r);
    (void)hipFree(w->s);
    (void)hipFree(w->d[0]);
    (void)hipFree(w->d[1]);
    (void)hipFree(w->p);
    (void)hipFree(w->dinv);
    (void)hipFree(w->state);
    (void)hipHostFree(w->host_state);
    w->f = w->r = w->s = w->d[0] = w->d[1] = w->p = w->dinv = nullptr;
    w->state = w->host_state = nullptr;
}

void ws_free(Workspace* w)
{
    ws_drop_graphs(w);
    (void)hipFree(w->kdev);
    if (w->capture_stream) (void)hipStreamDestroy(w->capture_stream);
    ws_free_vectors(w);
    (void)hipFree(w->kap32);
    (void)hipFree(w->part);
    (void)hipFree(w->spec);
    (void)hipFree(w->lr_gp);
    (void)hipFree(w->lr_h);
    (void)hipFree(w->hist);
    (void)hipFree(w->gam);
    delete w;
}

// workgroups of the streaming CG kernels of a grid
int ws_nbr(const Grid& g)
{
    const int64_t nb = (g.total + kBlock - 1) / kBlock;
    return (int)(nb < kMaxStreamBlocks ? nb : kMaxStreamBlocks);
}

// capacity of each partial buffer: the most workgroups any kernel of a pass
// writes partials from
int ws_npart(const Grid& g, int nbr, int extra_parts)
{
    int need = nbr;
    int ntile = choose_tile(g).blocks;
    if (march_max_blocks(g) > ntile) ntile = march_max_blocks(g);
    if (ntile > need) need = ntile;
    if (extra_parts > need) need = extra_parts;
    return need;
}

// The workspace of (current device, grid, stream), locked through *lease
// for the caller's solve.
uno_status ws_get(const Grid& g, const FftPlan* plan, const LowRankPlan* lr, int extra_parts, int hist_need, int nrhs,
                  hipStream_t stream, std::unique_lock<std::mutex>* lease, Workspace** out)
{
    int dev = 0;
    UNO_HIP(hipGetDevice(&dev));
    Workspace* w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        for (Workspace* c : g_ws)
            if (c->device == dev && c->stream == stream && c->n[0] == g.n[0] && c->n[1] == g.n[1] &&
                c->n[2] == g.n[2])
                w = c;
        if (!w) {
            w = new Workspace();
            w->device = dev;
            w->stream = stream;
            for (int b = 0; b < 3; ++b) w->n[b] = g.n[b];
            w->total = g.total;
            w->nbr = ws_nbr(g);
            g_ws.push_back(w);
        }
    }
    *lease = std::unique_lock<std::mutex>(w->mu);
    if (nrhs > w->nrhs_cap) {
        ws_drop_graphs(w);
        ws_free_vectors(w);
        const size_t vb = sizeof(double) * (size_t)g.total * nrhs;
        bool ok = hipMalloc(&w->f, vb) == hipSuccess && hipMalloc(&w->r, vb) == hipSuccess &&
                  hipMalloc(&w->s, vb) == hipSuccess && hipMalloc(&w->d[0], vb) == hipSuccess &&
                  hipMalloc(&w->d[1], vb) == hipSuccess && hipMalloc(&w->p, vb) == hipSuccess &&
                  hipMalloc(&w->dinv, vb) == hipSuccess &&
                  hipMalloc(&w->state, sizeof(CgState) * nrhs) == hipSuccess &&
                  hipHostMalloc(&w->host_state, sizeof(CgState) * nrhs, hipHostMallocDefault) == hipSuccess;
        if (!ok) {
            ws_free_vectors(w);
            w->nrhs_cap = 0;
            return UNO_ERR_NOMEM;
        }
        // (no memset of the states: the init kernels of every solve set them on
        // the solve's stream; a plain hipMemset would run on the null stream,
        // unordered with respect to a non-blocking solve stream)
        // partial buffers and histories are laid out per right-hand side
        (void)hipFree(w->part);
        (void)hipFree(w->hist);
        (void)hipFree(w->gam);
        w->part = w->hist = w->gam = nullptr;
        w->npart = w->hist_cap = 0;
        w->nrhs_cap = nrhs;
    }
    if (!w->kdev && hipMalloc(&w->kdev, sizeof(int)) != hipSuccess) return UNO_ERR_NOMEM;
    const int need = ws_npart(g, w->nbr, extra_parts);
    if (need > w->npart) {
        ws_drop_graphs(w);
        (void)hipFree(w->part);
        w->part = nullptr;
        if (hipMalloc(&w->part, sizeof(double) * 8 * (size_t)need * w->nrhs_cap) != hipSuccess) return UNO_ERR_NOMEM;
        w->npart = need;
    }
    if (plan && (plan->nspec > w->nspec || w->spec_cap < w->nrhs_cap)) {
        ws_drop_graphs(w);
        (void)hipFree(w->spec);
        w->spec = nullptr;
        w->nspec = w->spec_cap = 0;
        if (hipMalloc(&w->spec, sizeof(double2) * (size_t)plan->nspec * w->nrhs_cap) != hipSuccess)
            return UNO_ERR_NOMEM;
        w->nspec = plan->nspec;
        w->spec_cap = w->nrhs_cap;
    }
    if (lr) {
        int64_t ngp = 0, nh = 0;
        lowrank_scratch_size(lr, &ngp, &nh);
        if (ngp != w->lr_ngp || nh != w->lr_nh || w->lr_cap < w->nrhs_cap) {
            ws_drop_graphs(w);
            (void)hipFree(w->lr_gp);
            (void)hipFree(w->lr_h);
            w->lr_gp = w->lr_h = nullptr;
            w->lr_cap = 0;
            if (hipMalloc(&w->lr_gp, sizeof(double2) * (size_t)ngp * w->nrhs_cap) != hipSuccess ||
                hipMalloc(&w->lr_h, sizeof(double2) * (size_t)nh * w->nrhs_cap) != hipSuccess)
                return UNO_ERR_NOMEM;
            w->lr_ngp = ngp;
            w->lr_nh = nh;
            w->lr_cap = w->nrhs_cap;
        }
    }
    if (hist_need > w->hist_cap) {
        ws_drop_graphs(w);
        (void)hipFree(w->hist);
        (void)hipFree(w->gam);
        w->hist = w->gam = nullptr;
        w->hist_cap = 0;
        if (hipMalloc(&w->hist, sizeof(double) * (size_t)hist_need * w->nrhs_cap) != hipSuccess) return UNO_ERR_NOMEM;
        if (hipMalloc(&w->gam, sizeof(double) * (size_t)hist_need * w->nrhs_cap) != hipSuccess) return UNO_ERR_NOMEM;
        w->hist_cap = hist_need;
    }
    *out = w;
    return UNO_OK;
}

}  // namespace

uno_status ws_release_all()
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (Workspace* w : g_ws) {
        { std::lock_guard<std::mutex> wl(w->mu); }  // a solve still holding it finishes first
        ws_free(w);
    }
    g_ws.clear();
    return UNO_OK;
}

namespace {

// partial buffers of right-hand side 0 (right-hand side b: + b npart)
struct Parts {
    double* rmax;
    double* rs[2];
    double* dp;
    double* ss[2];  // sum(s), by pass parity
    double* ds[2];  // sum(d_new), by the parity of the d buffer
};

Parts parts_of(Workspace* w)
{
    Parts P;
    const size_t np = (size_t)w->npart * w->nrhs_cap;
    P.rmax = w->part;
    P.rs[0] = w->part + np;
    P.rs[1] = w->part + 2 * np;
    P.dp = w->part + 3 * np;
    P.ss[0] = w->part + 4 * np;
    P.ss[1] = w->part + 5 * np;
    P.ds[0] = w->part + 6 * np;
    P.ds[1] = w->part + 7 * np;
    return P;
}

// np_update: workgroups of the update kernel (they write the ||r||_inf
// partials read at the head of pass k > kr; pass kr, the last pass whose
// residual the init kernel took (0, a residual replacement or a restart),
// reads the init kernel's)
CgIter iter_of(Workspace* w, const Parts& P, int k, int k0, int kr, double rtol, int hist_len, int np_update,
               int64_t ks)
{
    CgIter it;
    memset(&it, 0, sizeof(it));
    it.k = k;
    it.k0 = k0;
    it.st = w->state;
    it.part_rmax = P.rmax;
    it.np_rmax = (k == kr) ? w->nbr : np_update;
    it.rtol = rtol;
    it.hist = w->hist;
    it.hist_len = hist_len;
    it.r = w->r;
    it.part_rs = P.rs[k & 1];
    it.part_ssum = P.ss[k & 1];
    it.vs = w->total;
    it.ps = w->npart;
    it.hs = w->hist_cap;
    it.ks = ks;
    it.kdev = w->capture_kdev;
    return it;
}

LrBatch lr_batch(Workspace* w, const uno_precond* pc, int nrhs)
{
    LrBatch b = lowrank_batch(pc->lr, w->lr_gp, w->lr_h, nrhs);
    b.bf = w->lr_bf;
    return b;
}

}  // namespace

// One CG pass k for nrhs right-hand sides (grid y).  T: precision of the
// operator / preconditioner vectors (s, d, p, conductivities, D^-1); r, u
// and every reduction stay FP64.
template <typename T>
static uno_status enqueue_pass(const Grid& g, Workspace* w, int kind, const uno_precond* pc, const T* kappa,
                               int64_t ks, double* u, int k, int k0, int kr, double rtol, int hist_len, int nrhs,
                               hipStream_t st)
{
    const Parts P = parts_of(w);
    const int nb = w->nbr;
    T* dold = (T*)w->d[k & 1];
    T* dnew = (T*)w->d[(k + 1) & 1];
    T* sv = (T*)w->s;
    T* pv = (T*)w->p;
    int np_rs = nb;
    const MeanFree mf{P.ss[k & 1], P.ds[k & 1], P.ds[(k + 1) & 1]};
    if (kind == UNO_PREC_UNO && uno_use_lowrank(pc)) {
        CgIter it = iter_of(w, P, k, k0, kr, rtol, hist_len, lowrank_update_blocks(pc->lr, nrhs), ks);
        const LrBatch bt = lr_batch(w, pc, nrhs);
        if constexpr (sizeof(T) == sizeof(double)) {
            if (uno_use_fused(pc)) {
                // fused FP64 flow: B (head, Parseval partials) -> [C + matvec] -> [update + A of pass k+1];
                // ||r||^2 partials in rs[0], the learned-mode part of r.s in rs[1]
                int np_dp = 0;
                uno_status e = lowrank_fused_pass(pc->lr, g, (const double*)kappa, w->r, (const double*)dold,
                                                  (double*)dnew, (double*)pv, P.dp, it, P.rs[1], P.rs[0], w->gam, bt,
                                                  st, &np_dp);
                if (e != UNO_OK) return e;
                return lowrank_update_forward<double>(pc->lr, w->r, u, (const double*)dnew, (const double*)pv, it, P.dp,
                                                      np_dp, w->gam, P.rmax, P.rs[0], bt, st);
            }
        }
        // learned-mode flow: [B (head) + C] -> matvec -> [update + A of pass k+1]
        uno_status e = lowrank_finish<T>(pc->lr, w->r, sv, &it, &np_rs, bt, st);
        if (e != UNO_OK) return e;
        const int np_dp = launch_tile<T, true, false>(g, kappa, sv, dold, dnew, pv, P.dp, it, P.rs[k & 1], np_rs,
                                                      w->gam, st, mf, nrhs);
        UNO_HIP(hipGetLastError());
        return lowrank_update_forward<T>(pc->lr, w->r, u, dnew, pv, it, P.dp, np_dp, w->gam, P.rmax, nullptr, bt, st);
    }
    CgIter it = iter_of(w, P, k, k0, kr, rtol, hist_len, nb, ks);
    if (kind == UNO_PREC_UNO) {
        if (sizeof(T) != sizeof(double)) return UNO_ERR_ARG;  // spectral passes: FP64
        uno_status e = uno_apply_passes(g, pc->plan, pc->table, UNO_F64, w->r, w->s, UNO_F64, w->spec, &it, &np_rs, st,
                                        nrhs, w->nspec);
        if (e != UNO_OK) return e;
    }
    int np_dp;
    if (kind == UNO_PREC_UNO)
        np_dp = launch_tile<T, true, false>(g, kappa, sv, dold, dnew, pv, P.dp, it, P.rs[k & 1], np_rs, w->gam, st, mf,
                                            nrhs);
    else
        np_dp = launch_tile<T, true, true>(g, kappa, sv, dold, dnew, pv, P.dp, it, P.rs[k & 1], np_rs, w->gam, st, mf,
                                           nrhs);
    UNO_HIP(hipGetLastError());
    double* rs_next = P.rs[(k + 1) & 1];
    double* ss_next = P.ss[(k + 1) & 1];
    const T* dinv = (const T*)w->dinv;
    const dim3 grid(nb, nrhs);
    if (kind == UNO_PREC_NONE)
        uno_launch(UNO_KT_UPDATE, k_cg_update<T, 0>, grid, dim3(kBlock), 0, st, g.dev, dinv, w->r, u, (const T*)dnew,
                   (const T*)pv, sv, it, (const double*)P.dp, np_dp, (const double*)w->gam, P.rmax, rs_next, ss_next);
    else if (kind == UNO_PREC_JACOBI)
        uno_launch(UNO_KT_UPDATE, k_cg_update<T, 1>, grid, dim3(kBlock), 0, st, g.dev, dinv, w->r, u, (const T*)dnew,
                   (const T*)pv, sv, it, (const double*)P.dp, np_dp, (const double*)w->gam, P.rmax, rs_next, ss_next);
    else
        uno_launch(UNO_KT_UPDATE, k_cg_update<T, 2>, grid, dim3(kBlock), 0, st, g.dev, dinv, w->r, u, (const T*)dnew,
                   (const T*)pv, sv, it, (const double*)P.dp, np_dp, (const double*)w->gam, P.rmax, rs_next, ss_next);
    UNO_HIP(hipGetLastError());
    return UNO_OK;
}

// Residual replacement of the FP32 mode: when ||r|| has dropped by this
// factor since the last replacement, r is recomputed as f - A u in FP64 and
// the recurrence continues with it (the search direction is kept: the
// replaced residual differs from the recursive one by the FP32 operator's
// rounding only, so the directions stay conjugate to that accuracy and no
// Krylov space is lost, the reliable update of van der Vorst and Ye).  FP32
// stencil sums lose accuracy on smooth directions (cancellation ~ 1e-7
// cond(A)); the replacement keeps the recursive residual equal to the true
// one.  The factor was chosen by measurement when a replacement also
// restarted the direction (64^3 x 48 loads to 1e-6, FP32 ms per solve:
// 1e-1.5 0.81, 1e-2 0.73, 1e-2.5 0.94, 1e-3 0.83, 1e-4 0.77, 1e-5 0.85);
// short cycles also keep the last cycle's drift small.
constexpr double kRestartFactor = 1e-2;

// r = f - A u in FP64 for every right-hand side (A u goes to p, which the
// next pass rewrites anyway)
static void replace_residual(const Grid& g, Workspace* w, const double* kappa64, const double* u, int64_t ks,
                             int nrhs, hipStream_t st)
{
    CgIter bi;
    memset(&bi, 0, sizeof(bi));
    bi.vs = g.total;
    bi.ks = ks;
    launch_tile<double, false, false>(g, kappa64, u, nullptr, nullptr, (double*)w->p, nullptr, bi, nullptr, 0,
                                      nullptr, st, MeanFree{nullptr, nullptr, nullptr}, nrhs);
    hipLaunchKernelGGL(k_sub, dim3(w->nbr), dim3(kBlock), 0, st, g.total * nrhs, (const double*)w->f,
                       (const double*)w->p, w->r);
}

// Host side of the chunked CG loop (thermal and elastic).  pass(k, k0, kr)
// enqueues CG pass k of the cycle that started at pass k0 (d = s there),
// the residual last taken by the init kernel at pass kr; check(k, k0, kr)
// the convergence test after a chunk's last pass; the host reads the loop
// states between chunks.  FP32 mode (restarts): residual() forms
// r = f - A u in FP64 (the product in w->p), start(reset, k) takes the
// residual in w->r at pass k (s = P r and the partials pass k reads),
// true_res() writes ||f - A u||_inf and ||f||_inf of the product in w->p
// into the states.  A residual replacement replaces the residual of every
// running right-hand side together (at one pass index kr for all) as soon
// as one of them has dropped by kRestartFactor since its last replacement;
// the search directions continue, and loads that have ended keep their
// state.  When every load has ended, a load whose true residual is still
// above its tolerance (the recursive residual of the last cycle drifts from
// it by the FP32 operator's rounding) is reopened from that residual, with
// a restarted direction (k0 = k: its d is that of its last pass).
// Graph mode (key non-empty): after the first chunk, passes run as replays
// of one captured chunk of kGraphPasses passes (recorded once per
// workspace and key, the key holding every argument the passes are
// recorded with besides the workspace's own buffers); its kernels read the
// index of the chunk's first pass from w->kdev, which the last node
// advances.  Chunks then start at even pass indices, so the buffers chosen
// by pass parity are those of the recorded offsets.
constexpr int kGraphPasses = 8;

template <class Pass>
static uno_status graph_exec(Workspace* w, const std::vector<int64_t>& key, Pass pass, hipStream_t st,
                             hipGraphExec_t* out)
{
    for (auto& gr : w->graphs)
        if (gr.key == key) {
            *out = gr.exec;
            return UNO_OK;
        }
    if (w->graphs.size() >= 8) {  // a few live (grid, operand) combinations per stream
        (void)hipGraphExecDestroy(w->graphs.front().exec);
        w->graphs.erase(w->graphs.begin());
    }
    // recorded on a stream of the workspace's own (the caller's may be the
    // null stream, which cannot be captured); replayed on the caller's
    if (!w->capture_stream) UNO_HIP(hipStreamCreateWithFlags(&w->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = w->capture_stream;
    hipGraph_t graph = nullptr;
    UNO_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    w->capture_kdev = w->kdev;
    uno_status e = UNO_OK;
    // recorded at offsets 0 .. kGraphPasses - 1 with k0 = -1: every captured
    // pass lies past the first pass of its cycle
    for (int j = 0; j < kGraphPasses && e == UNO_OK; ++j) e = pass(j, -1, -1, cs);
    if (e == UNO_OK) hipLaunchKernelGGL(k_advance_pass, dim3(1), dim3(64), 0, cs, w->kdev, kGraphPasses);
    w->capture_kdev = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (e != UNO_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return e;
    }
    UNO_HIP(ec);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    UNO_HIP(ei);
    w->graphs.push_back(Workspace::Graph{key, exec});
    *out = exec;
    return UNO_OK;
}

template <class Pass, class Check, class Residual, class Start, class TrueRes>
static uno_status run_chunks(Workspace* w, const uno_solve_opts* o, int nrhs, bool restarts, hipStream_t st,
                             Pass pass, Check check, Residual residual, Start start, TrueRes true_res, int* k_end,
                             const std::vector<int64_t>& graph_key = {})
{
    const int chunk0 = o->graph_chunk > 0 ? o->graph_chunk : 8;
    const bool graphs = !graph_key.empty() && w->kdev && !restarts && chunk0 % 2 == 0;
    int k = 0, k0 = 0, kr = 0, chunk = chunk0;
    std::vector<int> prev_k(nrhs, -1);
    std::vector<double> prev_r(nrhs, -1.0);
    std::vector<double> cycle_r(nrhs, -1.0);
    auto read_states = [&]() -> uno_status {
        UNO_HIP(hipMemcpyAsync(w->host_state, w->state, sizeof(CgState) * nrhs, hipMemcpyDeviceToHost, st));
        UNO_HIP(hipStreamSynchronize(st));
        return UNO_OK;
    };
    auto live = [](const CgState& hs) { return hs.status == 0 && hs.done == INT_MAX; };
    uno_status e = UNO_OK;
    for (;;) {
        if (chunk > o->max_iter - k) chunk = o->max_iter - k;
        int c = 0;
        if (graphs && k >= chunk0) {
            const int m = chunk / kGraphPasses;
            if (m > 0) {
                hipGraphExec_t exec;
                if ((e = graph_exec(w, graph_key, pass, st, &exec)) != UNO_OK) return e;
                hipLaunchKernelGGL(k_set_pass, dim3(1), dim3(64), 0, st, w->kdev, k);
                UNO_HIP(hipGetLastError());
                for (int r = 0; r < m; ++r) UNO_HIP(hipGraphLaunch(exec, st));
                c = m * kGraphPasses;
                k += c;
            }
        }
        for (; c < chunk; ++c, ++k) {
            e = pass(k, k0, kr, st);
            if (e != UNO_OK) return e;
        }
        check(k, k0, kr);
        UNO_HIP(hipGetLastError());
        if ((e = read_states()) != UNO_OK) return e;
        bool running = false;
        for (int b = 0; b < nrhs; ++b)
            if (live(w->host_state[b])) running = true;
        if (!running && restarts && k < o->max_iter) {
            // exit check of the FP32 mode
            residual();
            true_res();
            UNO_HIP(hipGetLastError());
            if ((e = read_states()) != UNO_OK) return e;
            bool reopen = false;
            for (int b = 0; b < nrhs; ++b) {
                CgState& hs = w->host_state[b];
                if (hs.status != 0 || hs.done == INT_MAX || !(hs.dmax > hs.tol_abs)) continue;
                hs.done = INT_MAX;
                cycle_r[b] = hs.dmax;
                prev_r[b] = -1.0;
                reopen = true;
            }
            if (reopen) {
                UNO_HIP(hipMemcpyAsync(w->state, w->host_state, sizeof(CgState) * nrhs, hipMemcpyHostToDevice, st));
                if ((e = start(0, k)) != UNO_OK) return e;
                k0 = kr = k;
                chunk = chunk0;
                continue;
            }
        }
        if (!running || k >= o->max_iter) break;
        if (restarts) {
            bool due = false;
            for (int b = 0; b < nrhs; ++b) {
                const CgState& hs = w->host_state[b];
                if (!live(hs)) continue;
                if (cycle_r[b] < 0.0) cycle_r[b] = hs.r0max;
                if (hs.rmax_last <= kRestartFactor * cycle_r[b]) due = true;
            }
            if (due) {
                // residual replacement, every load at once, at pass k; the
                // search direction continues (k0 kept)
                residual();
                for (int b = 0; b < nrhs; ++b) {
                    const CgState& hs = w->host_state[b];
                    if (!live(hs)) continue;
                    cycle_r[b] = hs.rmax_last;
                    prev_r[b] = -1.0;
                }
                if ((e = start(0, k)) != UNO_OK) return e;
                kr = k;
                chunk = chunk0;
                continue;
            }
        }
        if (o->graph_chunk <= 0) {
            // predict the passes still needed from the observed contraction
            // rate; the slowest running right-hand side decides.  Three
            // quarters of the prediction: a pass launched after every load
            // has ended costs about as much as one more host check, and the
            // rate over one chunk is noisy (64^3 x 48 loads: 112 passes
            // launched for 106 needed, against 127 with a 5 % margin).  A
            // chunk is at most twice the last one: the maximum norm of a CG
            // residual can stall over a chunk, and a rate near 1 would
            // otherwise launch up to 256 passes past the last load's end
            // (measured in the FP32 mode: 337 launches for 106 passes)
            int next = 2;
            for (int b = 0; b < nrhs; ++b) {
                const CgState& hs = w->host_state[b];
                if (!live(hs)) continue;
                double target = hs.tol_abs;
                if (restarts) {
                    const double lvl = kRestartFactor * cycle_r[b];
                    if (lvl > target) target = lvl;
                }
                int nx = 16;
                if (prev_r[b] > 0.0 && hs.rmax_last > 0.0 && hs.k_last > prev_k[b] && hs.rmax_last < prev_r[b]) {
                    const double rate = std::pow(hs.rmax_last / prev_r[b], 1.0 / (hs.k_last - prev_k[b]));
                    const double need = std::log(target / hs.rmax_last) / std::log(rate);
                    nx = (int)std::ceil(need * 0.75);
                }
                if (nx > next) next = nx;
            }
            if (next > 2 * chunk) next = 2 * chunk;
            chunk = next < 2 ? 2 : (next > 256 ? 256 : next);
            if (graphs) chunk = (chunk + kGraphPasses - 1) / kGraphPasses * kGraphPasses;
        }
        for (int b = 0; b < nrhs; ++b) {
            prev_k[b] = w->host_state[b].k_last;
            prev_r[b] = w->host_state[b].rmax_last;
        }
    }
    *k_end = k;
    return UNO_OK;
}

// The CG loop for nrhs right-hand sides.  FP32 mode: the residual of every
// running right-hand side is replaced together (one pass index for all) as
// soon as one of them has dropped by the restart factor since its last
// replacement; search directions continue, and loads that have ended keep
// their state.
template <typename T>
static uno_status pcg_loop(const Grid& g, Workspace* w, const double* kappa64, const T* kappa, int64_t ks,
                           double* u, const uno_solve_opts* o, const uno_precond* pc, int hist_len, int nrhs,
                           hipStream_t st, int* k_end)
{
    const int nb = w->nbr;
    const Parts P = parts_of(w);
    T* sv = (T*)w->s;
    T* dinv = (T*)w->dinv;
    const bool lowrank = pc && uno_use_lowrank(pc);
    const int np_update = lowrank ? lowrank_update_blocks(pc->lr, nrhs) : nb;
    const bool restarts = sizeof(T) == sizeof(float);
    if (o->kind == UNO_PREC_JACOBI)  // one inverse diagonal per conductivity field
        for (int b = 0; b < (ks ? nrhs : 1); ++b)
            hipLaunchKernelGGL(k_inv_diag<T>, dim3(nb), dim3(kBlock), 0, st, g.dev, kappa64 + b * ks, dinv + b * ks);
    // (re)start of the recurrence at pass kk from the residual in w->r:
    // s = P r and the partials pass kk reads (r.s and sum(s) in the buffers
    // of kk's parity)
    auto start = [&](int reset, int kk) -> uno_status {
        const dim3 grid(nb, nrhs);
        double* rs0 = P.rs[kk & 1];
        double* ss0 = P.ss[kk & 1];
        if (o->kind == UNO_PREC_NONE)
            hipLaunchKernelGGL((k_cg_init<T, 0>), grid, dim3(kBlock), 0, st, g.dev, (const T*)dinv,
                               (const double*)w->r, sv, P.rmax, rs0, ss0, w->state, w->npart, ks, reset);
        else if (o->kind == UNO_PREC_JACOBI)
            hipLaunchKernelGGL((k_cg_init<T, 1>), grid, dim3(kBlock), 0, st, g.dev, (const T*)dinv,
                               (const double*)w->r, sv, P.rmax, rs0, ss0, w->state, w->npart, ks, reset);
        else
            hipLaunchKernelGGL((k_cg_init<T, 2>), grid, dim3(kBlock), 0, st, g.dev, (const T*)dinv,
                               (const double*)w->r, sv, P.rmax, rs0, ss0, w->state, w->npart, ks, reset);
        UNO_HIP(hipGetLastError());
        if (lowrank) {  // transform of r for the first pass (and ||r||^2 in the fused flow)
            const bool fused = sizeof(T) == sizeof(double) && uno_use_fused(pc);
            const CgIter strides = iter_of(w, P, 0, 0, 0, 0.0, 0, nb, ks);
            return lowrank_forward(pc->lr, w->r, fused ? P.rs[0] : nullptr, lr_batch(w, pc, nrhs), strides, st);
        }
        return UNO_OK;
    };
    uno_status e = start(1, 0);
    if (e != UNO_OK) return e;
    auto pass = [&](int k, int k0, int kr, hipStream_t sp) {
        return enqueue_pass<T>(g, w, o->kind, pc, kappa, ks, u, k, k0, kr, o->rtol, hist_len, nrhs, sp);
    };
    auto check = [&](int k, int k0, int kr) {
        const CgIter it = iter_of(w, P, k, k0, kr, o->rtol, hist_len, np_update, ks);
        hipLaunchKernelGGL(k_cg_check, dim3(1, nrhs), dim3(kBlock), 0, st, it);
    };
    auto residual = [&]() { replace_residual(g, w, kappa64, u, ks, nrhs, st); };
    auto true_res = [&]() {
        hipLaunchKernelGGL(k_resid_parts_b, dim3(nb, nrhs), dim3(kBlock), 0, st, g.total, (const double*)w->f,
                           (const double*)w->p, P.rs[0], P.rs[1], g.total, w->npart);
        hipLaunchKernelGGL(k_resid_final_b, dim3(1, nrhs), dim3(kBlock), 0, st, (const double*)P.rs[0],
                           (const double*)P.rs[1], nb, w->state, w->npart);
    };
    std::vector<int64_t> key;
    if (o->use_graphs && !restarts && !ktimer_active() && (!pc || lowrank)) {
        int64_t rt;
        memcpy(&rt, &o->rtol, sizeof(rt));
        key = {1, (int64_t)sizeof(T), o->kind, pc ? (int64_t)pc->serial : 0, pc ? pc->path : -1, nrhs, ks,
               (int64_t)(uintptr_t)kappa, (int64_t)(uintptr_t)kappa64, (int64_t)(uintptr_t)u, hist_len, rt};
    }
    return run_chunks(w, o, nrhs, restarts, st, pass, check, residual, start, true_res, k_end, key);
}

static uno_status pcg_run_ws(const Grid& g, Workspace* w, bool may_alloc, const double* kappa, int64_t ks, int nrhs,
                             const double* macro_loads3, const double* rhs, double* u, const uno_solve_opts* o,
                             uno_solve_info* info, double* res_hist, hipStream_t st);

// nrhs solves with one operator (and preconditioner); load b: macro_loads +
// 3 b (or rhs + b n), solution u + b n, info[b]
uno_status pcg_run_batch(const Grid& g, const double* kappa, int64_t ks, int nrhs, const double* macro_loads3,
                         const double* rhs, double* u, const uno_solve_opts* o, uno_solve_info* info, double* res_hist,
                         hipStream_t st)
{
    const uno_precond* pc = (o->kind == UNO_PREC_UNO) ? o->uno : nullptr;
    const bool mixed = (o->op_t == UNO_F32);
    if (mixed && pc && !uno_use_lowrank(pc)) return UNO_ERR_ARG;
    // BF16 mode: the FP32 mode with the learned-mode passes' table and
    // spectrum stored in BF16 (one nodal DOF)
    if (o->prec_t == UNO_BF16 && (!mixed || !pc || pc->nc != 1)) return UNO_ERR_ARG;
    // one loop for all right-hand sides, every pass kernel taking them along
    // grid y (the spectral passes too)
    Workspace* w = nullptr;
    std::unique_lock<std::mutex> lease;
    uno_status e = ws_get(g, pc ? &pc->plan : nullptr, pc ? pc->lr : nullptr, pc ? pc->rs_blocks : 0, o->max_iter + 1,
                          nrhs, st, &lease, &w);
    if (e != UNO_OK) return e;
    return pcg_run_ws(g, w, true, kappa, ks, nrhs, macro_loads3, rhs, u, o, info, res_hist, st);
}

// The solve of pcg_run_batch on a workspace sized for it (may_alloc: the
// FP32 conductivities may be allocated on demand; otherwise w holds them).
static uno_status pcg_run_ws(const Grid& g, Workspace* w, bool may_alloc, const double* kappa, int64_t ks, int nrhs,
                             const double* macro_loads3, const double* rhs, double* u, const uno_solve_opts* o,
                             uno_solve_info* info, double* res_hist, hipStream_t st)
{
    const uno_precond* pc = (o->kind == UNO_PREC_UNO) ? o->uno : nullptr;
    const bool mixed = (o->op_t == UNO_F32);
    if (o->prec_t == UNO_BF16 && (!mixed || !pc || pc->nc != 1 || !uno_use_lowrank(pc))) return UNO_ERR_ARG;
    w->lr_bf = o->prec_t == UNO_BF16;  // (the workspace is leased to this solve)
    const int hist_len = o->max_iter + 1;
    uno_status e = UNO_OK;
    const int nb = w->nbr;
    const Parts P = parts_of(w);
    const int64_t n = g.total;
    // rhs and initial residual r_0 = f - A u_0 (FP64), every right-hand side
    // in one launch each
    CgIter bi;
    memset(&bi, 0, sizeof(bi));
    bi.vs = n;
    bi.ks = ks;
    if (macro_loads3) {
        for (int b0 = 0; b0 < nrhs; b0 += kLoads3) {  // the loads travel as a kernel argument, kLoads3 a launch
            const int m = std::min(kLoads3, nrhs - b0);
            Loads3 L;
            memset(&L, 0, sizeof(L));
            for (int b = 0; b < m; ++b)
                for (int a = 0; a < 3; ++a) L.g[b][a] = macro_loads3[3 * (b0 + b) + a];
            hipLaunchKernelGGL(k_rhs_batch, dim3(nb, m), dim3(kBlock), 0, st, g.dev, kappa + b0 * ks, ks, L,
                               w->f + (int64_t)b0 * n);
        }
    } else {
        UNO_HIP(hipMemcpyAsync(w->f, rhs, sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, st));
    }
    launch_tile<double, false, false>(g, kappa, u, nullptr, nullptr, w->p, nullptr, bi, nullptr, 0, nullptr, st,
                                      MeanFree{nullptr, nullptr, nullptr}, nrhs);
    hipLaunchKernelGGL(k_sub, dim3(nb), dim3(kBlock), 0, st, n * nrhs, (const double*)w->f, (const double*)w->p,
                       w->r);
    UNO_HIP(hipGetLastError());
    int k = 0;
    if (mixed) {
        // FP32 conductivities: one field, or one per right-hand side
        const int nf = ks ? nrhs : 1;
        if (w->kap32_cap < nf) {
            if (!may_alloc) return UNO_ERR_SHAPE;
            ws_drop_graphs(w);
            (void)hipFree(w->kap32);
            w->kap32 = nullptr;
            w->kap32_cap = 0;
            if (hipMalloc(&w->kap32, sizeof(float) * n * nf) != hipSuccess) return UNO_ERR_NOMEM;
            w->kap32_cap = nf;
        }
        for (int b = 0; b < nf; ++b)
            hipLaunchKernelGGL(k_convert<float>, dim3(nb), dim3(kBlock), 0, st, n, kappa + b * ks, w->kap32 + b * n);
        e = pcg_loop<float>(g, w, kappa, w->kap32, ks, u, o, pc, hist_len, nrhs, st, &k);
    } else {
        e = pcg_loop<double>(g, w, kappa, kappa, ks, u, o, pc, hist_len, nrhs, st, &k);
    }
    if (e != UNO_OK) return e;
    std::vector<CgState> hs(w->host_state, w->host_state + nrhs);
    // zero-mean fluctuation (Sec. 5.1) and the true residual in FP64, every
    // right-hand side in one launch each
    {
        const dim3 grid(nb, nrhs);
        const int ps = w->npart;
        hipLaunchKernelGGL(k_sum_parts_b, grid, dim3(kBlock), 0, st, n, (const double*)u, P.dp, n, ps);
        hipLaunchKernelGGL(k_sub_mean_b, grid, dim3(kBlock), 0, st, n, u, (const double*)P.dp, nb, w->state, n, ps);
        launch_tile<double, false, false>(g, kappa, u, nullptr, nullptr, w->p, nullptr, bi, nullptr, 0, nullptr, st,
                                          MeanFree{nullptr, nullptr, nullptr}, nrhs);
        hipLaunchKernelGGL(k_resid_parts_b, grid, dim3(kBlock), 0, st, n, (const double*)w->f, (const double*)w->p,
                           P.rs[0], P.rs[1], n, ps);
        hipLaunchKernelGGL(k_resid_final_b, dim3(1, nrhs), dim3(kBlock), 0, st, (const double*)P.rs[0],
                           (const double*)P.rs[1], nb, w->state, ps);
        UNO_HIP(hipGetLastError());
    }
    UNO_HIP(hipMemcpyAsync(w->host_state, w->state, sizeof(CgState) * nrhs, hipMemcpyDeviceToHost, st));
    const int iters0 = (hs[0].done != INT_MAX) ? hs[0].done : (hs[0].status != 0 ? hs[0].fail_iter : k);
    if (res_hist && nrhs == 1) {
        int nh = iters0 + 1;
        if (nh > hist_len) nh = hist_len;
        UNO_HIP(hipMemcpyAsync(res_hist, w->hist, sizeof(double) * nh, hipMemcpyDeviceToHost, st));
    }
    UNO_HIP(hipStreamSynchronize(st));
    bool failed = false;
    for (int b = 0; b < nrhs; ++b) {
        const CgState& h = hs[b];
        const CgState& fin = w->host_state[b];
        if (h.status != 0) failed = true;
        if (info) {
            uno_solve_info& I = info[b];
            I.iters = (h.done != INT_MAX) ? h.done : (h.status != 0 ? h.fail_iter : k);
            I.converged = (h.status == 0 && h.done != INT_MAX) ? 1 : 0;
            I.rel_res = h.r0max > 0.0 ? h.rmax_last / h.r0max : 0.0;
            I.true_rel_res = fin.fmax > 0.0 ? fin.dmax / fin.fmax : 0.0;
            I.r0_norm = h.r0max;
        }
    }
    return failed ? UNO_ERR_BREAKDOWN : UNO_OK;
}

// ---------------------------------------------------------------------------
// Linear elasticity (c = 3, Sec. 5.2): Jacobi-CG, plain CG or UNO-CG on the
// planar 3n-vectors, nrhs macroscopic strains carried by every pass kernel.
// The update and init kernels run on the 3n-vector as on a scalar field; the
// operator is the elastic march (it tests convergence at the head of the
// pass unless the UNO passes do).  lks: stride of the Lame fields per
// right-hand side (0 if shared).  FP32 mode (UNO only): s, d, p and the Lame
// fields in FP32, r, u, reductions and the stop test in FP64, with the
// thermal mode's residual replacement and exit check (r = f - A u by the
// FP64 operator).

// per-component mean of the 3n-vectors v + b N (b < nrhs) removed
static void el_remove_means(Workspace* w, const Parts& P, double* v, int64_t n, int nrhs, hipStream_t st)
{
    const int nb = w->nbr;
    for (int b = 0; b < nrhs; ++b) {
        double* pd = P.dp + (int64_t)b * w->npart;
        for (int c = 0; c < 3; ++c) {
            double* vc = v + b * 3 * n + c * n;
            hipLaunchKernelGGL(k_sum_parts, dim3(nb), dim3(kBlock), 0, st, n, (const double*)vc, pd);
            hipLaunchKernelGGL(k_sub_mean, dim3(nb), dim3(kBlock), 0, st, n, vc, (const double*)pd, nb, w->state + b);
        }
    }
}

// r = f - A u (FP64) for every right-hand side, A u in w->p
static uno_status el_residual(const ElDev& E, const Grid& g, Workspace* w, const double* lam, const double* mu,
                              int64_t lks, const double* u, int nrhs, hipStream_t st)
{
    const int64_t N = 3 * g.total;
    CgIter none;
    memset(&none, 0, sizeof(none));
    for (int b = 0; b < nrhs; ++b) {
        uno_status e = launch_el_apply<double, false, false>(E, g, lam + b * lks, mu + b * lks, 0, u + b * N, nullptr,
                                                             nullptr, w->p + b * N, nullptr, none, nullptr, 0,
                                                             nullptr, 1, st);
        if (e != UNO_OK) return e;
    }
    hipLaunchKernelGGL(k_sub, dim3(w->nbr), dim3(kBlock), 0, st, N * nrhs, (const double*)w->f, (const double*)w->p,
                       w->r);
    return hip_status(hipGetLastError());
}

template <typename T>
static uno_status el_loop(const ElDev& E, const Grid& g, const GridDev& gd, Workspace* w, const double* lam,
                          const double* mu, const T* lamT, const T* muT, int64_t lks, double* u,
                          const uno_solve_opts* o, const uno_precond* pc, int nrhs, hipStream_t st, int* k_end)
{
    const int nb = w->nbr;
    const Parts P = parts_of(w);
    const int hist_len = o->max_iter + 1;
    const int64_t dks = lks ? 3 * g.total : 0;  // Jacobi diagonals follow the Lame fields
    const bool restarts = sizeof(T) == sizeof(float);
    T* sv = (T*)w->s;
    T* pv = (T*)w->p;
    LrBatch bt{};
    int np_update = nb;
    if (pc) {
        bt = lowrank_batch(pc->lr, w->lr_gp, w->lr_h, nrhs);
        np_update = lowrank_update_blocks(pc->lr, nrhs);
    }
    // (re)start at pass kk from w->r: ||r||_inf partials (and s_0 = P r_0 for
    // Jacobi / none, r.s into the partials of kk's parity), the UNO flow's
    // first transform
    auto start = [&](int reset, int kk) -> uno_status {
        const dim3 grid(nb, nrhs);
        double* rs0 = P.rs[kk & 1];
        double* ss0 = P.ss[kk & 1];
        if (o->kind == UNO_PREC_JACOBI)
            hipLaunchKernelGGL((k_cg_init<T, 1>), grid, dim3(kBlock), 0, st, gd, (const T*)w->dinv,
                               (const double*)w->r, sv, P.rmax, rs0, ss0, w->state, w->npart, dks, reset);
        else if (o->kind == UNO_PREC_UNO)
            hipLaunchKernelGGL((k_cg_init<T, 2>), grid, dim3(kBlock), 0, st, gd, (const T*)w->dinv,
                               (const double*)w->r, sv, P.rmax, rs0, ss0, w->state, w->npart, dks, reset);
        else
            hipLaunchKernelGGL((k_cg_init<T, 0>), grid, dim3(kBlock), 0, st, gd, (const T*)w->dinv,
                               (const double*)w->r, sv, P.rmax, rs0, ss0, w->state, w->npart, dks, reset);
        UNO_HIP(hipGetLastError());
        if (pc) return lowrank_forward(pc->lr, w->r, nullptr, bt, iter_of(w, P, 0, 0, 0, 0.0, 0, nb, dks), st);
        return UNO_OK;
    };
    uno_status e = start(1, 0);
    if (e != UNO_OK) return e;
    // UNO flow per pass: [B (head) + C: s = P r, r.s] -> [d = s + beta d, p = A d, d.p]
    // -> [update + pass A of the next pass]
    auto pass = [&](int k, int k0, int kr, hipStream_t sp) -> uno_status {
        CgIter it = iter_of(w, P, k, k0, kr, o->rtol, hist_len, np_update, dks);
        T* dold = (T*)w->d[k & 1];
        T* dnew = (T*)w->d[(k + 1) & 1];
        if (pc) {
            int np_rs = 0;
            uno_status e2 = lowrank_finish<T>(pc->lr, w->r, sv, &it, &np_rs, bt, sp);
            if (e2 != UNO_OK) return e2;
            e2 = launch_el_apply<T, true, false>(E, g, lamT, muT, lks, sv, dold, dnew, pv, P.dp, it, P.rs[k & 1],
                                                 np_rs, w->gam, nrhs, sp);
            if (e2 != UNO_OK) return e2;
            return lowrank_update_forward<T>(pc->lr, w->r, u, (const T*)dnew, (const T*)pv, it, P.dp,
                                             el_march_blocks(g, nrhs), w->gam, P.rmax, nullptr, bt, sp);
        }
        if constexpr (sizeof(T) == sizeof(double)) {
            uno_status e2 = launch_el_apply<double, true, true>(E, g, lam, mu, lks, w->s, (const double*)dold,
                                                                (double*)dnew, w->p, P.dp, it, P.rs[k & 1], nb,
                                                                w->gam, nrhs, sp);
            if (e2 != UNO_OK) return e2;
            const int np_dp = el_march_blocks(g, nrhs);
            double* rs_next = P.rs[(k + 1) & 1];
            double* ss_next = P.ss[(k + 1) & 1];
            const dim3 grid(nb, nrhs);
            if (o->kind == UNO_PREC_JACOBI)
                uno_launch(UNO_KT_UPDATE, k_cg_update<double, 1>, grid, dim3(kBlock), 0, sp, gd,
                           (const double*)w->dinv, w->r, u, (const double*)dnew, (const double*)w->p, w->s, it,
                           (const double*)P.dp, np_dp, (const double*)w->gam, P.rmax, rs_next, ss_next);
            else
                uno_launch(UNO_KT_UPDATE, k_cg_update<double, 0>, grid, dim3(kBlock), 0, sp, gd,
                           (const double*)w->dinv, w->r, u, (const double*)dnew, (const double*)w->p, w->s, it,
                           (const double*)P.dp, np_dp, (const double*)w->gam, P.rmax, rs_next, ss_next);
            return hip_status(hipGetLastError());
        }
        return UNO_ERR_ARG;  // FP32 mode runs UNO-CG only
    };
    auto check = [&](int k, int k0, int kr) {
        const CgIter it = iter_of(w, P, k, k0, kr, o->rtol, hist_len, np_update, dks);
        hipLaunchKernelGGL(k_cg_check, dim3(1, nrhs), dim3(kBlock), 0, st, it);
    };
    const int64_t n = g.total, N = 3 * n;
    auto residual = [&]() {
        (void)el_residual(E, g, w, lam, mu, lks, u, nrhs, st);
        el_remove_means(w, P, w->r, n, nrhs, st);  // as for r_0: the rounding residue lies outside range(A)
    };
    auto true_res = [&]() {
        hipLaunchKernelGGL(k_resid_parts_b, dim3(nb, nrhs), dim3(kBlock), 0, st, N, (const double*)w->f,
                           (const double*)w->p, P.rs[0], P.rs[1], N, w->npart);
        hipLaunchKernelGGL(k_resid_final_b, dim3(1, nrhs), dim3(kBlock), 0, st, (const double*)P.rs[0],
                           (const double*)P.rs[1], nb, w->state, w->npart);
    };
    std::vector<int64_t> key;
    if (o->use_graphs && !restarts && !ktimer_active()) {
        int64_t rt;
        memcpy(&rt, &o->rtol, sizeof(rt));
        key = {2, (int64_t)sizeof(T), o->kind, pc ? (int64_t)pc->serial : 0, nrhs, lks, (int64_t)(uintptr_t)lam,
               (int64_t)(uintptr_t)mu, (int64_t)(uintptr_t)lamT, (int64_t)(uintptr_t)muT, (int64_t)(uintptr_t)u,
               hist_len, rt};
    }
    return run_chunks(w, o, nrhs, restarts, st, pass, check, residual, start, true_res, k_end, key);
}

uno_status pcg_run_el(const Grid& g, const double* lam, const double* mu, int64_t lks, int nrhs, const double* eps6,
                      double* u, const uno_solve_opts* o, uno_solve_info* info, hipStream_t st)
{
    if (o->kind != UNO_PREC_NONE && o->kind != UNO_PREC_JACOBI && o->kind != UNO_PREC_UNO) return UNO_ERR_ARG;
    const bool f64 = o->op_t == UNO_F64 && o->prec_t == UNO_F64;
    const bool mixed = o->op_t == UNO_F32 && o->prec_t == UNO_F32;
    if (!f64 && !(mixed && o->kind == UNO_PREC_UNO)) return UNO_ERR_ARG;
    const uno_precond* pc = (o->kind == UNO_PREC_UNO) ? o->uno : nullptr;
    if (o->kind == UNO_PREC_UNO && !(pc && pc->nc == 3 && pc->lr)) return UNO_ERR_ARG;
    ElDev E;
    uno_status e = el_dev(g, &E);
    if (e != UNO_OK) return e;
    const int64_t n = g.total, N = 3 * n;
    Grid gv = g;  // workspace of 3n-vectors, keyed apart from the scalar problems
    gv.n[0] = 3 * g.n[0];
    gv.total = N;
    GridDev gd = g.dev;
    gd.n = N;
    Workspace* w = nullptr;
    int extra = el_march_blocks(g, nrhs);
    if (pc && lowrank_max_blocks(pc->lr) > extra) extra = lowrank_max_blocks(pc->lr);
    std::unique_lock<std::mutex> lease;
    e = ws_get(gv, nullptr, pc ? pc->lr : nullptr, extra, o->max_iter + 1, nrhs, st, &lease, &w);
    if (e != UNO_OK) return e;
    const int nb = w->nbr;
    const Parts P = parts_of(w);
    for (int b = 0; b < nrhs; ++b) {
        e = launch_el_rhs(E, g, lam + b * lks, mu + b * lks, eps6 + 6 * b, w->f + b * N, st);
        if (e != UNO_OK) return e;
    }
    e = el_residual(E, g, w, lam, mu, lks, u, nrhs, st);
    if (e != UNO_OK) return e;
    // f and r_0 sum to zero per component in exact arithmetic (the
    // translations span the kernel of A); the rounding residue of those
    // sums lies outside the range of A and would stall CG once the
    // consistent part is resolved, so it is removed here
    el_remove_means(w, P, w->f, n, nrhs, st);
    el_remove_means(w, P, w->r, n, nrhs, st);
    if (o->kind == UNO_PREC_JACOBI) {
        e = launch_el_inv_diag(E, g, lam, mu, lks, lks ? nrhs : 1, w->dinv, st);
        if (e != UNO_OK) return e;
    }
    int k = 0;
    if (mixed) {
        // FP32 Lame fields: lambda then mu, one pair per field
        const int nf = lks ? nrhs : 1;
        if (w->kap32_cap < nf) {  // a field of the 3n-vector workspace holds both (2n <= 3n floats)
            ws_drop_graphs(w);
            (void)hipFree(w->kap32);
            w->kap32 = nullptr;
            w->kap32_cap = 0;
            if (hipMalloc(&w->kap32, sizeof(float) * N * nf) != hipSuccess) return UNO_ERR_NOMEM;
            w->kap32_cap = nf;
        }
        float* lam32 = w->kap32;
        float* mu32 = w->kap32 + n * nf;
        hipLaunchKernelGGL(k_convert<float>, dim3(nb), dim3(kBlock), 0, st, n * nf, lam, lam32);
        hipLaunchKernelGGL(k_convert<float>, dim3(nb), dim3(kBlock), 0, st, n * nf, mu, mu32);
        e = el_loop<float>(E, g, gd, w, lam, mu, lam32, mu32, lks, u, o, pc, nrhs, st, &k);
    } else {
        e = el_loop<double>(E, g, gd, w, lam, mu, lam, mu, lks, u, o, pc, nrhs, st, &k);
    }
    if (e != UNO_OK) return e;
    std::vector<CgState> hs(w->host_state, w->host_state + nrhs);
    // zero-mean components and the true residual in FP64
    el_remove_means(w, P, u, n, nrhs, st);
    e = el_residual(E, g, w, lam, mu, lks, u, nrhs, st);
    if (e != UNO_OK) return e;
    {
        const dim3 grid(nb, nrhs);
        hipLaunchKernelGGL(k_resid_parts_b, grid, dim3(kBlock), 0, st, N, (const double*)w->f, (const double*)w->p,
                           P.rs[0], P.rs[1], N, w->npart);
        hipLaunchKernelGGL(k_resid_final_b, dim3(1, nrhs), dim3(kBlock), 0, st, (const double*)P.rs[0],
                           (const double*)P.rs[1], nb, w->state, w->npart);
        UNO_HIP(hipGetLastError());
    }
    UNO_HIP(hipMemcpyAsync(w->host_state, w->state, sizeof(CgState) * nrhs, hipMemcpyDeviceToHost, st));
    UNO_HIP(hipStreamSynchronize(st));
    bool failed = false;
    for (int b = 0; b < nrhs; ++b) {
        const CgState& h = hs[b];
        const CgState& fin = w->host_state[b];
        if (h.status != 0) failed = true;
        if (info) {
            uno_solve_info& I = info[b];
            I.iters = (h.done != INT_MAX) ? h.done : (h.status != 0 ? h.fail_iter : k);
            I.converged = (h.status == 0 && h.done != INT_MAX) ? 1 : 0;
            I.rel_res = h.r0max > 0.0 ? h.rmax_last / h.r0max : 0.0;
            I.true_rel_res = fin.fmax > 0.0 ? fin.dmax / fin.fmax : 0.0;
            I.r0_norm = h.r0max;
        }
    }
    return failed ? UNO_ERR_BREAKDOWN : UNO_OK;
}

uno_status pcg_run(const Grid& g, const double* kappa, const double* macro_load3, const double* rhs, double* u,
                   const uno_solve_opts* o, uno_solve_info* info, double* res_hist, hipStream_t st)
{
    return pcg_run_batch(g, kappa, 0, 1, macro_load3, rhs, u, o, info, res_hist, st);
}

// ---------------------------------------------------------------------------
// Allocation-free solve: the CG workspace of one right-hand side is carved
// from a file-scope device array instead of being allocated, for callers
// that cannot allocate device memory.  Every call on a device shares that
// device's array (the calls are serialized by g_scratch_mu; each returns
// after its solve has finished) and finds the previous call's contents
// there: nothing in it needs to start at zero (the loop states are set by
// the init kernel, partials and histories are written before they are read,
// and the previous direction is not read on the first pass).

// kScratchDoubles doubles (24 MiB) per device: a 64^3 solve in FP64 needs
// 7 vectors of 2 MiB plus partials, histories and the learned-mode scratch.
constexpr size_t kScratchDoubles = (size_t)UNO_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's array (hipGetSymbolAddress once per
// device, with the device current); the host-side name `scratch` is never
// passed to a kernel or a copy
uno_status scratch_ptr(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return UNO_ERR_DEVICE;
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_status(e == hipSuccess ? hipErrorInvalidSymbol : e);
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return UNO_OK;
}
}  // namespace

uno_status pcg_run_noalloc(const Grid& g, const double* kappa, const double* macro_load3, const double* rhs,
                           double* u, const uno_solve_opts* o, uno_solve_info* info, double* res_hist, hipStream_t st)
{
    const uno_precond* pc = (o->kind == UNO_PREC_UNO) ? o->uno : nullptr;
    const bool mixed = (o->op_t == UNO_F32);
    if (mixed && pc && !uno_use_lowrank(pc)) return UNO_ERR_ARG;
    int dev = 0;
    UNO_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    double* base = nullptr;
    uno_status e = scratch_ptr(dev, &base);
    if (e != UNO_OK) return e;
    Workspace w;
    w.device = dev;
    w.stream = st;
    for (int b = 0; b < 3; ++b) w.n[b] = g.n[b];
    w.total = g.total;
    w.nbr = ws_nbr(g);
    w.npart = ws_npart(g, w.nbr, pc ? pc->rs_blocks : 0);
    w.nrhs_cap = 1;
    // sub-buffers at 256-byte boundaries
    const int64_t n = g.total;
    const int hist_len = o->max_iter + 1;
    size_t off = 0;
    auto take = [&](size_t doubles) {
        double* q = base + off;
        off += (doubles + 31) / 32 * 32;
        return q;
    };
    w.f = take(n);
    w.r = take(n);
    w.s = take(n);
    w.d[0] = take(n);
    w.d[1] = take(n);
    w.p = take(n);
    w.dinv = take(n);
    if (mixed) {
        w.kap32 = (float*)take((n + 1) / 2);
        w.kap32_cap = 1;
    }
    w.part = take(8 * (size_t)w.npart);
    w.state = (CgState*)take((sizeof(CgState) + 7) / 8);
    w.hist = take(hist_len);
    w.gam = take(hist_len);
    w.hist_cap = hist_len;
    if (pc && !uno_use_lowrank(pc)) {
        w.spec = (double2*)take(2 * (size_t)pc->plan.nspec);
        w.nspec = pc->plan.nspec;
        w.spec_cap = 1;
    }
    if (pc && pc->lr) {
        int64_t ngp = 0, nh = 0;
        lowrank_scratch_size(pc->lr, &ngp, &nh);
        w.lr_gp = (double2*)take(2 * (size_t)ngp);
        w.lr_h = (double2*)take(2 * (size_t)nh);
        w.lr_ngp = ngp;
        w.lr_nh = nh;
        w.lr_cap = 1;
    }
    if (off > kScratchDoubles) return UNO_ERR_SHAPE;  // beyond the array: use pcg_solve
    CgState host_state;  // the loop state read back between chunks (pageable)
    w.host_state = &host_state;
    return pcg_run_ws(g, &w, false, kappa, 0, 1, macro_load3, rhs, u, o, info, res_hist, st);
}

}  // namespace unocg
