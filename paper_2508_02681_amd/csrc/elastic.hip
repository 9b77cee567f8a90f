// Linear elasticity on the periodic voxel grid, d = 3, three nodal DOF
// (Sec. 5.2): the operator div((3 lambda P1 + 2 mu I_sym) sym(grad .)),
// discretized with trilinear hex8 elements (Sec. 3.1), strains and stresses
// in the Mandel basis (App. A).  Displacements are planar: component c of
// node i at u[c n + i].
//
// Node-centred gather: node i is corner s of the eight voxels e = i - s,
// s in {0,1}^3, and
//   (A u)_(i,a) = sum_s sum_t sum_b (lambda_e K^l + mu_e K^m)[(s,a),(t,b)] u_(e+t, b),
// with K^l, K^m the unit element matrices of the lambda and mu parts
// (24 x 24, exact 2-point Gauss integration), staged in LDS.
#include <cmath>
#include <cstring>
#include <vector>

#include "unocg_internal.h"
#include "reduce.h"
#include "cg_ctl.h"

namespace unocg {

// unit element matrices of the brick h0 x h1 x h2: K[0] lambda part, K[1] mu
// part, index (corner a * 3 + component c) * 24 + (corner b * 3 + component e)
void el_element_matrices(const double h[3], double K[2][576])
{
    const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
    const double s2 = std::sqrt(2.0);
    memset(K, 0, sizeof(double) * 2 * 576);
    for (int q = 0; q < 8; ++q) {
        const double xi[3] = {gp[(q >> 2) & 1], gp[(q >> 1) & 1], gp[q & 1]};
        const double w = h[0] * h[1] * h[2] / 8.0;
        double B[8][6][3];
        for (int a = 0; a < 8; ++a) {
            double g[3];
            for (int b = 0; b < 3; ++b) {
                const int sb = (a >> (2 - b)) & 1;
                double v = (sb ? 1.0 : -1.0) / h[b];
                for (int c = 0; c < 3; ++c) {
                    if (c == b) continue;
                    const int sc = (a >> (2 - c)) & 1;
                    v *= sc ? xi[c] : 1.0 - xi[c];
                }
                g[b] = v;
            }
            memset(B[a], 0, sizeof(B[a]));
            B[a][0][0] = g[0];
            B[a][1][1] = g[1];
            B[a][2][2] = g[2];
            B[a][3][0] = g[1] / s2; B[a][3][1] = g[0] / s2;
            B[a][4][0] = g[2] / s2; B[a][4][2] = g[0] / s2;
            B[a][5][1] = g[2] / s2; B[a][5][2] = g[1] / s2;
        }
        for (int a = 0; a < 8; ++a)
            for (int c = 0; c < 3; ++c)
                for (int b = 0; b < 8; ++b)
                    for (int e = 0; e < 3; ++e) {
                        // lambda part: (tr eps_a)(tr eps_b); mu part: 2 eps_a : eps_b (Mandel dot)
                        double tra = 0.0, trb = 0.0, dd = 0.0;
                        for (int k = 0; k < 3; ++k) {
                            tra += B[a][k][c];
                            trb += B[b][k][e];
                        }
                        for (int k = 0; k < 6; ++k) dd += B[a][k][c] * B[b][k][e];
                        K[0][(a * 3 + c) * 24 + b * 3 + e] += w * tra * trb;
                        K[1][(a * 3 + c) * 24 + b * 3 + e] += w * 2.0 * dd;
                    }
    }
}

__device__ __forceinline__ int wrap_el(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// CG variant: the operand is d = s + beta d_old (beta, d_old as in the
// thermal operator), d of the own node goes to d_new, p = A d, d.p partials.
// lks: stride between the Lame fields of the right-hand sides (0 if shared).
template <bool CG, bool HEAD>
__global__ void __launch_bounds__(256) k_el_apply(ElDev E, const double* __restrict__ lam, const double* __restrict__ mu,
                                                  int64_t lks, const double* __restrict__ s,
                                                  const double* __restrict__ dold, double* __restrict__ dnew,
                                                  double* __restrict__ p, double* __restrict__ part_dp, CgIter it,
                                                  const double* __restrict__ part_rs, int np_rs, double* gam)
{
    __shared__ double Ks[2 * 576];
    __shared__ double slots[4];
    const GridDev& g = E.g;
    const int64_t n = g.n;
    if (CG && blockIdx.y > 0) {
        const int64_t vo = (int64_t)blockIdx.y * it.vs, po = (int64_t)blockIdx.y * it.ps;
        lam += (int64_t)blockIdx.y * lks;
        mu += (int64_t)blockIdx.y * lks;
        s += vo;
        dold += vo;
        dnew += vo;
        p += vo;
        part_dp += po;
        part_rs += po;
        gam += (int64_t)blockIdx.y * it.hs;
        it = rhs_iter(it);
    }
    StateLoad sl;
    double head_share = 0.0, rs_share = 0.0, gprev = 1.0;
    if (CG) {
        sl = load_state(it.st);
        if (HEAD) head_share = load_share<OpMax>(it.part_rmax, it.np_rmax);
        rs_share = load_share<OpSum>(part_rs, np_rs);
        if (it.k > it.k0) gprev = gam[it.k - 1];
    }
    for (int j = threadIdx.x; j < 2 * 576; j += 256) Ks[j] = E.K[j];
    double beta = 0.0;
    bool first = true;
    if (CG) {
        if (HEAD) {
            if (head_decide(it, sl, head_share, slots)) return;
        } else if (ended(sl, it.k)) {
            return;
        }
        const int k = it.k;
        const double gk = combine_share<OpSum>(rs_share, slots);
        const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
        if (lead) gam[k] = gk;
        if (!(gk > 0.0) || !isfinite(gk)) {
            if (lead) { it.st->status = 1; it.st->fail_iter = k; }
            return;
        }
        first = (k == it.k0);
        beta = first ? 0.0 : gk / gprev;
    }
    __syncthreads();
    const bool use_old = CG && !first;
    double dot = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(i % g.n2);
        const int64_t q = i / g.n2;
        const int y = (int)(q % g.n1), x = (int)(q / g.n1);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int sc = 0; sc < 8; ++sc) {  // node i is corner sc of voxel e = i - sc
            const int ex = wrap_el(x - (sc >> 2), g.n0), ey = wrap_el(y - ((sc >> 1) & 1), g.n1),
                      ez = wrap_el(z - (sc & 1), g.n2);
            const int64_t e = ((int64_t)ex * g.n1 + ey) * g.n2 + ez;
            const double le = lam[e], me = mu[e];
            for (int t = 0; t < 8; ++t) {
                const int64_t j = ((int64_t)wrap_el(ex + (t >> 2), g.n0) * g.n1 + wrap_el(ey + ((t >> 1) & 1), g.n1)) *
                                      g.n2 + wrap_el(ez + (t & 1), g.n2);
                double dj[3];
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    dj[b] = s[b * n + j];
                    if (use_old) dj[b] += beta * dold[b * n + j];
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double* K0 = Ks + (sc * 3 + a) * 24 + t * 3;
                    const double* K1 = K0 + 576;
#pragma unroll
                    for (int b = 0; b < 3; ++b) acc[a] += (le * K0[b] + me * K1[b]) * dj[b];
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p[a * n + i] = acc[a];
            if (CG) {
                double di = s[a * n + i];
                if (use_old) di += beta * dold[a * n + i];
                dnew[a * n + i] = di;
                dot += di * acc[a];
            }
        }
    }
    if (CG) {
        const double bd = block_reduce<OpSum>(dot, slots);
        if (threadIdx.x == 0) part_dp[blockIdx.x] = bd;
    }
}

// inverse assembled diagonal, 3 per node (one field per right-hand side along grid y)
__global__ void __launch_bounds__(256) k_el_inv_diag(ElDev E, const double* __restrict__ lam,
                                                     const double* __restrict__ mu, int64_t ks,
                                                     double* __restrict__ dinv)
{
    const GridDev& g = E.g;
    const int64_t n = g.n;
    lam += (int64_t)blockIdx.y * ks;
    mu += (int64_t)blockIdx.y * ks;
    dinv += (int64_t)blockIdx.y * 3 * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(i % g.n2);
        const int64_t q = i / g.n2;
        const int y = (int)(q % g.n1), x = (int)(q / g.n1);
        double dg[3] = {0.0, 0.0, 0.0};
        for (int sc = 0; sc < 8; ++sc) {
            const int64_t e = ((int64_t)wrap_el(x - (sc >> 2), g.n0) * g.n1 + wrap_el(y - ((sc >> 1) & 1), g.n1)) *
                                  g.n2 + wrap_el(z - (sc & 1), g.n2);
            for (int a = 0; a < 3; ++a) {
                const int ii = (sc * 3 + a) * 24 + sc * 3 + a;
                dg[a] += lam[e] * E.K[ii] + mu[e] * E.K[576 + ii];
            }
        }
        for (int a = 0; a < 3; ++a) dinv[a * n + i] = 1.0 / dg[a];
    }
}

// f = -sum_e |Omega_e| grad N(centre)^T sigma_e, sigma_e = D_e eps_bar
__global__ void __launch_bounds__(256) k_el_rhs(ElDev E, const double* __restrict__ lam, const double* __restrict__ mu,
                                                double e0, double e1, double e2, double e3, double e4, double e5,
                                                double* __restrict__ f)
{
    const GridDev& g = E.g;
    const int64_t n = g.n;
    const double r2 = 1.0 / std::sqrt(2.0);
    const double tr = e0 + e1 + e2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(i % g.n2);
        const int64_t q = i / g.n2;
        const int y = (int)(q % g.n1), x = (int)(q / g.n1);
        double acc[3] = {0.0, 0.0, 0.0};
        for (int sc = 0; sc < 8; ++sc) {
            const int64_t e = ((int64_t)wrap_el(x - (sc >> 2), g.n0) * g.n1 + wrap_el(y - ((sc >> 1) & 1), g.n1)) *
                                  g.n2 + wrap_el(z - (sc & 1), g.n2);
            const double le = lam[e], me = mu[e];
            // stress tensor of D_e eps_bar (Mandel shear entries carry sqrt 2)
            double S[3][3];
            S[0][0] = le * tr + 2.0 * me * e0;
            S[1][1] = le * tr + 2.0 * me * e1;
            S[2][2] = le * tr + 2.0 * me * e2;
            S[0][1] = S[1][0] = 2.0 * me * e3 * r2;
            S[0][2] = S[2][0] = 2.0 * me * e4 * r2;
            S[1][2] = S[2][1] = 2.0 * me * e5 * r2;
            const double gr[3] = {((sc >> 2) ? 1.0 : -1.0) * E.gc[0], (((sc >> 1) & 1) ? 1.0 : -1.0) * E.gc[1],
                                  ((sc & 1) ? 1.0 : -1.0) * E.gc[2]};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) acc[a] -= E.hvol * S[a][b] * gr[b];
        }
        for (int a = 0; a < 3; ++a) f[a * n + i] = acc[a];
    }
}

// per-workgroup sums of the Mandel stress D_e (eps_bar + eps(u)(centre))
__global__ void __launch_bounds__(256) k_el_stress(ElDev E, const double* __restrict__ lam,
                                                   const double* __restrict__ mu, double e0, double e1, double e2,
                                                   double e3, double e4, double e5, const double* __restrict__ u,
                                                   double* __restrict__ part)
{
    __shared__ double slots[4];
    const GridDev& g = E.g;
    const int64_t n = g.n;
    const double r2 = std::sqrt(2.0);
    double sum[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(e % g.n2);
        const int64_t q = e / g.n2;
        const int y = (int)(q % g.n1), x = (int)(q / g.n1);
        double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // G[c][b] = d u_c / d x_b at the centre
        for (int t = 0; t < 8; ++t) {
            const int64_t j = ((int64_t)wrap_el(x + (t >> 2), g.n0) * g.n1 + wrap_el(y + ((t >> 1) & 1), g.n1)) *
                                  g.n2 + wrap_el(z + (t & 1), g.n2);
            const double sg[3] = {(t >> 2) ? 1.0 : -1.0, ((t >> 1) & 1) ? 1.0 : -1.0, (t & 1) ? 1.0 : -1.0};
            for (int c = 0; c < 3; ++c) {
                const double v = u[c * n + j];
                for (int b = 0; b < 3; ++b) G[c][b] += sg[b] * E.gc[b] * v;
            }
        }
        const double eps[6] = {e0 + G[0][0], e1 + G[1][1], e2 + G[2][2], e3 + (G[0][1] + G[1][0]) / r2,
                               e4 + (G[0][2] + G[2][0]) / r2, e5 + (G[1][2] + G[2][1]) / r2};
        const double le = lam[e], me = mu[e], tr = eps[0] + eps[1] + eps[2];
        for (int k = 0; k < 6; ++k) sum[k] += (k < 3 ? le * tr : 0.0) + 2.0 * me * eps[k];
    }
    for (int k = 0; k < 6; ++k) {
        const double b = block_reduce<OpSum>(sum[k], slots);
        if (threadIdx.x == 0) part[6 * blockIdx.x + k] = b;
    }
}

// ---------------------------------------------------------------------------
// host

namespace {
struct ElCache {
    int device;
    double h[3];
    double* K;
};
std::vector<ElCache> g_el;
}  // namespace

uno_status el_dev(const Grid& g, ElDev* out)
{
    int dev = 0;
    UNO_HIP(hipGetDevice(&dev));
    double* K = nullptr;
    for (const ElCache& c : g_el)
        if (c.device == dev && c.h[0] == g.h[0] && c.h[1] == g.h[1] && c.h[2] == g.h[2]) K = c.K;
    if (!K) {
        double Kh[2][576];
        el_element_matrices(g.h, Kh);
        if (hipMalloc(&K, sizeof(Kh)) != hipSuccess) return UNO_ERR_NOMEM;
        UNO_HIP(hipMemcpy(K, Kh, sizeof(Kh), hipMemcpyHostToDevice));
        g_el.push_back(ElCache{dev, {g.h[0], g.h[1], g.h[2]}, K});
    }
    out->g = g.dev;
    out->hvol = g.h[0] * g.h[1] * g.h[2];
    for (int b = 0; b < 3; ++b) out->gc[b] = 1.0 / (4.0 * g.h[b]);
    out->K = K;
    return UNO_OK;
}

void el_release_all()
{
    for (const ElCache& c : g_el) (void)hipFree(c.K);
    g_el.clear();
}

int el_blocks(const Grid& g)
{
    const int64_t nb = (g.total + 255) / 256;
    return (int)(nb < 1024 ? nb : 1024);
}

template <bool CG, bool HEAD>
uno_status launch_el_apply(const ElDev& E, const Grid& g, const double* lam, const double* mu, int64_t lks,
                           const double* s, const double* dold, double* dnew, double* p, double* part_dp,
                           const CgIter& it, const double* part_rs, int np_rs, double* gam, int nrhs, hipStream_t st)
{
    uno_launch(CG ? UNO_KT_MATVEC : UNO_KT_APPLY, k_el_apply<CG, HEAD>, dim3(el_blocks(g), nrhs), dim3(256), 0, st, E,
               lam, mu, lks, s, dold, dnew, p, part_dp, it, part_rs, np_rs, gam);
    return hip_status(hipGetLastError());
}
template uno_status launch_el_apply<false, false>(const ElDev&, const Grid&, const double*, const double*, int64_t,
                                                  const double*, const double*, double*, double*, double*,
                                                  const CgIter&, const double*, int, double*, int, hipStream_t);
template uno_status launch_el_apply<true, true>(const ElDev&, const Grid&, const double*, const double*, int64_t,
                                                const double*, const double*, double*, double*, double*,
                                                const CgIter&, const double*, int, double*, int, hipStream_t);

uno_status launch_el_inv_diag(const ElDev& E, const Grid& g, const double* lam, const double* mu, int64_t ks,
                              int nfields, double* dinv, hipStream_t st)
{
    hipLaunchKernelGGL(k_el_inv_diag, dim3(el_blocks(g), nfields), dim3(256), 0, st, E, lam, mu, ks, dinv);
    return hip_status(hipGetLastError());
}

uno_status launch_el_rhs(const ElDev& E, const Grid& g, const double* lam, const double* mu, const double* eps,
                         double* f, hipStream_t st)
{
    hipLaunchKernelGGL(k_el_rhs, dim3(el_blocks(g)), dim3(256), 0, st, E, lam, mu, eps[0], eps[1], eps[2], eps[3],
                       eps[4], eps[5], f);
    return hip_status(hipGetLastError());
}

uno_status el_stress_average(const ElDev& E, const Grid& g, const double* lam, const double* mu, const double* eps,
                             const double* u, double* out, hipStream_t st)
{
    const int nb = el_blocks(g);
    double* part = nullptr;
    if (hipMalloc(&part, sizeof(double) * 6 * nb) != hipSuccess) return UNO_ERR_NOMEM;
    hipLaunchKernelGGL(k_el_stress, dim3(nb), dim3(256), 0, st, E, lam, mu, eps[0], eps[1], eps[2], eps[3], eps[4],
                       eps[5], u, part);
    std::vector<double> h(6 * (size_t)nb);
    uno_status e = hip_status(hipGetLastError());
    if (e == UNO_OK) e = hip_status(hipMemcpyAsync(h.data(), part, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost, st));
    if (e == UNO_OK) e = hip_status(hipStreamSynchronize(st));
    (void)hipFree(part);
    if (e != UNO_OK) return e;
    for (int k = 0; k < 6; ++k) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += h[6 * b + k];
        out[k] = s / (double)g.total;
    }
    return UNO_OK;
}

}  // namespace unocg
