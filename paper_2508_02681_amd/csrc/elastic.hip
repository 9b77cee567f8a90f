// Linear elasticity on the periodic voxel grid, d = 3, three nodal DOF
// (Sec. 5.2): the operator div((3 lambda P1 + 2 mu I_sym) sym(grad .)),
// discretized with trilinear hex8 elements (Sec. 3.1), strains and stresses
// in the Mandel basis (App. A).  Displacements are planar: component c of
// node i at u[c n + i].
//
// The operator is applied voxel by voxel with the element integrals over
// the 2-point Gauss rule (exact for the trilinear brick) evaluated in the
// Walsh-Hadamard basis, where the Gauss interpolations are diagonal,
// marching along axis 0 with the corner forces summed in registers and LDS.
// The unit element matrices K^l, K^m of the lambda and mu parts (24 x 24)
// are kept for the Jacobi diagonal.
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

// In-place 3D Walsh-Hadamard transform of the eight corner values,
// x^(h) = sum_v x(v) (-1)^(h.v), v = 4a + 2b + c.
template <typename T>
__device__ __forceinline__ void had8(T x[8])
{
#pragma unroll
    for (int s = 1; s < 8; s <<= 1)
#pragma unroll
        for (int v = 0; v < 8; ++v)
            if (!(v & s)) {
                const T a = x[v], b = x[v | s];
                x[v] = a + b;
                x[v | s] = a - b;
            }
}

// index of h (bit of axis j clear) among the four such h, and back
__host__ __device__ constexpr int el_tpos(int h, int j)
{
    return ((h >> (3 - j)) << (2 - j)) | (h & ((1 << (2 - j)) - 1));
}
__host__ __device__ constexpr int el_tins(int t, int j)
{
    return ((t >> (2 - j)) << (3 - j)) | (t & ((1 << (2 - j)) - 1));
}
__host__ __device__ constexpr int el_pop(int h) { return (h & 1) + ((h >> 1) & 1) + ((h >> 2) & 1); }

// Element forces of one voxel, f = int B^T D B u over the exact 2-point
// Gauss rule, computed in the Walsh-Hadamard basis of the corners and of the
// Gauss points.  The 1D interpolation from the two ends of an edge to its
// two Gauss points is P = [[g0, g1], [g1, g0]] = H diag(1, r) H / 2 with
// H = [[1, 1], [1, -1]] and r = 1/sqrt 3, so in that basis every
// interpolation is a diagonal scaling:
//   gradient:  g^_ij(h) = -(2/h_j) r^|h| U^_i(h + e_j) for h_j = 0 (0 for
//              h_j = 1: the gradient along j does not vary along j),
//   stress:    s^_ij(h) = lam delta_ij sum_k g^_kk(h) + mu (g^_ij + g^_ji)(h)
//              (pointwise and constant on the voxel, so it commutes with the
//              transform),
//   forces:    Y_i(h + e_j) += -(2/h_j) r^|h| (w/8) s^_ij(h),
//              f_i = Hadamard(Y_i),
// |h| the number of set transverse bits, w/8 the Gauss weight times the
// voxel volume over the 8 of the inverse transform; lw, mw carry the w/8.
// U[i][v] in: corner values of component i; out: corner forces.
template <typename T>
__device__ __forceinline__ void el_element(const ElDev& E, T lw, T mw, T U[3][8])
{
#pragma unroll
    for (int i = 0; i < 3; ++i) had8(U[i]);
    T g[3][3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int h = el_tins(t, j);
                g[i][j][t] = (T)E.hc[j][el_pop(h)] * U[i][h | (4 >> j)];
            }
    T Y[3][8];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int v = 0; v < 8; ++v) Y[i][v] = (T)0;
#pragma unroll
    for (int h = 0; h < 8; ++h) {
        if (h == 7) continue;  // every direction has a set bit: no term
        T tr = (T)0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (!(h & (4 >> k))) tr += g[k][k][el_tpos(h, k)];
        const T ltr = lw * tr;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (h & (4 >> j)) continue;
            const T c = (T)E.hc[j][el_pop(h)];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T sij = g[i][j][el_tpos(h, j)];
                if (!(h & (4 >> i))) sij += g[j][i][el_tpos(h, i)];
                sij *= mw;
                if (i == j) sij += ltr;
                Y[i][h | (4 >> j)] += c * sij;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        had8(Y[i]);
#pragma unroll
        for (int v = 0; v < 8; ++v) U[i][v] = Y[i][v];
    }
}

// y = A u as a march along axis 0.  A workgroup of 16 x 16 threads owns a
// tile of 15 x 15 nodes in the (1, 2) plane and xb node planes; thread
// (ty, tz) computes the voxel whose lower corner is node (y0 - 1 + ty,
// z0 - 1 + tz) in each voxel plane x0 - 1 ... x0 + xb - 1 and owns that
// node when ty, tz >= 1.  The voxel's corner forces go to
//   corner a = 1 (next node plane): kept in registers for the next step,
//   corners b or c = 1 (other threads' nodes): exchanged through LDS,
// and the owner sums the four in-plane contributions.  The node planes
// pass through a ring of three LDS planes (two in use, one being filled).
//
// CG variant: the operand is d = s + beta d_old (beta from gamma_k /
// gamma_(k-1), gamma_k combined from the r.s partials), the owner writes
// d_new, p = A d and the d.p partial of the workgroup.  lks: stride of the
// Lame fields per right-hand side (0 if shared).
constexpr int kElT = 16;        // threads per tile side
constexpr int kElO = kElT - 1;  // owned nodes per tile side
constexpr int kElL = kElT + 1;  // LDS node tile side

template <typename T, bool CG, bool HEAD>
__global__ void __launch_bounds__(256) k_el_march(ElDev E, ElGeom eg, const T* __restrict__ lam,
                                                  const T* __restrict__ mu, int64_t lks,
                                                  const T* __restrict__ s, const T* __restrict__ dold,
                                                  T* __restrict__ dnew, T* __restrict__ p,
                                                  double* __restrict__ part_dp, CgIter it,
                                                  const double* __restrict__ part_rs, int np_rs, double* gam)
{
    resolve_pass(it);
    __shared__ T Dl[3][3][kElL * kElL];  // ring slot, component, node
    __shared__ T X[2][9][256];           // exchanged corner forces
    __shared__ double slots[4];
    const GridDev& g = E.g;
    const int64_t n = g.n;
    lam += (int64_t)blockIdx.y * lks;
    mu += (int64_t)blockIdx.y * lks;
    if (blockIdx.y > 0) {
        const int64_t vo = (int64_t)blockIdx.y * it.vs;
        s += vo;
        p += vo;
        if (CG) {
            dold += vo;
            dnew += vo;
            part_dp += (int64_t)blockIdx.y * it.ps;
            part_rs += (int64_t)blockIdx.y * it.ps;
            gam += (int64_t)blockIdx.y * it.hs;
            it = rhs_iter(it);
        }
    }
    const int t = threadIdx.x, ly = t >> 4, lz = t & 15;
    int bid = xcd_tile(blockIdx.x, gridDim.x);
    const int bz = bid % eg.tiles_z;
    bid /= eg.tiles_z;
    const int by = bid % eg.tiles_y, bx = bid / eg.tiles_y;
    const int y0 = by * kElO, z0 = bz * kElO, x0 = bx * eg.xb;
    const int nx = min(eg.xb, g.n0 - x0);
    const int64_t plane = (int64_t)g.n1 * g.n2;
    // this thread's node (and voxel) in the plane, and the extra node of the
    // LDS tile it loads (row 16, then column 16)
    const int64_t o0 = (int64_t)wrap_el(y0 - 1 + ly, g.n1) * g.n2 + wrap_el(z0 - 1 + lz, g.n2);
    const bool has_x = t < 2 * kElL - 1;
    const int xy = t < kElL ? kElT : t - kElL, xz = t < kElL ? t : kElT;
    // (threads without an extra node load their own node twice: every load
    // is unconditional, see fetch)
    const int64_t o1 = has_x ? (int64_t)wrap_el(y0 - 1 + xy, g.n1) * g.n2 + wrap_el(z0 - 1 + xz, g.n2) : o0;
    const int l0 = ly * kElL + lz, l1 = xy * kElL + xz;
    const bool own = ly >= 1 && lz >= 1 && y0 + ly - 1 < g.n1 && z0 + lz - 1 < g.n2;

    StateLoad sl;
    double head_share = 0.0, rs_share = 0.0, gprev = 1.0;
    if (CG) {
        sl = load_state(it.st);
        if (HEAD) head_share = load_share<OpMax>(it.part_rmax, it.np_rmax);
        rs_share = load_share<OpSum>(part_rs, np_rs);
        if (it.k > it.k0) gprev = gam[it.k - 1];
    }
    T beta = 0;
    bool use_old = false;
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
        use_old = k != it.k0;
        beta = use_old ? (T)(gk / gprev) : (T)0;
    }

    // node plane m (global x0 - 1 + m) of the operand, in registers between
    // its loads and its LDS store.  Every load is unconditional (d_old is
    // read on the first pass of a cycle too, and not used), so that no
    // branch lies between the loads of a plane and the wait for them, and
    // the waits before a store leave a later plane's loads in flight.  FP64:
    // two sets, the loads of plane j + 3 issued at step j (the element
    // arithmetic of two steps hides them); FP32 keeps one set (plane j + 2),
    // which holds its 4 waves per SIMD.
    constexpr bool DEEP = sizeof(T) == sizeof(double);
    struct Stage {
        T ps[3], pd[3], xs[3], xd[3];
    };
    Stage ra, rb;
    auto fetch = [&](Stage& R, int m) {
        const int64_t b = (int64_t)wrap_el(x0 - 1 + m, g.n0) * plane;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            R.ps[i] = s[i * n + b + o0];
            R.xs[i] = s[i * n + b + o1];
            if (CG) {
                R.pd[i] = dold[i * n + b + o0];
                R.xd[i] = dold[i * n + b + o1];
            }
        }
    };
    auto store = [&](const Stage& R, int m) {
        const int slot = m % 3;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T d = use_old ? R.ps[i] + beta * R.pd[i] : R.ps[i];
            Dl[slot][i][l0] = d;
            if (has_x) Dl[slot][i][l1] = use_old ? R.xs[i] + beta * R.xd[i] : R.xs[i];
            if (CG && own && m >= 1 && m <= nx) dnew[i * n + (int64_t)(x0 - 1 + m) * plane + o0] = d;
        }
    };
    fetch(ra, 0);
    if (DEEP) {
        fetch(rb, 1);
        store(ra, 0);
        store(rb, 1);
        fetch(ra, min(2, nx + 1));
    } else {
        store(ra, 0);
        fetch(ra, 1);
        store(ra, 1);
    }
    T le = lam[(int64_t)wrap_el(x0 - 1, g.n0) * plane + o0];
    T me = mu[(int64_t)wrap_el(x0 - 1, g.n0) * plane + o0];
    __syncthreads();

    T carry[3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) carry[i][k] = (T)0;
    double dot = 0.0;
    // steps in pairs, so that the register sets swap roles statically: `cur`
    // holds plane j + 2 (stored at the end of step j), `nxt` receives the
    // plane fetched at step j (the last steps reload plane nx + 1)
    for (int j0 = 0; j0 <= nx; j0 += 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = j0 + h;
            if (j > nx) break;
            Stage& cur = (DEEP && h) ? rb : ra;
            Stage& nxt = DEEP ? (h ? ra : rb) : ra;
            const bool more = j + 2 <= nx + 1;
            // Lame values of voxel plane x0 + j, used at step j + 1 (the last
            // step reloads plane x0 + nx - 1, unused); loaded before the
            // operand plane, so that their wait leaves that plane in flight
            const int64_t e = (int64_t)wrap_el(x0 + min(j, nx - 1), g.n0) * plane + o0;
            const T ln = lam[e], mn = mu[e];
            fetch(nxt, min(j + (DEEP ? 3 : 2), nx + 1));
            T U[3][8];
            const int sa = j % 3, sb = (j + 1) % 3;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                U[i][0] = Dl[sa][i][l0];
                U[i][1] = Dl[sa][i][l0 + 1];
                U[i][2] = Dl[sa][i][l0 + kElL];
                U[i][3] = Dl[sa][i][l0 + kElL + 1];
                U[i][4] = Dl[sb][i][l0];
                U[i][5] = Dl[sb][i][l0 + 1];
                U[i][6] = Dl[sb][i][l0 + kElL];
                U[i][7] = Dl[sb][i][l0 + kElL + 1];
            }
            const T dself[3] = {U[0][0], U[1][0], U[2][0]};
            el_element<T>(E, le * (T)E.w8, me * (T)E.w8, U);  // U becomes the corner forces
            // node plane j - 1 + x0: corners a = 0 of this voxel plus the carry
            T own_f[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T c1 = carry[i][1] + U[i][1], c2 = carry[i][2] + U[i][2], c3 = carry[i][3] + U[i][3];
                own_f[i] = carry[i][0] + U[i][0];
                if (j >= 1) {
                    X[j & 1][i * 3 + 0][t] = c1;  // corner (0, 1): node (ly, lz + 1)
                    X[j & 1][i * 3 + 1][t] = c2;  // corner (1, 0): node (ly + 1, lz)
                    X[j & 1][i * 3 + 2][t] = c3;  // corner (1, 1)
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) carry[i][k] = U[i][4 + k];
            }
            if (more) store(cur, j + 2);
            le = ln;
            me = mn;
            __syncthreads();
            if (j >= 1 && own) {
                const int64_t b = (int64_t)(x0 - 1 + j) * plane + o0;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const T y = own_f[i] + X[j & 1][i * 3 + 0][t - 1] + X[j & 1][i * 3 + 1][t - kElT] +
                                     X[j & 1][i * 3 + 2][t - kElT - 1];
                    p[i * n + b] = y;
                    if (CG) dot += (double)dself[i] * (double)y;
                }
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
    // element constants of the Hadamard-basis form: -(2/h_b) r^m, r = 1/sqrt 3,
    // and the Gauss weight times the voxel volume over 8
    const double rr = 1.0 / std::sqrt(3.0);
    for (int b = 0; b < 3; ++b)
        for (int m = 0; m < 3; ++m) out->hc[b][m] = -2.0 / g.h[b] * (m == 0 ? 1.0 : (m == 1 ? rr : rr * rr));
    out->w8 = g.h[0] * g.h[1] * g.h[2] / 64.0;
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

// tiles of 15 x 15 owned nodes in the (1, 2) plane; node planes per
// workgroup chosen for about 4096 workgroups over all right-hand sides
// (two fit a CU), at least 4 (each workgroup also computes the voxel plane
// below its first node plane)
ElGeom el_geom(const Grid& g, int nrhs)
{
    ElGeom eg;
    eg.tiles_y = (g.n[1] + kElO - 1) / kElO;
    eg.tiles_z = (g.n[2] + kElO - 1) / kElO;
    const int64_t tiles = (int64_t)eg.tiles_y * eg.tiles_z * (nrhs > 0 ? nrhs : 1);
    int xb = (int)((g.n[0] * tiles + 4095) / 4096);
    if (xb < 4) xb = 4;
    if (xb > g.n[0]) xb = g.n[0];
    eg.tiles_x = (g.n[0] + xb - 1) / xb;
    eg.xb = (g.n[0] + eg.tiles_x - 1) / eg.tiles_x;  // even split of the planes
    return eg;
}

int el_march_blocks(const Grid& g, int nrhs)
{
    const ElGeom eg = el_geom(g, nrhs);
    return eg.tiles_x * eg.tiles_y * eg.tiles_z;
}

template <typename T, bool CG, bool HEAD>
uno_status launch_el_apply(const ElDev& E, const Grid& g, const T* lam, const T* mu, int64_t lks, const T* s,
                           const T* dold, T* dnew, T* p, double* part_dp, const CgIter& it, const double* part_rs,
                           int np_rs, double* gam, int nrhs, hipStream_t st)
{
    const ElGeom eg = el_geom(g, nrhs);
    uno_launch(CG ? UNO_KT_MATVEC : UNO_KT_APPLY, k_el_march<T, CG, HEAD>,
               dim3(eg.tiles_x * eg.tiles_y * eg.tiles_z, nrhs), dim3(256), 0, st, E, eg, lam, mu, lks, s, dold,
               dnew, p, part_dp, it, part_rs, np_rs, gam);
    return hip_status(hipGetLastError());
}
#define UNO_EL_APPLY(T, CG, HEAD)                                                                               \
    template uno_status launch_el_apply<T, CG, HEAD>(const ElDev&, const Grid&, const T*, const T*, int64_t,  \
                                                     const T*, const T*, T*, T*, double*, const CgIter&,     \
                                                     const double*, int, double*, int, hipStream_t);
UNO_EL_APPLY(double, false, false)
UNO_EL_APPLY(double, true, false)
UNO_EL_APPLY(double, true, true)
UNO_EL_APPLY(float, true, false)
#undef UNO_EL_APPLY

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
