// Gradient of the effective conductivity with respect to the voxel
// conductivities.
//
// kappa_bar is read from the solutions t_a of the cell problems for the loads
// g_a (Sec. 5.1); in energy form, g_a . kappa_bar g_b = (1/|Omega|) sum_e
// kappa_e int_e (g_a + grad t_a).(g_b + grad t_b).  The cell problem is
// self-adjoint and its weak form holds for every field of the FE space
// (Sec. 3.1), so the solution of one load is the adjoint state of the other
// and the field sensitivities drop out: the total derivative with respect to
// kappa_e is the element energy density
//   D_ab(e) = (1/N_e) [ g_a.g_b + g_a.grad t_b(c_e) + g_b.grad t_a(c_e)
//                       + t_a^T K t_b / |Omega_e| ],
// with K the unit-conductivity element stiffness (corner couplings w[m] of
// the operator) and grad t(c_e) the element-centre gradient (the element
// mean of the gradient of a multilinear field).  No adjoint solve is needed.
// With G = [g_1 .. g_d], kappa_bar = G^-T E G^-1, hence
//   d kappa_bar_ij / d kappa_e = (G^-T D(e) G^-1)_ij.
#include <cmath>
#include <cstring>
#include <utility>

#include "unocg_internal.h"

namespace unocg {

struct GradLoads {
    int nl;            // number of loads (= d)
    double g[3][3];    // loads, embedded in 3D (g[a][axis])
    double m[3][3];    // full Jacobian: G^-1; weighted: G^-1 W G^-T
};

__device__ __forceinline__ int wrap1(int v, int n) { return v >= n ? v - n : v; }

// WEIGHTED: out[e] = sum_ab m_ab D_ab(e); else out[(i nl + j) n + e] = sum_ab m_ai D_ab m_bj
template <bool WEIGHTED>
__global__ void __launch_bounds__(kBlock) k_kbar_grad(GridDev g, GradLoads L, const double* __restrict__ u,
                                                      double* __restrict__ out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.n; e += (int64_t)gridDim.x * blockDim.x) {
        const int z = (int)(e % g.n2);
        const int64_t q = e / g.n2;
        const int y = (int)(q % g.n1), x = (int)(q / g.n1);
        int64_t node[8];
#pragma unroll
        for (int s = 0; s < 8; ++s)
            node[s] = ((int64_t)wrap1(x + (s >> 2), g.n0) * g.n1 + wrap1(y + ((s >> 1) & 1), g.n1)) * g.n2 +
                      wrap1(z + (s & 1), g.n2);
        double t[3][8], gc[3][3];
        for (int a = 0; a < L.nl; ++a) {
            const double* ua = u + (int64_t)a * g.n;
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const double v = ua[node[s]];
                t[a][s] = v;
                d0 += (s >> 2) ? v : -v;
                d1 += ((s >> 1) & 1) ? v : -v;
                d2 += (s & 1) ? v : -v;
            }
            gc[a][0] = d0 * g.gcoef[0];
            gc[a][1] = d1 * g.gcoef[1];
            gc[a][2] = d2 * g.gcoef[2];
        }
        const double inv_ne = 1.0 / (double)g.n, inv_vol = 1.0 / g.hvol;
        double D[3][3];
        for (int a = 0; a < L.nl; ++a)
            for (int b = a; b < L.nl; ++b) {
                double gg = 0.0, cross = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    gg += L.g[a][c] * L.g[b][c];
                    cross += L.g[a][c] * gc[b][c] + L.g[b][c] * gc[a][c];
                }
                double en = 0.0;  // t_a^T K t_b
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    double row = 0.0;
#pragma unroll
                    for (int s2 = 0; s2 < 8; ++s2) row += g.w[s ^ s2] * t[b][s2];
                    en += t[a][s] * row;
                }
                D[a][b] = D[b][a] = inv_ne * (gg + cross + en * inv_vol);
            }
        if (WEIGHTED) {
            double acc = 0.0;
            for (int a = 0; a < L.nl; ++a)
                for (int b = 0; b < L.nl; ++b) acc += L.m[a][b] * D[a][b];
            out[e] = acc;
        } else {
            for (int i = 0; i < L.nl; ++i)
                for (int j = 0; j < L.nl; ++j) {
                    double acc = 0.0;
                    for (int a = 0; a < L.nl; ++a)
                        for (int b = 0; b < L.nl; ++b) acc += L.m[a][i] * D[a][b] * L.m[b][j];
                    out[(int64_t)(i * L.nl + j) * g.n + e] = acc;
                }
        }
    }
}

}  // namespace unocg

using namespace unocg;

namespace {

// inverse of a d x d matrix (d <= 3), false if singular
bool invert(int d, const double a[3][3], double r[3][3])
{
    double m[3][6];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < 2 * d; ++j) m[i][j] = (j < d) ? a[i][j] : (j - d == i ? 1.0 : 0.0);
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int i = c + 1; i < d; ++i)
            if (std::fabs(m[i][c]) > std::fabs(m[piv][c])) piv = i;
        if (!(std::fabs(m[piv][c]) > 1e-300)) return false;
        for (int j = 0; j < 2 * d; ++j) std::swap(m[c][j], m[piv][j]);
        const double p = m[c][c];
        for (int j = 0; j < 2 * d; ++j) m[c][j] /= p;
        for (int i = 0; i < d; ++i) {
            if (i == c) continue;
            const double f = m[i][c];
            for (int j = 0; j < 2 * d; ++j) m[i][j] -= f * m[c][j];
        }
    }
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) r[i][j] = m[i][j + d];
    return true;
}

}  // namespace

extern "C" uno_status effective_tensor_grad(const uno_grid* grid, int32_t nload, const double* loads, const double* u,
                                            const double* weights, double* out, void* stream)
{
    Grid g;
    uno_status e = make_grid(grid, &g);
    if (e != UNO_OK) return e;
    const int d = grid->dim;
    if (nload != d || !loads || !u || !out) return UNO_ERR_ARG;
    GradLoads L;
    memset(&L, 0, sizeof(L));
    L.nl = d;
    double G[3][3] = {{0}}, Gi[3][3];
    for (int a = 0; a < d; ++a)
        for (int c = 0; c < d; ++c) {
            const double v = loads[a * d + c];
            if (!std::isfinite(v)) return UNO_ERR_ARG;
            G[c][a] = v;                 // columns are the loads
            L.g[a][3 - d + c] = v;       // embedded axes
        }
    if (!invert(d, G, Gi)) return UNO_ERR_ARG;
    if (weights) {
        // sum_ij W_ij (G^-T D G^-1)_ij = sum_ab (G^-1 W G^-T)_ab D_ab
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                double acc = 0.0;
                for (int i = 0; i < d; ++i)
                    for (int j = 0; j < d; ++j) acc += Gi[a][i] * weights[i * d + j] * Gi[b][j];
                L.m[a][b] = acc;
            }
    } else {
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) L.m[a][b] = Gi[a][b];
    }
    const int64_t nb = (g.total + kBlock - 1) / kBlock;
    const int blocks = (int)(nb < 4096 ? nb : 4096);
    if (weights)
        hipLaunchKernelGGL(k_kbar_grad<true>, dim3(blocks), dim3(kBlock), 0, (hipStream_t)stream, g.dev, L, u, out);
    else
        hipLaunchKernelGGL(k_kbar_grad<false>, dim3(blocks), dim3(kBlock), 0, (hipStream_t)stream, g.dev, L, u, out);
    return hip_status(hipGetLastError());
}
