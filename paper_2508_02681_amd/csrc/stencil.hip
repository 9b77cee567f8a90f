// Matrix-free operator, Jacobi diagonal, right-hand side and flux average of
// the periodic voxel FE discretization (Sec. 3.1, Sec. 5.1 of the paper).
//
// Node-centred formulation.  Node i touches the 8 voxels i + sigma,
// sigma in {-1,0}^3 (node i is their corner -sigma).  Assembling the
// element matrices (exact integration of the multilinear element, a tensor
// product of 1D stiffness and mass matrices) gives
//   (A u)_i = sum_{delta in {-1,0,1}^3} w[m(delta)] * kappa_sum(i, delta) * u_{i+delta}
// where m(delta) flags the axes along which delta is non-zero and
// kappa_sum adds the conductivities of the voxels that contain both nodes
// (axis b: delta_b = -1 -> sigma_b = -1; +1 -> sigma_b = 0; 0 -> both).
#include "unocg_internal.h"
#include "reduce.h"
#include "stencil_tile.h"

#include <cstring>

namespace unocg {

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ void load_kappa8(const GridDev& g, const T* __restrict__ kappa, int x, int y, int z,
                                            T k[2][2][2])
{
#pragma unroll
    for (int s0 = 0; s0 < 2; ++s0)
#pragma unroll
        for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                int xx = wrapi(x - 1 + s0, g.n0), yy = wrapi(y - 1 + s1, g.n1), zz = wrapi(z - 1 + s2, g.n2);
                k[s0][s1][s2] = kappa[((int64_t)xx * g.n1 + yy) * g.n2 + zz];
            }
}

// out = r / diag(A), diag = cdiag * sum of the 8 voxel conductivities.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_jacobi_node(GridDev g, const T* __restrict__ kappa,
                                                        const T* __restrict__ r, T* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    int z = (int)(i % g.n2);
    int64_t t = i / g.n2;
    int yy = (int)(t % g.n1);
    int x = (int)(t / g.n1);
    T k[2][2][2];
    load_kappa8(g, kappa, x, yy, z, k);
    T s = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += k[q >> 2][(q >> 1) & 1][q & 1];
    out[i] = r[i] / ((T)g.cdiag * s);
}

// f_i = -sum_sigma kappa_sigma |Omega_e| sum_b dN/dx_b(centre) gbar_b with
// dN/dx_b(centre) = (2 s_b - 1) / (4 h_b) for corner s = -sigma.
template <typename TK, typename T>
__global__ void __launch_bounds__(kBlock) k_rhs_node(GridDev g, const TK* __restrict__ kappa, double g0, double g1,
                                                     double g2, T* __restrict__ f)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    int z = (int)(i % g.n2);
    int64_t t = i / g.n2;
    int yy = (int)(t % g.n1);
    int x = (int)(t / g.n1);
    TK k[2][2][2];
    load_kappa8(g, kappa, x, yy, z, k);
    const double c0 = g0 * g.gcoef[0], c1 = g1 * g.gcoef[1], c2 = g2 * g.gcoef[2];
    double acc = 0.0;
#pragma unroll
    for (int s0 = 0; s0 < 2; ++s0)
#pragma unroll
        for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                // index s_b = 0 is sigma_b = -1 (node is the upper corner, 2s-1 = +1)
                double dirsum = (s0 ? -c0 : c0) + (s1 ? -c1 : c1) + (s2 ? -c2 : c2);
                acc += (double)k[s0][s1][s2] * dirsum;
            }
    f[i] = (T)(-g.hvol * acc);
}

// Per-voxel flux kappa_e (gbar + grad u(centre_e)), summed per workgroup.
template <typename TK>
__global__ void __launch_bounds__(kBlock) k_flux_voxel(GridDev g, const TK* __restrict__ kappa, double g0,
                                                       double g1, double g2, const double* __restrict__ u,
                                                       double* __restrict__ partials)
{
    __shared__ double slots[kBlock / 64];
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    if (e < g.n) {
        int z = (int)(e % g.n2);
        int64_t t = e / g.n2;
        int yy = (int)(t % g.n1);
        int x = (int)(t / g.n1);
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int s0 = 0; s0 < 2; ++s0)
#pragma unroll
            for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    int xx = wrapi(x + s0, g.n0), y2 = wrapi(yy + s1, g.n1), zz = wrapi(z + s2, g.n2);
                    double v = u[((int64_t)xx * g.n1 + y2) * g.n2 + zz];
                    d0 += s0 ? v : -v;
                    d1 += s1 ? v : -v;
                    d2 += s2 ? v : -v;
                }
        double ke = (double)kappa[e];
        q0 = ke * (g0 + d0 * g.gcoef[0]);
        q1 = ke * (g1 + d1 * g.gcoef[1]);
        q2 = ke * (g2 + d2 * g.gcoef[2]);
    }
    double r0 = block_reduce<OpSum>(q0, slots);
    double r1 = block_reduce<OpSum>(q1, slots);
    double r2 = block_reduce<OpSum>(q2, slots);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = r0;
        partials[3 * blockIdx.x + 1] = r1;
        partials[3 * blockIdx.x + 2] = r2;
    }
}

static int nblocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

uno_status launch_fe_apply(const Grid& g, const void* kappa, const void* u, void* y, uno_dtype t, hipStream_t s)
{
    CgIter none;
    memset(&none, 0, sizeof(none));
    if (t == UNO_F64)
        launch_tile<double, false, false>(g, (const double*)kappa, (const double*)u, nullptr, nullptr, (double*)y,
                                          nullptr, none, nullptr, 0, nullptr, s);
    else
        launch_tile<float, false, false>(g, (const float*)kappa, (const float*)u, nullptr, nullptr, (float*)y, nullptr,
                                         none, nullptr, 0, nullptr, s);
    return hip_status(hipGetLastError());
}

uno_status launch_jacobi(const Grid& g, const void* kappa, const void* r, void* out, uno_dtype t, hipStream_t s)
{
    int nb = nblocks_for(g.total);
    if (t == UNO_F64)
        hipLaunchKernelGGL(k_jacobi_node<double>, dim3(nb), dim3(kBlock), 0, s, g.dev, (const double*)kappa,
                           (const double*)r, (double*)out);
    else
        hipLaunchKernelGGL(k_jacobi_node<float>, dim3(nb), dim3(kBlock), 0, s, g.dev, (const float*)kappa,
                           (const float*)r, (float*)out);
    return hip_status(hipGetLastError());
}

uno_status launch_rhs(const Grid& g, const void* kappa, uno_dtype kt, const double gbar[3], void* f, uno_dtype t,
                      hipStream_t s)
{
    int nb = nblocks_for(g.total);
    if (kt == UNO_F64 && t == UNO_F64)
        hipLaunchKernelGGL((k_rhs_node<double, double>), dim3(nb), dim3(kBlock), 0, s, g.dev, (const double*)kappa,
                           gbar[0], gbar[1], gbar[2], (double*)f);
    else if (kt == UNO_F32 && t == UNO_F32)
        hipLaunchKernelGGL((k_rhs_node<float, float>), dim3(nb), dim3(kBlock), 0, s, g.dev, (const float*)kappa,
                           gbar[0], gbar[1], gbar[2], (float*)f);
    else if (kt == UNO_F32 && t == UNO_F64)
        hipLaunchKernelGGL((k_rhs_node<float, double>), dim3(nb), dim3(kBlock), 0, s, g.dev, (const float*)kappa,
                           gbar[0], gbar[1], gbar[2], (double*)f);
    else
        return UNO_ERR_ARG;
    return hip_status(hipGetLastError());
}

uno_status launch_flux(const Grid& g, const void* kappa, uno_dtype kt, const double gbar[3], const double* u,
                       double* partials, int* nblocks, hipStream_t s)
{
    int nb = nblocks_for(g.total);
    *nblocks = nb;
    if (kt == UNO_F64)
        hipLaunchKernelGGL(k_flux_voxel<double>, dim3(nb), dim3(kBlock), 0, s, g.dev, (const double*)kappa, gbar[0],
                           gbar[1], gbar[2], u, partials);
    else
        hipLaunchKernelGGL(k_flux_voxel<float>, dim3(nb), dim3(kBlock), 0, s, g.dev, (const float*)kappa, gbar[0],
                           gbar[1], gbar[2], u, partials);
    return hip_status(hipGetLastError());
}

}  // namespace unocg
