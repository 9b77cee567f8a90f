// Internal declarations of the gfx950 UNO-CG library (not part of the ABI).
//
// Every grid is handled as a 3D periodic voxel grid n0 x n1 x n2 (last axis
// contiguous).  A 2D problem n1 x n2 is embedded as 1 x n1 x n2 with a unit
// voxel edge along the dummy axis: with one voxel layer the trilinear element
// collapses onto the bilinear one (both node layers coincide), so operator,
// rhs and fluxes are exactly the 2D ones.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/unocg.h"

namespace unocg {

constexpr int kBlock = 256;          // threads per workgroup of streaming kernels
constexpr int kMaxFftStages = 16;

// Grid descriptor passed to kernels by value.
struct GridDev {
    int n0, n1, n2;   // voxels = nodes per axis
    int64_t n;        // n0 n1 n2
    double w[8];      // stencil weight per offset pattern m = (m0<<2)|(m1<<1)|m2,
                      // m_b = 1 iff the neighbour differs along axis b
    double cdiag;     // diag A = cdiag * sum of the 8 voxel conductivities at a node
    double hvol;      // voxel volume
    double gcoef[3];  // element-centre gradient factor per axis: 1 / (4 h_b)
};

// Host view of a problem grid.
struct Grid {
    int dim;          // 2 or 3 as given by the caller
    int n[3];         // embedded 3D sizes
    double h[3];      // embedded voxel edges
    int64_t total;
    GridDev dev;
};

uno_status make_grid(const uno_grid* g, Grid* out);

// complex helpers
template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };

// Optional per-family kernel timing: when family `fam` is being timed the
// launch carries start/stop events recorded around the dispatch itself
// (hipExtLaunchKernelGGL), otherwise it is a plain launch.
bool ktimer_take(int fam, hipEvent_t* a, hipEvent_t* b);
bool ktimer_active();  // a kernel family is being timed (no stream capture then)
void tune_release_all();  // forget the recorded operator shapes
uint64_t precond_serial();
void ktimer_push(hipEvent_t a, hipEvent_t b);

// Workgroups of a launch go to the 8 XCDs in turn (workgroup i to XCD
// i mod 8, along grid x), and each XCD has an L2 of its own.  Tile kernels
// whose neighbouring tiles share halo planes map workgroup i of n to this
// tile index, so that each XCD works on one contiguous range of tiles and
// the shared lines meet in one L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int i, int n)
{
    const int q = n >> 3, r = n & 7, x = i & 7, j = i >> 3;
    return x * q + (x < r ? x : r) + j;
}

template <typename... Formals, typename... Args>
inline void uno_launch(int fam, void (*kernel)(Formals...), dim3 grid, dim3 block, size_t sh, hipStream_t st,
                       Args... args)
{
    hipEvent_t a, b;
    if (fam != UNO_KT_NONE && ktimer_take(fam, &a, &b)) {
        hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)sh, st, a, b, 0u, args...);
        ktimer_push(a, b);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, sh, st, args...);
    }
}

// Status of the last HIP error inside a launch helper
uno_status hip_status(hipError_t e);

#define UNO_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_status(e_);    \
    } while (0)

// ---------------------------------------------------------------------------
// Stencil family (stencil.hip)
uno_status launch_fe_apply(const Grid& g, const void* kappa, const void* u, void* y, uno_dtype t,
                           hipStream_t s);
uno_status launch_jacobi(const Grid& g, const void* kappa, const void* r, void* out, uno_dtype t,
                         hipStream_t s);
uno_status launch_rhs(const Grid& g, const void* kappa, uno_dtype kt, const double gbar[3], void* f,
                      uno_dtype t, hipStream_t s);
// per-block partial flux sums: out has 3 * nblocks doubles, returns nblocks
uno_status launch_flux(const Grid& g, const void* kappa, uno_dtype kt, const double gbar[3],
                       const double* u, double* partials, int* nblocks, hipStream_t s);

// ---------------------------------------------------------------------------
// FFT family (fft.hip)
struct AxisPlan {
    int n;
    int nstages;
    int radix[kMaxFftStages];
    double2* tw64;    // exp(-2 pi i j / n), j < n
    float2* tw32;
};

struct FftPlan {
    AxisPlan ax[3];
    int nh;           // n2 / 2 + 1
    int64_t nspec;    // n0 n1 nh complex values
};

// twiddles_only: the tables exp(-2 pi i j / n_b) for any n_b (what the
// learned-mode passes use), without the factorization the full passes need
uno_status fft_plan_create(const Grid& g, FftPlan* p, bool twiddles_only = false);
void fft_plan_destroy(FftPlan* p);

struct CgIter;  // per-pass control of the CG loop (cg_ctl.h)

// s = (1/n) F^H diag(table) F r.  `spec` scratch holds nspec complex values of
// the vector precision.  it != nullptr: the passes belong to CG pass it->k,
// the first one runs the convergence test of that pass, every one returns at
// once when the loop has ended, and the last one writes per-workgroup r.s
// partials (their count is returned in *np_rs).  nrhs > 1 (FP64 inside CG
// only): right-hand side b along grid y, its vectors at + b it->vs, its
// spectrum at + b sst.
uno_status uno_apply_passes(const Grid& g, const FftPlan& p, const void* table, uno_dtype table_t,
                            const void* r, void* s, uno_dtype vec_t, void* spec, const CgIter* it, int* np_rs,
                            hipStream_t stream, int nrhs = 1, int64_t sst = 0);

// Forward transform of nbatch real fields into half spectra (training).
uno_status fft_forward_real(const Grid& g, const FftPlan& p, const double* x, double2* spec,
                            hipStream_t stream);

// ---------------------------------------------------------------------------
// CG (cg.hip): solver state kept on the device
struct CgState {
    double r0max;     // ||r_0||_inf
    double tol_abs;   // rtol * r0max
    double rmax_last; // last reduced ||r||_inf
    double mean;      // mean of u at the end
    double fmax, dmax;  // ||f||_inf, ||f - A u||_inf at the end
    int done;         // passes completed when the loop ended (INT_MAX while running)
    int status;       // 0 ok, 1 breakdown
    int k_last;       // pass index of rmax_last
    int fail_iter;    // pass of a breakdown
};

// ---------------------------------------------------------------------------
// UNO apply restricted to the learned modes (lowrank.hip)
struct LowRankPlan;
// row-chunk partials and H of nrhs right-hand sides (the plan's own for one),
// and the row split of pass A for that many: rb rows per workgroup, nch
// chunks per x-slab (fewer, longer chunks when many right-hand sides fill
// the chip anyway; pass B then gathers less)
struct LrBatch {
    double2* Gp;
    double2* H;
    int nrhs;
    int rb, nch;   // pass A: rows per workgroup, row chunks per slab
    int yc;        // pass C: rows per workgroup
    int cb;        // pass B: columns per workgroup (outside the fused flow)
    bool bf = false;  // BF16 storage of Gp, H and the table (one nodal DOF, outside the fused flow)
};
// nc = 1: cblock kxn x kyn x kzn corrections, W the bypass; nc = 3: six
// entries per block mode (q1..q6) and the bypass block Wq (6 entries)
uno_status lowrank_create(const Grid& g, const FftPlan& fp, int M, double W, const std::vector<double>& cblock,
                          LowRankPlan** out, int nc = 1, const double* Wq = nullptr);
void lowrank_destroy(LowRankPlan* p);
int lowrank_max_blocks(const LowRankPlan* p);
int lowrank_update_blocks(const LowRankPlan* p, int nrhs);
LrBatch lowrank_batch(const LowRankPlan* p, double2* Gp, double2* H, int nrhs);
void lowrank_scratch_size(const LowRankPlan* p, int64_t* ngp, int64_t* nh);
uno_status lowrank_apply(const LowRankPlan* p, const double* r, double* s, hipStream_t st);
uno_status lowrank_forward(const LowRankPlan* p, const double* r, double* part_rr, const LrBatch& bt,
                           const CgIter& strides, hipStream_t st);
template <typename T>
uno_status lowrank_update_forward(const LowRankPlan* p, double* r, double* u, const T* d, const T* pv,
                                  const CgIter& it, const double* part_dp, int np_dp, const double* gam,
                                  double* part_rmax, double* part_rr, const LrBatch& bt, hipStream_t st);
bool lowrank_fused(const LowRankPlan* p);
uno_status lowrank_fused_pass(const LowRankPlan* p, const Grid& g, const double* kappa, const double* r,
                              const double* dold, double* dnew, double* pv, double* part_dp, const CgIter& it,
                              double* part_corr, const double* part_rr, double* gam, const LrBatch& bt,
                              hipStream_t st, int* np_dp);
template <typename T>
uno_status lowrank_finish(const LowRankPlan* p, const double* r, T* s, const CgIter* it, int* np_rs,
                          const LrBatch& bt, hipStream_t st);
int fft_c2r_blocks(const Grid& g, const FftPlan& p);

// linear elasticity, c = 3 (elastic.hip)
struct ElDev {
    GridDev g;
    double hvol;
    double gc[3];        // centre gradient factor per axis 1 / (4 h_b)
    double hc[3][3];     // -(2/h_b) r^m, r = 1/sqrt 3 (Hadamard-basis element)
    double w8;           // Gauss weight times voxel volume / 8
    const double* K;     // 2 x 576 unit element matrices (device)
};
struct ElGeom {
    int tiles_y, tiles_z, xb, tiles_x;
};
ElGeom el_geom(const Grid& g, int nrhs);
int el_march_blocks(const Grid& g, int nrhs);
uno_status el_dev(const Grid& g, ElDev* out);
void el_release_all();
int el_blocks(const Grid& g);
template <typename T, bool CG, bool HEAD>
uno_status launch_el_apply(const ElDev& E, const Grid& g, const T* lam, const T* mu, int64_t lks, const T* s,
                           const T* dold, T* dnew, T* p, double* part_dp, const CgIter& it, const double* part_rs,
                           int np_rs, double* gam, int nrhs, hipStream_t st);
uno_status launch_el_inv_diag(const ElDev& E, const Grid& g, const double* lam, const double* mu, int64_t ks,
                              int nfields, double* dinv, hipStream_t st);
uno_status launch_el_rhs(const ElDev& E, const Grid& g, const double* lam, const double* mu, const double* eps,
                         double* f, hipStream_t st);
uno_status el_stress_average(const ElDev& E, const Grid& g, const double* lam, const double* mu, const double* eps,
                             const double* u, double* out, hipStream_t st);

}  // namespace unocg

// uno_precond layout (opaque to callers)
struct uno_precond {
    unocg::Grid grid;
    unocg::FftPlan plan;
    int M;
    uno_dtype table_t;    // precision the table values were rounded to
    double* table;        // device half spectrum, scaled by 1/n (FP64 applies)
    float* table32;       // the same in FP32 (FP32 applies)
    double* table_host;   // unscaled Phi on the half spectrum (after rounding)
    void* spec;           // scratch spectrum (FP64 complex, nspec values)
    unocg::LowRankPlan* lr;  // learned-mode passes (UNO tables only), or null
    int path;             // UNO_PATH_*
    int nc;               // nodal DOF the preconditioner acts on (1, or 3 for elasticity)
    int rs_blocks;        // most r.s partials any apply path writes
    int device;
    uint64_t serial;      // distinct for every preconditioner the process creates (keys captured graphs)
};

// apply path of a preconditioner in FP64
inline bool uno_use_lowrank(const uno_precond* p)
{
    return p->lr != nullptr && p->path != UNO_PATH_SPECTRAL;
}

// learned-mode passes with the last one folded into the operator (FP64 CG)
inline bool uno_use_fused(const uno_precond* p)
{
    return uno_use_lowrank(p) && p->path == UNO_PATH_FUSED && unocg::lowrank_fused(p->lr);
}
