// UNO preconditioner apply restricted to the learned modes.
//
// The UNO table is Phi(k) = W on every mode outside the learned block
// [-M..M]^(d-1) x [-M..M] (Sec. 4.2.2: modes outside K and its conjugate set
// carry only the bypass) and 0 at k = 0, so with C = Phi - W (zero outside
// the block, -W at k = 0) the operator s = T^H Phi T r of eq. (FNOCG-prec-
// fields-disc) is exactly
//   s = W r + T^H (C o T r),
// and the second term only needs the DFT coefficients of r on the block.
// For real r and a table with C(-k) = C(k) it is
//   (1/n) Re sum_{k in block, k_z >= 0} w(k_z) C(k) R(k) exp(+2 pi i k.x / N),
// with R(k) = sum_x r(x) exp(-2 pi i k.x / N), w = 1 for k_z = 0, 2 else.
// Three passes (the table stored here already holds w(k_z) C(k) / n):
//   A. per x-slab: partial DFT along z (k_z in [0, M]) then along y
//      (k_y in [-M, M]) -> G[x][k_y][k_z]      (also the CG convergence test)
//   B. per (k_y, k_z) column: partial DFT along x, multiply by the table,
//      inverse along x -> H[x][k_y][k_z]
//   C. per x-slab and row chunk: inverse along y, real inverse along z,
//      s = W r + correction (and the r.s partials inside CG).
// The passes move about 3 vectors of the grid (read r twice, write s) plus a
// small coefficient buffer, instead of five passes over the half spectrum.
#include <cmath>
#include <cstring>

#include "unocg_internal.h"
#include "reduce.h"
#include "cg_ctl.h"

namespace unocg {

struct LowRankDev {
    int n0, n1, n2;
    int mx, m;          // learned half-widths along x (0 for one voxel layer) and y, z
    int kxn, kyn, kzn;  // 2mx+1, 2m+1, m+1
    double W;           // bypass theta0^2
    const double2* twx; // exp(-2 pi i j / n_b) tables
    const double2* twy;
    const double2* twz;
};

__device__ __forceinline__ int mod_n(int64_t v, int n)
{
    int r = (int)(v % n);
    return r < 0 ? r + n : r;
}

// Pass A: one workgroup per (x-slab, k_z chunk).
__global__ void __launch_bounds__(256) k_lr_fwd(LowRankDev L, int kz_chunk, const double* __restrict__ r,
                                                double2* __restrict__ G, CgIter it)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    if (it.st && head_check(it, slots)) return;
    const int nchunks = (L.kzn + kz_chunk - 1) / kz_chunk;
    const int x = blockIdx.x / nchunks;
    const int kz0 = (blockIdx.x % nchunks) * kz_chunk;
    const int nkz = min(kz_chunk, L.kzn - kz0);
    double2* twz = (double2*)smem;          // n2
    double2* twy = twz + L.n2;              // n1
    double2* Z = twy + L.n1;                // n1 x nkz
    for (int j = threadIdx.x; j < L.n2; j += blockDim.x) twz[j] = L.twz[j];
    for (int j = threadIdx.x; j < L.n1; j += blockDim.x) twy[j] = L.twy[j];
    __syncthreads();
    const double* slab = r + (int64_t)x * L.n1 * L.n2;
    // Z[y][kz] = sum_z r(x, y, z) exp(-2 pi i kz z / n2)
    for (int q = threadIdx.x; q < L.n1 * nkz; q += blockDim.x) {
        const int y = q / nkz, kz = kz0 + q % nkz;
        const double* row = slab + (int64_t)y * L.n2;
        double re = 0.0, im = 0.0;
        int t = 0;
        for (int z = 0; z < L.n2; ++z) {
            const double v = row[z];
            const double2 w = twz[t];
            re += v * w.x;
            im += v * w.y;
            t += kz;
            if (t >= L.n2) t -= L.n2;
        }
        Z[q] = make_double2(re, im);
    }
    __syncthreads();
    // G[x][ky][kz] = sum_y Z[y][kz] exp(-2 pi i ky y / n1), ky in [-m, m]
    for (int q = threadIdx.x; q < L.kyn * nkz; q += blockDim.x) {
        const int kyi = q / nkz, kzl = q % nkz;
        const int ky = kyi - L.m;
        const int step = mod_n(ky, L.n1);
        double re = 0.0, im = 0.0;
        int t = 0;
        for (int y = 0; y < L.n1; ++y) {
            const double2 a = Z[y * nkz + kzl];
            const double2 w = twy[t];
            re += a.x * w.x - a.y * w.y;
            im += a.x * w.y + a.y * w.x;
            t += step;
            if (t >= L.n1) t -= L.n1;
        }
        G[((int64_t)x * L.kyn + kyi) * L.kzn + kz0 + kzl] = make_double2(re, im);
    }
}

// Pass B: one wavefront per (k_y, k_z) column.
__global__ void __launch_bounds__(64) k_lr_mid(LowRankDev L, const double* __restrict__ C,
                                               const double2* __restrict__ G, double2* __restrict__ H, CgIter it)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (it.st && loop_ended(it.st, it.k)) return;
    const int col = blockIdx.x;  // ky index * kzn + kz
    const int plane = L.kyn * L.kzn;
    double2* twx = (double2*)smem;  // n0
    double2* gx = twx + L.n0;       // n0
    double2* X = gx + L.n0;         // kxn
    for (int j = threadIdx.x; j < L.n0; j += blockDim.x) {
        twx[j] = L.twx[j];
        gx[j] = G[(int64_t)j * plane + col];
    }
    __syncthreads();
    for (int kxi = threadIdx.x; kxi < L.kxn; kxi += blockDim.x) {
        const int kx = kxi - L.mx;
        const int step = mod_n(kx, L.n0);
        double re = 0.0, im = 0.0;
        int t = 0;
        for (int x = 0; x < L.n0; ++x) {
            const double2 a = gx[x];
            const double2 w = twx[t];
            re += a.x * w.x - a.y * w.y;
            im += a.x * w.y + a.y * w.x;
            t += step;
            if (t >= L.n0) t -= L.n0;
        }
        const double c = C[(int64_t)kxi * plane + col];
        X[kxi] = make_double2(re * c, im * c);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < L.n0; x += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int kxi = 0; kxi < L.kxn; ++kxi) {
            const int kx = kxi - L.mx;
            const double2 w = twx[mod_n((int64_t)kx * x, L.n0)];  // conj gives exp(+i ...)
            const double2 a = X[kxi];
            re += a.x * w.x + a.y * w.y;
            im += a.y * w.x - a.x * w.y;
        }
        H[(int64_t)x * plane + col] = make_double2(re, im);
    }
}

// Pass C: one workgroup per (x-slab, chunk of rows y).
template <bool CG>
__global__ void __launch_bounds__(256) k_lr_inv(LowRankDev L, int y_chunk, const double* __restrict__ r,
                                                const double2* __restrict__ H, double* __restrict__ s, CgIter it)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    if (CG && loop_ended(it.st, it.k)) return;
    const int nch = (L.n1 + y_chunk - 1) / y_chunk;
    const int x = blockIdx.x / nch;
    const int y0 = (blockIdx.x % nch) * y_chunk;
    const int ny = min(y_chunk, L.n1 - y0);
    const int plane = L.kyn * L.kzn;
    double2* twz = (double2*)smem;       // n2
    double2* twy = twz + L.n2;           // n1
    double2* Hs = twy + L.n1;            // kyn x kzn
    double2* V = Hs + plane;             // ny x kzn
    for (int j = threadIdx.x; j < L.n2; j += blockDim.x) twz[j] = L.twz[j];
    for (int j = threadIdx.x; j < L.n1; j += blockDim.x) twy[j] = L.twy[j];
    for (int j = threadIdx.x; j < plane; j += blockDim.x) Hs[j] = H[(int64_t)x * plane + j];
    __syncthreads();
    // V[y][kz] = sum_ky H[x][ky][kz] exp(+2 pi i ky y / n1)
    for (int q = threadIdx.x; q < ny * L.kzn; q += blockDim.x) {
        const int yl = q / L.kzn, kz = q % L.kzn;
        const int y = y0 + yl;
        double re = 0.0, im = 0.0;
        for (int kyi = 0; kyi < L.kyn; ++kyi) {
            const int ky = kyi - L.m;
            const double2 w = twy[mod_n((int64_t)ky * y, L.n1)];
            const double2 a = Hs[kyi * L.kzn + kz];
            re += a.x * w.x + a.y * w.y;
            im += a.y * w.x - a.x * w.y;
        }
        V[q] = make_double2(re, im);
    }
    __syncthreads();
    // s = W r + Re sum_kz V[y][kz] exp(+2 pi i kz z / n2)
    double acc = 0.0;
    for (int q = threadIdx.x; q < ny * L.n2; q += blockDim.x) {
        const int yl = q / L.n2, z = q % L.n2;
        double c = 0.0;
        int t = 0;
        for (int kz = 0; kz < L.kzn; ++kz) {
            const double2 w = twz[t];
            const double2 a = V[yl * L.kzn + kz];
            c += a.x * w.x + a.y * w.y;  // Re(a * conj(w))
            t += z;
            if (t >= L.n2) t -= L.n2;
        }
        const int64_t i = ((int64_t)x * L.n1 + y0 + yl) * L.n2 + z;
        const double rv = r[i];
        const double sv = L.W * rv + c;
        s[i] = sv;
        if (CG) acc += rv * sv;
    }
    if (CG) {
        const double b = block_reduce<OpSum>(acc, slots);
        if (threadIdx.x == 0) it.part_rs[blockIdx.x] = b;
    }
}

// ----------------------------------------------------------------------------
// host

struct LowRankPlan {
    LowRankDev dev;
    double* table;    // kxn x kyn x kzn, w(kz) C(k) / n
    double2* G;       // n0 x kyn x kzn
    double2* H;
    int kz_chunk, y_chunk;
    int blocks_a, blocks_c;
};

static int pick_chunk(int total, int per_slab_target) { return (total + per_slab_target - 1) / per_slab_target; }

uno_status lowrank_create(const Grid& g, const FftPlan& fp, int M, double W, const std::vector<double>& cblock,
                          LowRankPlan** out)
{
    LowRankPlan* p = new LowRankPlan();
    memset(p, 0, sizeof(*p));
    LowRankDev& L = p->dev;
    L.n0 = g.n[0];
    L.n1 = g.n[1];
    L.n2 = g.n[2];
    L.mx = (g.n[0] == 1) ? 0 : M;
    L.m = M;
    L.kxn = 2 * L.mx + 1;
    L.kyn = 2 * M + 1;
    L.kzn = M + 1;
    L.W = W;
    L.twx = fp.ax[0].tw64;
    L.twy = fp.ax[1].tw64;
    L.twz = fp.ax[2].tw64;
    const int64_t nb = (int64_t)L.kxn * L.kyn * L.kzn;
    const int64_t ng = (int64_t)L.n0 * L.kyn * L.kzn;
    if ((int64_t)cblock.size() != nb) { delete p; return UNO_ERR_ARG; }
    // about four workgroups per slab in passes A and C
    p->kz_chunk = pick_chunk(L.kzn, g.n[0] >= 64 ? 4 : (g.n[0] >= 16 ? 8 : 16));
    p->y_chunk = pick_chunk(L.n1, g.n[0] >= 64 ? 4 : (g.n[0] >= 16 ? 8 : 16));
    if (p->kz_chunk < 1) p->kz_chunk = 1;
    if (p->y_chunk < 1) p->y_chunk = 1;
    const size_t lds_a = sizeof(double2) * ((size_t)L.n2 + L.n1 + (size_t)L.n1 * p->kz_chunk);
    const size_t lds_c = sizeof(double2) * ((size_t)L.n2 + L.n1 + (size_t)L.kyn * L.kzn + (size_t)p->y_chunk * L.kzn);
    const size_t lds_b = sizeof(double2) * (2 * (size_t)L.n0 + L.kxn);
    if (lds_a > 60 * 1024 || lds_b > 60 * 1024 || lds_c > 60 * 1024) { delete p; return UNO_ERR_SHAPE; }
    if (hipMalloc(&p->table, sizeof(double) * nb) != hipSuccess || hipMalloc(&p->G, sizeof(double2) * ng) != hipSuccess ||
        hipMalloc(&p->H, sizeof(double2) * ng) != hipSuccess) {
        (void)hipFree(p->table);
        (void)hipFree(p->G);
        delete p;
        return UNO_ERR_NOMEM;
    }
    UNO_HIP(hipMemcpy(p->table, cblock.data(), sizeof(double) * nb, hipMemcpyHostToDevice));
    p->blocks_a = L.n0 * ((L.kzn + p->kz_chunk - 1) / p->kz_chunk);
    p->blocks_c = L.n0 * ((L.n1 + p->y_chunk - 1) / p->y_chunk);
    *out = p;
    return UNO_OK;
}

void lowrank_destroy(LowRankPlan* p)
{
    if (!p) return;
    (void)hipFree(p->table);
    (void)hipFree(p->G);
    (void)hipFree(p->H);
    delete p;
}

int lowrank_rs_blocks(const LowRankPlan* p) { return p->blocks_c; }

uno_status lowrank_apply(const LowRankPlan* p, const double* r, double* s, const CgIter* itp, int* np_rs,
                         hipStream_t st)
{
    const LowRankDev& L = p->dev;
    CgIter it;
    memset(&it, 0, sizeof(it));
    if (itp) it = *itp;
    KTimer kt;
    {
        size_t sh = sizeof(double2) * ((size_t)L.n2 + L.n1 + (size_t)L.n1 * p->kz_chunk);
        ktimer_begin(&kt, UNO_KT_FFT_FWD, st);
        hipLaunchKernelGGL(k_lr_fwd, dim3(p->blocks_a), dim3(256), sh, st, L, p->kz_chunk, r, p->G, it);
        ktimer_end(&kt);
        UNO_HIP(hipGetLastError());
    }
    {
        size_t sh = sizeof(double2) * (2 * (size_t)L.n0 + L.kxn);
        ktimer_begin(&kt, UNO_KT_FFT_MID, st);
        hipLaunchKernelGGL(k_lr_mid, dim3(L.kyn * L.kzn), dim3(64), sh, st, L, (const double*)p->table,
                           (const double2*)p->G, p->H, it);
        ktimer_end(&kt);
        UNO_HIP(hipGetLastError());
    }
    {
        size_t sh = sizeof(double2) * ((size_t)L.n2 + L.n1 + (size_t)L.kyn * L.kzn + (size_t)p->y_chunk * L.kzn);
        ktimer_begin(&kt, UNO_KT_FFT_INV, st);
        if (itp)
            hipLaunchKernelGGL(k_lr_inv<true>, dim3(p->blocks_c), dim3(256), sh, st, L, p->y_chunk, r,
                               (const double2*)p->H, s, it);
        else
            hipLaunchKernelGGL(k_lr_inv<false>, dim3(p->blocks_c), dim3(256), sh, st, L, p->y_chunk, r,
                               (const double2*)p->H, s, it);
        ktimer_end(&kt);
        UNO_HIP(hipGetLastError());
    }
    if (np_rs) *np_rs = p->blocks_c;
    return UNO_OK;
}

}  // namespace unocg
