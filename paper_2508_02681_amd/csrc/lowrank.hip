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

// Pass A on the rows y0 .. y0+ny-1 of slab x: Z[y][kz] = sum_z r e^{-i kz z},
// then the partial y-sum of these rows, Gp[x][chunk][ky][kz] =
// sum_{y in rows} Z[y][kz] e^{-i ky y}; pass B adds the chunks in order.
// UPDATE (inside CG): the rows are first updated, r <- r - alpha p,
// u <- u + alpha d, and partials of ||r||_inf are written; the transformed
// rows are then those of the new residual (for the next pass).
template <bool UPDATE, typename TD>
__global__ void __launch_bounds__(256) k_lr_fwd(LowRankDev L, int ny_chunk, double* __restrict__ r,
                                                double* __restrict__ u, const TD* __restrict__ d,
                                                const TD* __restrict__ p, double2* __restrict__ Gp, CgIter it,
                                                const double* __restrict__ part_dp, int np_dp,
                                                const double* __restrict__ gam, double* __restrict__ part_rmax)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    const int nch = (L.n1 + ny_chunk - 1) / ny_chunk;
    const int x = blockIdx.x / nch, ch = blockIdx.x % nch;
    const int y0 = ch * ny_chunk;
    const int ny = min(ny_chunk, L.n1 - y0);
    double2* twz = (double2*)smem;                 // n2
    double2* twy = twz + L.n2;                     // n1
    double2* Z = twy + L.n1;                       // ny_chunk x kzn
    double* R = (double*)(Z + ny_chunk * L.kzn);   // ny_chunk x n2
    const int64_t base = ((int64_t)x * L.n1 + y0) * L.n2;
    const int cnt = ny * L.n2;
    double m = 0.0;
    // all global loads first (state, partials, gamma, the first PF elements
    // of the four vectors, twiddles); decisions come after
    constexpr int PF = 4;
    StateLoad sl;
    double dp_share = 0.0, gk = 0.0;
    double rv[PF], pv[PF], uv[PF], dv[PF];
    if (UPDATE) {
        sl = load_state(it.st);
        dp_share = load_share<OpSum>(part_dp, np_dp);
        gk = gam[it.k];
    }
#pragma unroll
    for (int j = 0; j < PF; ++j) {
        const int q = threadIdx.x + 256 * j;
        rv[j] = pv[j] = uv[j] = dv[j] = 0.0;
        if (q < cnt) {
            rv[j] = r[base + q];
            if (UPDATE) {
                pv[j] = (double)p[base + q];
                uv[j] = u[base + q];
                dv[j] = (double)d[base + q];
            }
        }
    }
    for (int j = threadIdx.x; j < L.n2; j += 256) twz[j] = L.twz[j];
    for (int j = threadIdx.x; j < L.n1; j += 256) twy[j] = L.twy[j];
    if (UPDATE) {
        if (ended(sl, it.k)) return;
        const double dp = combine_share<OpSum>(dp_share, slots);
        if (!(dp > 0.0) || !isfinite(dp)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) { it.st->status = 1; it.st->fail_iter = it.k; }
            return;
        }
        const double alpha = gk / dp;
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int q = threadIdx.x + 256 * j;
            if (q < cnt) {
                const double rn = rv[j] - alpha * pv[j];
                r[base + q] = rn;
                u[base + q] = uv[j] + alpha * dv[j];
                R[q] = rn;
                m = OpMax::apply(m, fabs(rn));
            }
        }
        for (int q = threadIdx.x + 256 * PF; q < cnt; q += 256) {
            const int64_t i = base + q;
            const double rn = r[i] - alpha * (double)p[i];
            r[i] = rn;
            u[i] += alpha * (double)d[i];
            R[q] = rn;
            m = OpMax::apply(m, fabs(rn));
        }
    } else {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int q = threadIdx.x + 256 * j;
            if (q < cnt) R[q] = rv[j];
        }
        for (int q = threadIdx.x + 256 * PF; q < cnt; q += 256) R[q] = r[base + q];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < ny * L.kzn; q += 256) {
        const int yl = q / L.kzn, kz = q % L.kzn;
        const double* row = R + yl * L.n2;
        double re = 0.0, im = 0.0;
        int t = 0;
#pragma unroll 8
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
    const int plane = L.kyn * L.kzn;
    for (int q = threadIdx.x; q < plane; q += 256) {
        const int kyi = q / L.kzn, kz = q % L.kzn;
        const int step = mod_n(kyi - L.m, L.n1);
        int t = mod_n((int64_t)(kyi - L.m) * y0, L.n1);
        double re = 0.0, im = 0.0;
#pragma unroll 4
        for (int yl = 0; yl < ny; ++yl) {
            const double2 a = Z[yl * L.kzn + kz];
            const double2 w = twy[t];
            re += a.x * w.x - a.y * w.y;
            im += a.x * w.y + a.y * w.x;
            t += step;
            if (t >= L.n1) t -= L.n1;
        }
        Gp[((int64_t)x * nch + ch) * plane + q] = make_double2(re, im);
    }
    if (UPDATE) {
        const double bm = block_reduce<OpMax>(m, slots);
        if (threadIdx.x == 0) part_rmax[blockIdx.x] = bm;
    }
}

// Pass B: one wavefront per (k_y, k_z) column: add the row-chunk partials,
// transform along x, multiply by the table, transform back.  Inside CG it is
// the first kernel of a pass and runs the convergence test.
__global__ void __launch_bounds__(64) k_lr_mid(LowRankDev L, int nch, const double* __restrict__ C,
                                               const double2* __restrict__ Gp, double2* __restrict__ H, CgIter it)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    const int col = blockIdx.x;  // ky index * kzn + kz
    const int plane = L.kyn * L.kzn;
    double2* twx = (double2*)smem;  // n0
    double2* gx = twx + L.n0;       // n0
    double2* X = gx + L.n0;         // kxn
    // loads first: state and ||r||_inf partials (head of the CG pass), the
    // row-chunk partials of this column, twiddles and the table entries
    StateLoad sl;
    double share = 0.0;
    if (it.st) {
        sl = load_state(it.st);
        share = load_share<OpMax>(it.part_rmax, it.np_rmax);
    }
    for (int j = threadIdx.x; j < L.n0; j += blockDim.x) {
        twx[j] = L.twx[j];
        double re = 0.0, im = 0.0;
        for (int c = 0; c < nch; ++c) {
            const double2 a = Gp[((int64_t)j * nch + c) * plane + col];
            re += a.x;
            im += a.y;
        }
        gx[j] = make_double2(re, im);
    }
    if (it.st && head_decide(it, sl, share, slots)) return;
    __syncthreads();
    for (int kxi = threadIdx.x; kxi < L.kxn; kxi += blockDim.x) {
        const int step = mod_n(kxi - L.mx, L.n0);
        double re = 0.0, im = 0.0;
        int t = 0;
#pragma unroll 8
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
        const int step = mod_n(x, L.n0);
        int t = mod_n((int64_t)(-L.mx) * x, L.n0);
        double re = 0.0, im = 0.0;
        for (int kxi = 0; kxi < L.kxn; ++kxi) {
            const double2 w = twx[t];  // conj(w) = exp(+2 pi i kx x / n0)
            const double2 a = X[kxi];
            re += a.x * w.x + a.y * w.y;
            im += a.y * w.x - a.x * w.y;
            t += step;
            if (t >= L.n0) t -= L.n0;
        }
        H[(int64_t)x * plane + col] = make_double2(re, im);
    }
}

// Pass C: one workgroup per (x-slab, chunk of rows y).
template <bool CG, typename TS>
__global__ void __launch_bounds__(256) k_lr_inv(LowRankDev L, int y_chunk, const double* __restrict__ r,
                                                const double2* __restrict__ H, TS* __restrict__ s, CgIter it)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    const int nch = (L.n1 + y_chunk - 1) / y_chunk;
    const int x = blockIdx.x / nch;
    const int y0 = (blockIdx.x % nch) * y_chunk;
    const int ny = min(y_chunk, L.n1 - y0);
    const int plane = L.kyn * L.kzn;
    double2* twz = (double2*)smem;       // n2
    double2* twy = twz + L.n2;           // n1
    double2* Hs = twy + L.n1;            // kyn x kzn
    double2* V = Hs + plane;             // ny x kzn
    // loads first: state, the coefficient plane, twiddles and this thread's r
    StateLoad sl;
    if (CG) sl = load_state(it.st);
    const int cnt = ny * L.n2;
    const int64_t base = ((int64_t)x * L.n1 + y0) * L.n2;
    constexpr int PF = 4;
    double rv[PF];
#pragma unroll
    for (int j = 0; j < PF; ++j) {
        const int q = threadIdx.x + 256 * j;
        rv[j] = (q < cnt) ? r[base + q] : 0.0;
    }
    for (int j = threadIdx.x; j < L.n2; j += blockDim.x) twz[j] = L.twz[j];
    for (int j = threadIdx.x; j < L.n1; j += blockDim.x) twy[j] = L.twy[j];
    for (int j = threadIdx.x; j < plane; j += blockDim.x) Hs[j] = H[(int64_t)x * plane + j];
    if (CG && ended(sl, it.k)) return;
    __syncthreads();
    // V[y][kz] = sum_ky H[x][ky][kz] exp(+2 pi i ky y / n1)
    for (int q = threadIdx.x; q < ny * L.kzn; q += blockDim.x) {
        const int yl = q / L.kzn, kz = q % L.kzn;
        const int y = y0 + yl;
        const int step = mod_n(y, L.n1);
        int t = mod_n((int64_t)(-L.m) * y, L.n1);
        double re = 0.0, im = 0.0;
        for (int kyi = 0; kyi < L.kyn; ++kyi) {
            const double2 w = twy[t];
            const double2 a = Hs[kyi * L.kzn + kz];
            re += a.x * w.x + a.y * w.y;
            im += a.y * w.x - a.x * w.y;
            t += step;
            if (t >= L.n1) t -= L.n1;
        }
        V[q] = make_double2(re, im);
    }
    __syncthreads();
    // s = W r + Re sum_kz V[y][kz] exp(+2 pi i kz z / n2)
    auto node = [&](int q, double rq, double& ss) -> double {
        const int yl = q / L.n2, z = q % L.n2;
        double c = 0.0;
        int t = 0;
#pragma unroll 4
        for (int kz = 0; kz < L.kzn; ++kz) {
            const double2 w = twz[t];
            const double2 a = V[yl * L.kzn + kz];
            c += a.x * w.x + a.y * w.y;  // Re(a * conj(w))
            t += z;
            if (t >= L.n2) t -= L.n2;
        }
        const TS sv = (TS)(L.W * rq + c);
        s[base + q] = sv;
        ss += (double)sv;
        return rq * (double)sv;
    };
    double acc = 0.0, ssum = 0.0;
#pragma unroll
    for (int j = 0; j < PF; ++j) {
        const int q = threadIdx.x + 256 * j;
        if (q < cnt) acc += node(q, rv[j], ssum);
    }
    for (int q = threadIdx.x + 256 * PF; q < cnt; q += 256) acc += node(q, r[base + q], ssum);
    if (CG) {
        const double b = block_reduce<OpSum>(acc, slots);
        if (threadIdx.x == 0) it.part_rs[blockIdx.x] = b;
        if (sizeof(TS) == 4) {
            const double bs = block_reduce<OpSum>(ssum, slots);
            if (threadIdx.x == 0) it.part_ssum[blockIdx.x] = bs;
        }
    }
}

// ----------------------------------------------------------------------------
// host

struct LowRankPlan {
    LowRankDev dev;
    double* table;    // kxn x kyn x kzn, w(kz) C(k) / n
    double2* Gp;      // n0 x nch_a x kyn x kzn row-chunk partials
    double2* H;       // n0 x kyn x kzn
    int ya, yc;       // rows per workgroup of passes A and C
    int nch_a;
    int blocks_a, blocks_c;
    size_t lds_a, lds_b, lds_c;
};

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
    if ((int64_t)cblock.size() != nb) { delete p; return UNO_ERR_ARG; }
    // rows per workgroup: about 1024 nodes, so the streaming part of pass A
    // (the CG update) and pass C spread over n / 1024 workgroups
    int rows = 1024 / L.n2;
    if (rows < 1) rows = 1;
    if (rows > L.n1) rows = L.n1;
    p->ya = p->yc = rows;
    p->nch_a = (L.n1 + p->ya - 1) / p->ya;
    p->blocks_a = L.n0 * p->nch_a;
    p->blocks_c = L.n0 * ((L.n1 + p->yc - 1) / p->yc);
    const int plane = L.kyn * L.kzn;
    p->lds_a = sizeof(double2) * ((size_t)L.n2 + L.n1 + (size_t)p->ya * L.kzn) + sizeof(double) * (size_t)p->ya * L.n2;
    p->lds_b = sizeof(double2) * (2 * (size_t)L.n0 + L.kxn);
    p->lds_c = sizeof(double2) * ((size_t)L.n2 + L.n1 + (size_t)plane + (size_t)p->yc * L.kzn);
    if (p->lds_a > 60 * 1024 || p->lds_b > 60 * 1024 || p->lds_c > 60 * 1024) { delete p; return UNO_ERR_SHAPE; }
    const int64_t ngp = (int64_t)L.n0 * p->nch_a * plane;
    const int64_t nh = (int64_t)L.n0 * plane;
    if (hipMalloc(&p->table, sizeof(double) * nb) != hipSuccess ||
        hipMalloc(&p->Gp, sizeof(double2) * ngp) != hipSuccess || hipMalloc(&p->H, sizeof(double2) * nh) != hipSuccess) {
        (void)hipFree(p->table);
        (void)hipFree(p->Gp);
        delete p;
        return UNO_ERR_NOMEM;
    }
    UNO_HIP(hipMemcpy(p->table, cblock.data(), sizeof(double) * nb, hipMemcpyHostToDevice));
    *out = p;
    return UNO_OK;
}

void lowrank_destroy(LowRankPlan* p)
{
    if (!p) return;
    (void)hipFree(p->table);
    (void)hipFree(p->Gp);
    (void)hipFree(p->H);
    delete p;
}

int lowrank_max_blocks(const LowRankPlan* p) { return p->blocks_a > p->blocks_c ? p->blocks_a : p->blocks_c; }
int lowrank_update_blocks(const LowRankPlan* p) { return p->blocks_a; }

static CgIter no_iter()
{
    CgIter it;
    memset(&it, 0, sizeof(it));
    return it;
}

// pass A on r (no update); also the initial transform of the CG loop
uno_status lowrank_forward(const LowRankPlan* p, const double* r, hipStream_t st)
{
    uno_launch(UNO_KT_FFT_FWD, k_lr_fwd<false, double>, dim3(p->blocks_a), dim3(256), p->lds_a, st, p->dev, p->ya,
               (double*)r, (double*)nullptr, (const double*)nullptr, (const double*)nullptr, p->Gp, no_iter(),
               (const double*)nullptr, 0, (const double*)nullptr, (double*)nullptr);
    return hip_status(hipGetLastError());
}

// CG update of pass k fused with pass A of pass k + 1
template <typename T>
uno_status lowrank_update_forward(const LowRankPlan* p, double* r, double* u, const T* d, const T* pv,
                                  const CgIter& it, const double* part_dp, int np_dp, const double* gam,
                                  double* part_rmax, hipStream_t st)
{
    uno_launch(UNO_KT_UPDATE, k_lr_fwd<true, T>, dim3(p->blocks_a), dim3(256), p->lds_a, st, p->dev, p->ya, r, u, d, pv,
               p->Gp, it, part_dp, np_dp, gam, part_rmax);
    return hip_status(hipGetLastError());
}

// passes B and C (B tests convergence inside CG); C writes s and r.s partials
template <typename T>
uno_status lowrank_finish(const LowRankPlan* p, const double* r, T* s, const CgIter* itp, int* np_rs,
                          hipStream_t st)
{
    const LowRankDev& L = p->dev;
    const CgIter it = itp ? *itp : no_iter();
    uno_launch(UNO_KT_FFT_MID, k_lr_mid, dim3(L.kyn * L.kzn), dim3(64), p->lds_b, st, L, p->nch_a,
               (const double*)p->table, (const double2*)p->Gp, p->H, it);
    UNO_HIP(hipGetLastError());
    if (itp)
        uno_launch(UNO_KT_FFT_INV, k_lr_inv<true, T>, dim3(p->blocks_c), dim3(256), p->lds_c, st, L, p->yc, r,
                   (const double2*)p->H, s, it);
    else
        uno_launch(UNO_KT_FFT_INV, k_lr_inv<false, T>, dim3(p->blocks_c), dim3(256), p->lds_c, st, L, p->yc, r,
                   (const double2*)p->H, s, it);
    UNO_HIP(hipGetLastError());
    if (np_rs) *np_rs = p->blocks_c;
    return UNO_OK;
}

uno_status lowrank_apply(const LowRankPlan* p, const double* r, double* s, hipStream_t st)
{
    uno_status e = lowrank_forward(p, r, st);
    if (e != UNO_OK) return e;
    return lowrank_finish<double>(p, r, s, nullptr, nullptr, st);
}

template uno_status lowrank_finish<double>(const LowRankPlan*, const double*, double*, const CgIter*, int*, hipStream_t);
template uno_status lowrank_finish<float>(const LowRankPlan*, const double*, float*, const CgIter*, int*, hipStream_t);
template uno_status lowrank_update_forward<double>(const LowRankPlan*, double*, double*, const double*, const double*,
                                                   const CgIter&, const double*, int, const double*, double*, hipStream_t);
template uno_status lowrank_update_forward<float>(const LowRankPlan*, double*, double*, const float*, const float*,
                                                  const CgIter&, const double*, int, const double*, double*, hipStream_t);

}  // namespace unocg
