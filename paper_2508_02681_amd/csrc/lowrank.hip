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
//
// Three nodal DOF (c = 3, App. B): Phi(k) is a symmetric 3 x 3 block per
// mode and W the bypass block psi(w^0), so s = W r + T^H (C o T r) with the
// 3 x 3 blocks C = Phi - W mixing the components.  Vectors are planar
// (component c at + c n), so passes A and C run over the 3 n0 slabs of the
// stacked components unchanged; pass B transforms the three components of a
// column along x, mixes them by C(k) and transforms back, and pass C adds
// the bypass product W r at each node.
#include <cmath>
#include <cstring>
#include <type_traits>

#include "unocg_internal.h"
#include "reduce.h"
#include "cg_ctl.h"
#include "stencil_tile.h"

namespace unocg {

struct LowRankDev {
    int n0, n1, n2;
    int mx, m;          // learned half-widths along x (0 for one voxel layer) and y, z
    int kxn, kyn, kzn;  // 2mx+1, 2m+1, m+1
    double W;           // bypass theta0^2 (c = 1)
    int nc;             // nodal DOF: 1, or 3 (planar components, slabs c n0 + x)
    double Wq[6];       // c = 3: bypass block entries q1..q6 (Phi_11, Phi_22, Phi_12, Phi_33, Phi_23, Phi_13)
    int64_t gps, hsz;   // per right-hand side: row-chunk partial and H sizes (double2)
    const double2* twx; // exp(-2 pi i j / n_b) tables
    const double2* twy;
    const double2* twz;
};

// v mod n in [0, n); 32-bit (every use has |v| <= n^2 / 2 with n < 46341):
// a 64-bit remainder is a long instruction sequence on this GPU
__device__ __forceinline__ int mod_n(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// Storage of the preconditioner's spectrum and table.  FP64 (double2 per
// complex value, double per table entry), or in the BF16 mode two BF16
// numbers in 32 bits per complex value (real part in the low half) and one
// per table entry: values are rounded to FP32 and then to the nearest BF16
// (ties to even), and widened exactly on load; the arithmetic stays FP64.
__device__ __forceinline__ uint32_t bf16_bits(double v)
{
    const uint32_t b = __float_as_uint((float)v);
    return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ double2 sp_get(const double2* p, int64_t i) { return p[i]; }
__device__ __forceinline__ double2 sp_get(const uint32_t* p, int64_t i)
{
    const uint32_t v = p[i];
    return make_double2((double)__uint_as_float(v << 16), (double)__uint_as_float(v & 0xffff0000u));
}
__device__ __forceinline__ void sp_put(double2* p, int64_t i, double2 v) { p[i] = v; }
__device__ __forceinline__ void sp_put(uint32_t* p, int64_t i, double2 v)
{
    p[i] = bf16_bits(v.x) | (bf16_bits(v.y) << 16);
}
__device__ __forceinline__ double tab_get(const double* c, int64_t i) { return c[i]; }
__device__ __forceinline__ double tab_get(const uint16_t* c, int64_t i)
{
    return (double)__uint_as_float((uint32_t)c[i] << 16);
}
template <bool BF>
using SpT = std::conditional_t<BF, uint32_t, double2>;
template <bool BF>
using TabT = std::conditional_t<BF, uint16_t, double>;

// Pass A on the rows [y_b, y_e) of slab x (one workgroup), taken ya rows at
// a time: Z[y][kz] = sum_z r e^{-i kz z}, then the partial y-sum over the
// workgroup's rows, Gp[x][chunk][ky][kz] = sum_y Z[y][kz] e^{-i ky y}
// (accumulated in LDS over the row groups); pass B adds the chunks in order.
// UPDATE (inside CG): the rows are first updated, r <- r - alpha p,
// u <- u + alpha d, and partials of ||r||_inf are written; the transformed
// rows are then those of the new residual (for the next pass).
template <bool UPDATE, typename TD, int PF, bool BF = false>
__global__ void __launch_bounds__(256) k_lr_fwd(LowRankDev L, int ya, int rb, double* __restrict__ r,
                                                double* __restrict__ u, const TD* __restrict__ d,
                                                const TD* __restrict__ p, SpT<BF>* __restrict__ Gp, CgIter it,
                                                const double* __restrict__ part_dp, int np_dp,
                                                const double* __restrict__ gam, double* __restrict__ part_rmax,
                                                double* __restrict__ part_rr)
{
    resolve_pass(it);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    if (blockIdx.y > 0) {  // right-hand side blockIdx.y of a batch
        const int64_t vo = (int64_t)blockIdx.y * it.vs, po = (int64_t)blockIdx.y * it.ps;
        r += vo;
        if (UPDATE) {
            u += vo;
            d += vo;
            p += vo;
            part_dp += po;
            gam += (int64_t)blockIdx.y * it.hs;
            part_rmax += po;
        }
        Gp += (int64_t)blockIdx.y * L.gps;
        if (part_rr) part_rr += po;
        it = rhs_iter(it);
    }
    const int nch = (L.n1 + rb - 1) / rb;
    const int x = blockIdx.x / nch, ch = blockIdx.x % nch;
    const int yb = ch * rb, ye = min(L.n1, yb + rb);
    const int plane = L.kyn * L.kzn;
    double2* twz = (double2*)smem;                 // n2
    double2* twy = twz + L.n2;                     // n1
    double2* Z = twy + L.n1;                       // ya x kzn
    double2* Gacc = Z + ya * L.kzn;                // plane
    double* R = (double*)(Gacc + plane);           // ya rows of n2 + 1 (padded against bank conflicts)
    const int rs = L.n2 + 1;
    double m = 0.0, sq = 0.0;
    // all global loads first (state, partials, gamma, the first PF elements
    // per thread of the four vectors of the first row group, twiddles);
    // decisions after
    StateLoad sl;
    double dp_share = 0.0, gk = 0.0;
    // d and p stay in their storage type until used: a conversion at the
    // load would wait for it and serialise the prefetch with the transform
    double rv[PF], uv[PF];
    TD pv[PF], dv[PF];
    if (UPDATE) {
        sl = load_state(it.st);
        dp_share = load_share<OpSum>(part_dp, np_dp);
        gk = gam[it.k];
    }
    // the first PF elements per thread of row group y0 into registers (the
    // next group is fetched while the current one is transformed)
    auto prefetch = [&](int y0) {
        const int ny = min(ya, ye - y0);
        const int64_t base = ((int64_t)x * L.n1 + y0) * L.n2;
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int q = threadIdx.x + 256 * j;
            rv[j] = uv[j] = 0.0;
            pv[j] = dv[j] = TD(0);
            if (q < ny * L.n2) {
                rv[j] = r[base + q];
                if (UPDATE) {
                    pv[j] = p[base + q];
                    uv[j] = u[base + q];
                    dv[j] = d[base + q];
                }
            }
        }
    };
    prefetch(yb);
    int rq[PF];  // padded LDS slot of element q: q + q / n2
#pragma unroll
    for (int j = 0; j < PF; ++j) {
        const int q = threadIdx.x + 256 * j;
        rq[j] = q + q / L.n2;
    }
    for (int j = threadIdx.x; j < L.n2; j += 256) twz[j] = L.twz[j];
    for (int j = threadIdx.x; j < L.n1; j += 256) twy[j] = L.twy[j];
    double alpha = 0.0;
    if (UPDATE) {
        if (ended(sl, it.k)) return;
        const double dp = combine_share<OpSum>(dp_share, slots);
        if (!(dp > 0.0) || !isfinite(dp)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) { it.st->status = 1; it.st->fail_iter = it.k; }
            return;
        }
        alpha = gk / dp;
    }
    for (int q = threadIdx.x; q < plane; q += 256) Gacc[q] = make_double2(0.0, 0.0);
    for (int y0 = yb; y0 < ye; y0 += ya) {
        const int ny = min(ya, ye - y0);
        const int cnt = ny * L.n2;
        const int64_t base = ((int64_t)x * L.n1 + y0) * L.n2;
        {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const int q = threadIdx.x + 256 * j;
                if (q < cnt) {
                    double v = rv[j];
                    if (UPDATE) {
                        v = rv[j] - alpha * (double)pv[j];
                        r[base + q] = v;
                        u[base + q] = uv[j] + alpha * (double)dv[j];
                        m = OpMax::apply(m, fabs(v));
                    }
                    R[rq[j]] = v;
                    sq += v * v;
                }
            }
        }
        for (int q = threadIdx.x + 256 * PF; q < cnt; q += 256) {
            const int64_t i = base + q;
            double v = r[i];
            if (UPDATE) {
                v -= alpha * (double)p[i];
                r[i] = v;
                u[i] += alpha * (double)d[i];
                m = OpMax::apply(m, fabs(v));
            }
            R[q + q / L.n2] = v;
            sq += v * v;
        }
        if (y0 + ya < ye) prefetch(y0 + ya);
        __syncthreads();
        // Z[y][kz] = sum_z R[y][z] w^z, w = twz[kz], by Horner's rule in w^2
        // over the even and the odd z (two independent chains), then E + w O
        for (int q = threadIdx.x; q < ny * L.kzn; q += 256) {
            const int yl = q / L.kzn, kz = q % L.kzn;
            const double* row = R + yl * rs;
            const double2 w = twz[kz], w2 = twz[mod_n(2 * kz, L.n2)];
            double er = 0.0, ei = 0.0, or_ = 0.0, oi = 0.0;
            int z = (L.n2 - 1) & ~1;  // last even z
            if (z + 1 < L.n2) or_ = row[z + 1];
            er = row[z];
#pragma unroll 4
            for (z -= 2; z >= 0; z -= 2) {
                const double ve = row[z], vo = row[z + 1];
                const double ner = fma(er, w2.x, fma(-ei, w2.y, ve));
                ei = fma(er, w2.y, ei * w2.x);
                er = ner;
                const double nor = fma(or_, w2.x, fma(-oi, w2.y, vo));
                oi = fma(or_, w2.y, oi * w2.x);
                or_ = nor;
            }
            Z[q] = make_double2(er + or_ * w.x - oi * w.y, ei + or_ * w.y + oi * w.x);
        }
        __syncthreads();
        // Gacc[ky][kz] += w^y0 sum_yl Z[yl][kz] w^yl, w = twy[ky mod n1], by
        // Horner's rule over the rows of the group
        for (int q = threadIdx.x; q < plane; q += 256) {
            const int kyi = q / L.kzn, kz = q % L.kzn;
            const double2 w = twy[mod_n(kyi - L.m, L.n1)];
            const double2 ph = twy[mod_n((kyi - L.m) * y0, L.n1)];
            double re = 0.0, im = 0.0;
#pragma unroll 4
            for (int yl = ny - 1; yl >= 0; --yl) {
                const double2 a = Z[yl * L.kzn + kz];
                const double nre = fma(re, w.x, fma(-im, w.y, a.x));
                im = fma(re, w.y, fma(im, w.x, a.y));
                re = nre;
            }
            Gacc[q].x += re * ph.x - im * ph.y;
            Gacc[q].y += re * ph.y + im * ph.x;
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < plane; q += 256) sp_put(Gp, ((int64_t)x * nch + ch) * plane + q, Gacc[q]);
    if (UPDATE) {
        const double bm = block_reduce<OpMax>(m, slots);
        if (threadIdx.x == 0) part_rmax[blockIdx.x] = bm;
    }
    if (part_rr) {  // ||r||^2 partials: r.s by Parseval in the fused flow
        const double bs = block_reduce<OpSum>(sq, slots);
        if (threadIdx.x == 0) part_rr[blockIdx.x] = bs;
    }
}

// Pass B: one workgroup of 256 threads per group of CB consecutive (k_y,
// k_z) columns: add the row-chunk partials (reads of CB adjacent columns are
// contiguous), transform along x, multiply by the table, transform back.
// Inside CG it is the first kernel of a pass and runs the convergence test.
// Both x-transforms are evaluated with Horner's rule in the unit-modulus
// phase factor, split into even and odd powers (two independent chains).
//
// With part_corr, it also writes per workgroup sum C(k) |X(k)|^2 over its
// columns: by Parseval, r.s = W ||r||^2 + (sum of these), since the table
// holds w(k_z) (Phi(k) - W) / n and X is the unnormalized DFT of r on the
// block.
constexpr int kMidQB = 2;  // gathered (column, x) entries per thread held in registers

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One Horner step (re, im) <- (re, im) w + h in complex arithmetic, as four
// nested fused multiply-adds (the compiler contracts the plain expression
// into six operations)
__device__ __forceinline__ void horner_step(double& re, double& im, double2 w, double2 h)
{
    const double nr = fma(re, w.x, fma(-im, w.y, h.x));
    im = fma(re, w.y, fma(im, w.x, h.y));
    re = nr;
}

// sum_{j < m} a[j * stride] w^j, by Horner on even and odd j in w^2
__device__ __forceinline__ double2 horner_eo(const double2* a, int stride, int m, double2 w)
{
    const double2 w2 = cmul(w, w);
    double er = 0.0, ei = 0.0, orr = 0.0, oi = 0.0;
    int j = (m - 1) & ~1;  // highest even index
    if (j + 1 < m) {       // m even: the odd chain starts one step higher
        const double2 h = a[(j + 1) * stride];
        orr = h.x;
        oi = h.y;
    }
#pragma unroll 4
    for (; j >= 2; j -= 2) {  // both chains
        horner_step(er, ei, w2, a[j * stride]);
        horner_step(orr, oi, w2, a[(j - 1) * stride]);
    }
    horner_step(er, ei, w2, a[0]);  // j = 0: the even chain only
    // E(w^2) + w O(w^2), E holding the even j, O the odd j
    return make_double2(er + (orr * w.x - oi * w.y), ei + (orr * w.y + oi * w.x));
}

// sum_{c < nch} src[c stride], added in the order c = 0, 1, ...; the loads
// are issued four at a time so that they are in flight together
template <typename SP>
__device__ __forceinline__ double2 chunk_sum(const SP* __restrict__ src, int nch, int64_t stride)
{
    double re = 0.0, im = 0.0;
    int c = 0;
    for (; c + 4 <= nch; c += 4) {
        const double2 v0 = sp_get(src, c * stride), v1 = sp_get(src, (c + 1) * stride);
        const double2 v2 = sp_get(src, (c + 2) * stride), v3 = sp_get(src, (c + 3) * stride);
        re += v0.x;
        im += v0.y;
        re += v1.x;
        im += v1.y;
        re += v2.x;
        im += v2.y;
        re += v3.x;
        im += v3.y;
    }
    for (; c < nch; ++c) {
        const double2 v = sp_get(src, c * stride);
        re += v.x;
        im += v.y;
    }
    return make_double2(re, im);
}

template <int CB, bool BF = false>  // columns per workgroup, BF16 storage
__global__ void __launch_bounds__(256) k_lr_mid(LowRankDev L, int nch, const TabT<BF>* __restrict__ C,
                                                const SpT<BF>* __restrict__ Gp, SpT<BF>* __restrict__ H, CgIter it,
                                                double* __restrict__ part_corr)
{
    resolve_pass(it);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    if (blockIdx.y > 0) {
        Gp += (int64_t)blockIdx.y * L.gps;
        H += (int64_t)blockIdx.y * L.hsz;
        if (part_corr) part_corr += (int64_t)blockIdx.y * it.ps;
        it = rhs_iter(it);
    }
    const int plane = L.kyn * L.kzn;
    const int col0 = blockIdx.x * CB;
    double2* gx = (double2*)smem;  // [x][cl]
    double2* X = gx + L.n0 * CB;   // [kx][cl]
    // loads first: state and ||r||_inf partials (head of the CG pass) and
    // this thread's first gathered entries
    StateLoad sl;
    double share = 0.0;
    if (it.st) {
        sl = load_state(it.st);
        share = load_share<OpMax>(it.part_rmax, it.np_rmax);
    }
    const int ng = L.n0 * CB;
    auto gather = [&](int q) {
        const int cl = q % CB, x = q / CB;
        const int col = col0 + cl;
        if (col >= plane) return make_double2(0.0, 0.0);
        return chunk_sum(Gp + (int64_t)x * nch * plane + col, nch, plane);
    };
    double2 gv[kMidQB];
#pragma unroll
    for (int u = 0; u < kMidQB; ++u) {
        const int q = threadIdx.x + 256 * u;
        gv[u] = (q < ng) ? gather(q) : make_double2(0.0, 0.0);
    }
    if (it.st && head_decide(it, sl, share, slots)) return;
#pragma unroll
    for (int u = 0; u < kMidQB; ++u) {
        const int q = threadIdx.x + 256 * u;
        if (q < ng) gx[q] = gv[u];
    }
    for (int q = threadIdx.x + 256 * kMidQB; q < ng; q += 256) gx[q] = gather(q);
    __syncthreads();
    // X[kx][cl] = C(k) sum_x g[x] exp(-2 pi i (kx - mx) x / n0).  With few
    // (kx, column) items per workgroup (few columns per workgroup: few
    // right-hand sides) the x range is cut into P parts of at least 8
    // points, each a Horner chain of its own times the phase of its first
    // point, added in part order: P times shorter dependent chains
    double corr = 0.0;
    const int items = L.kxn * CB;
    int P = 256 / items;
    if (P > 8) P = 8;
    if (P > L.n0 / 8) P = L.n0 / 8;
    if (P <= 1) {
        for (int o = threadIdx.x; o < items; o += 256) {
            const int cl = o % CB, kxi = o / CB;
            const int col = col0 + cl;
            const double2 w = L.twx[mod_n(kxi - L.mx, L.n0)];
            const double2 v = horner_eo(gx + cl, CB, L.n0, w);
            const double c = (col < plane) ? tab_get(C, (int64_t)kxi * plane + col) : 0.0;
            X[o] = make_double2(v.x * c, v.y * c);
            corr += c * (v.x * v.x + v.y * v.y);
        }
    } else {
        double2* Xp = X + items;  // P x items partial sums (P items <= 256)
        const int len = (L.n0 + P - 1) / P;
        for (int o = threadIdx.x; o < P * items; o += 256) {
            const int part = o / items, oi = o - part * items;
            const int cl = oi % CB, kx = oi / CB - L.mx;
            const int x0 = part * len, m = min(len, L.n0 - x0);
            double2 v = make_double2(0.0, 0.0);
            if (m > 0) {
                v = horner_eo(gx + x0 * CB + cl, CB, m, L.twx[mod_n(kx, L.n0)]);
                v = cmul(v, L.twx[mod_n(kx * x0, L.n0)]);  // exp(-2 pi i kx x0 / n0)
            }
            Xp[o] = v;
        }
        __syncthreads();
        for (int o = threadIdx.x; o < items; o += 256) {
            double2 v = Xp[o];
            for (int part = 1; part < P; ++part) {
                v.x += Xp[part * items + o].x;
                v.y += Xp[part * items + o].y;
            }
            const int cl = o % CB, kxi = o / CB;
            const int col = col0 + cl;
            const double c = (col < plane) ? tab_get(C, (int64_t)kxi * plane + col) : 0.0;
            X[o] = make_double2(v.x * c, v.y * c);
            corr += c * (v.x * v.x + v.y * v.y);
        }
    }
    if (part_corr) {
        const double b = block_reduce<OpSum>(corr, slots);
        if (threadIdx.x == 0) part_corr[blockIdx.x] = b;
    }
    __syncthreads();
    // H[x][col] = sum_kx X[kx] exp(+2 pi i (kx - mx) x / n0)
    for (int o = threadIdx.x; o < ng; o += 256) {
        const int cl = o % CB, x = o / CB;
        const int col = col0 + cl;
        if (col >= plane) continue;
        const double2 t = L.twx[x];                       // exp(-2 pi i x / n0)
        const double2 w = make_double2(t.x, -t.y);        // exp(+2 pi i x / n0)
        const double2 v = horner_eo(X + cl, CB, L.kxn, w);
        const double2 sh = L.twx[mod_n(L.mx * x, L.n0)];  // exp(-2 pi i mx x / n0)
        sp_put(H, (int64_t)x * plane + col, cmul(v, sh));
    }
}

// Pass B for three components: the workgroup gathers the (k_y, k_z)
// columns of the three component slabs, transforms each along x, mixes them
// by the 3 x 3 block of the table (C6: entries q1..q6 per mode, times
// w(k_z) / n) and transforms the three results back.  Inside CG it also runs
// the convergence test at the head of the pass.
__global__ void __launch_bounds__(256) k_lr_mid3(LowRankDev L, int nch, int cb, const double* __restrict__ C6,
                                                 const double2* __restrict__ Gp, double2* __restrict__ H, CgIter it)
{
    resolve_pass(it);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    if (blockIdx.y > 0) {
        Gp += (int64_t)blockIdx.y * L.gps;
        H += (int64_t)blockIdx.y * L.hsz;
        it = rhs_iter(it);
    }
    const int plane = L.kyn * L.kzn;
    const int col0 = blockIdx.x * cb;
    const int ncol = L.n0 * cb, nxk = L.kxn * cb;
    double2* gx = (double2*)smem;   // [c][x][cl]
    double2* X = gx + 3 * ncol;     // [c][kx][cl]
    StateLoad sl;
    double share = 0.0;
    if (it.st) {
        sl = load_state(it.st);
        share = load_share<OpMax>(it.part_rmax, it.np_rmax);
    }
    const int ng = 3 * ncol;
    auto gather = [&](int q) {  // q = c ncol + x cb + cl
        const int c = q / ncol, rem = q % ncol;
        const int cl = rem % cb, x = rem / cb;
        const int col = col0 + cl;
        if (col >= plane) return make_double2(0.0, 0.0);
        return chunk_sum(Gp + (int64_t)(c * L.n0 + x) * nch * plane + col, nch, plane);
    };
    double2 gv[kMidQB];
#pragma unroll
    for (int u = 0; u < kMidQB; ++u) {
        const int q = threadIdx.x + 256 * u;
        gv[u] = (q < ng) ? gather(q) : make_double2(0.0, 0.0);
    }
    if (it.st && head_decide(it, sl, share, slots)) return;
#pragma unroll
    for (int u = 0; u < kMidQB; ++u) {
        const int q = threadIdx.x + 256 * u;
        if (q < ng) gx[q] = gv[u];
    }
    for (int q = threadIdx.x + 256 * kMidQB; q < ng; q += 256) gx[q] = gather(q);
    __syncthreads();
    for (int o = threadIdx.x; o < nxk; o += 256) {
        const int cl = o % cb, kxi = o / cb;
        const int col = col0 + cl;
        const double2 w = L.twx[mod_n(kxi - L.mx, L.n0)];
        const double2 a = horner_eo(gx + cl, cb, L.n0, w);
        const double2 b = horner_eo(gx + ncol + cl, cb, L.n0, w);
        const double2 c = horner_eo(gx + 2 * ncol + cl, cb, L.n0, w);
        double q[6] = {0, 0, 0, 0, 0, 0};
        if (col < plane) {
            const double* t = C6 + ((int64_t)kxi * plane + col) * 6;
#pragma unroll
            for (int e = 0; e < 6; ++e) q[e] = t[e];
        }
        // [q1 q3 q6; q3 q2 q5; q6 q5 q4] (a, b, c)
        X[o] = make_double2(q[0] * a.x + q[2] * b.x + q[5] * c.x, q[0] * a.y + q[2] * b.y + q[5] * c.y);
        X[nxk + o] = make_double2(q[2] * a.x + q[1] * b.x + q[4] * c.x, q[2] * a.y + q[1] * b.y + q[4] * c.y);
        X[2 * nxk + o] = make_double2(q[5] * a.x + q[4] * b.x + q[3] * c.x, q[5] * a.y + q[4] * b.y + q[3] * c.y);
    }
    __syncthreads();
    for (int o = threadIdx.x; o < 3 * ncol; o += 256) {
        const int c = o / ncol, rem = o % ncol;
        const int cl = rem % cb, x = rem / cb;
        const int col = col0 + cl;
        if (col >= plane) continue;
        const double2 t = L.twx[x];
        const double2 w = make_double2(t.x, -t.y);
        const double2 v = horner_eo(X + c * nxk + cl, cb, L.kxn, w);
        const double2 sh = L.twx[mod_n(L.mx * x, L.n0)];
        H[(int64_t)(c * L.n0 + x) * plane + col] = cmul(v, sh);
    }
}

// Pass C for one component (the form the scalar problems use): one
// workgroup per (x-slab, chunk of rows y).  Along y the partial
// inverse transform is evaluated with Horner's rule in the unit-modulus
// phase factor: a thread owns one k_z column for two rows (each H value read
// from LDS feeds two chains).  Along z only the real part is needed, and the
// points z and n2 - z share it: with V_k = a_k + i b_k and theta = 2 pi z / n2,
//   Re sum_k V_k e^{+i k theta} = C - S,  Re sum_k V_k e^{-i k theta} = C + S,
//   C = sum_k a_k cos k theta,  S = sum_k b_k sin k theta,
// both by Clenshaw's recurrence y_k = c_k + 2 cos(theta) y_(k+1) - y_(k+2)
// (two operations per step and series for two points, half of a complex
// Horner step per point).  A thread owns pairs (z, n2 - z) of one row
// (each V value feeds all its pairs) and also loads, updates and writes
// exactly those nodes.  (For three components the pairs' recurrence state
// costs more registers than the halved arithmetic saves: k_lr_inv below.)
template <bool CG, typename TS, bool BF = false>
__global__ void __launch_bounds__(256) k_lr_inv_pairs(LowRankDev L, int y_chunk, const double* __restrict__ r,
                                                      const SpT<BF>* __restrict__ H, TS* __restrict__ s, CgIter it)
{
    resolve_pass(it);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    if (blockIdx.y > 0) {
        const int64_t vo = (int64_t)blockIdx.y * it.vs;
        r += vo;
        s += vo;
        H += (int64_t)blockIdx.y * L.hsz;
        it = rhs_iter(it);
    }
    const int nch = (L.n1 + y_chunk - 1) / y_chunk;
    const int x = blockIdx.x / nch;
    const int y0 = (blockIdx.x % nch) * y_chunk;
    const int ny = min(y_chunk, L.n1 - y0);
    const int plane = L.kyn * L.kzn;
    double2* Hs = (double2*)smem;  // kyn x kzn
    double2* V = Hs + plane;       // ny x kzn
    // pairs of this thread: row t / tpr, pair j = t % tpr + tpr i, points
    // z = j and n2 - j (one point for j = 0 and j = n2 / 2)
    const int tpr = 256 / y_chunk;
    const int row = threadIdx.x / tpr, part = threadIdx.x % tpr;
    const bool row_ok = row < ny;
    const int npair = L.n2 / 2 + 1;
    const int ppt = (npair + tpr - 1) / tpr;
    constexpr int ZB = 4;  // pairs held in registers per round
    const int64_t rbase = ((int64_t)x * L.n1 + y0 + row) * L.n2;
    // loads first: state, the coefficient plane and this thread's r
    StateLoad sl;
    if (CG) sl = load_state(it.st);
    double rv[ZB], rw[ZB];  // r at z = j and at n2 - j
    auto load_r = [&](int i0) {
#pragma unroll
        for (int i = 0; i < ZB; ++i) {
            const int j = part + tpr * (i0 + i);
            const bool ok = row_ok && j < npair && i0 + i < ppt;
            const int zm = j == 0 ? 0 : L.n2 - j;
            rv[i] = ok ? r[rbase + j] : 0.0;
            rw[i] = (ok && zm != j) ? r[rbase + zm] : 0.0;
        }
    };
    load_r(0);
    for (int j = threadIdx.x; j < plane; j += blockDim.x) Hs[j] = sp_get(H, (int64_t)x * plane + j);
    if (CG && ended(sl, it.k)) return;
    __syncthreads();
    // V[y][kz] = exp(-i M phi_y) sum_kyi H[kyi][kz] w_y^kyi, w_y = exp(+2 pi i y / n1)
    {
        const int yh = (ny + 1) / 2;
        for (int t = threadIdx.x; t < yh * L.kzn; t += blockDim.x) {
            const int ya = t % yh, kz = t / yh;
            const int yb = (ya + yh < ny) ? ya + yh : ya;
            const double2 ta = L.twy[y0 + ya], tb = L.twy[y0 + yb];
            const double2 wa = make_double2(ta.x, -ta.y), wb = make_double2(tb.x, -tb.y);
            const double2* hcol = Hs + kz;
            double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
            for (int kyi = L.kyn - 1; kyi >= 0; --kyi) {
                const double2 h = hcol[kyi * L.kzn];
                horner_step(ar, ai, wa, h);
                horner_step(br, bi, wb, h);
            }
            const double2 sa = L.twy[mod_n(L.m * (y0 + ya), L.n1)];
            const double2 sb = L.twy[mod_n(L.m * (y0 + yb), L.n1)];
            V[ya * L.kzn + kz] = make_double2(ar * sa.x - ai * sa.y, ar * sa.y + ai * sa.x);
            if (yb != ya) V[yb * L.kzn + kz] = make_double2(br * sb.x - bi * sb.y, br * sb.y + bi * sb.x);
        }
    }
    __syncthreads();
    // s = W r + Re sum_kz V[row][kz] w_z^kz, w_z = exp(+2 pi i z / n2), for
    // the pair (z, n2 - z) by Clenshaw's recurrence in cos(2 pi z / n2)
    double acc = 0.0, ssum = 0.0;
    if (row_ok) {
        const double2* vrow = V + row * L.kzn;
        for (int i0 = 0; i0 < ppt; i0 += ZB) {
            double c2[ZB], sn[ZB], b1[ZB], b2[ZB], d1[ZB], d2[ZB];
            if (i0 > 0) load_r(i0);
#pragma unroll
            for (int i = 0; i < ZB; ++i) {
                const int j = part + tpr * (i0 + i);
                const double2 tz = L.twz[j < npair ? j : 0];  // exp(-2 pi i j / n2)
                c2[i] = 2.0 * tz.x;
                sn[i] = -tz.y;
                b1[i] = b2[i] = d1[i] = d2[i] = 0.0;
            }
            for (int kz = L.kzn - 1; kz >= 1; --kz) {
                const double2 v = vrow[kz];
#pragma unroll
                for (int i = 0; i < ZB; ++i) {
                    const double nb = fma(c2[i], b1[i], v.x) - b2[i];
                    b2[i] = b1[i];
                    b1[i] = nb;
                    const double nd = fma(c2[i], d1[i], v.y) - d2[i];
                    d2[i] = d1[i];
                    d1[i] = nd;
                }
            }
            const double a0 = vrow[0].x;
#pragma unroll
            for (int i = 0; i < ZB; ++i) {
                const int j = part + tpr * (i0 + i);
                if (j >= npair || i0 + i >= ppt) continue;
                const int zm = j == 0 ? 0 : L.n2 - j;
                const double C = fma(0.5 * c2[i], b1[i], a0) - b2[i];
                const double S = d1[i] * sn[i];
                const TS sp = (TS)(L.W * rv[i] + (C - S));
                s[rbase + j] = sp;
                ssum += (double)sp;
                acc += rv[i] * (double)sp;
                if (zm != j) {
                    const TS sm = (TS)(L.W * rw[i] + (C + S));
                    s[rbase + zm] = sm;
                    ssum += (double)sm;
                    acc += rw[i] * (double)sm;
                }
            }
        }
    }
    if (CG) {
        const double b = block_reduce<OpSum>(acc, slots);
        if (threadIdx.x == 0) it.part_rs[blockIdx.x] = b;
        if (sizeof(TS) == 4) {
            const double bs = block_reduce<OpSum>(ssum, slots);
            if (threadIdx.x == 0) it.part_ssum[blockIdx.x] = bs;
        }
    }
}

// Pass C: one workgroup per (x-slab, chunk of rows y).  Both partial
// inverse transforms are evaluated with Horner's rule in the unit-modulus
// phase factor: along y a thread owns one k_z column for two rows (each H
// value read from LDS feeds two chains); along z a thread owns zpt points of
// one row (each V value feeds zpt chains) and also loads, updates and writes
// exactly those nodes.  NC = 3: the workgroup takes the three components of
// its slab, so each node's three residual values are read once for the
// bypass block and the three corrections.
template <bool CG, typename TS, int NC>
__global__ void __launch_bounds__(256) k_lr_inv(LowRankDev L, int y_chunk, const double* __restrict__ r,
                                                const double2* __restrict__ H, TS* __restrict__ s, CgIter it)
{
    resolve_pass(it);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[4];
    if (blockIdx.y > 0) {
        const int64_t vo = (int64_t)blockIdx.y * it.vs;
        r += vo;
        s += vo;
        H += (int64_t)blockIdx.y * L.hsz;
        it = rhs_iter(it);
    }
    const int nch = (L.n1 + y_chunk - 1) / y_chunk;
    const int x = blockIdx.x / nch;
    const int y0 = (blockIdx.x % nch) * y_chunk;
    const int ny = min(y_chunk, L.n1 - y0);
    const int plane = L.kyn * L.kzn;
    const int64_t cs = (int64_t)L.n0 * L.n1 * L.n2;  // component stride (NC = 3)
    double2* Hs = (double2*)smem;        // NC x kyn x kzn
    double2* V = Hs + NC * plane;        // NC x ny x kzn
    // z points of this thread: row t / tpr, z = t % tpr + tpr i
    const int tpr = 256 / y_chunk;
    const int row = threadIdx.x / tpr, part = threadIdx.x % tpr;
    const bool row_ok = row < ny;
    const int zpt = (L.n2 + tpr - 1) / tpr;
    constexpr int ZB = NC == 1 ? 4 : 2;  // z points held in registers per round
    const int64_t rbase = ((int64_t)x * L.n1 + y0 + row) * L.n2;
    // loads first: state, the coefficient planes, phase factors and this thread's r
    StateLoad sl;
    if (CG) sl = load_state(it.st);
    double rv[NC][ZB];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i = 0; i < ZB; ++i) {
            const int z = part + tpr * i;
            rv[c][i] = (row_ok && z < L.n2 && i < zpt) ? r[c * cs + rbase + z] : 0.0;
        }
    for (int j = threadIdx.x; j < NC * plane; j += blockDim.x) {
        const int c = j / plane, jj = j - c * plane;
        Hs[j] = H[(int64_t)(c * L.n0 + x) * plane + jj];
    }
    if (CG && ended(sl, it.k)) return;
    __syncthreads();
    // V[c][y][kz] = exp(-i M phi_y) sum_kyi H[c][kyi][kz] w_y^kyi, w_y = exp(+2 pi i y / n1)
    {
        const int yh = (ny + 1) / 2;
        for (int t = threadIdx.x; t < NC * yh * L.kzn; t += blockDim.x) {
            const int c = t / (yh * L.kzn), tt = t - c * yh * L.kzn;
            const int ya = tt % yh, kz = tt / yh;
            const int yb = (ya + yh < ny) ? ya + yh : ya;
            const double2 ta = L.twy[y0 + ya], tb = L.twy[y0 + yb];
            const double2 wa = make_double2(ta.x, -ta.y), wb = make_double2(tb.x, -tb.y);
            const double2* hcol = Hs + c * plane + kz;
            double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
            for (int kyi = L.kyn - 1; kyi >= 0; --kyi) {
                const double2 h = hcol[kyi * L.kzn];
                horner_step(ar, ai, wa, h);
                horner_step(br, bi, wb, h);
            }
            const double2 sa = L.twy[mod_n(L.m * (y0 + ya), L.n1)];
            const double2 sb = L.twy[mod_n(L.m * (y0 + yb), L.n1)];
            double2* vc = V + (int64_t)c * ny * L.kzn;
            vc[ya * L.kzn + kz] = make_double2(ar * sa.x - ai * sa.y, ar * sa.y + ai * sa.x);
            if (yb != ya) vc[yb * L.kzn + kz] = make_double2(br * sb.x - bi * sb.y, br * sb.y + bi * sb.x);
        }
    }
    __syncthreads();
    // s = W r + Re sum_kz V[row][kz] w_z^kz, w_z = exp(+2 pi i z / n2)
    double acc = 0.0, ssum = 0.0;
    if (row_ok) {
        for (int i0 = 0; i0 < zpt; i0 += ZB) {
            double ar[NC][ZB], ai[NC][ZB];
            double2 w[ZB];
#pragma unroll
            for (int i = 0; i < ZB; ++i) {
                const int z = part + tpr * (i0 + i);
                const double2 tz = L.twz[z < L.n2 ? z : 0];
                w[i] = make_double2(tz.x, -tz.y);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    ar[c][i] = ai[c][i] = 0.0;
                    // this round's residual values, loaded ahead of the chains
                    if (i0 > 0) rv[c][i] = (z < L.n2) ? r[c * cs + rbase + z] : 0.0;
                }
            }
            for (int kz = L.kzn - 1; kz >= 0; --kz) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double2 v = V[((int64_t)c * ny + row) * L.kzn + kz];
#pragma unroll
                    for (int i = 0; i < ZB; ++i) horner_step(ar[c][i], ai[c][i], w[i], v);
                }
            }
#pragma unroll
            for (int i = 0; i < ZB; ++i) {
                const int z = part + tpr * (i0 + i);
                if (z < L.n2) {
                    double rq[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) rq[c] = rv[c][i];
                    if (NC == 1) {
                        const TS sv = (TS)(L.W * rq[0] + ar[0][i]);
                        s[rbase + z] = sv;
                        ssum += (double)sv;
                        acc += rq[0] * (double)sv;
                    } else {
                        // bypass block [q1 q3 q6; q3 q2 q5; q6 q5 q4]
                        const double* q = L.Wq;
                        const double b0 = q[0] * rq[0] + q[2] * rq[1 % NC] + q[5] * rq[2 % NC];
                        const double b1 = q[2] * rq[0] + q[1] * rq[1 % NC] + q[4] * rq[2 % NC];
                        const double b2 = q[5] * rq[0] + q[4] * rq[1 % NC] + q[3] * rq[2 % NC];
                        const TS s0 = (TS)(b0 + ar[0][i]), s1 = (TS)(b1 + ar[1 % NC][i]),
                                 s2 = (TS)(b2 + ar[2 % NC][i]);
                        s[rbase + z] = s0;
                        s[cs + rbase + z] = s1;
                        s[2 * cs + rbase + z] = s2;
                        ssum += (double)s0 + (double)s1 + (double)s2;
                        acc += rq[0] * (double)s0 + rq[1 % NC] * (double)s1 + rq[2 % NC] * (double)s2;
                    }
                }
            }
        }
    }
    if (CG) {
        const double b = block_reduce<OpSum>(acc, slots);
        if (threadIdx.x == 0) it.part_rs[blockIdx.x] = b;
        if (sizeof(TS) == 4) {
            const double bs = block_reduce<OpSum>(ssum, slots);
            if (threadIdx.x == 0) it.part_ssum[blockIdx.x] = bs;
        }
    }
}

// Fused flow inside FP64 CG: pass C folded into the operator apply.  The
// tile kernel evaluates s = W r + correction itself on its tile and halo
// (from r and the H planes of its x-range), so s is never stored, and r.s
// comes from Parseval: r.s = W ||r||^2 + sum_k C(k) |X(k)|^2 (partials of
// pass A and pass B).  Then, as in the operator-apply tile kernel,
// d = s + beta d_old, p = A d and the d.p partials.
//
// The corrections are evaluated with Horner's rule in the unit-modulus
// phase factor: along y, V[x][y][k_z] = sum_{k_y} H[x][k_y][k_z] w_y^{k_y}
// with w_y = exp(+2 pi i y / n1); along z, Re sum_{k_z} V w_z^{k_z}.  (The
// two contractions are small and latency-bound here; written for the FP64
// matrix cores they measured slower on this chip.)
struct LrTileArgs {
    const double* part_rr;    // ||r||^2 partials (pass A)
    int np_rr;
    const double* part_corr;  // sum C |X|^2 partials (pass B)
    int np_corr;
};

// double2 elements of dynamic LDS of k_lr_tile: H planes and V
__host__ __device__ inline int lr_tile_dyn_elems(int dx, int dy, int kyn, int kzn)
{
    return dx * kyn * kzn + dx * dy * kzn;
}

template <int TX, int TZ, bool NEAR>
__global__ void __launch_bounds__(256) k_lr_tile(GridDev g, TileGeom tg, LowRankDev L, const double* __restrict__ kappa,
                                                 const double* __restrict__ r, const double2* __restrict__ H,
                                                 const double* __restrict__ dold, double* __restrict__ dnew,
                                                 double* __restrict__ p, double* __restrict__ part_dp, CgIter it,
                                                 LrTileArgs a, double* gam)
{
    resolve_pass(it);
    constexpr int TY = 256 / TZ;
    constexpr int DX = TX + 2, DY = TY + 2, DZ = TZ + 2;
    constexpr int KX = TX + 1, KY = TY + 1, KZ = TZ + 1;
    constexpr int HB = 2;  // H values per thread and plane held in registers (the rest is copied after)
    __shared__ double Dl[DX * DY * DZ];
    __shared__ double Kl[KX * KY * KZ];
    __shared__ double2 wz[DZ], wy[DY], wyM[DY];
    __shared__ double slots[4];
    extern __shared__ __align__(16) unsigned char smem[];
    const int plane = L.kyn * L.kzn;
    double2* Hl = (double2*)smem;  // DX planes of H   [xl][k_y][k_z]
    double2* V = Hl + DX * plane;  // y-inverse of H   [xl][yl][k_z]

    int b = blockIdx.x;
    const int tzi = b % tg.tiles_z;
    b /= tg.tiles_z;
    const int tyi = b % tg.tiles_y;
    const int txi = b / tg.tiles_y;
    const int x0 = txi * TX, y0 = tyi * TY, z0 = tzi * TZ;
    if (blockIdx.y > 0) {  // right-hand side blockIdx.y of a batch
        const int64_t vo = (int64_t)blockIdx.y * it.vs, po = (int64_t)blockIdx.y * it.ps;
        kappa += (int64_t)blockIdx.y * it.ks;
        r += vo;
        dold += vo;
        dnew += vo;
        p += vo;
        H += (int64_t)blockIdx.y * L.hsz;
        part_dp += po;
        a.part_rr += po;
        a.part_corr += po;
        gam += (int64_t)blockIdx.y * it.hs;
        it = rhs_iter(it);
    }

    // every global load first: state, both partial sets, previous gamma, r
    // and d_old on the halo, conductivities, H planes, phase factors
    const StateLoad sl = load_state(it.st);
    const double rr_share = load_share<OpSum>(a.part_rr, a.np_rr);
    const double cr_share = load_share<OpSum>(a.part_corr, a.np_corr);
    const double gprev = (it.k > it.k0) ? gam[it.k - 1] : 1.0;
    constexpr int ND = DX * DY * DZ, NK = KX * KY * KZ;
    constexpr int PD = (ND + 255) / 256, PK = (NK + 255) / 256;
    auto wrapc = [](int v, int n) {
        if constexpr (NEAR) return wrap_near(v, n);
        else return wrap_mod(v, n);
    };
    double rv[PD], dv[PD], kv[PK];
    double2 hv[DX][HB];
#pragma unroll
    for (int xl = 0; xl < DX; ++xl) {
        const double2* hp = H + (int64_t)wrapc(x0 - 1 + xl, g.n0) * plane;
#pragma unroll
        for (int u = 0; u < HB; ++u) {
            const int c = threadIdx.x + 256 * u;
            hv[xl][u] = (c < plane) ? hp[c] : make_double2(0.0, 0.0);
        }
    }
#pragma unroll
    for (int j = 0; j < PD; ++j) {
        const int q = threadIdx.x + 256 * j;
        rv[j] = dv[j] = 0.0;
        if (q < ND) {
            const int zl = q % DZ, t = q / DZ;
            const int yl = t % DY, xl = t / DY;
            const int x = wrapc(x0 - 1 + xl, g.n0), y = wrapc(y0 - 1 + yl, g.n1), z = wrapc(z0 - 1 + zl, g.n2);
            const int64_t idx = ((int64_t)x * g.n1 + y) * g.n2 + z;
            rv[j] = r[idx];
            if (it.k > it.k0) dv[j] = dold[idx];
        }
    }
#pragma unroll
    for (int j = 0; j < PK; ++j) {
        const int q = threadIdx.x + 256 * j;
        kv[j] = 0.0;
        if (q < NK) {
            const int zl = q % KZ, t = q / KZ;
            const int yl = t % KY, xl = t / KY;
            const int x = wrapc(x0 - 1 + xl, g.n0), y = wrapc(y0 - 1 + yl, g.n1), z = wrapc(z0 - 1 + zl, g.n2);
            kv[j] = kappa[((int64_t)x * g.n1 + y) * g.n2 + z];
        }
    }
    // phase factors of the tile: w_z, w_y (conjugates of the exp(-...) tables) and w_y^{-M}
    double2 tw = make_double2(0.0, 0.0);
    {
        const int t = threadIdx.x;
        if (t < DZ) {
            tw = L.twz[wrapc(z0 - 1 + t, g.n2)];
        } else if (t < DZ + DY) {
            tw = L.twy[wrapc(y0 - 1 + (t - DZ), g.n1)];
        } else if (t < DZ + 2 * DY) {
            const int y = wrapc(y0 - 1 + (t - DZ - DY), g.n1);
            tw = L.twy[(L.m * y) % g.n1];
        }
    }
    if (ended(sl, it.k)) return;
    const int k = it.k;
    const double rr = combine_share<OpSum>(rr_share, slots);
    const double cr = combine_share<OpSum>(cr_share, slots);
    const double gk = L.W * rr + cr;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (lead) gam[k] = gk;
    if (!(gk > 0.0) || !isfinite(gk)) {
        if (lead) { it.st->status = 1; it.st->fail_iter = k; }
        return;
    }
    const bool first = (k == it.k0);
    const double beta = first ? 0.0 : gk / gprev;
    // LDS: staged W r + beta d_old (the correction is added below),
    // conductivities, H planes, phase factors
#pragma unroll
    for (int j = 0; j < PD; ++j) {
        const int q = threadIdx.x + 256 * j;
        if (q < ND) Dl[q] = first ? L.W * rv[j] : L.W * rv[j] + beta * dv[j];
    }
#pragma unroll
    for (int j = 0; j < PK; ++j) {
        const int q = threadIdx.x + 256 * j;
        if (q < NK) Kl[q] = kv[j];
    }
#pragma unroll
    for (int xl = 0; xl < DX; ++xl) {
#pragma unroll
        for (int u = 0; u < HB; ++u) {
            const int c = threadIdx.x + 256 * u;
            if (c < plane) Hl[xl * plane + c] = hv[xl][u];
        }
        if (plane > 256 * HB) {
            const double2* hp = H + (int64_t)wrapc(x0 - 1 + xl, g.n0) * plane;
            for (int c = threadIdx.x + 256 * HB; c < plane; c += 256) Hl[xl * plane + c] = hp[c];
        }
    }
    {
        const int t = threadIdx.x;
        if (t < DZ) wz[t] = make_double2(tw.x, -tw.y);
        else if (t < DZ + DY) wy[t - DZ] = make_double2(tw.x, -tw.y);
        else if (t < DZ + 2 * DY) wyM[t - DZ - DY] = tw;
    }
    __syncthreads();
    // V[xl][yl][kz]: inverse partial DFT along y, Horner in w_y.  A thread
    // owns one (xl, kz) column and a pair of rows yl, yl + YH, so each H value
    // read from LDS feeds two independent chains.
    {
        constexpr int YH = (DY + 1) / 2;
        const int nt = DX * L.kzn * YH;
        for (int t = threadIdx.x; t < nt; t += 256) {
            const int ya = t % YH, c = t / YH;
            const int kz = c % L.kzn, xl = c / L.kzn;
            const int yb = (ya + YH < DY) ? ya + YH : ya;
            const double2 wa = wy[ya], wb = wy[yb];
            const double2* hcol = Hl + xl * plane + kz;
            double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
            auto step = [&](const double2 h) {
                horner_step(ar, ai, wa, h);
                horner_step(br, bi, wb, h);
            };
            int kyi = L.kyn - 1;
            for (; kyi >= 3; kyi -= 4) {  // four LDS reads in flight per round
                const double2 h0 = hcol[kyi * L.kzn], h1 = hcol[(kyi - 1) * L.kzn];
                const double2 h2 = hcol[(kyi - 2) * L.kzn], h3 = hcol[(kyi - 3) * L.kzn];
                step(h0);
                step(h1);
                step(h2);
                step(h3);
            }
            for (; kyi >= 0; --kyi) step(hcol[kyi * L.kzn]);
            const double2 sa = wyM[ya], sb = wyM[yb];  // times w_y^-M
            V[(xl * DY + ya) * L.kzn + kz] = make_double2(ar * sa.x - ai * sa.y, ar * sa.y + ai * sa.x);
            if (yb != ya) V[(xl * DY + yb) * L.kzn + kz] = make_double2(br * sb.x - bi * sb.y, br * sb.y + bi * sb.x);
        }
    }
    __syncthreads();
    // s = (W r + beta d_old, already staged) + Re sum_kz V w_z^kz: a thread
    // owns ZPT points of one staged row, so each V value read from LDS feeds
    // ZPT independent Horner chains
    {
        constexpr int ROWS = DX * DY;
        constexpr int TPR = (256 / ROWS) > 0 ? 256 / ROWS : 1;
        constexpr int ZPT = (DZ + TPR - 1) / TPR;
        for (int t = threadIdx.x; t < ROWS * TPR; t += 256) {
            const int row = t / TPR, part = t % TPR;
            double ar[ZPT], ai[ZPT];
            double2 w[ZPT];
#pragma unroll
            for (int i = 0; i < ZPT; ++i) {
                const int zl = part + TPR * i;
                w[i] = wz[zl < DZ ? zl : 0];
                ar[i] = ai[i] = 0.0;
            }
            const double2* vrow = V + row * L.kzn;
            auto step = [&](const double2 v) {
#pragma unroll
                for (int i = 0; i < ZPT; ++i) {
                    const double nr = ar[i] * w[i].x - ai[i] * w[i].y + v.x;
                    ai[i] = ar[i] * w[i].y + ai[i] * w[i].x + v.y;
                    ar[i] = nr;
                }
            };
            int kz = L.kzn - 1;
            for (; kz >= 3; kz -= 4) {
                const double2 v0 = vrow[kz], v1 = vrow[kz - 1], v2 = vrow[kz - 2], v3 = vrow[kz - 3];
                step(v0);
                step(v1);
                step(v2);
                step(v3);
            }
            for (; kz >= 0; --kz) step(vrow[kz]);
#pragma unroll
            for (int i = 0; i < ZPT; ++i) {
                const int zl = part + TPR * i;
                if (zl < DZ) Dl[row * DZ + zl] += ar[i];
            }
        }
    }
    __syncthreads();

    const int tz = threadIdx.x % TZ, ty = threadIdx.x / TZ;
    const int y = y0 + ty, z = z0 + tz;
    const bool yz_ok = (y < g.n1) && (z < g.n2);
    double dm[3][3], d0[3][3], dq[3][3], km[2][2], kp[2][2];
#pragma unroll
    for (int bb = 0; bb < 3; ++bb)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dm[bb][c] = Dl[(0 * DY + ty + bb) * DZ + tz + c];
            d0[bb][c] = Dl[(1 * DY + ty + bb) * DZ + tz + c];
        }
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int c = 0; c < 2; ++c) km[bb][c] = Kl[(0 * KY + ty + bb) * KZ + tz + c];
    double dot = 0.0;
#pragma unroll
    for (int xi = 0; xi < TX; ++xi) {
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int c = 0; c < 3; ++c) dq[bb][c] = Dl[((xi + 2) * DY + ty + bb) * DZ + tz + c];
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int c = 0; c < 2; ++c) kp[bb][c] = Kl[((xi + 1) * KY + ty + bb) * KZ + tz + c];
        const int x = x0 + xi;
        if (yz_ok && x < g.n0) {
            const double acc = stencil_node<double>(g, dm, d0, dq, km, kp);
            const int64_t i = ((int64_t)x * g.n1 + y) * g.n2 + z;
            p[i] = acc;
            dnew[i] = d0[1][1];
            dot += d0[1][1] * acc;
        }
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dm[bb][c] = d0[bb][c];
                d0[bb][c] = dq[bb][c];
            }
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int c = 0; c < 2; ++c) km[bb][c] = kp[bb][c];
    }
    const double bd = block_reduce<OpSum>(dot, slots);
    if (threadIdx.x == 0) part_dp[blockIdx.x] = bd;
}

// ----------------------------------------------------------------------------
// host

struct LowRankPlan {
    LowRankDev dev;
    double* table;    // kxn x kyn x kzn, w(kz) C(k) / n
    uint16_t* table_bf;  // the same in BF16 (one nodal DOF; the BF16 preconditioner mode)
    double2* Gp;      // n0 x nch_a x kyn x kzn row-chunk partials
    double2* H;       // n0 x kyn x kzn
    int ya, yc;       // rows per group of pass A (in LDS at once), fewest rows per workgroup of pass C
    int yc_max;       // most rows per workgroup of pass C (its LDS is sized for them)
    int rb;           // rows per workgroup of pass A
    int nch_a;
    int slabs;        // x-slabs of passes A and C: nc n0
    int blocks_a, blocks_c;
    size_t lds_a, lds_b, lds_c;
    int cb_mid, blocks_mid;  // columns per workgroup of pass B, its workgroups
    bool fused;       // the fused operator tile fits (FP64 CG flow)
    TileChoice tile;  // its tile shape
    size_t lds_t;     // its dynamic LDS
};

// static LDS of k_lr_tile<TX, TZ> plus the dynamic part (H planes, V)
static size_t lr_tile_lds(const LowRankDev& L, int tx, int tz, size_t* dyn)
{
    const int ty = 256 / tz;
    const size_t dx = tx + 2, dy = ty + 2, dz = tz + 2;
    const size_t stat = sizeof(double) * (dx * dy * dz + (size_t)(tx + 1) * (ty + 1) * (tz + 1)) + 4 * sizeof(double) +
                        sizeof(double2) * (dz + 2 * dy);
    *dyn = sizeof(double2) * (size_t)lr_tile_dyn_elems((int)dx, (int)dy, L.kyn, L.kzn);
    return stat + *dyn;
}

uno_status lowrank_create(const Grid& g, const FftPlan& fp, int M, double W, const std::vector<double>& cblock,
                          LowRankPlan** out, int nc, const double* Wq)
{
    if (nc != 1 && nc != 3) return UNO_ERR_ARG;
    // the kernels form the phase indices M j (j < n) in 32-bit integers
    for (int b = 0; b < 3; ++b)
        if ((int64_t)M * g.n[b] >= ((int64_t)1 << 30)) return UNO_ERR_SHAPE;
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
    L.nc = nc;
    for (int e = 0; e < 6; ++e) L.Wq[e] = (nc == 3) ? Wq[e] : 0.0;
    L.twx = fp.ax[0].tw64;
    L.twy = fp.ax[1].tw64;
    L.twz = fp.ax[2].tw64;
    const int64_t nb = (int64_t)L.kxn * L.kyn * L.kzn;
    const int64_t ntab = nb * (nc == 3 ? 6 : 1);
    if ((int64_t)cblock.size() != ntab) { delete p; return UNO_ERR_ARG; }
    p->slabs = nc * L.n0;
    // rows per workgroup: about 1024 nodes, so the streaming part of pass A
    // (the CG update) and pass C spread over n / 1024 workgroups
    int rows = 1024 / L.n2;
    if (rows < 1) rows = 1;
    if (rows > L.n1) rows = L.n1;
    // pass A takes at least 8 rows per group where rows are long (fewer
    // group steps per workgroup: 192^3 x 3 loads 239 -> 211 us with 10 rows
    // instead of 5), its first 2048 elements prefetched
    p->ya = rows >= 8 || 2 * rows > L.n1 ? rows : 2 * rows;
    p->yc = rows < 256 ? rows : 256;  // pass C: at least one thread per row
    // pass A: a workgroup sums its rows' partial DFTs itself, so the row
    // chunks pass B gathers stay few: enough workgroups for one right-hand
    // side to fill the chip (about 2048, at most 64 chunks per slab), each
    // taking its rows ya at a time; batches take fewer chunks
    {
        int want = (2048 + p->slabs - 1) / p->slabs;
        if (want > 64) want = 64;
        int rb = (L.n1 + want - 1) / want;
        rb = ((rb + p->ya - 1) / p->ya) * p->ya;
        if (rb > L.n1) rb = L.n1;
        if (p->ya > rb) p->ya = rb;
        p->rb = rb;
    }
    p->nch_a = (L.n1 + p->rb - 1) / p->rb;
    p->blocks_a = p->slabs * p->nch_a;
    p->blocks_c = L.n0 * ((L.n1 + p->yc - 1) / p->yc);  // pass C takes all components of a slab
    const int plane = L.kyn * L.kzn;
    p->lds_a = sizeof(double2) * ((size_t)L.n2 + L.n1 + (size_t)p->ya * L.kzn + plane) +
               sizeof(double) * (size_t)p->ya * (L.n2 + 1);
    p->cb_mid = 8;
    while (p->cb_mid > 1 && sizeof(double2) * (size_t)nc * p->cb_mid * (L.n0 + L.kxn) > 48 * 1024) p->cb_mid /= 2;
    p->blocks_mid = (L.kyn * L.kzn + p->cb_mid - 1) / p->cb_mid;
    p->lds_b = sizeof(double2) * ((size_t)nc * p->cb_mid * (L.n0 + L.kxn) + 256);
    // pass C takes up to 64 rows per workgroup when many right-hand sides
    // fill the chip (fewer loads of the H plane per node, longer z chains)
    p->yc_max = p->yc;
    for (int y = 64; y > p->yc; y /= 2)
        if (y <= L.n1 && sizeof(double2) * (size_t)nc * ((size_t)plane + (size_t)y * L.kzn) <= 60 * 1024) {
            p->yc_max = y;
            break;
        }
    p->lds_c = sizeof(double2) * (size_t)nc * ((size_t)plane + (size_t)p->yc_max * L.kzn);
    if (p->lds_a > 60 * 1024 || p->lds_b > 60 * 1024 || p->lds_c > 60 * 1024) { delete p; return UNO_ERR_SHAPE; }
    // fused operator tile: the apply's tile shape, 2-deep in x if 4 does not fit
    p->tile = choose_tile(g);
    size_t dyn = 0;
    if (p->tile.tx == 4 && lr_tile_lds(L, 4, p->tile.tz, &dyn) > 64 * 1024) {
        p->tile.tx = 2;
        p->tile.blocks = ((g.n[0] + 1) / 2) * p->tile.geom.tiles_y * p->tile.geom.tiles_z;
    }
    p->fused = nc == 1 && lr_tile_lds(L, p->tile.tx, p->tile.tz, &dyn) <= 64 * 1024;
    p->lds_t = dyn;
    const int64_t ngp = (int64_t)p->slabs * p->nch_a * plane;
    const int64_t nh = (int64_t)p->slabs * plane;
    L.gps = ngp;
    L.hsz = nh;
    if (hipMalloc(&p->table, sizeof(double) * ntab) != hipSuccess ||
        hipMalloc(&p->Gp, sizeof(double2) * ngp) != hipSuccess || hipMalloc(&p->H, sizeof(double2) * nh) != hipSuccess ||
        (nc == 1 && hipMalloc(&p->table_bf, sizeof(uint16_t) * ntab) != hipSuccess)) {
        (void)hipFree(p->table);
        (void)hipFree(p->Gp);
        (void)hipFree(p->H);
        delete p;
        return UNO_ERR_NOMEM;
    }
    UNO_HIP(hipMemcpy(p->table, cblock.data(), sizeof(double) * ntab, hipMemcpyHostToDevice));
    if (nc == 1) {  // rounded to FP32, then to the nearest BF16 (ties to even), as the kernels round
        std::vector<uint16_t> tb(ntab);
        for (int64_t i = 0; i < ntab; ++i) {
            const float f = (float)cblock[i];
            uint32_t b;
            memcpy(&b, &f, sizeof(b));
            tb[i] = (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
        }
        UNO_HIP(hipMemcpy(p->table_bf, tb.data(), sizeof(uint16_t) * ntab, hipMemcpyHostToDevice));
    }
    *out = p;
    return UNO_OK;
}

void lowrank_destroy(LowRankPlan* p)
{
    if (!p) return;
    (void)hipFree(p->table);
    (void)hipFree(p->table_bf);
    (void)hipFree(p->Gp);
    (void)hipFree(p->H);
    delete p;
}

int lowrank_max_blocks(const LowRankPlan* p)
{
    int m = p->blocks_a > p->blocks_c ? p->blocks_a : p->blocks_c;
    const int cols = p->dev.kyn * p->dev.kzn;
    if (cols > m) m = cols;
    if (p->tile.blocks > m) m = p->tile.blocks;
    return m;
}
bool lowrank_fused(const LowRankPlan* p) { return p->fused; }
LrBatch lowrank_batch(const LowRankPlan* p, double2* Gp, double2* H, int nrhs)
{
    LrBatch b{Gp, H, nrhs, p->rb, p->nch_a, p->yc, p->cb_mid};
    // pass B: fewer columns per workgroup while a launch has under about
    // 1024 workgroups (each column is transformed alone, so the grouping
    // changes no result)
    while (b.cb > 1 && (int64_t)((p->dev.kyn * p->dev.kzn + b.cb - 1) / b.cb) * nrhs < 1024) b.cb /= 2;
    // pass C: rows per workgroup (measured: 192^3 x 3 loads 127 us with 64
    // rows, 92 us with 16; 64^3 x 48 loads 63 us with 64 rows, 75 us with 32)
    if (p->dev.nc == 1) {
        // one component (k_lr_inv_pairs, 256 / yc threads per row): the
        // most rows per workgroup that still give 2048 workgroups with at
        // most 9 point pairs per thread, else the plan's fewest rows
        const LowRankDev& L = p->dev;
        const int npair = L.n2 / 2 + 1;
        b.yc = p->yc;
        for (int y = p->yc_max; y > p->yc; y /= 2) {
            const int tpr = 256 / y, ppt = (npair + tpr - 1) / tpr;
            const int64_t wg = (int64_t)L.n0 * ((L.n1 + y - 1) / y) * nrhs;
            if (ppt <= 9 && wg >= 2048) {
                b.yc = y;
                break;
            }
        }
    } else {  // three components (k_lr_inv): about 2048 workgroups per launch
        const int64_t want = ((int64_t)p->dev.n0 * p->dev.n1 * nrhs + 2047) / 2048;
        int yc = p->yc;
        while (yc < p->yc_max && yc < want) yc *= 2;
        b.yc = yc < p->yc_max ? yc : p->yc_max;
    }
    // at least ~2048 workgroups of pass A per launch; no more chunks than the plan's
    const int64_t per = (int64_t)p->slabs * nrhs;
    int nch = (int)((2048 + per - 1) / per);
    if (nch < p->nch_a) {
        if (nch < 1) nch = 1;
        int rb = (p->dev.n1 + nch - 1) / nch;
        rb = ((rb + p->ya - 1) / p->ya) * p->ya;
        if (rb > p->dev.n1) rb = p->dev.n1;
        b.rb = rb;
        b.nch = (p->dev.n1 + rb - 1) / rb;
    }
    return b;
}
int lowrank_update_blocks(const LowRankPlan* p, int nrhs)
{
    return p->slabs * lowrank_batch(p, nullptr, nullptr, nrhs).nch;
}
void lowrank_scratch_size(const LowRankPlan* p, int64_t* ngp, int64_t* nh)
{
    *ngp = p->dev.gps;
    *nh = p->dev.hsz;
}

static CgIter no_iter()
{
    CgIter it;
    memset(&it, 0, sizeof(it));
    return it;
}

static LrBatch own(const LowRankPlan* p) { return lowrank_batch(p, p->Gp, p->H, 1); }

// pass A on r (no update); also the initial transform of the CG loop
// (part_rr, nullable: ||r||^2 partials for the fused flow; `strides`: the
// vector and partial strides of a batch)
uno_status lowrank_forward(const LowRankPlan* p, const double* r, double* part_rr, const LrBatch& bt,
                           const CgIter& strides, hipStream_t st)
{
    const dim3 grid(p->slabs * bt.nch, bt.nrhs);
    const bool pf8 = p->ya * p->dev.n2 > 1024;
    if (bt.bf) {
        if (p->dev.nc != 1) return UNO_ERR_ARG;
        uint32_t* gb = (uint32_t*)bt.Gp;
        if (pf8)
            uno_launch(UNO_KT_FFT_FWD, k_lr_fwd<false, double, 8, true>, grid, dim3(256), p->lds_a, st, p->dev, p->ya,
                       bt.rb, (double*)r, (double*)nullptr, (const double*)nullptr, (const double*)nullptr, gb,
                       strides, (const double*)nullptr, 0, (const double*)nullptr, (double*)nullptr, part_rr);
        else
            uno_launch(UNO_KT_FFT_FWD, k_lr_fwd<false, double, 4, true>, grid, dim3(256), p->lds_a, st, p->dev, p->ya,
                       bt.rb, (double*)r, (double*)nullptr, (const double*)nullptr, (const double*)nullptr, gb,
                       strides, (const double*)nullptr, 0, (const double*)nullptr, (double*)nullptr, part_rr);
        return hip_status(hipGetLastError());
    }
    if (pf8)
        uno_launch(UNO_KT_FFT_FWD, k_lr_fwd<false, double, 8>, grid, dim3(256), p->lds_a, st, p->dev, p->ya, bt.rb,
                   (double*)r, (double*)nullptr, (const double*)nullptr, (const double*)nullptr, bt.Gp, strides,
                   (const double*)nullptr, 0, (const double*)nullptr, (double*)nullptr, part_rr);
    else
        uno_launch(UNO_KT_FFT_FWD, k_lr_fwd<false, double, 4>, grid, dim3(256), p->lds_a, st, p->dev, p->ya, bt.rb,
                   (double*)r, (double*)nullptr, (const double*)nullptr, (const double*)nullptr, bt.Gp, strides,
                   (const double*)nullptr, 0, (const double*)nullptr, (double*)nullptr, part_rr);
    return hip_status(hipGetLastError());
}

// CG update of pass k fused with pass A of pass k + 1
template <typename T>
uno_status lowrank_update_forward(const LowRankPlan* p, double* r, double* u, const T* d, const T* pv,
                                  const CgIter& it, const double* part_dp, int np_dp, const double* gam,
                                  double* part_rmax, double* part_rr, const LrBatch& bt, hipStream_t st)
{
    const dim3 grid(p->slabs * bt.nch, bt.nrhs);
    const bool pf8 = p->ya * p->dev.n2 > 1024;
    if constexpr (sizeof(T) == sizeof(float)) {  // the BF16 mode runs with the FP32 vectors
        if (bt.bf) {
            if (p->dev.nc != 1) return UNO_ERR_ARG;
            uint32_t* gb = (uint32_t*)bt.Gp;
            if (pf8)
                uno_launch(UNO_KT_UPDATE, k_lr_fwd<true, T, 8, true>, grid, dim3(256), p->lds_a, st, p->dev, p->ya,
                           bt.rb, r, u, d, pv, gb, it, part_dp, np_dp, gam, part_rmax, part_rr);
            else
                uno_launch(UNO_KT_UPDATE, k_lr_fwd<true, T, 4, true>, grid, dim3(256), p->lds_a, st, p->dev, p->ya,
                           bt.rb, r, u, d, pv, gb, it, part_dp, np_dp, gam, part_rmax, part_rr);
            return hip_status(hipGetLastError());
        }
    }
    if (bt.bf) return UNO_ERR_ARG;
    if (pf8)
        uno_launch(UNO_KT_UPDATE, k_lr_fwd<true, T, 8>, grid, dim3(256), p->lds_a, st, p->dev, p->ya, bt.rb, r, u, d,
                   pv, bt.Gp, it, part_dp, np_dp, gam, part_rmax, part_rr);
    else
        uno_launch(UNO_KT_UPDATE, k_lr_fwd<true, T, 4>, grid, dim3(256), p->lds_a, st, p->dev, p->ya, bt.rb, r, u, d,
                   pv, bt.Gp, it, part_dp, np_dp, gam, part_rmax, part_rr);
    return hip_status(hipGetLastError());
}

template <int TX, bool NEAR>
static void launch_lr_tile(const LowRankPlan* p, const GridDev& g, const double* kappa, const double* r,
                           const double* dold, double* dnew, double* pv, double* part_dp, const CgIter& it,
                           const LrTileArgs& a, double* gam, const LrBatch& bt, hipStream_t st)
{
    const TileChoice& c = p->tile;
    const dim3 grid(c.blocks, bt.nrhs), blk(256);
    const double2* H = bt.H;
    switch (c.tz) {
        case 64:
            uno_launch(UNO_KT_MATVEC, k_lr_tile<TX, 64, NEAR>, grid, blk, p->lds_t, st, g, c.geom, p->dev, kappa, r, H,
                       dold, dnew, pv, part_dp, it, a, gam);
            break;
        case 32:
            uno_launch(UNO_KT_MATVEC, k_lr_tile<TX, 32, NEAR>, grid, blk, p->lds_t, st, g, c.geom, p->dev, kappa, r, H,
                       dold, dnew, pv, part_dp, it, a, gam);
            break;
        default:
            uno_launch(UNO_KT_MATVEC, k_lr_tile<TX, 16, NEAR>, grid, blk, p->lds_t, st, g, c.geom, p->dev, kappa, r, H,
                       dold, dnew, pv, part_dp, it, a, gam);
            break;
    }
}

template <int TX>
static void launch_lr_tile_tx(const LowRankPlan* p, const GridDev& g, const double* kappa, const double* r,
                              const double* dold, double* dnew, double* pv, double* part_dp, const CgIter& it,
                              const LrTileArgs& a, double* gam, const LrBatch& bt, hipStream_t st)
{
    if (tile_near(p->tile, g))
        launch_lr_tile<TX, true>(p, g, kappa, r, dold, dnew, pv, part_dp, it, a, gam, bt, st);
    else
        launch_lr_tile<TX, false>(p, g, kappa, r, dold, dnew, pv, part_dp, it, a, gam, bt, st);
}

// pass B with cb (8, 4, 2 or 1) columns per workgroup as a constant
static void launch_mid(const LowRankPlan* p, const LrBatch& bt, int cb, const CgIter& it, double* part_corr,
                       hipStream_t st)
{
    const LowRankDev& L = p->dev;
    const dim3 grid((L.kyn * L.kzn + cb - 1) / cb, bt.nrhs), blk(256);
    const size_t lds = sizeof(double2) * ((size_t)cb * (L.n0 + L.kxn) + 256);  // + the x-range partials
    if (bt.bf) {
        const uint16_t* Cb = p->table_bf;
        const uint32_t* Gb = (const uint32_t*)bt.Gp;
        uint32_t* Hb = (uint32_t*)bt.H;
        switch (cb) {
            case 8:
                uno_launch(UNO_KT_FFT_MID, k_lr_mid<8, true>, grid, blk, lds, st, L, bt.nch, Cb, Gb, Hb, it,
                           part_corr);
                break;
            case 4:
                uno_launch(UNO_KT_FFT_MID, k_lr_mid<4, true>, grid, blk, lds, st, L, bt.nch, Cb, Gb, Hb, it,
                           part_corr);
                break;
            case 2:
                uno_launch(UNO_KT_FFT_MID, k_lr_mid<2, true>, grid, blk, lds, st, L, bt.nch, Cb, Gb, Hb, it,
                           part_corr);
                break;
            default:
                uno_launch(UNO_KT_FFT_MID, k_lr_mid<1, true>, grid, blk, lds, st, L, bt.nch, Cb, Gb, Hb, it,
                           part_corr);
                break;
        }
        return;
    }
    const double* C = (const double*)p->table;
    const double2* Gp = bt.Gp;
    switch (cb) {
        case 8:
            uno_launch(UNO_KT_FFT_MID, k_lr_mid<8>, grid, blk, lds, st, L, bt.nch, C, Gp, bt.H, it, part_corr);
            break;
        case 4:
            uno_launch(UNO_KT_FFT_MID, k_lr_mid<4>, grid, blk, lds, st, L, bt.nch, C, Gp, bt.H, it, part_corr);
            break;
        case 2:
            uno_launch(UNO_KT_FFT_MID, k_lr_mid<2>, grid, blk, lds, st, L, bt.nch, C, Gp, bt.H, it, part_corr);
            break;
        default:
            uno_launch(UNO_KT_FFT_MID, k_lr_mid<1>, grid, blk, lds, st, L, bt.nch, C, Gp, bt.H, it, part_corr);
            break;
    }
}

// Fused FP64 CG pass, first half: pass B (convergence test, H, Parseval
// partials into part_corr), then the tile kernel (s on the fly, gamma,
// d = s + beta d_old, p = A d, d.p partials).  Returns the d.p partial count.
uno_status lowrank_fused_pass(const LowRankPlan* p, const Grid& g, const double* kappa, const double* r,
                              const double* dold, double* dnew, double* pv, double* part_dp, const CgIter& it,
                              double* part_corr, const double* part_rr, double* gam, const LrBatch& bt,
                              hipStream_t st, int* np_dp)
{
    if (!p->fused || bt.bf) return UNO_ERR_SHAPE;
    launch_mid(p, bt, p->cb_mid, it, part_corr, st);  // the plan's grouping: part_corr has blocks_mid partials
    UNO_HIP(hipGetLastError());
    const LrTileArgs a{part_rr, p->dev.n0 * bt.nch, part_corr, p->blocks_mid};
    if (p->tile.tx == 1)
        launch_lr_tile_tx<1>(p, g.dev, kappa, r, dold, dnew, pv, part_dp, it, a, gam, bt, st);
    else if (p->tile.tx == 2)
        launch_lr_tile_tx<2>(p, g.dev, kappa, r, dold, dnew, pv, part_dp, it, a, gam, bt, st);
    else
        launch_lr_tile_tx<4>(p, g.dev, kappa, r, dold, dnew, pv, part_dp, it, a, gam, bt, st);
    UNO_HIP(hipGetLastError());
    *np_dp = p->tile.blocks;
    return UNO_OK;
}

// passes B and C (B tests convergence inside CG); C writes s and r.s partials
template <typename T>
uno_status lowrank_finish(const LowRankPlan* p, const double* r, T* s, const CgIter* itp, int* np_rs,
                          const LrBatch& bt, hipStream_t st)
{
    const LowRankDev& L = p->dev;
    const CgIter it = itp ? *itp : no_iter();
    if (bt.bf && (L.nc != 1 || sizeof(T) != sizeof(float))) return UNO_ERR_ARG;
    if (L.nc == 3)
        uno_launch(UNO_KT_FFT_MID, k_lr_mid3, dim3((L.kyn * L.kzn + bt.cb - 1) / bt.cb, bt.nrhs), dim3(256),
                   sizeof(double2) * 3 * (size_t)bt.cb * (L.n0 + L.kxn), st, L, bt.nch, bt.cb,
                   (const double*)p->table, (const double2*)bt.Gp, bt.H, it);
    else
        launch_mid(p, bt, bt.cb, it, nullptr, st);
    UNO_HIP(hipGetLastError());
    const int nbc = L.n0 * ((L.n1 + bt.yc - 1) / bt.yc);
    const dim3 grid(nbc, bt.nrhs);
    if constexpr (sizeof(T) == sizeof(float)) {
        if (bt.bf) {
            const uint32_t* Hb = (const uint32_t*)bt.H;
            if (itp)
                uno_launch(UNO_KT_FFT_INV, k_lr_inv_pairs<true, T, true>, grid, dim3(256), p->lds_c, st, L, bt.yc, r,
                           Hb, s, it);
            else
                uno_launch(UNO_KT_FFT_INV, k_lr_inv_pairs<false, T, true>, grid, dim3(256), p->lds_c, st, L, bt.yc, r,
                           Hb, s, it);
            UNO_HIP(hipGetLastError());
            if (np_rs) *np_rs = nbc;
            return UNO_OK;
        }
    }
    if (itp) {
        if (L.nc == 3)
            uno_launch(UNO_KT_FFT_INV, k_lr_inv<true, T, 3>, grid, dim3(256), p->lds_c, st, L, bt.yc, r,
                       (const double2*)bt.H, s, it);
        else
            uno_launch(UNO_KT_FFT_INV, k_lr_inv_pairs<true, T>, grid, dim3(256), p->lds_c, st, L, bt.yc, r,
                       (const double2*)bt.H, s, it);
    } else {
        if (L.nc == 3)
            uno_launch(UNO_KT_FFT_INV, k_lr_inv<false, T, 3>, grid, dim3(256), p->lds_c, st, L, bt.yc, r,
                       (const double2*)bt.H, s, it);
        else
            uno_launch(UNO_KT_FFT_INV, k_lr_inv_pairs<false, T>, grid, dim3(256), p->lds_c, st, L, bt.yc, r,
                       (const double2*)bt.H, s, it);
    }
    UNO_HIP(hipGetLastError());
    if (np_rs) *np_rs = nbc;
    return UNO_OK;
}

uno_status lowrank_apply(const LowRankPlan* p, const double* r, double* s, hipStream_t st)
{
    uno_status e = lowrank_forward(p, r, nullptr, own(p), no_iter(), st);
    if (e != UNO_OK) return e;
    return lowrank_finish<double>(p, r, s, nullptr, nullptr, own(p), st);
}

template uno_status lowrank_finish<double>(const LowRankPlan*, const double*, double*, const CgIter*, int*,
                                           const LrBatch&, hipStream_t);
template uno_status lowrank_finish<float>(const LowRankPlan*, const double*, float*, const CgIter*, int*,
                                          const LrBatch&, hipStream_t);
template uno_status lowrank_update_forward<double>(const LowRankPlan*, double*, double*, const double*, const double*,
                                                   const CgIter&, const double*, int, const double*, double*, double*,
                                                   const LrBatch&, hipStream_t);
template uno_status lowrank_update_forward<float>(const LowRankPlan*, double*, double*, const float*, const float*,
                                                  const CgIter&, const double*, int, const double*, double*, double*,
                                                  const LrBatch&, hipStream_t);

}  // namespace unocg
