// Unitary DFT of the UNO preconditioner (Sec. 4.2.1: T unitary, T^-1 = T^H;
// for periodic problems T is the DFT with a real transform along the last
// axis and full transforms along the others, Sec. 2.2 "Fourier Neural
// Operators").  s = T^H Q T r is computed as five passes over a
// half-spectrum buffer S[x][y][kz] (kz < n2/2 + 1):
//   1. real-to-complex along z: two real rows are transformed as one complex
//      row a + i b and separated by the conjugate symmetry of real data;
//   2. complex transform along y;
//   3. complex transform along x, multiply by the table, inverse along x;
//   4. inverse along y;
//   5. complex-to-real along z (two rows at a time), optionally with r.s.
// Each pass keeps a batch of lines in LDS and runs a mixed-radix (2,3,4,5)
// Stockham transform there (autosort: no bit reversal), one butterfly per
// thread per stage.  Transforms are unnormalised; the table carries 1/n.
#include <cmath>
#include <cstring>

#include "unocg_internal.h"
#include "reduce.h"
#include "cg_ctl.h"

namespace unocg {

struct AxisDev {
    int n;
    int nstages;
    int radix[kMaxFftStages];
    const void* tw;  // double2 or float2 table, exp(-2 pi i j / n)
};

template <typename T> struct V2;
template <> struct V2<double> {
    using t = double2;
    __device__ static double2 mk(double x, double y) { return make_double2(x, y); }
};
template <> struct V2<float> {
    using t = float2;
    __device__ static float2 mk(float x, float y) { return make_float2(x, y); }
};

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b)
{
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// multiply by sign * i
template <int SIGN, typename C> __device__ __forceinline__ C mul_si(C a)
{
    C r;
    if (SIGN < 0) { r.x = a.y; r.y = -a.x; }
    else { r.x = -a.y; r.y = a.x; }
    return r;
}
template <typename C> __device__ __forceinline__ C cconj(C a) { a.y = -a.y; return a; }
template <typename C, typename S> __device__ __forceinline__ C cscale(C a, S s) { a.x *= s; a.y *= s; return a; }

// In-register small DFTs X_p = sum_q v_q exp(SIGN 2 pi i q p / R).
template <int SIGN, typename C> __device__ __forceinline__ void dft2(C* v)
{
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
template <int SIGN, typename C> __device__ __forceinline__ void dft4(C* v)
{
    C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    C s13 = cadd(v[1], v[3]), d13 = mul_si<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}
template <int SIGN, typename C> __device__ __forceinline__ void dft3(C* v)
{
    using S = decltype(v[0].x);
    const S h = (S)0.86602540378443864676;  // sqrt(3)/2
    C t = cadd(v[1], v[2]);
    C u = cscale(mul_si<SIGN>(csub(v[1], v[2])), h);
    C m = csub(v[0], cscale(t, (S)0.5));
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, u);
    v[2] = csub(m, u);
}
template <int SIGN, typename C> __device__ __forceinline__ void dft5(C* v)
{
    using S = decltype(v[0].x);
    const S c1 = (S)0.30901699437494742410, c2 = (S)-0.80901699437494742410;
    const S s1 = (S)0.95105651629515357212, s2 = (S)0.58778525229247312917;
    C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    C p1 = cadd(v[0], cadd(cscale(a1, c1), cscale(a2, c2)));
    C p2 = cadd(v[0], cadd(cscale(a1, c2), cscale(a2, c1)));
    C q1 = mul_si<SIGN>(cadd(cscale(b1, s1), cscale(b2, s2)));
    C q2 = mul_si<SIGN>(csub(cscale(b1, s2), cscale(b2, s1)));
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
}

// One Stockham stage for all lines held in LDS.  Element (line, j) lives at
// INTERLEAVED ? j * nl + line : line * n + j.
template <typename T, int SIGN, int R, bool INTERLEAVED>
__device__ __forceinline__ void stage(const typename V2<T>::t* __restrict__ in, typename V2<T>::t* __restrict__ out,
                                      int n, int nl, int ns, const typename V2<T>::t* __restrict__ tw)
{
    using C = typename V2<T>::t;
    const int nb = n / R;
    const int twstride = n / (ns * R);
    for (int q = threadIdx.x; q < nl * nb; q += blockDim.x) {
        int line, j;
        if (INTERLEAVED) { line = q % nl; j = q / nl; }
        else { line = q / nb; j = q % nb; }
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int jj = j + r * nb;
            v[r] = in[INTERLEAVED ? jj * nl + line : line * n + jj];
        }
        const int k = j % ns;
#pragma unroll
        for (int r = 1; r < R; ++r) {
            C w = tw[r * k * twstride];
            if (SIGN > 0) w = cconj(w);
            v[r] = cmul(v[r], w);
        }
        if (R == 2) dft2<SIGN>(v);
        if (R == 3) dft3<SIGN>(v);
        if (R == 4) dft4<SIGN>(v);
        if (R == 5) dft5<SIGN>(v);
        const int d = (j / ns) * ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int jj = d + r * ns;
            out[INTERLEAVED ? jj * nl + line : line * n + jj] = v[r];
        }
    }
}

// Full transform of the nl lines in buf0; returns the buffer holding the result.
template <typename T, int SIGN, bool INTERLEAVED>
__device__ typename V2<T>::t* transform_lds(typename V2<T>::t* buf0, typename V2<T>::t* buf1, int nl,
                                            const AxisDev& ax)
{
    using C = typename V2<T>::t;
    const C* tw = (const C*)ax.tw;
    C* in = buf0;
    C* out = buf1;
    int ns = 1;
    for (int st = 0; st < ax.nstages; ++st) {
        const int R = ax.radix[st];
        __syncthreads();
        switch (R) {
            case 2: stage<T, SIGN, 2, INTERLEAVED>(in, out, ax.n, nl, ns, tw); break;
            case 3: stage<T, SIGN, 3, INTERLEAVED>(in, out, ax.n, nl, ns, tw); break;
            case 4: stage<T, SIGN, 4, INTERLEAVED>(in, out, ax.n, nl, ns, tw); break;
            default: stage<T, SIGN, 5, INTERLEAVED>(in, out, ax.n, nl, ns, tw); break;
        }
        ns *= R;
        C* t = in;
        in = out;
        out = t;
    }
    __syncthreads();
    return in;
}

// Pass 1: real rows (length n2) -> half spectra, nl row pairs per workgroup.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fft_r2c_z(int64_t rows, int nl, AxisDev ax, int nh,
                                                      const T* __restrict__ x, typename V2<T>::t* __restrict__ S,
                                                      int64_t sst, CgIter it)
{
    using C = typename V2<T>::t;
    __shared__ double slots[kBlock / 64];
    if (blockIdx.y > 0) {  // right-hand side blockIdx.y of a batch
        x += (int64_t)blockIdx.y * it.vs;
        S += (int64_t)blockIdx.y * sst;
        it = rhs_iter(it);
    }
    if (it.st && head_check(it, slots)) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = ax.n;
    C* buf0 = (C*)smem;
    C* buf1 = buf0 + (size_t)nl * n;
    const int64_t pair0 = (int64_t)blockIdx.x * nl;
    for (int q = threadIdx.x; q < nl * n; q += blockDim.x) {
        int p = q / n, j = q % n;
        int64_t ra = 2 * (pair0 + p), rb = ra + 1;
        T a = (ra < rows) ? x[ra * n + j] : (T)0;
        T b = (rb < rows) ? x[rb * n + j] : (T)0;
        buf0[q] = V2<T>::mk(a, b);
    }
    C* X = transform_lds<T, -1, false>(buf0, buf1, nl, ax);
    for (int q = threadIdx.x; q < nl * nh; q += blockDim.x) {
        int p = q / nh, k = q % nh;
        int64_t ra = 2 * (pair0 + p), rb = ra + 1;
        if (ra >= rows) continue;
        C xk = X[p * n + k], xm = cconj(X[p * n + (k == 0 ? 0 : n - k)]);
        C A = cscale(cadd(xk, xm), (T)0.5);
        C B = cscale(mul_si<-1>(csub(xk, xm)), (T)0.5);  // (xk - xm) / (2i)
        S[ra * nh + k] = A;
        if (rb < rows) S[rb * nh + k] = B;
    }
}

// Passes 2-4: transforms along a strided axis.  Line l = (outer, inner),
// element j at outer * n * st + j * st + inner.  MID: forward, multiply by the
// table (same layout as S), inverse.
template <typename T, int SIGN, bool MID, typename TT>
__global__ void __launch_bounds__(kBlock) k_fft_strided(int64_t nlines, int64_t st, int nl, AxisDev ax,
                                                        typename V2<T>::t* __restrict__ S, int64_t sst,
                                                        const TT* __restrict__ table, CgIter it)
{
    using C = typename V2<T>::t;
    if (blockIdx.y > 0) {
        S += (int64_t)blockIdx.y * sst;
        it = rhs_iter(it);
    }
    if (it.st && loop_ended(it.st, it.k)) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = ax.n;
    C* buf0 = (C*)smem;
    C* buf1 = buf0 + (size_t)nl * n;
    const int64_t l0 = (int64_t)blockIdx.x * nl;
    for (int q = threadIdx.x; q < nl * n; q += blockDim.x) {
        int line = q % nl, j = q / nl;
        int64_t l = l0 + line;
        C v = V2<T>::mk(0, 0);
        if (l < nlines) {
            int64_t outer = l / st, inner = l % st;
            v = S[(outer * n + j) * st + inner];
        }
        buf0[q] = v;
    }
    C* X;
    if (MID) {
        X = transform_lds<T, -1, true>(buf0, buf1, nl, ax);
        for (int q = threadIdx.x; q < nl * n; q += blockDim.x) {
            int line = q % nl, j = q / nl;
            int64_t l = l0 + line;
            if (l < nlines) {
                int64_t outer = l / st, inner = l % st;
                T w = (T)table[(outer * n + j) * st + inner];
                X[q] = cscale(X[q], w);
            }
        }
        C* other = (X == buf0) ? buf1 : buf0;
        X = transform_lds<T, +1, true>(X, other, nl, ax);
    } else {
        X = transform_lds<T, SIGN, true>(buf0, buf1, nl, ax);
    }
    for (int q = threadIdx.x; q < nl * n; q += blockDim.x) {
        int line = q % nl, j = q / nl;
        int64_t l = l0 + line;
        if (l < nlines) {
            int64_t outer = l / st, inner = l % st;
            S[(outer * n + j) * st + inner] = X[q];
        }
    }
}

// Pass 5: half spectra -> real rows, two rows per complex transform.  Inside
// CG it also writes the per-workgroup partials of r.s (FP64).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fft_c2r_z(int64_t rows, int nl, AxisDev ax, int nh,
                                                      const typename V2<T>::t* __restrict__ S, int64_t sst,
                                                      T* __restrict__ out, CgIter it)
{
    using C = typename V2<T>::t;
    if (blockIdx.y > 0) {
        S += (int64_t)blockIdx.y * sst;
        out += (int64_t)blockIdx.y * it.vs;
        it = rhs_iter(it);
    }
    if (it.st && loop_ended(it.st, it.k)) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double slots[kBlock / 64];
    const double* __restrict__ rdot = it.st ? it.r : nullptr;
    const int n = ax.n;
    C* buf0 = (C*)smem;
    C* buf1 = buf0 + (size_t)nl * n;
    const int64_t pair0 = (int64_t)blockIdx.x * nl;
    const bool even = (n % 2) == 0;
    for (int q = threadIdx.x; q < nl * n; q += blockDim.x) {
        int p = q / n, k = q % n;
        int64_t ra = 2 * (pair0 + p), rb = ra + 1;
        C A = V2<T>::mk(0, 0), B = V2<T>::mk(0, 0);
        if (ra < rows) {
            int kk = (k < nh) ? k : n - k;
            A = S[ra * nh + kk];
            if (rb < rows) B = S[rb * nh + kk];
            if (kk == 0 || (even && kk == n / 2)) { A.y = 0; B.y = 0; }  // real part at DC / Nyquist
            if (k >= nh) { A = cconj(A); B = cconj(B); }
        }
        buf0[q] = cadd(A, mul_si<+1>(B));  // A + i B
    }
    C* X = transform_lds<T, +1, false>(buf0, buf1, nl, ax);
    double acc = 0.0;
    for (int q = threadIdx.x; q < nl * n; q += blockDim.x) {
        int p = q / n, j = q % n;
        int64_t ra = 2 * (pair0 + p), rb = ra + 1;
        if (ra >= rows) continue;
        C v = X[q];
        out[ra * n + j] = v.x;
        if (rb < rows) out[rb * n + j] = v.y;
        if (rdot) {
            acc += rdot[ra * n + j] * (double)v.x;
            if (rb < rows) acc += rdot[rb * n + j] * (double)v.y;
        }
    }
    if (rdot) {
        double bsum = block_reduce<OpSum>(acc, slots);
        if (threadIdx.x == 0) it.part_rs[blockIdx.x] = bsum;
    }
}

// ----------------------------------------------------------------------------
// host side

static bool factorize(int n, AxisPlan* a)
{
    if (n < 1 || n > 2048) return false;  // LDS holds two line buffers of <= 64 KiB
    a->n = n;
    a->nstages = 0;
    int m = n;
    const int order[4] = {4, 2, 3, 5};
    for (int oi = 0; oi < 4; ++oi) {
        int R = order[oi];
        while (m % R == 0) {
            if (a->nstages >= kMaxFftStages) return false;
            a->radix[a->nstages++] = R;
            m /= R;
        }
    }
    return m == 1;
}

uno_status fft_plan_create(const Grid& g, FftPlan* p, bool twiddles_only)
{
    memset(p, 0, sizeof(*p));
    for (int b = 0; b < 3; ++b) {
        AxisPlan& a = p->ax[b];
        if (twiddles_only) {
            if (g.n[b] < 1) return UNO_ERR_SHAPE;
            a.n = g.n[b];
        } else if (!factorize(g.n[b], &a)) {
            return UNO_ERR_SHAPE;
        }
        std::vector<double2> t64(a.n);
        std::vector<float2> t32(a.n);
        for (int j = 0; j < a.n; ++j) {
            long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)a.n;
            double c = (double)cosl(ang), s = (double)-sinl(ang);
            t64[j] = make_double2(c, s);
            t32[j] = make_float2((float)c, (float)s);
        }
        if (hipMalloc(&a.tw64, sizeof(double2) * a.n) != hipSuccess) return UNO_ERR_NOMEM;
        if (hipMalloc(&a.tw32, sizeof(float2) * a.n) != hipSuccess) return UNO_ERR_NOMEM;
        UNO_HIP(hipMemcpy(a.tw64, t64.data(), sizeof(double2) * a.n, hipMemcpyHostToDevice));
        UNO_HIP(hipMemcpy(a.tw32, t32.data(), sizeof(float2) * a.n, hipMemcpyHostToDevice));
    }
    p->nh = g.n[2] / 2 + 1;
    p->nspec = (int64_t)g.n[0] * g.n[1] * p->nh;
    return UNO_OK;
}

void fft_plan_destroy(FftPlan* p)
{
    for (int b = 0; b < 3; ++b) {
        if (p->ax[b].tw64) (void)hipFree(p->ax[b].tw64);
        if (p->ax[b].tw32) (void)hipFree(p->ax[b].tw32);
        p->ax[b].tw64 = nullptr;
        p->ax[b].tw32 = nullptr;
    }
}

static AxisDev axis_dev(const AxisPlan& a, bool f64)
{
    AxisDev d;
    d.n = a.n;
    d.nstages = a.nstages;
    for (int i = 0; i < kMaxFftStages; ++i) d.radix[i] = a.radix[i];
    d.tw = f64 ? (const void*)a.tw64 : (const void*)a.tw32;
    return d;
}

// lines per workgroup: about 512 complex values in LDS per buffer
static int lines_per_block(int n) { return n >= 512 ? 1 : 512 / n; }

// workgroups of the last (complex-to-real) pass = number of r.s partials
int fft_c2r_blocks(const Grid& g, const FftPlan& p)
{
    const int nl = lines_per_block(p.ax[2].n);
    const int64_t pairs = ((int64_t)g.n[0] * g.n[1] + 1) / 2;
    return (int)((pairs + nl - 1) / nl);
}

// nrhs right-hand sides along grid y: vectors at + b it.vs, spectra at
// + b sst (one when itp is null)
template <typename T, typename TT>
static uno_status run_passes(const Grid& g, const FftPlan& p, const TT* table, const T* r, T* s,
                             typename V2<T>::t* S, const CgIter* itp, int* np_rs, hipStream_t stream, bool f64,
                             int nrhs, int64_t sst)
{
    using C = typename V2<T>::t;
    CgIter it;
    memset(&it, 0, sizeof(it));
    if (itp) it = *itp;
    const int64_t rows = (int64_t)g.n[0] * g.n[1];
    const int nh = p.nh;
    // pass 1
    {
        AxisDev az = axis_dev(p.ax[2], f64);
        int nl = lines_per_block(az.n);
        int64_t pairs = (rows + 1) / 2;
        int nb = (int)((pairs + nl - 1) / nl);
        size_t sh = 2 * sizeof(C) * (size_t)nl * az.n;
        uno_launch(UNO_KT_FFT_FWD, k_fft_r2c_z<T>, dim3(nb, nrhs), dim3(kBlock), sh, stream, rows, nl, az, nh, r, S, sst,
                   it);
        UNO_HIP(hipGetLastError());
    }
    // pass 2: y forward (st = nh, outer = n0)
    AxisDev ay = axis_dev(p.ax[1], f64);
    if (ay.n > 1) {
        int nl = lines_per_block(ay.n);
        int64_t nlines = (int64_t)g.n[0] * nh;
        int nb = (int)((nlines + nl - 1) / nl);
        size_t sh = 2 * sizeof(C) * (size_t)nl * ay.n;
        hipLaunchKernelGGL((k_fft_strided<T, -1, false, TT>), dim3(nb, nrhs), dim3(kBlock), sh, stream, nlines,
                           (int64_t)nh, nl, ay, S, sst, table, it);
        UNO_HIP(hipGetLastError());
    }
    // pass 3: x forward, multiply, inverse (st = n1 nh, outer = 1)
    {
        AxisDev ax = axis_dev(p.ax[0], f64);
        int nl = lines_per_block(ax.n);
        int64_t nlines = (int64_t)g.n[1] * nh;
        int nb = (int)((nlines + nl - 1) / nl);
        size_t sh = 2 * sizeof(C) * (size_t)nl * ax.n;
        uno_launch(UNO_KT_FFT_MID, k_fft_strided<T, -1, true, TT>, dim3(nb, nrhs), dim3(kBlock), sh, stream, nlines,
                   nlines, nl, ax, S, sst, table, it);
        UNO_HIP(hipGetLastError());
    }
    // pass 4: y inverse
    if (ay.n > 1) {
        int nl = lines_per_block(ay.n);
        int64_t nlines = (int64_t)g.n[0] * nh;
        int nb = (int)((nlines + nl - 1) / nl);
        size_t sh = 2 * sizeof(C) * (size_t)nl * ay.n;
        hipLaunchKernelGGL((k_fft_strided<T, +1, false, TT>), dim3(nb, nrhs), dim3(kBlock), sh, stream, nlines,
                           (int64_t)nh, nl, ay, S, sst, table, it);
        UNO_HIP(hipGetLastError());
    }
    // pass 5
    {
        AxisDev az = axis_dev(p.ax[2], f64);
        int nl = lines_per_block(az.n);
        int64_t pairs = (rows + 1) / 2;
        int nb = (int)((pairs + nl - 1) / nl);
        size_t sh = 2 * sizeof(C) * (size_t)nl * az.n;
        uno_launch(UNO_KT_FFT_INV, k_fft_c2r_z<T>, dim3(nb, nrhs), dim3(kBlock), sh, stream, rows, nl, az, nh,
                   (const C*)S, sst, s, it);
        if (np_rs) *np_rs = nb;
        UNO_HIP(hipGetLastError());
    }
    return UNO_OK;
}

uno_status uno_apply_passes(const Grid& g, const FftPlan& p, const void* table, uno_dtype table_t, const void* r,
                            void* s, uno_dtype vec_t, void* spec, const CgIter* it, int* np_rs, hipStream_t stream,
                            int nrhs, int64_t sst)
{
    if (nrhs < 1 || (nrhs > 1 && !it)) return UNO_ERR_ARG;  // batches carry their strides in it
    if (vec_t == UNO_F64) {
        if (table_t != UNO_F64) return UNO_ERR_ARG;
        return run_passes<double, double>(g, p, (const double*)table, (const double*)r, (double*)s, (double2*)spec, it,
                                          np_rs, stream, true, nrhs, sst);
    }
    if (vec_t == UNO_F32) {
        if (it) return UNO_ERR_ARG;  // the FP32 path forms r.s in the CG update kernels
        if (table_t == UNO_F32)
            return run_passes<float, float>(g, p, (const float*)table, (const float*)r, (float*)s, (float2*)spec,
                                            nullptr, nullptr, stream, false, 1, 0);
        return UNO_ERR_ARG;
    }
    return UNO_ERR_ARG;
}

// Forward real transform only (passes 1 and 2 and the forward x transform),
// for feature accumulation: spec receives F x on the half spectrum.
uno_status fft_forward_real(const Grid& g, const FftPlan& p, const double* x, double2* spec, hipStream_t stream)
{
    CgIter none;
    memset(&none, 0, sizeof(none));
    const int64_t rows = (int64_t)g.n[0] * g.n[1];
    const int nh = p.nh;
    AxisDev az = axis_dev(p.ax[2], true);
    {
        int nl = lines_per_block(az.n);
        int64_t pairs = (rows + 1) / 2;
        int nb = (int)((pairs + nl - 1) / nl);
        size_t sh = 2 * sizeof(double2) * (size_t)nl * az.n;
        hipLaunchKernelGGL(k_fft_r2c_z<double>, dim3(nb), dim3(kBlock), sh, stream, rows, nl, az, nh, x, spec,
                           (int64_t)0, none);
        UNO_HIP(hipGetLastError());
    }
    AxisDev ay = axis_dev(p.ax[1], true);
    if (ay.n > 1) {
        int nl = lines_per_block(ay.n);
        int64_t nlines = (int64_t)g.n[0] * nh;
        int nb = (int)((nlines + nl - 1) / nl);
        size_t sh = 2 * sizeof(double2) * (size_t)nl * ay.n;
        hipLaunchKernelGGL((k_fft_strided<double, -1, false, double>), dim3(nb), dim3(kBlock), sh, stream, nlines,
                           (int64_t)nh, nl, ay, spec, (int64_t)0, (const double*)nullptr, none);
        UNO_HIP(hipGetLastError());
    }
    AxisDev ax = axis_dev(p.ax[0], true);
    if (ax.n > 1) {
        int nl = lines_per_block(ax.n);
        int64_t nlines = (int64_t)g.n[1] * nh;
        int nb = (int)((nlines + nl - 1) / nl);
        size_t sh = 2 * sizeof(double2) * (size_t)nl * ax.n;
        hipLaunchKernelGGL((k_fft_strided<double, -1, false, double>), dim3(nb), dim3(kBlock), sh, stream, nlines,
                           nlines, nl, ax, spec, (int64_t)0, (const double*)nullptr, none);
        UNO_HIP(hipGetLastError());
    }
    return UNO_OK;
}

}  // namespace unocg
