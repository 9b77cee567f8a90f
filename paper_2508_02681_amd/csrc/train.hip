// Second-order training of the UNO weights for one nodal DOF (Sec. 4.4).
//
// Features (eq. (features-c-1)) are accumulated on the half spectrum from
// forward transforms computed by the same FFT kernels as the preconditioner:
//   alpha(k) += |f^(k)|^2 / Ns,  beta(k) += 2 Re(conj f^(k) u^(k)) / Ns,
// hats being the unitary DFT.  The loss in the table values v(k) is
//   L = sum_k alpha(k) v(k)^2 - beta(k) v(k) + const,
// a sum of convex quadratics, and the parametrization
//   v(k) = a + b_g(k)  (a = theta0^2, b = theta_i^2 >= 0, groups g of modes
//   sharing one learned value), v(k) = a on the other modes k != 0,
// makes the exact minimiser a one-dimensional search over a: for a fixed a,
// b_g = max(0, B_g / (2 A_g) - a); the remaining function of a is a convex
// piecewise quadratic whose root of the derivative is found between sorted
// breakpoints.  The Newton iteration of Algorithm 4 converges to this point.
#include <algorithm>
#include <cmath>
#include <vector>

#include "unocg_internal.h"
#include "reduce.h"

namespace unocg {

__global__ void __launch_bounds__(kBlock) k_feat_accum(int64_t ns, const double2* __restrict__ F,
                                                       const double2* __restrict__ U, double scale,
                                                       double* __restrict__ alpha, double* __restrict__ beta)
{
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= ns) return;
    double2 f = F[l], u = U[l];
    alpha[l] += scale * (f.x * f.x + f.y * f.y);
    beta[l] += 2.0 * scale * (f.x * u.x + f.y * u.y);
}


// ---- Loss and gradient in the weights (a first-order training step) ----
// L(theta) = sum over the full spectrum of alpha Phi^2 - beta Phi (the
// sample loss (1/Ns) sum_j ||P_theta f_j - u_j||^2 of Algorithm 3 up to the
// constant delta, by Parseval), kept on the half spectrum with the
// multiplicity of the conjugate pair.  Phi(k) = W + 0.5 (psi_s(k) + psi_s(-k))
// with W = theta_0^2 and psi_s = theta_s^2 on learned modes (and their
// conjugates), so dL/dtheta_0 = 2 theta_0 sum_{k != 0} q(k) and a slot whose
// mode has k_d > 0 gets 2 theta_s q(k_s), one with k_d = 0 gets
// theta_s (q(k_s) + q(-k_s)), where q = mult (2 alpha Phi - beta).
struct TrainDev {
    int d, M;
    int n0, n1, n2, nh;
    int64_t nspec, nw;
};

__device__ __forceinline__ int centred_dev(int i, int n) { return (2 * i <= n) ? i : i - n; }

__device__ inline int64_t slot_dev(int d, int M, const int* k)
{
    int64_t lin = 0, zero = 0;
    bool nz = false;
    for (int b = 0; b < d; ++b) {
        const int lo = (b == d - 1) ? 0 : -M;
        const int span = (b == d - 1) ? M + 1 : 2 * M + 1;
        if (k[b] < lo || k[b] > M) return 0;
        lin = lin * span + (k[b] - lo);
        zero = zero * span + (-lo);
        nz |= (k[b] != 0);
    }
    if (!nz) return 0;
    return lin < zero ? lin + 1 : lin;
}

// learned value of mode k (its own slot or, for a conjugate mode, that of -k)
__device__ inline double psi_dev(const TrainDev& t, const double* __restrict__ th, const int* k)
{
    int64_t s = slot_dev(t.d, t.M, k);
    if (s == 0 && k[t.d - 1] < 0) {
        int mk[3];
        for (int b = 0; b < t.d; ++b) mk[b] = -k[b];
        s = slot_dev(t.d, t.M, mk);
    }
    return s ? th[s] * th[s] : 0.0;
}

__device__ inline double phi_dev(const TrainDev& t, const double* __restrict__ th, const int* k)
{
    int mk[3];
    for (int b = 0; b < t.d; ++b) mk[b] = -k[b];
    return th[0] * th[0] + 0.5 * (psi_dev(t, th, k) + psi_dev(t, th, mk));
}

// mode of half-spectrum entry l, in the problem's dimension
__device__ inline void mode_of(const TrainDev& t, int64_t l, int* k, int* kz)
{
    *kz = (int)(l % t.nh);
    const int64_t r = l / t.nh;
    const int iy = (int)(r % t.n1), ix = (int)(r / t.n1);
    if (t.d == 3) { k[0] = centred_dev(ix, t.n0); k[1] = centred_dev(iy, t.n1); k[2] = *kz; }
    else { k[0] = centred_dev(iy, t.n1); k[1] = *kz; }
}

__device__ inline double mult_of(const TrainDev& t, int kz)
{
    return (kz == 0 || (t.n2 % 2 == 0 && kz == t.n2 / 2)) ? 1.0 : 2.0;
}

// per-workgroup partial sums of the loss and of q over k != 0
__global__ void __launch_bounds__(kBlock) k_train_loss(TrainDev t, const double* __restrict__ th,
                                                       const double* __restrict__ alpha,
                                                       const double* __restrict__ beta, double* __restrict__ part)
{
    __shared__ double slots[kBlock / 64];
    double L = 0.0, Q = 0.0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < t.nspec; l += (int64_t)gridDim.x * blockDim.x) {
        if (l == 0) continue;  // zero mode: Phi = 0
        int k[3], kz;
        mode_of(t, l, k, &kz);
        const double m = mult_of(t, kz), ph = phi_dev(t, th, k), a = alpha[l], b = beta[l];
        L += m * (a * ph * ph - b * ph);
        Q += m * (2.0 * a * ph - b);
    }
    const double bl = block_reduce<OpSum>(L, slots);
    const double bq = block_reduce<OpSum>(Q, slots);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = bl;
        part[2 * blockIdx.x + 1] = bq;
    }
}

// dL/dtheta_s for the learned slots s = 1 .. nw-1 (one thread per slot)
__global__ void __launch_bounds__(kBlock) k_train_slot_grad(TrainDev t, const double* __restrict__ th,
                                                            const double* __restrict__ alpha,
                                                            const double* __restrict__ beta,
                                                            double* __restrict__ grad)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (s >= t.nw) return;
    // mode k_s of slot s (lexicographic over [-M..M]^(d-1) x [0..M], zero skipped)
    int64_t zero = 0;
    for (int b = 0; b < t.d; ++b) zero = zero * ((b == t.d - 1) ? t.M + 1 : 2 * t.M + 1) + ((b == t.d - 1) ? 0 : t.M);
    int64_t lin = (s <= zero) ? s - 1 : s;
    int k[3];
    for (int b = t.d - 1; b >= 0; --b) {
        const int span = (b == t.d - 1) ? t.M + 1 : 2 * t.M + 1;
        const int lo = (b == t.d - 1) ? 0 : -t.M;
        k[b] = (int)(lin % span) + lo;
        lin /= span;
    }
    auto entry = [&](const int* kk) -> int64_t {
        const int kzz = kk[t.d - 1];
        const int ky = kk[t.d - 2];
        const int kx = (t.d == 3) ? kk[0] : 0;
        const int ix = (kx % t.n0 + t.n0) % t.n0, iy = (ky % t.n1 + t.n1) % t.n1;
        return ((int64_t)ix * t.n1 + iy) * t.nh + kzz;
    };
    const double ph = phi_dev(t, th, k);
    const int64_t l1 = entry(k);
    const double q1 = mult_of(t, k[t.d - 1]) * (2.0 * alpha[l1] * ph - beta[l1]);
    if (k[t.d - 1] > 0) {
        grad[s] = 2.0 * th[s] * q1;
    } else {
        int mk[3];
        for (int b = 0; b < t.d; ++b) mk[b] = -k[b];
        const int64_t l2 = entry(mk);
        const double q2 = 2.0 * alpha[l2] * ph - beta[l2];
        grad[s] = th[s] * (q1 + q2);
    }
}

}  // namespace unocg

using namespace unocg;

namespace {
int centred_i(int i, int n) { return (2 * i <= n) ? i : i - n; }

int64_t slot_in_K(int d, int M, const int* k)
{
    int64_t lin = 0, zero = 0;
    bool nz = false;
    for (int b = 0; b < d; ++b) {
        const int lo = (b == d - 1) ? 0 : -M;
        const int span = (b == d - 1) ? M + 1 : 2 * M + 1;
        if (k[b] < lo || k[b] > M) return 0;
        lin = lin * span + (k[b] - lo);
        zero = zero * span + (-lo);
        nz |= (k[b] != 0);
    }
    if (!nz) return 0;
    return lin < zero ? lin + 1 : lin;
}
}  // namespace

extern "C" {

uno_status uno_train_accumulate(const uno_grid* grid, int32_t ns, const double* f, const double* u,
                                double ns_total, double* alpha, double* beta, void* stream)
{
    Grid g;
    uno_status e = make_grid(grid, &g);
    if (e != UNO_OK) return e;
    if (ns < 0 || !(ns_total > 0.0) || !alpha || !beta || (ns > 0 && (!f || !u))) return UNO_ERR_ARG;
    FftPlan plan;
    e = fft_plan_create(g, &plan);
    if (e != UNO_OK) { fft_plan_destroy(&plan); return e; }
    double2 *F = nullptr, *U = nullptr;
    if (hipMalloc(&F, sizeof(double2) * plan.nspec) != hipSuccess ||
        hipMalloc(&U, sizeof(double2) * plan.nspec) != hipSuccess) {
        (void)hipFree(F);
        fft_plan_destroy(&plan);
        return UNO_ERR_NOMEM;
    }
    hipStream_t st = (hipStream_t)stream;
    const double scale = 1.0 / (ns_total * (double)g.total);
    const int nb = (int)((plan.nspec + kBlock - 1) / kBlock);
    for (int j = 0; j < ns && e == UNO_OK; ++j) {
        e = fft_forward_real(g, plan, f + (int64_t)j * g.total, F, st);
        if (e == UNO_OK) e = fft_forward_real(g, plan, u + (int64_t)j * g.total, U, st);
        if (e == UNO_OK) {
            hipLaunchKernelGGL(k_feat_accum, dim3(nb), dim3(kBlock), 0, st, plan.nspec, F, U, scale, alpha, beta);
            e = hip_status(hipGetLastError());
        }
    }
    if (hipStreamSynchronize(st) != hipSuccess && e == UNO_OK) e = UNO_ERR_DEVICE;
    (void)hipFree(F);
    (void)hipFree(U);
    fft_plan_destroy(&plan);
    return e;
}

uno_status uno_train_loss_grad(const uno_grid* grid, int32_t M, const double* alpha, const double* beta,
                               const double* theta, int64_t ntheta, double* loss, double* grad, void* stream)
{
    Grid g;
    uno_status e = make_grid(grid, &g);
    if (e != UNO_OK) return e;
    const int d = grid->dim;
    if (!alpha || !beta || !theta || !loss || !grad || M < 0) return UNO_ERR_ARG;
    for (int b = 0; b < d; ++b)
        if (2 * M + 1 > grid->n[b]) return UNO_ERR_SHAPE;
    int64_t nw = M + 1;
    for (int b = 0; b + 1 < d; ++b) nw *= 2 * M + 1;
    if (ntheta != nw) return UNO_ERR_SHAPE;
    for (int64_t i = 0; i < ntheta; ++i)
        if (!std::isfinite(theta[i])) return UNO_ERR_ARG;
    TrainDev t;
    t.d = d;
    t.M = M;
    t.n0 = g.n[0];
    t.n1 = g.n[1];
    t.n2 = g.n[2];
    t.nh = g.n[2] / 2 + 1;
    t.nspec = (int64_t)g.n[0] * g.n[1] * t.nh;
    t.nw = nw;
    const int nb = (int)std::min<int64_t>((t.nspec + kBlock - 1) / kBlock, 1024);
    double *th = nullptr, *part = nullptr, *gd = nullptr;
    if (hipMalloc(&th, sizeof(double) * nw) != hipSuccess || hipMalloc(&part, sizeof(double) * 2 * nb) != hipSuccess ||
        hipMalloc(&gd, sizeof(double) * nw) != hipSuccess) {
        (void)hipFree(th);
        (void)hipFree(part);
        return UNO_ERR_NOMEM;
    }
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> hp(2 * (size_t)nb);
    e = hip_status(hipMemcpyAsync(th, theta, sizeof(double) * nw, hipMemcpyHostToDevice, st));
    if (e == UNO_OK) {
        hipLaunchKernelGGL(k_train_loss, dim3(nb), dim3(kBlock), 0, st, t, (const double*)th, alpha, beta, part);
        if (nw > 1)
            hipLaunchKernelGGL(k_train_slot_grad, dim3((unsigned)((nw - 1 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                               st, t, (const double*)th, alpha, beta, gd);
        e = hip_status(hipGetLastError());
    }
    if (e == UNO_OK) e = hip_status(hipMemcpyAsync(hp.data(), part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, st));
    if (e == UNO_OK && nw > 1)
        e = hip_status(hipMemcpyAsync(grad + 1, gd + 1, sizeof(double) * (nw - 1), hipMemcpyDeviceToHost, st));
    if (e == UNO_OK) e = hip_status(hipStreamSynchronize(st));
    if (e == UNO_OK) {
        double L = 0.0, Q = 0.0;
        for (int b = 0; b < nb; ++b) {
            L += hp[2 * b];
            Q += hp[2 * b + 1];
        }
        *loss = L;
        grad[0] = 2.0 * theta[0] * Q;
    }
    (void)hipFree(th);
    (void)hipFree(part);
    (void)hipFree(gd);
    return e;
}

uno_status uno_train_fit(const uno_grid* grid, int32_t M, const double* alpha, const double* beta, double* theta,
                         int64_t ntheta, void* stream)
{
    Grid g;
    uno_status e = make_grid(grid, &g);
    if (e != UNO_OK) return e;
    const int d = grid->dim;
    if (!alpha || !beta || !theta || M < 0) return UNO_ERR_ARG;
    for (int b = 0; b < d; ++b)
        if (2 * M + 1 > grid->n[b]) return UNO_ERR_SHAPE;
    int64_t nw = M + 1;
    for (int b = 0; b + 1 < d; ++b) nw *= 2 * M + 1;
    if (ntheta != nw) return UNO_ERR_SHAPE;
    const int nh = g.n[2] / 2 + 1;
    const int64_t nspec = (int64_t)g.n[0] * g.n[1] * nh;
    std::vector<double> A(nspec), B(nspec);
    hipStream_t st = (hipStream_t)stream;
    UNO_HIP(hipMemcpyAsync(A.data(), alpha, sizeof(double) * nspec, hipMemcpyDeviceToHost, st));
    UNO_HIP(hipMemcpyAsync(B.data(), beta, sizeof(double) * nspec, hipMemcpyDeviceToHost, st));
    UNO_HIP(hipStreamSynchronize(st));

    // per-slot sums; a pair (k, -k) on the plane k_d = 0 is keyed by the smaller slot
    std::vector<double> Ag(nw, 0.0), Bg(nw, 0.0);
    std::vector<int64_t> key(nw);
    for (int64_t s = 0; s < nw; ++s) key[s] = s;
    double Au = 0.0, Bu = 0.0;
    const bool even = (g.n[2] % 2) == 0;
    for (int ix = 0; ix < g.n[0]; ++ix)
        for (int iy = 0; iy < g.n[1]; ++iy)
            for (int kz = 0; kz < nh; ++kz) {
                const int64_t l = ((int64_t)ix * g.n[1] + iy) * nh + kz;
                if (l == 0) continue;  // zero mode: excluded, its table value is fixed to 0
                const double mult = (kz == 0 || (even && kz == g.n[2] / 2)) ? 1.0 : 2.0;
                int k[3], mk[3];
                if (d == 3) { k[0] = centred_i(ix, g.n[0]); k[1] = centred_i(iy, g.n[1]); k[2] = kz; }
                else { k[0] = centred_i(iy, g.n[1]); k[1] = kz; }
                const int64_t s = slot_in_K(d, M, k);
                if (s == 0) {
                    Au += mult * A[l];
                    Bu += mult * B[l];
                    continue;
                }
                int64_t gk = s;
                if (k[d - 1] == 0) {
                    for (int b = 0; b < d; ++b) mk[b] = -k[b];
                    const int64_t s2 = slot_in_K(d, M, mk);
                    gk = std::min(s, s2);
                    key[s] = gk;
                    key[s2] = gk;
                }
                Ag[gk] += mult * A[l];
                Bg[gk] += mult * B[l];
            }
    struct Brk { double c, A, B; };
    std::vector<Brk> br;
    for (int64_t s = 1; s < nw; ++s)
        if (key[s] == s && Ag[s] > 0.0) br.push_back({Bg[s] / (2.0 * Ag[s]), Ag[s], Bg[s]});
    std::sort(br.begin(), br.end(), [](const Brk& x, const Brk& y) { return x.c < y.c; });
    // derivative 2 SA a - SB with the groups whose breakpoint lies below a
    double SA = Au, SB = Bu, a = 0.0;
    size_t i = 0;
    while (i < br.size() && br[i].c <= 0.0) { SA += br[i].A; SB += br[i].B; ++i; }
    for (;;) {
        double cand = SA > 0.0 ? SB / (2.0 * SA) : 0.0;
        if (cand < 0.0) cand = 0.0;
        const double hi = i < br.size() ? br[i].c : INFINITY;
        if (cand <= hi) { a = cand; break; }
        SA += br[i].A;
        SB += br[i].B;
        ++i;
    }
    theta[0] = std::sqrt(a);
    for (int64_t s = 1; s < nw; ++s) {
        const int64_t gk = key[s];
        const double c = Ag[gk] > 0.0 ? Bg[gk] / (2.0 * Ag[gk]) : -INFINITY;
        theta[s] = (c > a) ? std::sqrt(c - a) : 0.0;
    }
    return UNO_OK;
}

}  // extern "C"
