// Second-order training of the UNO weights for three nodal DOF (Sec. 4.4
// with App. B).
//
// Features: with hats the unitary DFT of each component (x, y, z),
//   alpha_1 = <|f^_x|^2>, alpha_2 = <|f^_y|^2>, alpha_4 = <|f^_z|^2>,
//   alpha_3 = <2 Re(conj f^_x f^_y)>, alpha_5 = <2 Re(conj f^_y f^_z)>,
//   alpha_6 = <2 Re(conj f^_x f^_z)>,
//   beta_1 = <2 Re(conj f^_x u^_x)>, beta_2, beta_4 likewise,
//   beta_3 = <2 Re(conj f^_x u^_y + conj f^_y u^_x)>, beta_5 (y, z), beta_6 (x, z),
// accumulated on the half spectrum from the forward transforms of the FFT
// kernels.  The loss per mode is the quadratic of App. B in the table
// entries q1..q6 of Phi(k); it is linear in the features, so the modes that
// share one table value are summed first: the modes outside the learned set
// (Phi = psi(w^0)), each learned mode with k_d > 0 together with its
// conjugate, and each pair k, -k on the plane k_d = 0 (its two slots are
// tied to one weight vector, so Phi = psi(w^0) + psi(w^g) on every group).
// Algorithm 4 then runs on the host over w^0 and one w^g per group: Newton
// steps with the gradient and Hessian of the chain rule through psi, a
// Levenberg-Marquardt shift keeping every step a descent step, the linear
// system solved through the 6 x 6 blocks (w^0 couples to every group,
// groups only to w^0: an arrowhead matrix, eliminated by its Schur
// complement on w^0).
#include <cmath>
#include <cstring>
#include <vector>

#include "unocg_internal.h"

namespace unocg {

// x-, y-, z-spectra of f (F0..F2) and u (U0..U2), nspec each
__global__ void __launch_bounds__(kBlock) k_feat3_accum(int64_t ns, const double2* __restrict__ F,
                                                        const double2* __restrict__ U, double scale,
                                                        double* __restrict__ alpha, double* __restrict__ beta)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= ns) return;
    const double2 fx = F[l], fy = F[ns + l], fz = F[2 * ns + l];
    const double2 ux = U[l], uy = U[ns + l], uz = U[2 * ns + l];
    // Re(conj a b)
    auto re = [](double2 a, double2 b) { return a.x * b.x + a.y * b.y; };
    alpha[l] += scale * re(fx, fx);
    alpha[ns + l] += scale * re(fy, fy);
    alpha[2 * ns + l] += 2.0 * scale * re(fx, fy);
    alpha[3 * ns + l] += scale * re(fz, fz);
    alpha[4 * ns + l] += 2.0 * scale * re(fy, fz);
    alpha[5 * ns + l] += 2.0 * scale * re(fx, fz);
    beta[l] += 2.0 * scale * re(fx, ux);
    beta[ns + l] += 2.0 * scale * re(fy, uy);
    beta[2 * ns + l] += 2.0 * scale * (re(fx, uy) + re(fy, ux));
    beta[3 * ns + l] += 2.0 * scale * re(fz, uz);
    beta[4 * ns + l] += 2.0 * scale * (re(fy, uz) + re(fz, uy));
    beta[5 * ns + l] += 2.0 * scale * (re(fx, uz) + re(fz, ux));
}

namespace {

int centred3(int i, int n) { return (2 * i <= n) ? i : i - n; }

// slot of k in K = [-M..M]^2 x [0..M] \ {0} (1-based), 0 if outside
int64_t slot3(int M, const int* k)
{
    int64_t lin = 0, zero = 0;
    bool nz = false;
    for (int b = 0; b < 3; ++b) {
        const int lo = (b == 2) ? 0 : -M;
        const int span = (b == 2) ? M + 1 : 2 * M + 1;
        if (k[b] < lo || k[b] > M) return 0;
        lin = lin * span + (k[b] - lo);
        zero = zero * span + (-lo);
        nz |= (k[b] != 0);
    }
    if (!nz) return 0;
    return lin < zero ? lin + 1 : lin;
}

// q = psi(w): (Phi_11, Phi_22, Phi_12, Phi_33, Phi_23, Phi_13) of L L^T,
// L = [w0 0 0; w2 w1 0; w5 w4 w3]
void psi(const double* w, double q[6])
{
    q[0] = w[0] * w[0];
    q[1] = w[2] * w[2] + w[1] * w[1];
    q[2] = w[0] * w[2];
    q[3] = w[5] * w[5] + w[4] * w[4] + w[3] * w[3];
    q[4] = w[2] * w[5] + w[1] * w[4];
    q[5] = w[0] * w[5];
}

// J[e][m] = d q_e / d w_m
void psi_jac(const double* w, double J[6][6])
{
    memset(J, 0, sizeof(double) * 36);
    J[0][0] = 2.0 * w[0];
    J[1][1] = 2.0 * w[1];
    J[1][2] = 2.0 * w[2];
    J[2][0] = w[2];
    J[2][2] = w[0];
    J[3][3] = 2.0 * w[3];
    J[3][4] = 2.0 * w[4];
    J[3][5] = 2.0 * w[5];
    J[4][1] = w[4];
    J[4][2] = w[5];
    J[4][4] = w[1];
    J[4][5] = w[2];
    J[5][0] = w[5];
    J[5][5] = w[0];
}

// sum_e c_e d^2 q_e / dw dw (psi is quadratic: constant second derivatives)
void psi_curv(const double c[6], double H[6][6])
{
    memset(H, 0, sizeof(double) * 36);
    H[0][0] = 2.0 * c[0];
    H[1][1] = 2.0 * c[1];
    H[2][2] = 2.0 * c[1];
    H[0][2] = H[2][0] = c[2];
    H[3][3] = H[4][4] = H[5][5] = 2.0 * c[3];
    H[1][4] = H[4][1] = c[4];
    H[2][5] = H[5][2] = c[4];
    H[0][5] = H[5][0] = c[5];
}

// loss of App. B for one group (feature sums a, b), its gradient and
// Hessian in q
double grp_loss(const double* q, const double* a, const double* b)
{
    const double q1 = q[0], q2 = q[1], q3 = q[2], q4 = q[3], q5 = q[4], q6 = q[5];
    return a[0] * (q1 * q1 + q3 * q3 + q6 * q6) + a[1] * (q2 * q2 + q3 * q3 + q5 * q5) +
           a[2] * (q1 * q3 + q2 * q3 + q5 * q6) + a[3] * (q4 * q4 + q5 * q5 + q6 * q6) +
           a[4] * (q2 * q5 + q3 * q6 + q4 * q5) + a[5] * (q1 * q6 + q3 * q5 + q4 * q6) -
           (b[0] * q1 + b[1] * q2 + b[2] * q3 + b[3] * q4 + b[4] * q5 + b[5] * q6);
}

void grp_grad(const double* q, const double* a, const double* b, double g[6])
{
    const double q1 = q[0], q2 = q[1], q3 = q[2], q4 = q[3], q5 = q[4], q6 = q[5];
    g[0] = 2 * a[0] * q1 + a[2] * q3 + a[5] * q6 - b[0];
    g[1] = 2 * a[1] * q2 + a[2] * q3 + a[4] * q5 - b[1];
    g[2] = 2 * (a[0] + a[1]) * q3 + a[2] * (q1 + q2) + a[4] * q6 + a[5] * q5 - b[2];
    g[3] = 2 * a[3] * q4 + a[4] * q5 + a[5] * q6 - b[3];
    g[4] = 2 * (a[1] + a[3]) * q5 + a[2] * q6 + a[4] * (q2 + q4) + a[5] * q3 - b[4];
    g[5] = 2 * (a[0] + a[3]) * q6 + a[2] * q5 + a[4] * q3 + a[5] * (q1 + q4) - b[5];
}

void grp_hess(const double* a, double H[6][6])
{
    memset(H, 0, sizeof(double) * 36);
    H[0][0] = 2 * a[0];
    H[1][1] = 2 * a[1];
    H[2][2] = 2 * (a[0] + a[1]);
    H[3][3] = 2 * a[3];
    H[4][4] = 2 * (a[1] + a[3]);
    H[5][5] = 2 * (a[0] + a[3]);
    H[0][2] = H[2][0] = a[2];
    H[1][2] = H[2][1] = a[2];
    H[0][5] = H[5][0] = a[5];
    H[1][4] = H[4][1] = a[4];
    H[2][4] = H[4][2] = a[5];
    H[2][5] = H[5][2] = a[4];
    H[3][4] = H[4][3] = a[4];
    H[3][5] = H[5][3] = a[5];
    H[4][5] = H[5][4] = a[2];
}

// x = A^-1 y for a 6 x 6 matrix (Gaussian elimination with partial
// pivoting); false if A is singular to working precision
bool solve6(const double A_in[6][6], const double* y, double* x)
{
    double A[6][7];
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < 6; ++j) A[i][j] = A_in[i][j];
        A[i][6] = y[i];
    }
    for (int c = 0; c < 6; ++c) {
        int p = c;
        for (int i = c + 1; i < 6; ++i)
            if (std::fabs(A[i][c]) > std::fabs(A[p][c])) p = i;
        if (!(std::fabs(A[p][c]) > 1e-300)) return false;
        if (p != c)
            for (int j = 0; j < 7; ++j) std::swap(A[p][j], A[c][j]);
        for (int i = c + 1; i < 6; ++i) {
            const double f = A[i][c] / A[c][c];
            for (int j = c; j < 7; ++j) A[i][j] -= f * A[c][j];
        }
    }
    for (int i = 5; i >= 0; --i) {
        double v = A[i][6];
        for (int j = i + 1; j < 6; ++j) v -= A[i][j] * x[j];
        x[i] = v / A[i][i];
    }
    return std::isfinite(x[0] + x[1] + x[2] + x[3] + x[4] + x[5]);
}

struct Groups {
    std::vector<double> a, b;   // 6 per group; group 0: modes outside K (bypass only)
    std::vector<int64_t> key;   // slot -> group (0: none)
    int ng = 0;
};

double total_loss(const Groups& G, const std::vector<double>& w)
{
    double q0[6];
    psi(w.data(), q0);
    double L = grp_loss(q0, &G.a[0], &G.b[0]);
    for (int g = 1; g < G.ng; ++g) {
        double q[6], t[6];
        psi(&w[6 * g], t);
        for (int e = 0; e < 6; ++e) q[e] = q0[e] + t[e];
        L += grp_loss(q, &G.a[6 * g], &G.b[6 * g]);
    }
    return L;
}

}  // namespace
}  // namespace unocg

using namespace unocg;

extern "C" {

uno_status el_uno_train_accumulate(const uno_grid* grid, int32_t ns, const double* f, const double* u,
                                   double ns_total, double* alpha, double* beta, void* stream)
{
    Grid g;
    uno_status e = make_grid(grid, &g);
    if (e != UNO_OK) return e;
    if (grid->dim != 3 || ns < 0 || !(ns_total > 0.0) || !alpha || !beta || (ns > 0 && (!f || !u)))
        return UNO_ERR_ARG;
    FftPlan plan;
    e = fft_plan_create(g, &plan);
    if (e != UNO_OK) { fft_plan_destroy(&plan); return e; }
    double2* buf = nullptr;  // F0..F2, U0..U2
    if (hipMalloc(&buf, sizeof(double2) * 6 * plan.nspec) != hipSuccess) {
        fft_plan_destroy(&plan);
        return UNO_ERR_NOMEM;
    }
    hipStream_t st = (hipStream_t)stream;
    const double scale = 1.0 / (ns_total * (double)g.total);  // unitary transforms
    const int nb = (int)((plan.nspec + kBlock - 1) / kBlock);
    const int64_t n = g.total;
    for (int j = 0; j < ns && e == UNO_OK; ++j) {
        for (int c = 0; c < 3 && e == UNO_OK; ++c) {
            e = fft_forward_real(g, plan, f + (int64_t)j * 3 * n + c * n, buf + c * plan.nspec, st);
            if (e == UNO_OK) e = fft_forward_real(g, plan, u + (int64_t)j * 3 * n + c * n, buf + (3 + c) * plan.nspec, st);
        }
        if (e == UNO_OK) {
            hipLaunchKernelGGL(k_feat3_accum, dim3(nb), dim3(kBlock), 0, st, plan.nspec, (const double2*)buf,
                               (const double2*)(buf + 3 * plan.nspec), scale, alpha, beta);
            e = hip_status(hipGetLastError());
        }
    }
    if (hipStreamSynchronize(st) != hipSuccess && e == UNO_OK) e = UNO_ERR_DEVICE;
    (void)hipFree(buf);
    fft_plan_destroy(&plan);
    return e;
}

uno_status el_uno_train_fit(const uno_grid* grid, int32_t M, const double* alpha, const double* beta,
                            int32_t max_epochs, double* theta, int64_t ntheta, double* loss, void* stream)
{
    Grid g;
    uno_status e = make_grid(grid, &g);
    if (e != UNO_OK) return e;
    if (grid->dim != 3 || !alpha || !beta || !theta || M < 0 || max_epochs < 0) return UNO_ERR_ARG;
    for (int b = 0; b < 3; ++b)
        if (2 * M + 1 > g.n[b]) return UNO_ERR_SHAPE;
    const int64_t nslot = (int64_t)(2 * M + 1) * (2 * M + 1) * (M + 1);  // 1 + |K|
    if (ntheta != 6 * nslot) return UNO_ERR_SHAPE;
    const int nh = g.n[2] / 2 + 1;
    const int64_t nspec = (int64_t)g.n[0] * g.n[1] * nh;
    std::vector<double> A(6 * nspec), B(6 * nspec);
    hipStream_t st = (hipStream_t)stream;
    UNO_HIP(hipMemcpyAsync(A.data(), alpha, sizeof(double) * 6 * nspec, hipMemcpyDeviceToHost, st));
    UNO_HIP(hipMemcpyAsync(B.data(), beta, sizeof(double) * 6 * nspec, hipMemcpyDeviceToHost, st));
    UNO_HIP(hipStreamSynchronize(st));

    // feature sums per group (a pair k, -k on k_z = 0 is one group)
    Groups G;
    G.key.assign(nslot, 0);
    G.ng = 1;
    G.a.assign(6, 0.0);
    G.b.assign(6, 0.0);
    const bool even = (g.n[2] % 2) == 0;
    for (int ix = 0; ix < g.n[0]; ++ix)
        for (int iy = 0; iy < g.n[1]; ++iy)
            for (int kz = 0; kz < nh; ++kz) {
                const int64_t l = ((int64_t)ix * g.n[1] + iy) * nh + kz;
                if (l == 0) continue;  // zero mode: table fixed to 0
                const double mult = (kz == 0 || (even && kz == g.n[2] / 2)) ? 1.0 : 2.0;
                const int k[3] = {centred3(ix, g.n[0]), centred3(iy, g.n[1]), kz};
                const int64_t s = slot3(M, k);
                int64_t grp = 0;
                if (s) {
                    if (!G.key[s]) {
                        G.key[s] = G.ng++;
                        G.a.resize(6 * G.ng, 0.0);
                        G.b.resize(6 * G.ng, 0.0);
                        if (kz == 0) {
                            const int mk[3] = {-k[0], -k[1], 0};
                            G.key[slot3(M, mk)] = G.key[s];
                        }
                    }
                    grp = G.key[s];
                }
                for (int c = 0; c < 6; ++c) {
                    G.a[6 * grp + c] += mult * A[c * nspec + l];
                    G.b[6 * grp + c] += mult * B[c * nspec + l];
                }
            }

    // start: psi = a I on every group, a the best multiple of the identity
    std::vector<double> w(6 * (size_t)G.ng, 0.0);
    {
        double sa = 0.0, sb = 0.0;
        for (int gg = 0; gg < G.ng; ++gg) {
            sa += G.a[6 * gg] + G.a[6 * gg + 1] + G.a[6 * gg + 3];
            sb += G.b[6 * gg] + G.b[6 * gg + 1] + G.b[6 * gg + 3];
        }
        const double aiso = (sa > 0.0 && sb > 0.0) ? sb / (2.0 * sa) : 1.0;
        const double w0 = std::sqrt(aiso / 2.0);
        for (int gg = 0; gg < G.ng; ++gg) w[6 * gg] = w[6 * gg + 1] = w[6 * gg + 3] = w0;
    }
    double L = total_loss(G, w);
    double lam = -1.0, g0max = -1.0;
    std::vector<double> hist{L};
    std::vector<double> grad(6 * (size_t)G.ng), dw(6 * (size_t)G.ng), wn(6 * (size_t)G.ng);
    std::vector<double> Hgg(36 * (size_t)G.ng), H0g(36 * (size_t)G.ng);
    for (int ep = 0; ep < max_epochs; ++ep) {
        // gradient and Hessian blocks
        double q0[6], J0[6][6], H00[6][6];
        psi(w.data(), q0);
        psi_jac(w.data(), J0);
        memset(H00, 0, sizeof(H00));
        std::fill(grad.begin(), grad.end(), 0.0);
        for (int gg = 0; gg < G.ng; ++gg) {
            double q[6], Jg[6][6], gq[6], Hq[6][6];
            memcpy(q, q0, sizeof(q));
            if (gg > 0) {
                double t[6];
                psi(&w[6 * gg], t);
                for (int c = 0; c < 6; ++c) q[c] += t[c];
                psi_jac(&w[6 * gg], Jg);
            }
            grp_grad(q, &G.a[6 * gg], &G.b[6 * gg], gq);
            grp_hess(&G.a[6 * gg], Hq);
            // J0^T Hq J0 + curvature into H00; J0^T gq into grad0
            double HJ0[6][6], HJg[6][6], C[6][6];
            for (int i = 0; i < 6; ++i)
                for (int m = 0; m < 6; ++m) {
                    double v0 = 0.0, vg = 0.0;
                    for (int j = 0; j < 6; ++j) {
                        v0 += Hq[i][j] * J0[j][m];
                        if (gg > 0) vg += Hq[i][j] * Jg[j][m];
                    }
                    HJ0[i][m] = v0;
                    HJg[i][m] = vg;
                }
            psi_curv(gq, C);
            for (int m = 0; m < 6; ++m) {
                double gv = 0.0;
                for (int i = 0; i < 6; ++i) gv += J0[i][m] * gq[i];
                grad[m] += gv;
                for (int p = 0; p < 6; ++p) {
                    double v = C[m][p];
                    for (int i = 0; i < 6; ++i) v += J0[i][m] * HJ0[i][p];
                    H00[m][p] += v;
                }
            }
            if (gg == 0) continue;
            double* hg = &Hgg[36 * (size_t)gg];
            double* h0 = &H0g[36 * (size_t)gg];
            for (int m = 0; m < 6; ++m) {
                double gv = 0.0;
                for (int i = 0; i < 6; ++i) gv += Jg[i][m] * gq[i];
                grad[6 * gg + m] = gv;
                for (int p = 0; p < 6; ++p) {
                    double vg = C[m][p], v0 = 0.0;
                    for (int i = 0; i < 6; ++i) {
                        vg += Jg[i][m] * HJg[i][p];
                        v0 += J0[i][m] * HJg[i][p];
                    }
                    hg[m * 6 + p] = vg;
                    h0[m * 6 + p] = v0;  // d2L / dw0_m dwg_p
                }
            }
        }
        double gmax = 0.0, dmax = 0.0;
        for (double v : grad) gmax = std::fmax(gmax, std::fabs(v));
        for (int m = 0; m < 6; ++m) dmax = std::fmax(dmax, std::fabs(H00[m][m]));
        if (g0max < 0.0) g0max = gmax;
        if (!(gmax > 1e-10 * g0max)) break;
        const size_t nh_ = hist.size();
        if (nh_ >= 3 && hist[nh_ - 3] - hist[nh_ - 1] <= 1e-14 * std::fabs(hist[nh_ - 1])) break;
        if (lam < 0.0) lam = 1e-6 * (dmax > 0.0 ? dmax : 1.0);
        bool accepted = false;
        while (!accepted) {
            // (H + lam I) dw = -grad through the Schur complement on w0
            double S[6][6], rhs0[6];
            bool ok = true;
            for (int m = 0; m < 6; ++m) {
                rhs0[m] = -grad[m];
                for (int p = 0; p < 6; ++p) S[m][p] = H00[m][p] + (m == p ? lam : 0.0);
            }
            std::vector<double> Zg(36 * (size_t)G.ng), zg(6 * (size_t)G.ng);  // (Hgg+lam)^-1 Hg0, (Hgg+lam)^-1 (-g_g)
            for (int gg = 1; gg < G.ng && ok; ++gg) {
                double Hs[6][6];
                const double* hg = &Hgg[36 * (size_t)gg];
                const double* h0 = &H0g[36 * (size_t)gg];
                for (int m = 0; m < 6; ++m)
                    for (int p = 0; p < 6; ++p) Hs[m][p] = hg[m * 6 + p] + (m == p ? lam : 0.0);
                double y[6], x[6];
                for (int m = 0; m < 6; ++m) y[m] = -grad[6 * gg + m];
                ok = solve6(Hs, y, x);
                for (int m = 0; m < 6; ++m) zg[6 * gg + m] = x[m];
                for (int c = 0; c < 6 && ok; ++c) {  // column c of Hg0 = row c of H0g^T
                    for (int m = 0; m < 6; ++m) y[m] = h0[c * 6 + m];
                    ok = solve6(Hs, y, x);
                    for (int m = 0; m < 6; ++m) Zg[36 * (size_t)gg + m * 6 + c] = x[m];
                }
                if (!ok) break;
                // S -= H0g Z, rhs0 -= H0g z
                for (int m = 0; m < 6; ++m) {
                    for (int p = 0; p < 6; ++p) {
                        double v = 0.0;
                        for (int i = 0; i < 6; ++i) v += h0[m * 6 + i] * Zg[36 * (size_t)gg + i * 6 + p];
                        S[m][p] -= v;
                    }
                    double v = 0.0;
                    for (int i = 0; i < 6; ++i) v += h0[m * 6 + i] * zg[6 * gg + i];
                    rhs0[m] -= v;
                }
            }
            double d0[6] = {0, 0, 0, 0, 0, 0};
            if (ok) ok = solve6(S, rhs0, d0);
            if (ok) {
                for (int m = 0; m < 6; ++m) dw[m] = d0[m];
                for (int gg = 1; gg < G.ng; ++gg)
                    for (int m = 0; m < 6; ++m) {
                        double v = zg[6 * gg + m];
                        for (int c = 0; c < 6; ++c) v -= Zg[36 * (size_t)gg + m * 6 + c] * d0[c];
                        dw[6 * gg + m] = v;
                    }
                for (size_t i = 0; i < w.size(); ++i) wn[i] = w[i] + dw[i];
                const double Ln = total_loss(G, wn);
                if (Ln <= L) {
                    w.swap(wn);
                    L = Ln;
                    lam = std::fmax(lam / 3.0, 1e-300);
                    accepted = true;
                    break;
                }
            }
            lam *= 4.0;
            if (lam > 1e300) break;
        }
        if (!accepted) break;
        hist.push_back(L);
    }
    // weights per slot: the group's (both slots of a pair)
    for (int c = 0; c < 6; ++c) theta[c] = w[c];
    for (int64_t s = 1; s < nslot; ++s) {
        const int64_t gg = G.key[s];
        for (int c = 0; c < 6; ++c) theta[6 * s + c] = gg ? w[6 * gg + c] : 0.0;
    }
    if (loss) *loss = L;
    return UNO_OK;
}

}  // extern "C"
