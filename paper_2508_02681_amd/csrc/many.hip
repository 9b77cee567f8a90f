// Many independent problems of uneven sizes in one call (the batched
// solution of Sec. 4.5 applied to the many-query setting of Sec. 1).
//
// Problems are grouped into classes of equal grid (and preconditioner).
// The load cases of a class become the right-hand sides of the batched CG
// (every pass kernel takes them along grid y, each with its own
// conductivity field, scalars and stopping test), in launches of up to 256;
// the classes follow one another on the caller's stream, largest first.
// (Classes on concurrent streams were tried: the learned-mode flow then
// lost the agreement between its recursive and true residuals on some load
// cases, cause not yet found, so the classes run in order.)
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "unocg_internal.h"

namespace unocg {

uno_status pcg_run_batch(const Grid& g, const double* kappa, int64_t ks, int nrhs, const double* macro_loads3,
                         const double* rhs, double* u, const uno_solve_opts* o, uno_solve_info* info, double* res_hist,
                         hipStream_t st);

namespace {

constexpr int kMaxRhs = 256;     // right-hand sides per launch
struct Rhs {
    int prob, load;
};

struct Class {
    Grid g;
    const uno_precond* pc;
    std::vector<Rhs> rhs;
    uno_status status = UNO_OK;
};

// one class: gather fields, batched solves of up to kMaxRhs, scatter
void run_class(Class* c, const uno_problem* probs, uno_solve_opts o, hipStream_t st)
{
    o.uno = c->pc;
    const Grid& g = c->g;
    const int64_t n = g.total;
    const int d = g.dim;
    const int nr = (int)std::min<size_t>(c->rhs.size(), kMaxRhs);
    double *kap = nullptr, *u = nullptr;
    uno_status e = UNO_OK;
    if (hipMalloc(&kap, sizeof(double) * n * nr) != hipSuccess || hipMalloc(&u, sizeof(double) * n * nr) != hipSuccess)
        e = UNO_ERR_NOMEM;
    bool broke = false;
    std::vector<double> g3;
    std::vector<uno_solve_info> info;
    for (size_t b0 = 0; b0 < c->rhs.size() && e == UNO_OK; b0 += kMaxRhs) {
        const int m = (int)std::min<size_t>(kMaxRhs, c->rhs.size() - b0);
        g3.assign(3 * (size_t)m, 0.0);
        info.assign(m, uno_solve_info{});
        for (int j = 0; j < m && e == UNO_OK; ++j) {
            const Rhs& r = c->rhs[b0 + j];
            const uno_problem& P = probs[r.prob];
            for (int a = 0; a < d; ++a) g3[3 * j + 3 - d + a] = P.loads[r.load * d + a];
            if (hipMemcpyAsync(kap + j * n, P.kappa, sizeof(double) * n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(u + j * n, P.u + r.load * n, sizeof(double) * n, hipMemcpyDeviceToDevice, st) !=
                    hipSuccess)
                e = UNO_ERR_DEVICE;
        }
        if (e != UNO_OK) break;
        uno_status s = pcg_run_batch(g, kap, n, m, g3.data(), nullptr, u, &o, info.data(), nullptr, st);
        if (s == UNO_ERR_BREAKDOWN) broke = true;
        else if (s != UNO_OK) { e = s; break; }
        for (int j = 0; j < m && e == UNO_OK; ++j) {
            const Rhs& r = c->rhs[b0 + j];
            const uno_problem& P = probs[r.prob];
            if (hipMemcpyAsync(P.u + r.load * n, u + j * n, sizeof(double) * n, hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
                e = UNO_ERR_DEVICE;
            if (P.info) P.info[r.load] = info[j];
        }
    }
    if (hipStreamSynchronize(st) != hipSuccess && e == UNO_OK) e = UNO_ERR_DEVICE;
    (void)hipFree(kap);
    (void)hipFree(u);
    c->status = (e == UNO_OK && broke) ? UNO_ERR_BREAKDOWN : e;
}

}  // namespace
}  // namespace unocg

using namespace unocg;

extern "C" uno_status pcg_solve_many(int32_t nprob, const uno_problem* probs, const uno_solve_opts* opts,
                                     void* stream)
{
    if (nprob < 0 || (nprob > 0 && !probs) || !opts) return UNO_ERR_ARG;
    if (!(opts->rtol >= 0.0) || opts->max_iter < 1) return UNO_ERR_ARG;
    if (opts->kind < UNO_PREC_NONE || opts->kind > UNO_PREC_UNO) return UNO_ERR_ARG;
    const bool f64 = opts->op_t == UNO_F64 && opts->prec_t == UNO_F64;
    const bool f32 = opts->op_t == UNO_F32 && opts->prec_t == UNO_F32;
    if (!f64 && !f32) return UNO_ERR_ARG;
    // classes of equal grid shape, spacing and preconditioner
    std::map<std::tuple<int, int, int, int, double, double, double, const void*>, int> key;
    std::vector<Class> cls;
    for (int i = 0; i < nprob; ++i) {
        const uno_problem& P = probs[i];
        Grid g;
        uno_status e = make_grid(&P.grid, &g);
        if (e != UNO_OK) return e;
        if (!P.kappa || !P.u || !P.loads || P.nload < 1 || P.nload > 3) return UNO_ERR_ARG;
        for (int k = 0; k < P.nload * P.grid.dim; ++k)
            if (!std::isfinite(P.loads[k])) return UNO_ERR_ARG;
        const uno_precond* pc = nullptr;
        if (opts->kind == UNO_PREC_UNO) {
            pc = P.uno;
            if (!pc || pc->nc != 1) return UNO_ERR_ARG;
            if (pc->grid.n[0] != g.n[0] || pc->grid.n[1] != g.n[1] || pc->grid.n[2] != g.n[2]) return UNO_ERR_SHAPE;
            if (f32 && !uno_use_lowrank(pc)) return UNO_ERR_ARG;  // FP32 UNO runs the learned-mode passes
        }
        const auto k = std::make_tuple(g.dim, g.n[0], g.n[1], g.n[2], g.h[0], g.h[1], g.h[2], (const void*)pc);
        auto it = key.find(k);
        int c;
        if (it == key.end()) {
            c = (int)cls.size();
            key[k] = c;
            cls.push_back(Class{g, pc, {}, UNO_OK});
        } else {
            c = it->second;
        }
        for (int l = 0; l < P.nload; ++l) cls[c].rhs.push_back(Rhs{i, l});
    }
    if (cls.empty()) return UNO_OK;
    hipStream_t st = (hipStream_t)stream;
    uno_status worst = UNO_OK;
    std::vector<int> order(cls.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return cls[a].g.total * cls[a].rhs.size() > cls[b].g.total * cls[b].rhs.size(); });
    for (int q : order) {
        run_class(&cls[q], probs, *opts, st);
        if (cls[q].status == UNO_ERR_BREAKDOWN) worst = UNO_ERR_BREAKDOWN;
        else if (cls[q].status != UNO_OK) return cls[q].status;
    }
    return worst;
}
