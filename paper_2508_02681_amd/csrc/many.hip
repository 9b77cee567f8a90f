// Many independent problems of uneven sizes in one call (the batched
// solution of Sec. 4.5 applied to the many-query setting of Sec. 1).
//
// Problems are grouped into classes of equal grid (and preconditioner).
// The load cases of a class become the right-hand sides of the batched CG
// (every pass kernel takes them along grid y, each with its own
// conductivity field, scalars and stopping test), in launches of up to 256.
// Small grids leave most of the chip idle in a single launch, so the
// classes run concurrently: one host thread per class drives its batched
// loop on a stream of its own (a CG workspace belongs to one stream), all
// forked from and joined back into the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "unocg_internal.h"

namespace unocg {

uno_status pcg_run_batch(const Grid& g, const double* kappa, int64_t ks, int nrhs, const double* macro_loads3,
                         const double* rhs, double* u, const uno_solve_opts* o, uno_solve_info* info, double* res_hist,
                         hipStream_t st);

namespace {

constexpr int kMaxRhs = 256;     // right-hand sides per launch
constexpr int kMaxStreams = 8;   // classes in flight at once

struct Rhs {
    int prob, load;
};

struct Class {
    Grid g;
    const uno_precond* pc;
    std::vector<Rhs> rhs;
    double* kap = nullptr;  // gathered conductivities and solutions of one launch
    double* u = nullptr;
    uno_status status = UNO_OK;
};

// streams of the pool of a device (created on first use, default priority,
// not synchronizing with the null stream; ordered by events instead)
std::mutex g_smu;
std::vector<std::pair<int, std::vector<hipStream_t>>> g_streams;

uno_status pool_streams(int dev, int count, std::vector<hipStream_t>* out)
{
    std::lock_guard<std::mutex> lk(g_smu);
    std::vector<hipStream_t>* p = nullptr;
    for (auto& q : g_streams)
        if (q.first == dev) p = &q.second;
    if (!p) {
        g_streams.emplace_back(dev, std::vector<hipStream_t>());
        p = &g_streams.back().second;
    }
    while ((int)p->size() < count) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return UNO_ERR_DEVICE;
        p->push_back(st);
    }
    out->assign(p->begin(), p->begin() + count);
    return UNO_OK;
}

// one class on stream st: gather fields, batched solves of up to kMaxRhs, scatter
void run_class(Class* c, const uno_problem* probs, uno_solve_opts o, hipStream_t st)
{
    o.uno = c->pc;
    const Grid& g = c->g;
    const int64_t n = g.total;
    const int d = g.dim;
    double *kap = c->kap, *u = c->u;
    uno_status e = UNO_OK;
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
    const bool f32 = opts->op_t == UNO_F32 && (opts->prec_t == UNO_F32 ||
                                               (opts->prec_t == UNO_BF16 && opts->kind == UNO_PREC_UNO));
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
            cls.push_back(Class{g, pc, {}, nullptr, nullptr, UNO_OK});
        } else {
            c = it->second;
        }
        for (int l = 0; l < P.nload; ++l) cls[c].rhs.push_back(Rhs{i, l});
    }
    if (cls.empty()) return UNO_OK;
    hipStream_t caller = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return UNO_ERR_DEVICE;
    std::vector<int> order(cls.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return cls[a].g.total * cls[a].rhs.size() > cls[b].g.total * cls[b].rhs.size(); });
    // gather buffers of every class, allocated here so that no class thread
    // allocates or frees while the others run
    uno_status worst = UNO_OK;
    for (Class& c : cls) {
        const size_t nr = std::min<size_t>(c.rhs.size(), kMaxRhs);
        const size_t bytes = sizeof(double) * (size_t)c.g.total * nr;
        if (hipMalloc(&c.kap, bytes) != hipSuccess || hipMalloc(&c.u, bytes) != hipSuccess) {
            worst = UNO_ERR_NOMEM;
            break;
        }
    }
    const int nst = (int)std::min<size_t>(cls.size(), kMaxStreams);
    std::vector<hipStream_t> streams;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins(nst, nullptr);
    if (worst == UNO_OK) worst = pool_streams(dev, nst, &streams);
    if (worst == UNO_OK && hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) worst = UNO_ERR_DEVICE;
    for (int i = 0; i < nst && worst == UNO_OK; ++i)
        if (hipEventCreateWithFlags(&joins[i], hipEventDisableTiming) != hipSuccess) worst = UNO_ERR_DEVICE;
    if (worst == UNO_OK && hipEventRecord(fork, caller) != hipSuccess) worst = UNO_ERR_DEVICE;
    for (int i = 0; i < nst && worst == UNO_OK; ++i)
        if (hipStreamWaitEvent(streams[i], fork, 0) != hipSuccess) worst = UNO_ERR_DEVICE;
    if (worst == UNO_OK) {
        // nst threads, thread i taking classes i, i + nst, ... of the order on stream i
        std::vector<std::thread> th;
        for (int i = 0; i < nst; ++i)
            th.emplace_back([&, i]() {
                if (hipSetDevice(dev) != hipSuccess) {
                    for (size_t q = i; q < order.size(); q += nst) cls[order[q]].status = UNO_ERR_DEVICE;
                    return;
                }
                for (size_t q = i; q < order.size(); q += nst) run_class(&cls[order[q]], probs, *opts, streams[i]);
            });
        for (auto& t : th) t.join();
        for (int i = 0; i < nst; ++i)
            if (hipEventRecord(joins[i], streams[i]) != hipSuccess || hipStreamWaitEvent(caller, joins[i], 0) != hipSuccess)
                worst = UNO_ERR_DEVICE;
        for (const Class& c : cls) {
            if (c.status == UNO_ERR_BREAKDOWN && worst == UNO_OK) worst = UNO_ERR_BREAKDOWN;
            else if (c.status != UNO_OK && c.status != UNO_ERR_BREAKDOWN) worst = c.status;
        }
    }
    // every class thread has synchronized its stream; the buffers are idle
    for (int i = 0; i < nst; ++i)
        if (joins[i]) (void)hipEventDestroy(joins[i]);
    if (fork) (void)hipEventDestroy(fork);
    for (Class& c : cls) {
        (void)hipFree(c.kap);
        (void)hipFree(c.u);
    }
    return worst;
}
