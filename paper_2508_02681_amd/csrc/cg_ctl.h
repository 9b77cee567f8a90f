// Control of the device-resident CG loop shared by the CG and FFT kernels.
//
// The host enqueues pass k = 0, 1, 2, ... without waiting; the scalars of a
// pass are combined from per-workgroup partials by the kernels that need
// them.  The first kernel of pass k reduces ||r_k||_inf and ends the loop
// when it is <= rtol ||r_0||_inf (Algorithm 1, while condition); every other
// kernel returns at once once the loop has ended.
#pragma once

#include <climits>

#include "unocg_internal.h"
#include "reduce.h"

namespace unocg {

struct CgIter {
    int k;                    // pass index
    int k0;                   // first pass of the current cycle (0, or a residual replacement)
    CgState* st;
    const double* part_rmax;  // ||r_k||_inf partials (init kernel or update of pass k-1)
    int np_rmax;
    double rtol;
    double* hist;             // ||r_k||_inf history (hist_len entries)
    int hist_len;
    const double* r;          // FP64 residual (for r.s in the preconditioner's last pass)
    double* part_rs;          // r.s partials of pass k
    double* part_ssum;        // sum(s) partials of pass k (FP32 mode: mean removal)
    // several right-hand sides solved together (blockIdx.y = rhs index):
    // strides between their vectors, partial buffers and scalar histories
    int64_t vs;
    int ps;
    int hs;
    int64_t ks;   // stride between the conductivity (and Jacobi) fields: 0 when shared
    // graph-captured passes: k is the offset of the pass within the captured
    // chunk and *kdev (device) the index of the chunk's first pass, set
    // before the chunk runs (null: k is the pass index itself)
    const int* kdev;
};

// The pass index of a kernel's CG pass (first statement of every pass kernel).
__device__ __forceinline__ void resolve_pass(CgIter& it)
{
    if (it.kdev) it.k += *it.kdev;
}

// The control of right-hand side blockIdx.y (state, partials, history).
__device__ __forceinline__ CgIter rhs_iter(CgIter c)
{
    const int b = blockIdx.y;
    if (b == 0) return c;
    if (c.st) c.st += b;
    const int64_t po = (int64_t)b * c.ps;
    if (c.part_rmax) c.part_rmax += po;
    if (c.part_rs) c.part_rs += po;
    if (c.part_ssum) c.part_ssum += po;
    if (c.hist) c.hist += (int64_t)b * c.hs;
    if (c.r) c.r += (int64_t)b * c.vs;
    return c;
}

__device__ __forceinline__ bool loop_ended(const CgState* st, int k)
{
    return st->status != 0 || st->done <= k;
}

// This thread's share of a partial array, combined with Op (loads only).
template <class Op>
__device__ __forceinline__ double load_share(const double* __restrict__ parts, int np)
{
    double v = Op::ident();
    for (int i = threadIdx.x; i < np; i += blockDim.x) v = Op::apply(v, parts[i]);
    return v;
}

// Block-wide combination of the per-thread shares; every thread gets it.
template <class Op>
__device__ __forceinline__ double combine_share(double v, double* slots)
{
    v = block_reduce<Op>(v, slots);
    __syncthreads();
    if (threadIdx.x == 0) slots[0] = v;
    __syncthreads();
    v = slots[0];
    __syncthreads();
    return v;
}

// Values a kernel of pass k reads from the loop state, loaded at entry
// together with everything else so that all global loads overlap.
struct StateLoad {
    int done, status;
    double tol_abs;
};

__device__ __forceinline__ StateLoad load_state(const CgState* st)
{
    StateLoad s;
    s.done = st->done;
    s.status = st->status;
    s.tol_abs = st->tol_abs;
    return s;
}

__device__ __forceinline__ bool ended(const StateLoad& s, int k) { return s.status != 0 || s.done <= k; }

// Convergence test at the head of pass k from preloaded values (`share` is
// this thread's share of the ||r_k||_inf partials); true when the workgroup
// must exit.
__device__ inline bool head_decide(const CgIter& c, const StateLoad& sl, double share, double* slots)
{
    if (ended(sl, c.k)) return true;
    const double rm = combine_share<OpMax>(share, slots);
    const double tol = (c.k == 0) ? c.rtol * rm : sl.tol_abs;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (lead) {
        if (c.k == 0) {
            c.st->r0max = rm;
            c.st->tol_abs = tol;
        }
        c.st->rmax_last = rm;
        c.st->k_last = c.k;
        if (c.hist && c.k < c.hist_len) c.hist[c.k] = rm;
    }
    if (!(rm == rm)) {
        if (lead) { c.st->status = 1; c.st->fail_iter = c.k; }
        return true;
    }
    if (rm <= tol) {
        if (lead) c.st->done = c.k;
        return true;
    }
    return false;
}

// Convergence test at the head of pass k; true when the workgroup must exit.
__device__ inline bool head_check(const CgIter& c, double* slots)
{
    const StateLoad sl = load_state(c.st);
    const double share = load_share<OpMax>(c.part_rmax, c.np_rmax);
    return head_decide(c, sl, share, slots);
}

}  // namespace unocg
