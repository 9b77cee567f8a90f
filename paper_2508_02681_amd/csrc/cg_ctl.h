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
    CgState* st;
    const double* part_rmax;  // ||r_k||_inf partials (init kernel or update of pass k-1)
    int np_rmax;
    double rtol;
    double* hist;             // ||r_k||_inf history (hist_len entries)
    int hist_len;
    const double* r;          // FP64 residual (for r.s in the preconditioner's last pass)
    double* part_rs;          // r.s partials of pass k
};

__device__ __forceinline__ bool loop_ended(const CgState* st, int k)
{
    return st->status != 0 || st->done <= k;
}

// Convergence test at the head of pass k; true when the workgroup must exit.
__device__ inline bool head_check(const CgIter& c, double* slots)
{
    if (loop_ended(c.st, c.k)) return true;
    const double rm = reduce_parts<OpMax>(c.part_rmax, c.np_rmax, slots);
    const double tol = (c.k == 0) ? c.rtol * rm : c.st->tol_abs;
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

}  // namespace unocg
