// Deterministic FP64 reductions for wave64 workgroups.
//
// A workgroup reduces its values with cross-lane shuffles and one LDS slot
// per wavefront, writes one partial per workgroup, and the last workgroup to
// arrive (device-scope counter) combines all partials in a fixed order.  The
// result therefore does not depend on scheduling, and the counter is left at
// zero for the next kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace unocg {

struct OpSum {
    __device__ static double apply(double a, double b) { return a + b; }
    __device__ static double ident() { return 0.0; }
};
struct OpMax {
    // used on absolute values; a NaN operand wins so that breakdowns surface
    __device__ static double apply(double a, double b) { return (a != a || a > b) ? a : b; }
    __device__ static double ident() { return 0.0; }
};

template <class Op>
__device__ inline double wave_reduce(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = Op::apply(v, __shfl_down(v, off, 64));
    return v;
}

// Result valid in thread 0.  `slots` holds blockDim.x / 64 doubles.
template <class Op>
__device__ inline double block_reduce(double v, double* slots)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_reduce<Op>(v);
    __syncthreads();
    if (lane == 0) slots[wid] = v;
    __syncthreads();
    double r = Op::ident();
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) r = Op::apply(r, slots[i]);
    return r;
}

// Publishes thread 0's block value(s) and tells whether this workgroup is the
// last to arrive.  Call from all threads; returns the same flag in all.
__device__ inline bool arrive_last(unsigned* counter, int* flag_lds)
{
    if (threadIdx.x == 0) {
        __threadfence();
        unsigned t = atomicAdd(counter, 1u);
        *flag_lds = (t == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    bool last = *flag_lds != 0;
    if (last) __threadfence();
    return last;
}

// Fixed-order combination of nparts partials by the whole (last) workgroup.
// Result valid in thread 0.
template <class Op>
__device__ inline double combine_partials(const double* parts, int nparts, double* slots)
{
    double v = Op::ident();
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        v = Op::apply(v, parts[i]);
    }
    return block_reduce<Op>(v, slots);
}

}  // namespace unocg
