// Deterministic FP64 reductions for wave64 workgroups.
//
// A workgroup reduces its values with cross-lane shuffles and one LDS slot
// per wavefront and writes one partial per workgroup.  The kernel that needs
// the scalar combines the partials itself, in every workgroup, in a fixed
// order: the result does not depend on scheduling and no device-scope fence
// (which would write back the whole L2 on this chip) is needed.
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

// Fixed-order combination of nparts partials (written by an earlier kernel)
// by a whole workgroup; every thread receives the result.  Kernel boundaries
// make the partials visible, so no fences are needed.
template <class Op>
__device__ inline double reduce_parts(const double* parts, int nparts, double* slots)
{
    double v = Op::ident();
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) v = Op::apply(v, parts[i]);
    v = block_reduce<Op>(v, slots);
    __syncthreads();
    if (threadIdx.x == 0) slots[0] = v;
    __syncthreads();
    v = slots[0];
    __syncthreads();
    return v;
}

}  // namespace unocg
