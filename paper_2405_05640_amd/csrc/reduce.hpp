// reduce.hpp -- one-workgroup finalize reductions of the Krylov loops.
#pragma once

#include <hip/hip_runtime.h>

#include "cg.hpp"

namespace sem {

// A scalar finalize (alpha, beta, the convergence test) needs the sum of the
// per-workgroup partials of the kernel before it.  One workgroup of kWide
// threads sums them and runs the finalize in the same launch when there are
// at most kDirectMax of them; with more, a kStage-workgroup stage kernel runs
// first (one workgroup reading ~25,000 partials per quantity was measured
// slower than the two launches on the 32^3 mesh; with ~6,000, as on the 16^3
// channel, the single launch wins by about 4 % of the CG iteration).
//
// Doing the sum inside the producing kernel (the workgroup that finishes
// last finalizes) was measured and rejected: each XCD has its own L2, so
// publishing a partial at agent scope writes back that L2 and reading them
// invalidates it.  With a fence in each of ~10^4 workgroups per launch the
// FP64 CG iteration on the 32^3 mesh took 1.5 ms (release and acquire
// fences split) to 3.9 ms (full fences), against 0.41 ms.
constexpr int kWide = 1024;
constexpr int64_t kDirectMax = 1 << 14;

// Fixed-order sums of a[0..n) and b[0..n) (b may be null) by one workgroup
// of kWide threads, every thread gets both: strided per-thread sums with up
// to sixteen loads in flight, a butterfly of cross-lane shuffles per
// wavefront, the wavefronts in order.  A finalize kernel calls this before
// it reads its state, so the loads of the partials and of the state overlap
// (the partial buffers are always readable).
__device__ inline void wide_sum2(const double *__restrict__ a, const double *__restrict__ b, int64_t n, double &sa,
                                 double &sb)
{
    __shared__ double red[2][kWide / 64];
    constexpr int U = 8;
    double s0 = 0.0, s1 = 0.0;
    int64_t q = threadIdx.x;
    for (; q + (U - 1) * kWide < n; q += U * kWide) {
        double t[U], u[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            t[k] = a[q + k * kWide];
            u[k] = b ? b[q + k * kWide] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            s0 += t[k];
            s1 += u[k];
        }
    }
    for (; q < n; q += kWide) {
        s0 += a[q];
        if (b) s1 += b[q];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_xor(s0, o);
        s1 += __shfl_xor(s1, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s0;
        red[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    sa = sb = 0.0;
#pragma unroll
    for (int w = 0; w < kWide / 64; ++w) {
        sa += red[0][w];
        sb += red[1][w];
    }
    __syncthreads();
}

__device__ inline double wide_sum(const double *__restrict__ a, int64_t n)
{
    double sa, sb;
    wide_sum2(a, nullptr, n, sa, sb);
    return sa;
}

}  // namespace sem
