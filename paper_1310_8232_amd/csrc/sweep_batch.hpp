// Batched z-march sweep over several grids (shots); shares the one-step
// sweep's body (sweep.hpp).
#pragma once

#include "sweep.hpp"

namespace p1310 {

// Several grids (shots) in one launch: the launch grid concatenates every
// shot's workgroups; wg_begin[s] is the first workgroup of shot s (increasing,
// wg_begin[0] = 0). Each shot keeps its own sizes, march depth, fields and
// source; `it` is the step. A workgroup finds its shot by binary search over
// wg_begin (log2 of the shot count in uniform loads).
template <int R, int BX, int BY, int RY, int VW, int PF, typename ST>
__global__ void __launch_bounds__(BX * BY) zmarch_batch_kernel(const SweepArgs *shots, const int *wg_begin,
                                                               int nshots, int xcd, int64_t it)
{
    int b = blockIdx.x;
    if (xcd > 1) b = xcd_order(b, gridDim.x, xcd);
    int lo = 0, hi = nshots - 1;  // the last shot whose first workgroup is <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (wg_begin[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    SweepArgs a = shots[lo];
    a.it = it;
    zmarch_body<R, BX, BY, RY, VW, PF, ST>(a, b - wg_begin[lo]);
}

}  // namespace p1310
