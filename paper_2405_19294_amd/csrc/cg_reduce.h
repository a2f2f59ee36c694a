// The alpha step of CG (Sec. 3.3) as a device function, shared by the
// one-workgroup scalar kernel and the hopping kernels that run it on the side
// (the second stage of the Sec. 3.2 two-stage reduction).
#pragma once

#include "kernels.h"

namespace hrw {

// Sum of p[0 .. nparts) in one fixed order, whatever the workgroup size (a
// multiple of 64): 256 virtual lanes, lane v summing p[v], p[v + 256], ...;
// each virtual wavefront of 64 lanes folded by the shuffle-down tree; the four
// wavefront sums added in order.  Every thread of the workgroup must call it;
// the result is valid in thread 0.  sh: 4 doubles of LDS.
__device__ inline double fixed_sum_256(const double *p, int nparts, double *sh)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int vw = w; vw < 4; vw += nw) {
        double v = strided_sum(p, vw * 64 + lane, nparts, 256);
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) sh[vw] = v;
    }
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) r += sh[k];
    __syncthreads();
    return r;
}

// <p, A p> of system rhs from its partial sums, then alpha = |r|^2 / <p, A p>
// (breakdown when <p, A p> is not positive and finite); inactive systems get
// alpha = 0.  Every thread of the workgroup must call it.
__device__ inline void cg_alpha_step(CgState *cs, const double *partial, int nparts, double *alpha_out, int rhs,
                                     double *sh)
{
    const double pap = fixed_sum_256(partial, nparts, sh);
    if (threadIdx.x == 0) {
        CgState c = cs[rhs];
        c.pap = pap;
        if (c.active) {
            if (!(pap > 0) || isinf(pap)) {
                c.status = CG_BREAKDOWN;
                c.active = 0;
                c.alpha = 0;
            } else {
                c.alpha = c.rr / pap;
            }
        } else {
            c.alpha = 0;
        }
        cs[rhs] = c;
        alpha_out[rhs] = c.alpha;
    }
}

// The alpha step carried by a hopping launch (a.red_cs set): the workgroups
// with blockIdx.x == 0 of a grid with one row per source, or the first
// workgroups of a one-row grid, each take the systems rhs = their index,
// index + grid width, ...  Called by every thread of a workgroup before any
// early return.
template <class S>
__device__ inline void hop_alpha_on_the_side(const HopArgs<S> &a, double *sh)
{
    if (!a.red_cs) return;
    if (gridDim.y > 1) {
        if (blockIdx.x != 0) return;
        const int rhs = blockIdx.y;
        cg_alpha_step(a.red_cs, a.red_partial + (size_t)rhs * a.red_pstride, a.red_nparts, a.red_alpha, rhs, sh);
    } else {
        for (int rhs = blockIdx.x; rhs < a.red_n; rhs += gridDim.x)
            cg_alpha_step(a.red_cs, a.red_partial + (size_t)rhs * a.red_pstride, a.red_nparts, a.red_alpha, rhs, sh);
    }
}

}  // namespace hrw
