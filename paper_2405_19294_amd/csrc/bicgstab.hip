// Stabilised bi-conjugate gradient (BiCGstab: van der Vorst, SIAM J. Sci.
// Stat. Comput. 13 (1992) 631), the second inverter family of arXiv
// 2405.19294 Sec. 3.3, applied to the even/odd Schur operator D_hat =
// 1 - kappa^2 H_eo H_oe (Sec. 3.1) itself rather than to its normal
// equations, so the condition number is not squared.
//
// Scheduling follows the CG driver: packed half fields in the caller's
// workspace, per-workgroup FP64 partials reduced in a fixed order by one small
// kernel per right-hand side that also evaluates the coefficients (no scalar
// crosses to the host inside an iteration), convergence polled through
// host-mapped flags two iterations behind the launches, and systems that are
// not iterating skipped by every hop and vector kernel.
//
// Mixed precision (inner FP32, or BF16 storage with FP32 arithmetic): the
// recurrences run on the low-precision fields while the solution accumulates
// in FP64.  Every `reliable_every` iterations, when |r|
// fell by `reliable_delta` since the last update, or at recursive
// convergence, the inner solution is folded into the FP64 one and the FP64
// true residual b - D_hat x replaces the recursive residual; rho is then
// re-evaluated against the shadow vector and the search direction kept
// (reliable updates, Sleijpen and van der Vorst, Computing 56 (1996) 141).
// Plain FP64 checks the true residual only at recursive convergence and, when
// it is still above tol, starts again from it with it as the new shadow
// vector.  A vanishing rho, <r0, v> or omega also starts again (both modes).
#include <math.h>
#include <string.h>

#include <chrono>
#include <type_traits>
#include <vector>

#include "engine.h"

namespace hrw {

// ------------------------------------------------------------------ state

struct BiState {      // per right-hand side, device
    double bb;        // |b|^2
    double tol2;      // tol^2 |b|^2
    double rr;        // |r|^2 of the recursion
    double rr_last;   // |r|^2 right after the last FP64 update
    double rr_true;   // last FP64 true |r|^2
    double rho[2], rho_old[2], alpha[2], omega[2], beta[2];  // complex (re, im)
    int status;       // CgStatus
    int iters;
    int restarts;     // new starts (true residual above tol in plain mode, or a vanished coefficient)
    int updates;      // FP64 true-residual evaluations
    int since;        // iterations since the last FP64 update
    int fresh;        // 1: the next iteration takes p = r
    int restart;      // 1: the pending FP64 update must start again (new shadow)
    int pad_;
};

// ------------------------------------------------------------------ device helpers

static __device__ inline double wg_sum(double v, double *sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += sh[k];
    __syncthreads();
    return r;
}

// sum of the nb partials of value k of one rhs, fixed order; valid in thread 0
static __device__ inline double part_sum(const double *partial, int pstride, int nb, int rhs, int k, double *sh)
{
    return wg_sum(strided_sum(partial + (size_t)rhs * pstride + (size_t)k * nb, threadIdx.x, nb, blockDim.x), sh);
}

// c = a / b; false when b = 0 or the quotient is not finite
static __device__ inline bool cdiv(const double a[2], const double b[2], double c[2])
{
    const double d = b[0] * b[0] + b[1] * b[1];
    c[0] = (a[0] * b[0] + a[1] * b[1]) / d;
    c[1] = (a[1] * b[0] - a[0] * b[1]) / d;
    return d > 0 && isfinite(c[0]) && isfinite(c[1]);
}

static __device__ inline void cmul(const double a[2], const double b[2], double c[2])
{
    const double re = a[0] * b[0] - a[1] * b[1];
    c[1] = a[0] * b[1] + a[1] * b[0];
    c[0] = re;
}

// beta = (rho / rho_old) (alpha / omega); false if not finite or omega = 0
static __device__ inline bool make_beta(BiState &c)
{
    double q1[2], q2[2];
    const bool ok = cdiv(c.rho, c.rho_old, q1) && cdiv(c.alpha, c.omega, q2);
    cmul(q1, q2, c.beta);
    return ok && isfinite(c.beta[0]) && isfinite(c.beta[1]);
}

static __device__ inline int host_flag(const BiState &c, int active)
{
    return active ? 1 : (c.status == CG_UPDATE_DUE ? 2 : 0);
}

#define BI_LOOP(n)                                                                                 \
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (n);                       \
         e += (size_t)gridDim.x * blockDim.x)

// ------------------------------------------------------------------ vector kernels

// p = r (fresh) or p = r + beta (p - omega v)
template <class S>
__global__ void __launch_bounds__(WG) bi_p_kernel(const cpx<S> *__restrict__ r, cpx<S> *__restrict__ p,
                                                  const cpx<S> *__restrict__ v, const BiState *st,
                                                  const int *active, size_t n, size_t rs)
{
    typedef typename acc_of<S>::type A;
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    const bool fresh = st[rhs].fresh != 0;
    const A br = (A)st[rhs].beta[0], bi = (A)st[rhs].beta[1];
    const A wr = (A)st[rhs].omega[0], wi = (A)st[rhs].omega[1];
    BI_LOOP(n)
    {
        A rr, ri;
        load_c(r + o + e, rr, ri);
        if (fresh) {
            store_c(p + o + e, rr, ri);
            continue;
        }
        A pr, pi, vr, vi;
        load_c(p + o + e, pr, pi);
        load_c(v + o + e, vr, vi);
        const A qr = pr - (wr * vr - wi * vi), qi = pi - (wr * vi + wi * vr);
        store_c(p + o + e, rr + (br * qr - bi * qi), ri + (br * qi + bi * qr));
    }
}

// partials of <a, b> (re, im) = sum conj(a) b
template <class S>
__global__ void __launch_bounds__(WG) bi_dot_kernel(const cpx<S> *__restrict__ a, const cpx<S> *__restrict__ b,
                                                    const int *active, size_t n, size_t rs, double *partial,
                                                    int pstride)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    double sr = 0, si = 0;
    BI_LOOP(n)
    {
        typename acc_of<S>::type ar, ai, br, bi;
        load_c(a + o + e, ar, ai);
        load_c(b + o + e, br, bi);
        sr += (double)ar * br + (double)ai * bi;
        si += (double)ar * bi - (double)ai * br;
    }
    const double tr = wg_sum(sr, sh), ti = wg_sum(si, sh);
    if (threadIdx.x == 0) {
        double *q = partial + (size_t)rhs * pstride + blockIdx.x;
        q[0] = tr;
        q[gridDim.x] = ti;
    }
}

// s = r - alpha v
template <class S>
__global__ void __launch_bounds__(WG) bi_s_kernel(const cpx<S> *__restrict__ r, const cpx<S> *__restrict__ v,
                                                  cpx<S> *__restrict__ s, const BiState *st, const int *active,
                                                  size_t n, size_t rs)
{
    typedef typename acc_of<S>::type A;
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    const A ar = (A)st[rhs].alpha[0], ai = (A)st[rhs].alpha[1];
    BI_LOOP(n)
    {
        A rr, ri, vr, vi;
        load_c(r + o + e, rr, ri);
        load_c(v + o + e, vr, vi);
        store_c(s + o + e, rr - (ar * vr - ai * vi), ri - (ar * vi + ai * vr));
    }
}

// partials of <t, s> (re, im) and |t|^2
template <class S>
__global__ void __launch_bounds__(WG) bi_ts_kernel(const cpx<S> *__restrict__ t, const cpx<S> *__restrict__ s,
                                                   const int *active, size_t n, size_t rs, double *partial,
                                                   int pstride)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    double sr = 0, si = 0, tt = 0;
    BI_LOOP(n)
    {
        typename acc_of<S>::type tr, ti, xr, xi;
        load_c(t + o + e, tr, ti);
        load_c(s + o + e, xr, xi);
        sr += (double)tr * xr + (double)ti * xi;
        si += (double)tr * xi - (double)ti * xr;
        tt += (double)tr * tr + (double)ti * ti;
    }
    const double a = wg_sum(sr, sh), b = wg_sum(si, sh), c = wg_sum(tt, sh);
    if (threadIdx.x == 0) {
        double *q = partial + (size_t)rhs * pstride + blockIdx.x;
        q[0] = a;
        q[gridDim.x] = b;
        q[2 * gridDim.x] = c;
    }
}

// x += alpha p + omega s; r = s - omega t; partials of |r|^2 and <r0, r> (re, im)
template <class S>
__global__ void __launch_bounds__(WG) bi_xr_kernel(cpx<S> *__restrict__ x, cpx<S> *__restrict__ r,
                                                   const cpx<S> *__restrict__ p, const cpx<S> *__restrict__ s,
                                                   const cpx<S> *__restrict__ t, const cpx<S> *__restrict__ r0,
                                                   const BiState *st, const int *active, size_t n, size_t rs,
                                                   double *partial, int pstride)
{
    typedef typename acc_of<S>::type A;
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    const A ar = (A)st[rhs].alpha[0], ai = (A)st[rhs].alpha[1];
    const A wr = (A)st[rhs].omega[0], wi = (A)st[rhs].omega[1];
    double nn = 0, dr = 0, di = 0;
    BI_LOOP(n)
    {
        A xr, xi, pr, pi, sr, si, tr, ti, hr, hi;
        load_c(x + o + e, xr, xi);
        load_c(p + o + e, pr, pi);
        load_c(s + o + e, sr, si);
        load_c(t + o + e, tr, ti);
        load_c(r0 + o + e, hr, hi);
        xr += (ar * pr - ai * pi) + (wr * sr - wi * si);
        xi += (ar * pi + ai * pr) + (wr * si + wi * sr);
        const A nr = sr - (wr * tr - wi * ti), ni = si - (wr * ti + wi * tr);
        store_c(x + o + e, xr, xi);
        store_c(r + o + e, nr, ni);
        // the partials see the stored residual (rounded for 16-bit storage)
        const A qr = conv<S>::to_acc(conv<S>::from_acc(nr)), qi = conv<S>::to_acc(conv<S>::from_acc(ni));
        nn += (double)qr * qr + (double)qi * qi;
        dr += (double)hr * qr + (double)hi * qi;
        di += (double)hr * qi - (double)hi * qr;
    }
    const double a = wg_sum(nn, sh), b = wg_sum(dr, sh), c = wg_sum(di, sh);
    if (threadIdx.x == 0) {
        double *q = partial + (size_t)rhs * pstride + blockIdx.x;
        q[0] = a;
        q[gridDim.x] = b;
        q[2 * gridDim.x] = c;
    }
}

// mixed precision, due systems: x64 += x_lo; x_lo = 0
template <class S>
__global__ void __launch_bounds__(WG) bi_fold_kernel(cpx<S> *__restrict__ xl, cpx<double> *__restrict__ x64,
                                                     const int *due, size_t n, size_t rs)
{
    typedef typename acc_of<S>::type A;
    const int rhs = blockIdx.y;
    if (!due[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    BI_LOOP(n)
    {
        A lr, li;
        load_c(xl + o + e, lr, li);
        double hr, hi;
        load_c(x64 + o + e, hr, hi);
        store_c(x64 + o + e, hr + (double)lr, hi + (double)li);
        store_c(xl + o + e, (A)0, (A)0);
    }
}

// due systems: r64 = b - q64; partials of |r64|^2 and <r0, r64> (re, im)
template <class S>
__global__ void __launch_bounds__(WG) bi_resid_kernel(const cpx<double> *__restrict__ b,
                                                      const cpx<double> *__restrict__ q,
                                                      cpx<double> *__restrict__ r64, const cpx<S> *__restrict__ r0,
                                                      const int *due, size_t n, size_t rs, double *partial,
                                                      int pstride)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.y;
    if (!due[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    double nn = 0, dr = 0, di = 0;
    BI_LOOP(n)
    {
        double br, bi, qr, qi;
        load_c(b + o + e, br, bi);
        load_c(q + o + e, qr, qi);
        typename acc_of<S>::type hr, hi;
        load_c(r0 + o + e, hr, hi);
        const double rr = br - qr, ri = bi - qi;
        store_c(r64 + o + e, rr, ri);
        nn += rr * rr + ri * ri;
        dr += (double)hr * rr + (double)hi * ri;
        di += (double)hr * ri - (double)hi * rr;
    }
    const double a = wg_sum(nn, sh), c = wg_sum(dr, sh), d = wg_sum(di, sh);
    if (threadIdx.x == 0) {
        double *p = partial + (size_t)rhs * pstride + blockIdx.x;
        p[0] = a;
        p[gridDim.x] = c;
        p[2 * gridDim.x] = d;
    }
}

// due systems that iterate again: r = r64 (rounded to S); after a new start also r0 = r
template <class S>
__global__ void __launch_bounds__(WG) bi_reseed_kernel(const cpx<double> *__restrict__ r64, cpx<S> *__restrict__ r,
                                                       cpx<S> *__restrict__ r0, const BiState *st, const int *due,
                                                       const int *active, size_t n, size_t rs)
{
    const int rhs = blockIdx.y;
    if (!due[rhs] || !active[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    const bool fresh = st[rhs].fresh != 0;
    BI_LOOP(n)
    {
        double hr, hi;
        load_c(r64 + o + e, hr, hi);
        cpx<S> w;
        w.re = conv<S>::from_f64(hr);
        w.im = conv<S>::from_f64(hi);
        r[o + e] = w;
        if (fresh) r0[o + e] = w;
    }
}

// ------------------------------------------------------------------ scalar kernels (one workgroup per rhs)

__global__ void __launch_bounds__(WG) bi_init_kernel(BiState *st, int *active, const double *partial, int pstride,
                                                     int nb, double tol, int *host)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    const double bb = part_sum(partial, pstride, nb, rhs, 0, sh);
    if (threadIdx.x == 0) {
        BiState c = {};
        c.bb = bb;
        c.tol2 = tol * tol * bb;
        c.rr = c.rr_last = c.rr_true = bb;
        c.rho[0] = bb;
        c.rho_old[0] = c.alpha[0] = c.omega[0] = 1.0;
        c.fresh = 1;
        int a = 0;
        if (!isfinite(bb)) c.status = CG_BREAKDOWN;
        else if (bb == 0) c.status = CG_DONE;
        else {
            c.status = CG_RUNNING;
            a = 1;
        }
        st[rhs] = c;
        active[rhs] = a;
        host[rhs] = host_flag(c, a);
    }
}

// alpha = rho / <r0, v>
__global__ void __launch_bounds__(WG) bi_alpha_kernel(BiState *st, int *active, const double *partial, int pstride,
                                                      int nb)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    if (!active[rhs]) return;
    const double d0 = part_sum(partial, pstride, nb, rhs, 0, sh);
    const double d1 = part_sum(partial, pstride, nb, rhs, 1, sh);
    if (threadIdx.x == 0) {
        // alpha = rho / <r0, v>, the arithmetic of cdiv on scalars (a local copy of the
        // state with its arrays went to scratch)
        BiState &c = st[rhs];
        const double a0 = c.rho[0], a1 = c.rho[1];
        const double d = d0 * d0 + d1 * d1;
        const double q0 = (a0 * d0 + a1 * d1) / d, q1 = (a1 * d0 - a0 * d1) / d;
        c.fresh = 0;
        if (d > 0 && isfinite(q0) && isfinite(q1)) {
            c.alpha[0] = q0;
            c.alpha[1] = q1;
        } else {
            c.alpha[0] = c.alpha[1] = 0;
            c.status = CG_UPDATE_DUE;
            c.restart = 1;
            active[rhs] = 0;
        }
    }
}

// omega = <t, s> / |t|^2 (0 when t = 0)
__global__ void __launch_bounds__(WG) bi_omega_kernel(BiState *st, const int *active, const double *partial,
                                                      int pstride, int nb)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    if (!active[rhs]) return;
    const double ts_r = part_sum(partial, pstride, nb, rhs, 0, sh);
    const double ts_i = part_sum(partial, pstride, nb, rhs, 1, sh);
    const double tt = part_sum(partial, pstride, nb, rhs, 2, sh);
    if (threadIdx.x == 0) {
        BiState c = st[rhs];
        c.omega[0] = tt > 0 ? ts_r / tt : 0.0;
        c.omega[1] = tt > 0 ? ts_i / tt : 0.0;
        st[rhs] = c;
    }
}

// end of an iteration: |r|^2, rho = <r0, r>, stopping and update decisions, beta
__global__ void __launch_bounds__(WG) bi_rho_kernel(BiState *st, int *active, const double *partial, int pstride,
                                                    int nb, int max_iter, ReliableSchedule sched, int *host)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    if (!active[rhs]) {
        if (threadIdx.x == 0) host[rhs] = host_flag(st[rhs], 0);
        return;
    }
    const double rr = part_sum(partial, pstride, nb, rhs, 0, sh);
    const double pr = part_sum(partial, pstride, nb, rhs, 1, sh);
    const double pi = part_sum(partial, pstride, nb, rhs, 2, sh);
    if (threadIdx.x == 0) {
        BiState c = st[rhs];
        int a = 1;
        ++c.iters;
        ++c.since;
        c.rr = rr;
        c.rho_old[0] = c.rho[0];
        c.rho_old[1] = c.rho[1];
        c.rho[0] = pr;
        c.rho[1] = pi;
        if (!isfinite(rr) || rr <= c.tol2) {
            c.status = CG_UPDATE_DUE;  // the FP64 check decides (a non-finite value ends as breakdown)
            a = 0;
        } else if (c.iters >= max_iter) {
            c.status = CG_MAXITER;
            a = 0;
        } else if ((sched.every > 0 && c.since >= sched.every) ||
                   (sched.delta2 > 0 && rr < sched.delta2 * c.rr_last)) {
            c.status = CG_UPDATE_DUE;
            a = 0;
        } else if (!make_beta(c)) {
            c.status = CG_UPDATE_DUE;
            c.restart = 1;
            a = 0;
        }
        st[rhs] = c;
        active[rhs] = a;
        host[rhs] = host_flag(c, a);
    }
}

__global__ void bi_mark_due_kernel(const BiState *st, int *due, int n, int all)
{
    const int j = threadIdx.x;
    if (j < n) due[j] = all || st[j].status == CG_UPDATE_DUE;
}

// After the FP64 true residual of the due systems: done, breakdown, or
// iterate again (reliable update in mixed mode, new start in plain mode or
// after a vanished coefficient).  `record_only`: store rr_true, decide nothing.
__global__ void __launch_bounds__(WG) bi_reliable_kernel(BiState *st, int *active, const int *due,
                                                         const double *partial, int pstride, int nb, int mixed,
                                                         int max_restarts, int record_only, int *host)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    if (!due[rhs]) return;
    const double rt = part_sum(partial, pstride, nb, rhs, 0, sh);
    const double dr = part_sum(partial, pstride, nb, rhs, 1, sh);
    const double di = part_sum(partial, pstride, nb, rhs, 2, sh);
    if (threadIdx.x != 0) return;
    BiState c = st[rhs];
    c.rr_true = rt;
    if (record_only) {
        st[rhs] = c;
        return;
    }
    ++c.updates;
    int a = 0;
    if (!isfinite(rt)) {
        c.status = CG_BREAKDOWN;
    } else if (rt <= c.tol2) {
        c.status = CG_DONE;
    } else {
        bool again = c.restart || !mixed;
        if (!again) {
            c.rho[0] = dr;
            c.rho[1] = di;
            again = !make_beta(c);
        }
        if (again && ++c.restarts > max_restarts) {
            c.status = CG_BREAKDOWN;
        } else {
            if (again) {
                c.fresh = 1;
                c.rho[0] = rt;
                c.rho[1] = 0;
            }
            c.rr = rt;
            c.rr_last = rt;
            c.since = 0;
            c.status = CG_RUNNING;
            a = 1;
        }
    }
    c.restart = 0;
    st[rhs] = c;
    active[rhs] = a;
    host[rhs] = host_flag(c, a);
}

// ------------------------------------------------------------------ host plan

struct BiField {
    char *base = nullptr;
    int dt = 0;
    size_t H = 0;
    bool two = false;  // both parity halves (canonical full-lattice fields)
    void *h(int q) const { return base + (two ? (size_t)q * H * dtype_cbytes(dt) : 0); }
};

struct BiPlan {
    int sys;
    bool mixed;
    int dl;          // inner dtype
    size_t H;        // elements of one packed half field
    size_t RS;       // rhs stride of the half fields
    size_t RS2;      // rhs stride of the two-half fields
    BiField x, r, r0, p, v, s, t, o;  // inner precision (o: odd temporary)
    BiField b, x64, r64, q64, o64;    // FP64 (x64 only in mixed mode)
    BiField bfull, dfull, efull;      // HRW_SYS_D_EO: full source, full solution, D x
    BiField w, u, w64, u64;           // clover: odd and even temporaries of D_hat_sw
    BiState *st;
    int *active;  // [0, MAX_RHS) active, [MAX_RHS, 2 MAX_RHS) due
    double *coef_k, *coef_k2, *coef_mk, *scal;
    double *part;
    int nb, pstride;
};

static BiField take_field(Arena &ar, int dt, size_t H, bool two, int n_rhs)
{
    BiField f;
    f.dt = dt;
    f.H = H;
    f.two = two;
    f.base = (char *)ar.take((two ? 2 : 1) * H * n_rhs * dtype_cbytes(dt));
    return f;
}

static void plan_bicg(Arena &ar, const Geom &g, int nr, int n_rhs, const hrw_solve_params *prm, BiPlan &P,
                      bool clover = false)
{
    P.sys = prm->system;
    P.dl = prm->inner_dtype;
    P.mixed = P.dl != 0;
    P.H = spinor_elems(g, nr);
    P.RS = P.H;
    P.RS2 = 2 * P.H;
    auto half = [&](int dt) { return take_field(ar, dt, P.H, false, n_rhs); };
    for (BiField *f : {&P.x, &P.r, &P.r0, &P.p, &P.v, &P.s, &P.t, &P.o}) *f = half(P.dl);
    for (BiField *f : {&P.b, &P.r64, &P.q64, &P.o64}) *f = half(0);
    if (P.mixed) P.x64 = half(0);
    if (clover) {
        P.w = half(P.dl);
        P.u = half(P.dl);
        P.w64 = half(0);
        P.u64 = half(0);
    }
    if (P.sys == HRW_SYS_D_EO) {
        P.bfull = take_field(ar, 0, P.H, true, n_rhs);
        P.dfull = take_field(ar, 0, P.H, true, n_rhs);
        P.efull = take_field(ar, 0, P.H, true, n_rhs);
    }
    P.st = (BiState *)ar.take(sizeof(BiState) * MAX_RHS);
    P.active = (int *)ar.take(sizeof(int) * 2 * MAX_RHS);
    P.coef_k = (double *)ar.take(sizeof(double) * MAX_RHS);
    P.coef_k2 = (double *)ar.take(sizeof(double) * MAX_RHS);
    P.coef_mk = (double *)ar.take(sizeof(double) * MAX_RHS);
    P.scal = (double *)ar.take(sizeof(double) * 2 * MAX_RHS);
    // the two-half residual of the D x = b check needs the larger grid
    P.nb = vec_grid(P.sys == HRW_SYS_D_EO ? 2 * P.H : P.H);
    P.pstride = 3 * P.nb;
    P.part = (double *)ar.take(sizeof(double) * (size_t)P.pstride * n_rhs);
}

int bicg_workspace(const Geom &g, int nr, int n_rhs, const hrw_solve_params *p, size_t *bytes, bool clover)
{
    Arena ar(nullptr, 0);
    BiPlan P;
    plan_bicg(ar, g, nr, n_rhs, p, P, clover);
    *bytes = ar.off + 256;
    return HRW_OK;
}

// ------------------------------------------------------------------ driver

struct BiRun {
    const hrw_gauge *g;
    BiPlan *P;
    Phases ph;
    int n;
    hipStream_t st;
    int nbh;  // vector-kernel blocks over one half field
    const hrw_clover *cl;  // clover term (D_hat_sw in place of D_hat), or null
};

// out = D_hat in (or D_hat_sw with a clover term) on the dtype of the fields (run: per rhs skip mask)
static int apply_dhat(BiRun &R, const BiField &in, const BiField &odd, const BiField &out, const int *run)
{
    if (R.cl) {
        const bool lo = in.dt != 0;
        const BiField &w = lo ? R.P->w : R.P->w64, &u = lo ? R.P->u : R.P->u64;
        return dsw_eo_packed(R.cl, R.ph, in.dt, R.n, false, R.P->RS, in.h(0), odd.h(0), w.h(0), u.h(0), out.h(0),
                             R.P->coef_k2, run, R.st);
    }
    HopCall a;
    a.dt = in.dt;
    a.n_rhs = R.n;
    a.rstride = R.P->RS;
    a.run = run;
    a.parity = 1;
    a.epi = EPI_PLAIN;
    a.in[0] = in.h(0);
    a.out[1] = odd.h(0);
    int rc = run_hop(R.g, R.ph, a, R.st);
    if (rc) return rc;
    HopCall b = a;
    b.parity = 0;
    b.epi = EPI_AXPY;
    b.coef = R.P->coef_k2;
    b.in[1] = odd.h(0);
    b.in[0] = nullptr;
    b.out[1] = nullptr;
    b.self[0] = in.h(0);
    b.out[0] = out.h(0);
    return run_hop(R.g, R.ph, b, R.st);
}

template <class S>
static int bi_iteration(BiRun &R, int max_iter, ReliableSchedule sched, int *host)
{
    BiPlan &P = *R.P;
    const dim3 grid(R.nbh, R.n);
    const size_t E = P.H, RS = P.RS;
    auto F = [](const BiField &f) { return (cpx<S> *)f.base; };
    int rc;
    bi_p_kernel<S><<<grid, WG, 0, R.st>>>(F(P.r), F(P.p), F(P.v), P.st, P.active, E, RS);
    HRW_HIP(hipGetLastError());
    if ((rc = apply_dhat(R, P.p, P.o, P.v, P.active))) return rc;
    bi_dot_kernel<S><<<grid, WG, 0, R.st>>>(F(P.r0), F(P.v), P.active, E, RS, P.part, P.pstride);
    HRW_HIP(hipGetLastError());
    bi_alpha_kernel<<<R.n, WG, 0, R.st>>>(P.st, P.active, P.part, P.pstride, R.nbh);
    HRW_HIP(hipGetLastError());
    bi_s_kernel<S><<<grid, WG, 0, R.st>>>(F(P.r), F(P.v), F(P.s), P.st, P.active, E, RS);
    HRW_HIP(hipGetLastError());
    if ((rc = apply_dhat(R, P.s, P.o, P.t, P.active))) return rc;
    bi_ts_kernel<S><<<grid, WG, 0, R.st>>>(F(P.t), F(P.s), P.active, E, RS, P.part, P.pstride);
    HRW_HIP(hipGetLastError());
    bi_omega_kernel<<<R.n, WG, 0, R.st>>>(P.st, P.active, P.part, P.pstride, R.nbh);
    HRW_HIP(hipGetLastError());
    bi_xr_kernel<S><<<grid, WG, 0, R.st>>>(F(P.x), F(P.r), F(P.p), F(P.s), F(P.t), F(P.r0), P.st, P.active, E, RS,
                                           P.part, P.pstride);
    HRW_HIP(hipGetLastError());
    bi_rho_kernel<<<R.n, WG, 0, R.st>>>(P.st, P.active, P.part, P.pstride, R.nbh, max_iter, sched, host);
    HRW_HIP(hipGetLastError());
    return HRW_OK;
}

// FP64 true residual of the systems in `due` (mixed: after folding x_lo into
// x64), partials of |r64|^2 and <r0, r64> in P.part
template <class S>
static int bi_true_residual(BiRun &R, const int *due)
{
    BiPlan &P = *R.P;
    const dim3 grid(R.nbh, R.n);
    if (P.mixed) {
        bi_fold_kernel<S><<<grid, WG, 0, R.st>>>((cpx<S> *)P.x.base, (cpx<double> *)P.x64.base, due, P.H, P.RS);
        HRW_HIP(hipGetLastError());
    }
    int rc = apply_dhat(R, P.mixed ? P.x64 : P.x, P.o64, P.q64, due);
    if (rc) return rc;
    bi_resid_kernel<S><<<grid, WG, 0, R.st>>>((const cpx<double> *)P.b.base, (const cpx<double> *)P.q64.base,
                                              (cpx<double> *)P.r64.base, (const cpx<S> *)P.r0.base, due, P.H, P.RS,
                                              P.part, P.pstride);
    HRW_HIP(hipGetLastError());
    return HRW_OK;
}

template <class S>
static int bi_reliable_pass(BiRun &R, int *host)
{
    BiPlan &P = *R.P;
    int *due = P.active + MAX_RHS;
    bi_mark_due_kernel<<<1, 64, 0, R.st>>>(P.st, due, R.n, 0);
    HRW_HIP(hipGetLastError());
    int rc = bi_true_residual<S>(R, due);
    if (rc) return rc;
    bi_reliable_kernel<<<R.n, WG, 0, R.st>>>(P.st, P.active, due, P.part, P.pstride, R.nbh, P.mixed ? 1 : 0,
                                             100, 0, host);
    HRW_HIP(hipGetLastError());
    bi_reseed_kernel<S><<<dim3(R.nbh, R.n), WG, 0, R.st>>>((const cpx<double> *)P.r64.base, (cpx<S> *)P.r.base,
                                                          (cpx<S> *)P.r0.base, P.st, due, P.active, P.H, P.RS);
    HRW_HIP(hipGetLastError());
    HRW_HIP(hipStreamSynchronize(R.st));
    return HRW_OK;
}

static bool bi_any(const int *host, int n, int v)
{
    for (int j = 0; j < n; ++j)
        if (host[j] == v) return true;
    return false;
}

template <class S>
static int bi_run(BiRun &R, const hrw_solve_params *prm, const HostFlags &hf, hipEvent_t ev[3])
{
    ReliableSchedule sched;
    sched.every = R.P->mixed ? (prm->reliable_every > 0 ? prm->reliable_every : 50) : 0;
    sched.delta2 = R.P->mixed ? prm->reliable_delta * prm->reliable_delta : 0.0;
    const int n = R.n;
    int rc;
    long long enq = 0;
    for (;;) {
        // iterate until nothing runs or some system waits for its FP64 check;
        // the flags are read two iterations behind the launches
        const long long e0 = enq;
        while (bi_any(hf.host, n, 1)) {
            if ((rc = bi_iteration<S>(R, prm->max_iter, sched, hf.dev))) return rc;
            HRW_HIP(hipEventRecord(ev[enq % 3], R.st));
            ++enq;
            if (enq - e0 >= 2) {
                HRW_HIP(hipEventSynchronize(ev[(enq - 2) % 3]));
                if (bi_any(hf.host, n, 2)) break;
            }
        }
        HRW_HIP(hipStreamSynchronize(R.st));
        if (bi_any(hf.host, n, 2)) {
            if ((rc = bi_reliable_pass<S>(R, hf.dev))) return rc;
            continue;
        }
        if (!bi_any(hf.host, n, 1)) return HRW_OK;
    }
}

template <class S>
static int bi_finish(BiRun &R, double *x_out, hrw_solve_result *res, std::chrono::steady_clock::time_point t0)
{
    BiPlan &P = *R.P;
    const hrw_gauge *g = R.g;
    const hipStream_t st = R.st;
    const int n = R.n;
    int *due = P.active + MAX_RHS;
    bi_mark_due_kernel<<<1, 64, 0, st>>>(P.st, due, n, 1);
    HRW_HIP(hipGetLastError());
    int rc = bi_true_residual<S>(R, due);
    if (rc) return rc;
    bi_reliable_kernel<<<n, WG, 0, st>>>(P.st, P.active, due, P.part, P.pstride, R.nbh, 0, 0, 1, nullptr);
    HRW_HIP(hipGetLastError());
    const BiField &X = P.mixed ? P.x64 : P.x;
    if (P.sys == HRW_SYS_DHAT_EO) {
        HRW_HIP(launch_unpack_spinor(0, g->nr, g->g, false, 0, n, X.h(0), nullptr, P.RS, x_out, st));
    } else {
        // x_e into the even half of dfull (the hops take one rhs stride for every operand),
        // x_o = b_o + kappa H_oe x_e into its odd half
        HRW_HIP(hipMemcpy2DAsync(P.dfull.h(0), P.RS2 * sizeof(cpx<double>), X.h(0), P.RS * sizeof(cpx<double>),
                                 P.H * sizeof(cpx<double>), n, hipMemcpyDeviceToDevice, st));
        HopCall c;
        c.dt = 0;
        c.n_rhs = n;
        c.rstride = P.RS2;
        c.parity = 1;
        c.epi = EPI_AXPY;
        c.coef = P.coef_mk;
        c.in[0] = P.dfull.h(0);
        c.self[1] = P.bfull.h(1);
        c.out[1] = R.cl ? P.efull.h(1) : P.dfull.h(1);
        if ((rc = run_hop(g, R.ph, c, st))) return rc;
        // with a clover term x_o = A_oo^-1 (b_o + kappa H_oe x_e)
        if (R.cl)
            HRW_HIP(launch_clover_mul(0, g->nr, g->g, R.cl->inv[0][1], P.efull.h(1), P.dfull.h(1), n, P.RS2, st));
        HRW_HIP(launch_unpack_spinor(0, g->nr, g->g, true, 0, n, P.dfull.h(0), P.dfull.h(1), P.RS2, x_out, st));
        // |b - D x| / |b| on the full lattice
        HopCall d;
        d.dt = 0;
        d.n_rhs = n;
        d.rstride = P.RS2;
        d.parity = -1;
        d.epi = EPI_AXPY;
        d.coef = P.coef_k;
        for (int q = 0; q < 2; ++q) {
            d.in[q] = P.dfull.h(q);
            d.self[q] = P.dfull.h(q);
            d.out[q] = P.efull.h(q);
        }
        if (R.cl) {
            // D_sw x = A x - kappa H x: self = A x (the epilogue reads self before it writes out in place)
            for (int q = 0; q < 2; ++q) {
                HRW_HIP(launch_clover_mul(0, g->nr, g->g, R.cl->a[0][q], P.dfull.h(q), P.efull.h(q), n, P.RS2, st));
                d.self[q] = P.efull.h(q);
            }
        }
        if ((rc = run_hop(g, R.ph, d, st))) return rc;
        const int nb2 = vec_grid(2 * P.H);
        HRW_HIP(launch_residual<double>((const cpx<double> *)P.bfull.base, (const cpx<double> *)P.efull.base,
                                        (cpx<double> *)P.dfull.base, 2 * P.H, P.RS2, n, P.part, P.pstride, nb2, st));
        HRW_HIP(launch_sum_partials(P.part, P.pstride, nb2, n, P.scal, st));
        HRW_HIP(launch_norm2<double>((const cpx<double> *)P.bfull.base, 2 * P.H, P.RS2, n, P.part, P.pstride, nb2,
                                     st));
        HRW_HIP(launch_sum_partials(P.part, P.pstride, nb2, n, P.scal + MAX_RHS, st));
    }
    std::vector<BiState> hs(n);
    HRW_HIP(hipMemcpyAsync(hs.data(), P.st, sizeof(BiState) * n, hipMemcpyDeviceToHost, st));
    double dres[2 * MAX_RHS] = {0};
    if (P.sys == HRW_SYS_D_EO)
        HRW_HIP(hipMemcpyAsync(dres, P.scal, sizeof(double) * 2 * MAX_RHS, hipMemcpyDeviceToHost, st));
    HRW_HIP(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int overall = HRW_OK;
    for (int j = 0; j < n; ++j) {
        const BiState &c = hs[j];
        hrw_solve_result &o = res[j];
        memset(&o, 0, sizeof o);
        o.iters = c.iters;
        o.reliable_updates = P.mixed ? c.updates : 0;
        o.restarts = c.restarts;
        o.true_rel_resid = c.bb > 0 ? sqrt(c.rr_true / c.bb) : 0.0;
        o.recursive_rel_resid = c.bb > 0 ? sqrt(c.rr / c.bb) : 0.0;
        o.d_rel_resid = dres[MAX_RHS + j] > 0 ? sqrt(dres[j] / dres[MAX_RHS + j]) : 0.0;
        o.seconds = secs;
        o.status = c.status == CG_DONE ? HRW_OK : c.status == CG_BREAKDOWN ? HRW_EBREAKDOWN : HRW_NOT_CONVERGED;
        if (o.status == HRW_EBREAKDOWN) overall = HRW_EBREAKDOWN;
        else if (o.status == HRW_NOT_CONVERGED && overall == HRW_OK) overall = HRW_NOT_CONVERGED;
    }
    return overall;
}

int bicgstab_solve(const hrw_gauge *g, const hrw_solve_params *prm, int n_rhs, const double *kappa,
                   const double *b_in, double *x_out, hrw_solve_result *res, void *ws, size_t ws_bytes,
                   hipStream_t st, const hrw_clover *cl)
{
    const auto t0 = std::chrono::steady_clock::now();
    Arena ar(ws, ws_bytes);
    BiPlan P;
    plan_bicg(ar, g->g, g->nr, n_rhs, prm, P, cl != nullptr);
    if (!ar.fits()) return fail(HRW_ENOMEM, "workspace too small: need %zu bytes, got %zu", ar.off + 256, ws_bytes);
    BiRun R{g, &P, make_phases(prm->theta), n_rhs, st, vec_grid(P.H), cl};
    int rc;
    double kv[MAX_RHS], k2[MAX_RHS], mk[MAX_RHS];
    for (int j = 0; j < n_rhs; ++j) {
        kv[j] = kappa[j];
        k2[j] = kappa[j] * kappa[j];
        mk[j] = -kappa[j];
    }
    // every field starts at zero: padding lanes stay zero and x starts at 0
    HRW_HIP(launch_zero(ar.base, ar.off, st));
    if ((rc = set_device_doubles(P.coef_k, kv, n_rhs, st))) return rc;
    if ((rc = set_device_doubles(P.coef_k2, k2, n_rhs, st))) return rc;
    if ((rc = set_device_doubles(P.coef_mk, mk, n_rhs, st))) return rc;
    if (P.sys == HRW_SYS_DHAT_EO) {
        HRW_HIP(launch_pack_spinor(0, g->nr, g->g, false, 0, n_rhs, b_in, P.b.h(0), nullptr, P.RS, st));
    } else {
        // b'_e = b_e + kappa H_eo b_o (with a clover term: b_e + kappa H_eo A_oo^-1 b_o)
        HRW_HIP(launch_pack_spinor(0, g->nr, g->g, true, 0, n_rhs, b_in, P.bfull.h(0), P.bfull.h(1), P.RS2, st));
        if (cl) HRW_HIP(launch_clover_mul(0, g->nr, g->g, cl->inv[0][1], P.bfull.h(1), P.efull.h(1), n_rhs, P.RS2, st));
        HopCall c;
        c.dt = 0;
        c.n_rhs = n_rhs;
        c.rstride = P.RS2;
        c.parity = 0;
        c.epi = EPI_AXPY;
        c.coef = P.coef_mk;
        c.in[1] = cl ? P.efull.h(1) : P.bfull.h(1);
        c.self[0] = P.bfull.h(0);
        c.out[0] = P.dfull.h(0);
        if ((rc = run_hop(g, R.ph, c, st))) return rc;
        HRW_HIP(hipMemcpy2DAsync(P.b.h(0), P.RS * sizeof(cpx<double>), P.dfull.h(0), P.RS2 * sizeof(cpx<double>),
                                 P.H * sizeof(cpx<double>), n_rhs, hipMemcpyDeviceToDevice, st));
    }
    HostFlags hf;
    if ((rc = host_flags_acquire(&hf))) return rc;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    struct Cleanup {
        HostFlags *hf;
        hipEvent_t *ev;
        ~Cleanup()
        {
            for (int k = 0; k < 3; ++k)
                if (ev[k]) (void)hipEventDestroy(ev[k]);
            host_flags_release(hf);
        }
    } cleanup{&hf, ev};
    for (int k = 0; k < 3; ++k)
        if (hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) != hipSuccess)
            return fail(HRW_EDEVICE, "event creation failed");
    HRW_HIP(launch_norm2<double>((const cpx<double> *)P.b.base, P.H, P.RS, n_rhs, P.part, P.pstride, R.nbh, st));
    bi_init_kernel<<<n_rhs, WG, 0, st>>>(P.st, P.active, P.part, P.pstride, R.nbh, prm->tol, hf.dev);
    HRW_HIP(hipGetLastError());
    // r = r0 = b in the inner precision (p = r is taken by the first iteration)
    HRW_HIP(launch_convert(0, P.b.base, P.dl, P.r.base, P.H * n_rhs, st));
    HRW_HIP(launch_convert(0, P.b.base, P.dl, P.r0.base, P.H * n_rhs, st));
    HRW_HIP(hipStreamSynchronize(st));
    bool ok = dispatch_dtype(P.dl, [&](auto sv) {
        typedef decltype(sv) S;
        if constexpr (std::is_same<S, double>::value || std::is_same<S, float>::value ||
                      std::is_same<S, bf16_t>::value) {
            rc = bi_run<S>(R, prm, hf, ev);
            if (!rc) rc = bi_finish<S>(R, x_out, res, t0);
        } else {
            rc = fail(HRW_EUNSUPPORTED, "BiCGstab runs with FP64, FP32 or BF16 inner fields");
        }
    });
    if (!ok) return fail(HRW_EINVAL, "bad inner dtype");
    if (rc < 0) return rc;
    if (timing().on) timing_harvest();
    return rc;
}

}  // namespace hrw
