// Site-wise linear algebra and reductions for the solvers (arXiv 2405.19294,
// Sec. 3.2: streaming spinor kernels; inner products and norms reduce a field
// to a number in two stages).  Here the first stage is fused into the kernel
// that produces the field (per-workgroup partials in FP64, wave shuffles then
// LDS, fixed order) and the second stage is one small kernel per right-hand
// side that also evaluates the CG coefficients on the device, so no scalar
// travels to the host inside the iteration.  Every reduction uses a fixed
// order: results are bitwise reproducible run to run.
#include <math.h>

#include "kernels.h"
#include "cg_reduce.h"

namespace hrw {

static __device__ inline double block_sum(double v, double *sh)
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

int vec_grid(size_t elems)
{
    size_t b = (elems + WG - 1) / WG;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

// ------------------------------------------------------------------ fills and copies

__global__ void __launch_bounds__(WG) zero_kernel(uint4 *p, size_t n16, unsigned char *tail, size_t ntail)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n16; t += stride)
        p[t] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_zero(void *dst, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return hipSuccess;
    // callers pass 16-byte aligned buffers; the tail (< 16 bytes) is cleared bytewise
    const size_t n16 = bytes / 16;
    const size_t ntail = bytes - n16 * 16;
    size_t b = (n16 + WG - 1) / WG;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    zero_kernel<<<(unsigned)b, WG, 0, st>>>((uint4 *)dst, n16, (unsigned char *)dst + n16 * 16, ntail);
    return hipGetLastError();
}

template <class S>
__global__ void __launch_bounds__(WG) copy_kernel(const cpx<S> *__restrict__ a, cpx<S> *__restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) b[t] = a[t];
}

template <class S>
hipError_t launch_copy(const cpx<S> *src, cpx<S> *dst, size_t elems, hipStream_t st)
{
    copy_kernel<S><<<vec_grid(elems), WG, 0, st>>>(src, dst, elems);
    return hipGetLastError();
}

template <class Ss, class Sd>
__global__ void __launch_bounds__(WG) convert_kernel(const cpx<Ss> *__restrict__ a, cpx<Sd> *__restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        typename acc_of<Ss>::type re, im;
        load_c(a + t, re, im);
        cpx<Sd> v;
        // FP64 sources round once to the destination format; others go through FP32
        if constexpr (std::is_same<Ss, double>::value) {
            v.re = conv<Sd>::from_f64(re);
            v.im = conv<Sd>::from_f64(im);
        } else {
            v.re = conv<Sd>::from_acc((typename acc_of<Sd>::type)re);
            v.im = conv<Sd>::from_acc((typename acc_of<Sd>::type)im);
        }
        b[t] = v;
    }
}

hipError_t launch_convert(int dt_src, const void *src, int dt_dst, void *dst, size_t elems,
                          hipStream_t st)
{
    bool ok = dispatch_dtype(dt_src, [&](auto sa) {
        typedef decltype(sa) Ss;
        dispatch_dtype(dt_dst, [&](auto sb) {
            typedef decltype(sb) Sd;
            convert_kernel<Ss, Sd><<<vec_grid(elems), WG, 0, st>>>((const cpx<Ss> *)src, (cpx<Sd> *)dst, elems);
        });
    });
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------ reductions

template <class S>
__global__ void __launch_bounds__(WG) norm2_kernel(const cpx<S> *__restrict__ a, size_t n, size_t rstride,
                                                    double *partial, int pstride)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.y;
    const cpx<S> *ar = a + (size_t)rhs * rstride;
    double s = 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        typename acc_of<S>::type re, im;
        load_c(ar + t, re, im);
        s += (double)re * re + (double)im * im;
    }
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) partial[(size_t)rhs * pstride + blockIdx.x] = tot;
}

template <class S>
hipError_t launch_norm2(const cpx<S> *a, size_t elems, size_t rstride, int n_rhs, double *partial,
                        int pstride, int nblocks, hipStream_t st)
{
    norm2_kernel<S><<<dim3(nblocks, n_rhs), WG, 0, st>>>(a, elems, rstride, partial, pstride);
    return hipGetLastError();
}

template <class S>
__global__ void __launch_bounds__(WG) residual_kernel(const cpx<S> *__restrict__ b, const cpx<S> *__restrict__ q,
                                                       cpx<S> *__restrict__ r, size_t n, size_t rstride,
                                                       double *partial, int pstride)
{
    typedef typename acc_of<S>::type A;
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.y;
    const size_t ro = (size_t)rhs * rstride;
    double s = 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        A br, bi, qr, qi;
        load_c(b + ro + t, br, bi);
        load_c(q + ro + t, qr, qi);
        const A vr = br - qr, vi = bi - qi;
        store_c(r + ro + t, vr, vi);
        s += (double)vr * vr + (double)vi * vi;
    }
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) partial[(size_t)rhs * pstride + blockIdx.x] = tot;
}

template <class S>
hipError_t launch_residual(const cpx<S> *b, const cpx<S> *q, cpx<S> *r, size_t elems, size_t rstride,
                           int n_rhs, double *partial, int pstride, int nblocks, hipStream_t st)
{
    residual_kernel<S><<<dim3(nblocks, n_rhs), WG, 0, st>>>(b, q, r, elems, rstride, partial, pstride);
    return hipGetLastError();
}

template <class S>
__global__ void __launch_bounds__(WG) xpay_kernel(const cpx<S> *__restrict__ r, cpx<S> *__restrict__ p,
                                                   const double *beta, const int *active, size_t n,
                                                   size_t rstride)
{
    typedef typename acc_of<S>::type A;
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const A bt = (A)beta[rhs];
    const size_t ro = (size_t)rhs * rstride;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        A rr, ri, pr, pi;
        load_c(r + ro + t, rr, ri);
        load_c(p + ro + t, pr, pi);
        store_c(p + ro + t, rr + bt * pr, ri + bt * pi);
    }
}

template <class S>
hipError_t launch_xpay(const cpx<S> *r, cpx<S> *p, const double *beta, const int *active, size_t elems,
                       size_t rstride, int n_rhs, hipStream_t st)
{
    xpay_kernel<S><<<dim3(vec_grid(elems), n_rhs), WG, 0, st>>>(r, p, beta, active, elems, rstride);
    return hipGetLastError();
}

template <class S>
__global__ void __launch_bounds__(WG) cg_xp_kernel(const cpx<S> *__restrict__ r, cpx<S> *__restrict__ p,
                                                    cpx<S> *__restrict__ x, const double *alpha, const double *beta,
                                                    const int *advanced, size_t n, size_t rstride)
{
    typedef typename acc_of<S>::type A;
    const int rhs = blockIdx.y;
    if (!advanced[rhs]) return;
    const A al = (A)alpha[rhs], bt = (A)beta[rhs];
    const size_t ro = (size_t)rhs * rstride;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        A rr, ri, pr, pi, xr, xi;
        load_c_nt(r + ro + t, rr, ri);
        load_c(p + ro + t, pr, pi);
        load_c_nt(x + ro + t, xr, xi);
        xr += al * pr;
        xi += al * pi;
        store_c_nt(x + ro + t, xr, xi);
        store_c(p + ro + t, rr + bt * pr, ri + bt * pi);
    }
}

template <class S>
hipError_t launch_cg_xp(const cpx<S> *r, cpx<S> *p, cpx<S> *x, const double *alpha, const double *beta,
                        const int *advanced, size_t elems, size_t rstride, int n_rhs, hipStream_t st)
{
    cg_xp_kernel<S><<<dim3(vec_grid(elems), n_rhs), WG, 0, st>>>(r, p, x, alpha, beta, advanced, elems, rstride);
    return hipGetLastError();
}

template <class Sx, class Sy>
__global__ void __launch_bounds__(WG) axpy_mixed_kernel(const cpx<Sx> *__restrict__ x, cpx<Sy> *__restrict__ y,
                                                         const double *a, size_t n, size_t rsx, size_t rsy)
{
    typedef typename acc_of<Sy>::type A;
    const int rhs = blockIdx.y;
    const A al = (A)a[rhs];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        typename acc_of<Sx>::type xr, xi;
        load_c(x + (size_t)rhs * rsx + t, xr, xi);
        A yr, yi;
        load_c(y + (size_t)rhs * rsy + t, yr, yi);
        store_c(y + (size_t)rhs * rsy + t, yr + al * (A)xr, yi + al * (A)xi);
    }
}

hipError_t launch_axpy_mixed(int dt_x, const void *x, int dt_y, void *y, const double *a, size_t elems,
                             size_t rstride_x, size_t rstride_y, int n_rhs, hipStream_t st)
{
    bool ok = dispatch_dtype(dt_x, [&](auto sx) {
        typedef decltype(sx) Sx;
        dispatch_dtype(dt_y, [&](auto sy) {
            typedef decltype(sy) Sy;
            axpy_mixed_kernel<Sx, Sy><<<dim3(vec_grid(elems), n_rhs), WG, 0, st>>>(
                (const cpx<Sx> *)x, (cpx<Sy> *)y, a, elems, rstride_x, rstride_y);
        });
    });
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

template <class Sl>
__global__ void __launch_bounds__(WG) fold_kernel(cpx<Sl> *__restrict__ xl, cpx<double> *__restrict__ x64,
                                                   const int *due, const CgState *cs, size_t n, size_t rstride)
{
    const int rhs = blockIdx.y;
    if (!due[rhs]) return;
    const double inv = 1.0 / cs[rhs].scale;
    const size_t ro = (size_t)rhs * rstride;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        typename acc_of<Sl>::type lr, li;
        load_c(xl + ro + t, lr, li);
        double hr, hi;
        load_c(x64 + ro + t, hr, hi);
        store_c(x64 + ro + t, hr + (double)lr * inv, hi + (double)li * inv);
        store_c(xl + ro + t, (typename acc_of<Sl>::type)0, (typename acc_of<Sl>::type)0);
    }
}

hipError_t launch_fold(int dt_lo, void *x_lo, double *x64, const int *due, const CgState *cs, size_t elems,
                       size_t rstride, int n_rhs, hipStream_t st)
{
    bool ok = dispatch_dtype(dt_lo, [&](auto sv) {
        typedef decltype(sv) Sl;
        fold_kernel<Sl><<<dim3(vec_grid(elems), n_rhs), WG, 0, st>>>((cpx<Sl> *)x_lo, (cpx<double> *)x64, due,
                                                                     cs, elems, rstride);
    });
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

template <class Sl>
__global__ void __launch_bounds__(WG) reseed_kernel(const cpx<double> *__restrict__ r64, cpx<Sl> *__restrict__ rl,
                                                     cpx<Sl> *__restrict__ pl, const int *due, const CgState *cs,
                                                     size_t n, size_t rstride)
{
    const int rhs = blockIdx.y;
    if (!due[rhs]) return;
    const double sn = cs[rhs].scale, so = 1.0 / cs[rhs].scale_prev;
    const size_t ro = (size_t)rhs * rstride;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const cpx<double> v = r64[ro + t];
        typename acc_of<Sl>::type orr, ori, opr, opi;
        load_c(rl + ro + t, orr, ori);
        load_c(pl + ro + t, opr, opi);
        cpx<Sl> w, q;
        w.re = conv<Sl>::from_f64(sn * v.re);
        w.im = conv<Sl>::from_f64(sn * v.im);
        q.re = conv<Sl>::from_f64(sn * ((double)opr * so + (v.re - (double)orr * so)));
        q.im = conv<Sl>::from_f64(sn * ((double)opi * so + (v.im - (double)ori * so)));
        rl[ro + t] = w;
        pl[ro + t] = q;
    }
}

hipError_t launch_reseed(int dt_lo, const double *r64, void *r_lo, void *p_lo, const int *due, const CgState *cs,
                         size_t elems, size_t rstride, int n_rhs, hipStream_t st)
{
    bool ok = dispatch_dtype(dt_lo, [&](auto sv) {
        typedef decltype(sv) Sl;
        reseed_kernel<Sl><<<dim3(vec_grid(elems), n_rhs), WG, 0, st>>>((const cpx<double> *)r64, (cpx<Sl> *)r_lo,
                                                                       (cpx<Sl> *)p_lo, due, cs, elems, rstride);
    });
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

template <class Sl>
__global__ void __launch_bounds__(WG) seed_kernel(const cpx<double> *__restrict__ b64, cpx<Sl> *__restrict__ rl,
                                                   cpx<Sl> *__restrict__ pl, const CgState *cs, size_t n,
                                                   size_t rstride)
{
    const int rhs = blockIdx.y;
    const double sc = cs[rhs].scale;
    const size_t ro = (size_t)rhs * rstride;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const cpx<double> v = b64[ro + t];
        cpx<Sl> w;
        w.re = conv<Sl>::from_f64(sc * v.re);
        w.im = conv<Sl>::from_f64(sc * v.im);
        rl[ro + t] = w;
        pl[ro + t] = w;
    }
}

hipError_t launch_seed(int dt_lo, const double *b64, void *r_lo, void *p_lo, const CgState *cs, size_t elems,
                       size_t rstride, int n_rhs, hipStream_t st)
{
    bool ok = dispatch_dtype(dt_lo, [&](auto sv) {
        typedef decltype(sv) Sl;
        seed_kernel<Sl><<<dim3(vec_grid(elems), n_rhs), WG, 0, st>>>((const cpx<double> *)b64, (cpx<Sl> *)r_lo,
                                                                     (cpx<Sl> *)p_lo, cs, elems, rstride);
    });
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// plain CG restart of the systems a true-residual check re-activated
// (due[rhs] && active[rhs]): r = p = r64
__global__ void __launch_bounds__(WG) restart_kernel(const cpx<double> *__restrict__ r64, cpx<double> *__restrict__ r,
                                                      cpx<double> *__restrict__ p, const int *due, const int *active,
                                                      size_t n, size_t rstride)
{
    const int rhs = blockIdx.y;
    if (!due[rhs] || !active[rhs]) return;
    const size_t ro = (size_t)rhs * rstride;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const cpx<double> v = r64[ro + t];
        r[ro + t] = v;
        p[ro + t] = v;
    }
}

hipError_t launch_restart(const double *r64, double *r, double *p, const int *due, const int *active, size_t elems,
                          size_t rstride, int n_rhs, hipStream_t st)
{
    restart_kernel<<<dim3(vec_grid(elems), n_rhs), WG, 0, st>>>((const cpx<double> *)r64, (cpx<double> *)r,
                                                                (cpx<double> *)p, due, active, elems, rstride);
    return hipGetLastError();
}

// ------------------------------------------------------------------ second stage + CG scalars

// sum of nparts partials of one rhs, in a fixed order; valid in thread 0
static __device__ double sum_parts(const double *partial, int nparts, double *sh)
{
    return block_sum(strided_sum(partial, threadIdx.x, nparts, blockDim.x), sh);
}

__global__ void __launch_bounds__(WG) sum_partials_kernel(const double *partial, int pstride, int nparts,
                                                           double *out)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    const double s = sum_parts(partial + (size_t)rhs * pstride, nparts, sh);
    if (threadIdx.x == 0) out[rhs] = s;
}

hipError_t launch_sum_partials(const double *partial, int pstride, int nparts, int n_rhs, double *out,
                               hipStream_t st)
{
    sum_partials_kernel<<<n_rhs, WG, 0, st>>>(partial, pstride, nparts, out);
    return hipGetLastError();
}

__global__ void __launch_bounds__(WG) cg_init_kernel(CgState *cs, const double *partial, int pstride,
                                                      int nparts, double tol, double scale_numer, int *active_out)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    const double s = sum_parts(partial + (size_t)rhs * pstride, nparts, sh);
    if (threadIdx.x == 0) {
        CgState c;
        c.scale = (scale_numer > 0 && s > 0 && !isinf(s)) ? sqrt(scale_numer / s) : 1.0;
        c.scale_prev = c.scale;
        c.rr = s * c.scale * c.scale;
        c.rr0 = s;
        c.pap = 0;
        c.alpha = 0;
        c.beta = 0;
        c.tol2 = tol * tol * s;
        c.rr_true = s;
        c.rr_last = c.rr;
        c.iters = 0;
        c.restarts = 0;
        c.updates = 0;
        c.since = 0;
        if (!(s == s) || isinf(s)) {
            c.status = CG_BREAKDOWN;
            c.active = 0;
        } else if (s == 0) {
            c.status = CG_DONE;
            c.active = 0;
        } else {
            c.status = CG_RUNNING;
            c.active = 1;
        }
        cs[rhs] = c;
        active_out[rhs] = c.active;
    }
}

hipError_t launch_cg_init(CgState *cs, const double *partial, int pstride, int nparts, int n_rhs,
                          double tol, double scale_numer, int *active_out, hipStream_t st)
{
    cg_init_kernel<<<n_rhs, WG, 0, st>>>(cs, partial, pstride, nparts, tol, scale_numer, active_out);
    return hipGetLastError();
}

__global__ void __launch_bounds__(WG) cg_alpha_kernel(CgState *cs, const double *partial, int pstride,
                                                       int nparts, double *alpha_out)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    cg_alpha_step(cs, partial + (size_t)rhs * pstride, nparts, alpha_out, rhs, sh);
}

hipError_t launch_cg_alpha(CgState *cs, const double *partial, int pstride, int nparts, int n_rhs,
                           double *alpha_out, hipStream_t st)
{
    cg_alpha_kernel<<<n_rhs, WG, 0, st>>>(cs, partial, pstride, nparts, alpha_out);
    return hipGetLastError();
}

// The beta step sits on the critical path of every CG iteration (the x / p
// update waits for it), so its partial sums are read by 1024 threads (four
// rounds of eight loads each at 32^4 instead of sixteen; 10.6 -> ~4 us); the
// summation order is fixed by that workgroup size.
constexpr int BETA_THREADS = 1024;

__global__ void __launch_bounds__(BETA_THREADS) cg_beta_kernel(CgState *cs, const double *partial, int pstride,
                                                               int nparts, int max_iter, ReliableSchedule sched,
                                                               double *beta_out, int *active_out, int *advanced_out,
                                                               volatile int *host_active)
{
    __shared__ double sh[BETA_THREADS / 64];
    const int rhs = blockIdx.x;
    const double rr_new = sum_parts(partial + (size_t)rhs * pstride, nparts, sh);
    if (threadIdx.x == 0) {
        CgState c = cs[rhs];
        advanced_out[rhs] = c.active;
        if (c.active) {
            c.iters += 1;
            c.since += 1;
            c.beta = rr_new / c.rr;
            c.rr = rr_new;
            if (!(rr_new == rr_new) || isinf(rr_new)) {
                c.status = CG_BREAKDOWN;
                c.active = 0;
            } else if (rr_new <= c.tol2 * c.scale * c.scale) {
                c.status = CG_RECURSIVE_DONE;
                c.active = 0;
            } else if (c.iters >= max_iter) {
                c.status = CG_MAXITER;
                c.active = 0;
            } else if ((sched.every > 0 && c.since >= sched.every) ||
                       (sched.delta2 > 0 && rr_new < sched.delta2 * c.rr_last)) {
                c.status = CG_UPDATE_DUE;
                c.active = 0;
            }
        } else {
            c.beta = 0;
        }
        cs[rhs] = c;
        beta_out[rhs] = c.beta;
        active_out[rhs] = c.active;
        // host flag: 1 running, 2 waiting for a reliable update or true-residual
        // check (recursion converged), 0 otherwise
        if (host_active)
            host_active[rhs] = c.active ? 1 : (c.status == CG_UPDATE_DUE || c.status == CG_RECURSIVE_DONE ? 2 : 0);
    }
}

hipError_t launch_cg_beta(CgState *cs, const double *partial, int pstride, int nparts, int n_rhs,
                          int max_iter, ReliableSchedule sched, double *beta_out, int *active_out,
                          int *advanced_out, int *host_active, hipStream_t st)
{
    cg_beta_kernel<<<n_rhs, BETA_THREADS, 0, st>>>(cs, partial, pstride, nparts, max_iter, sched, beta_out, active_out,
                                         advanced_out, host_active);
    return hipGetLastError();
}


template hipError_t launch_copy<double>(const cpx<double> *, cpx<double> *, size_t, hipStream_t);
template hipError_t launch_copy<float>(const cpx<float> *, cpx<float> *, size_t, hipStream_t);
template hipError_t launch_copy<bf16_t>(const cpx<bf16_t> *, cpx<bf16_t> *, size_t, hipStream_t);
template hipError_t launch_copy<f16_t>(const cpx<f16_t> *, cpx<f16_t> *, size_t, hipStream_t);
#define HRW_INST(S)                                                                                     \
    template hipError_t launch_norm2<S>(const cpx<S> *, size_t, size_t, int, double *, int, int,        \
                                        hipStream_t);                                                  \
    template hipError_t launch_residual<S>(const cpx<S> *, const cpx<S> *, cpx<S> *, size_t, size_t, int, \
                                           double *, int, int, hipStream_t);                           \
    template hipError_t launch_cg_xp<S>(const cpx<S> *, cpx<S> *, cpx<S> *, const double *, const double *, \
                                        const int *, size_t, size_t, int, hipStream_t);                       \
    template hipError_t launch_xpay<S>(const cpx<S> *, cpx<S> *, const double *, const int *, size_t,   \
                                       size_t, int, hipStream_t);
HRW_INST(double)
HRW_INST(float)
HRW_INST(bf16_t)
HRW_INST(f16_t)
#undef HRW_INST

}  // namespace hrw
