// QMR on the g5-symmetric Lanczos process (QMR-g5, the third inverter family
// of arXiv 2405.19294 Sec. 3.3) for D_hat x_e = b_e or D x = b through the
// even/odd Schur complement.  D_hat^+ = g5 D_hat g5, so D_hat is self-adjoint
// in the indefinite form [a, b] = <a, g5 b> and the two-sided Lanczos process
// takes one operator application per step:
//   alpha_n = [v_n, A v_n] / delta_n,  beta_n = rho_n delta_n / delta_{n-1},
//   w = A v_n - alpha_n v_n - beta_n v_{n-1},  rho_{n+1} = |w|,  v_{n+1} = w / rho_{n+1},
// with delta_n = [v_n, v_n]; the coefficients are real, so the quasi-minimal
// residual update (Givens rotations on the real tridiagonal matrix, three-term
// direction vectors) runs on real scalars.  The true residual is bounded by
// sqrt(k + 1) times the quasi-residual after k steps from the last start; when
// that bound reaches tol |b| (or rho or delta vanishes) the FP64 true residual
// is computed, and above tol the process starts again from it.  (Stopping on
// the quasi-residual alone can stall: a start from a residual at rounding
// level has [v, v] near zero and an almost empty Lanczos step.)
//
// Layout and scheduling follow the BiCGstab driver: packed half fields in the
// caller's workspace (no more than BiCGstab's, so its workspace size serves),
// per-workgroup FP64 partials reduced in a fixed order by one workgroup per
// system that also evaluates the coefficients, convergence flags polled two
// iterations behind the launches.  The Lanczos and direction vectors rotate
// through fixed buffers by pointer exchange on the host (the same exchange for
// every system), so no vector is copied.
#include <math.h>
#include <string.h>

#include <chrono>
#include <utility>
#include <vector>

#include "engine.h"

namespace hrw {

struct QState {        // per right-hand side, device
    double bb, tol2;   // |b|^2, tol^2 |b|^2
    double delta;      // [v_n, v_n]
    double beta;       // beta_n
    double alpha;
    double tau;        // rotated right-hand side, current row
    double c1, s1, c2, s2;      // rotations G_{n-1}, G_{n-2}
    double e, f, rr, ctau;      // direction update of this step: d = (v - f d1 - e d2) / rr, x += ctau d
    double rho_next;
    double rr_true;
    int status, iters, restarts, adv;
    int since;         // steps since the last start
};

static __device__ inline double q_wg_sum(double v, double *sh)
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

static __device__ inline double q_part_sum(const double *partial, int pstride, int nb, int rhs, int k, double *sh)
{
    return q_wg_sum(strided_sum(partial + (size_t)rhs * pstride + (size_t)k * nb, threadIdx.x, nb, blockDim.x), sh);
}

// The packed fields are in the hopping kernels' storage basis (q_s = psi_s -
// psi_{s+2}, q_{s+2} = psi_s + psi_{s+2}, T = sqrt(2) x unitary), in which g5 =
// diag(1, 1, -1, -1) of the chiral basis becomes the exchange of the spin
// pairs (s, s + 2): [a, b] = sum conj(a_s) b_{s+2} + conj(a_{s+2}) b_s.  The
// form and the norms both scale by 2 against the chiral basis, so every
// coefficient of the process is the chiral one.  The loops below run over the
// upper spin pairs (s = 0, 1): index u of the n / 2 of them gives the element
// e of spin s and its partner e + 2 N_R BLK of spin s + 2.
static __device__ inline size_t q_upper(size_t u, int nr)
{
    const size_t half_blk = (size_t)2 * nr * BLK;
    return (u / half_blk) * 2 * half_blk + u % half_blk;
}

#define Q_LOOP(n)                                                                                  \
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (n);                       \
         e += (size_t)gridDim.x * blockDim.x)

// partial of Re [v, w] = Re sum conj(v) g5 w
__global__ void __launch_bounds__(WG) q_jdot_kernel(const cpx<double> *__restrict__ v, const cpx<double> *__restrict__ w,
                                                    const int *active, size_t n, size_t rs, int nr, double *partial,
                                                    int pstride)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t o = (size_t)rhs * rs, pair = (size_t)2 * nr * BLK;
    double s = 0;
    Q_LOOP(n / 2)
    {
        const size_t eu = o + q_upper(e, nr), ed = eu + pair;
        const cpx<double> au = v[eu], ad = v[ed], bu = w[eu], bd = w[ed];
        s += (au.re * bd.re + au.im * bd.im) + (ad.re * bu.re + ad.im * bu.im);
    }
    const double t = q_wg_sum(s, sh);
    if (threadIdx.x == 0) partial[(size_t)rhs * pstride + blockIdx.x] = t;
}

// alpha = [v, A v] / delta; marks the systems that take this step
__global__ void __launch_bounds__(WG) q_alpha_kernel(QState *st, const int *active, const double *partial, int pstride,
                                                     int nb)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    const double s = active[rhs] ? q_part_sum(partial, pstride, nb, rhs, 0, sh) : 0.0;
    if (threadIdx.x == 0) {
        st[rhs].adv = active[rhs];
        if (active[rhs]) st[rhs].alpha = s / st[rhs].delta;
    }
}

// w = w - alpha v - beta vp; partials of |w|^2 and [w, w]
__global__ void __launch_bounds__(WG) q_lanczos_kernel(cpx<double> *__restrict__ w, const cpx<double> *__restrict__ v,
                                                       const cpx<double> *__restrict__ vp, const QState *st,
                                                       const int *active, size_t n, size_t rs, int nr, double *partial,
                                                       int pstride)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.y;
    if (!active[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    const double al = st[rhs].alpha, be = st[rhs].beta;
    const size_t pair = (size_t)2 * nr * BLK;
    double nn = 0, jj = 0;
    Q_LOOP(n / 2)
    {
        double re[2], im[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const size_t x = o + q_upper(e, nr) + h * pair;
            const cpx<double> a = w[x], b = v[x], c = vp[x];
            re[h] = a.re - al * b.re - be * c.re;
            im[h] = a.im - al * b.im - be * c.im;
            w[x] = {re[h], im[h]};
            nn += re[h] * re[h] + im[h] * im[h];
        }
        jj += 2 * (re[0] * re[1] + im[0] * im[1]);
    }
    const double t1 = q_wg_sum(nn, sh), t2 = q_wg_sum(jj, sh);
    if (threadIdx.x == 0) {
        double *p = partial + (size_t)rhs * pstride + blockIdx.x;
        p[0] = t1;
        p[gridDim.x] = t2;
    }
}

// rotations, direction coefficients, the next Lanczos coefficients and the stop decision
__global__ void __launch_bounds__(WG) q_rot_kernel(QState *st, int *active, const double *partial, int pstride, int nb,
                                                   int max_iter, int *host)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    if (!active[rhs]) {
        if (threadIdx.x == 0) host[rhs] = st[rhs].status == CG_UPDATE_DUE ? 2 : 0;
        return;
    }
    const double ww = q_part_sum(partial, pstride, nb, rhs, 0, sh);
    const double wj = q_part_sum(partial, pstride, nb, rhs, 1, sh);
    if (threadIdx.x != 0) return;
    QState c = st[rhs];
    const double rho = sqrt(ww);
    // column of T: beta (row n-1), alpha (row n), rho (row n+1)
    const double e = c.s2 * c.beta;
    const double f0 = c.c2 * c.beta;
    const double f = c.c1 * f0 + c.s1 * c.alpha;
    const double g0 = -c.s1 * f0 + c.c1 * c.alpha;
    const double rr = sqrt(g0 * g0 + ww);
    const double cn = g0 / rr, sn = rho / rr;
    c.e = e;
    c.f = f;
    c.rr = rr;
    c.ctau = cn * c.tau;
    c.tau = -sn * c.tau;
    c.c2 = c.c1;
    c.s2 = c.s1;
    c.c1 = cn;
    c.s1 = sn;
    c.rho_next = rho;
    ++c.iters;
    ++c.since;
    int a = 1;
    const double delta_next = rho > 0 ? wj / ww : 0.0;
    if (!isfinite(rr) || rr == 0) {
        c.ctau = 0;  // no usable step: check and start again
        c.status = CG_UPDATE_DUE;
        a = 0;
    } else if ((c.since + 1) * c.tau * c.tau <= c.tol2 || rho == 0 || !(delta_next == delta_next) ||
               delta_next == 0) {
        c.status = CG_UPDATE_DUE;
        a = 0;
    } else if (c.iters >= max_iter) {
        c.status = CG_MAXITER;
        a = 0;
    } else {
        c.beta = rho * delta_next / c.delta;
        c.delta = delta_next;
    }
    st[rhs] = c;
    active[rhs] = a;
    host[rhs] = a ? 1 : (c.status == CG_UPDATE_DUE ? 2 : 0);
}

// d_new = (v - f d1 - e d2) / rr into d2's buffer; x += ctau d_new; w = w / rho (the next v)
__global__ void __launch_bounds__(WG) q_update_kernel(const cpx<double> *__restrict__ v, const cpx<double> *__restrict__ d1,
                                                      cpx<double> *__restrict__ d2, cpx<double> *__restrict__ x,
                                                      cpx<double> *__restrict__ w, const QState *st, size_t n,
                                                      size_t rs)
{
    const int rhs = blockIdx.y;
    const QState &c = st[rhs];
    if (!c.adv) return;
    const size_t o = (size_t)rhs * rs;
    const double cf = c.f, ce = c.e, inv = 1.0 / c.rr, ct = c.ctau;
    const double sc = c.rho_next > 0 ? 1.0 / c.rho_next : 0.0;
    Q_LOOP(n)
    {
        const cpx<double> vv = v[o + e], a = d1[o + e], b = d2[o + e], xx = x[o + e], ww = w[o + e];
        const double dr = (vv.re - cf * a.re - ce * b.re) * inv, di = (vv.im - cf * a.im - ce * b.im) * inv;
        d2[o + e] = {dr, di};
        x[o + e] = {xx.re + ct * dr, xx.im + ct * di};
        w[o + e] = {ww.re * sc, ww.im * sc};
    }
}

// r = b - q with partials of |r|^2 and [r, r] (systems in due)
__global__ void __launch_bounds__(WG) q_resid_kernel(const cpx<double> *__restrict__ b, const cpx<double> *__restrict__ q,
                                                     cpx<double> *__restrict__ r, const int *due, size_t n, size_t rs,
                                                     int nr, double *partial, int pstride)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.y;
    if (!due[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    const size_t pair = (size_t)2 * nr * BLK;
    double nn = 0, jj = 0;
    Q_LOOP(n / 2)
    {
        double re[2], im[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const size_t x = o + q_upper(e, nr) + h * pair;
            const cpx<double> a = b[x], c = q[x];
            re[h] = a.re - c.re;
            im[h] = a.im - c.im;
            r[x] = {re[h], im[h]};
            nn += re[h] * re[h] + im[h] * im[h];
        }
        jj += 2 * (re[0] * re[1] + im[0] * im[1]);
    }
    const double t1 = q_wg_sum(nn, sh), t2 = q_wg_sum(jj, sh);
    if (threadIdx.x == 0) {
        double *p = partial + (size_t)rhs * pstride + blockIdx.x;
        p[0] = t1;
        p[gridDim.x] = t2;
    }
}

__global__ void q_mark_kernel(const QState *st, int *due, int n, int all)
{
    const int j = threadIdx.x;
    if (j < n) due[j] = all || st[j].status == CG_UPDATE_DUE;
}

// initial start (first = 1) or FP64 check of the due systems: done, breakdown, or a new start from r
__global__ void __launch_bounds__(WG) q_start_kernel(QState *st, int *active, const int *due, const double *partial,
                                                     int pstride, int nb, double tol, int first, int record_only,
                                                     int *host)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    if (!due[rhs]) return;
    const double rr = q_part_sum(partial, pstride, nb, rhs, 0, sh);
    const double rj = q_part_sum(partial, pstride, nb, rhs, 1, sh);
    if (threadIdx.x != 0) return;
    QState c = st[rhs];
    if (first) {
        c = QState{};
        c.bb = rr;
        c.tol2 = tol * tol * rr;
    }
    c.rr_true = rr;
    if (record_only) {
        st[rhs] = c;
        return;
    }
    int a = 0;
    if (!isfinite(rr)) {
        c.status = CG_BREAKDOWN;
    } else if (rr <= c.tol2) {
        c.status = CG_DONE;
    } else if (!first && ++c.restarts > 100) {
        c.status = CG_BREAKDOWN;
    } else {
        // v = r / |r|: delta = [r, r] / |r|^2, tau = |r|
        c.delta = rj / rr;
        c.beta = 0;
        c.tau = sqrt(rr);
        c.c1 = c.c2 = 1;
        c.s1 = c.s2 = 0;
        c.since = 0;
        c.status = CG_RUNNING;
        a = 1;
    }
    c.adv = 0;
    st[rhs] = c;
    active[rhs] = a;
    host[rhs] = a;
}

// v = r / |r|, vp = d1 = d2 = 0 for the systems that start (again)
__global__ void __launch_bounds__(WG) q_seed_kernel(const cpx<double> *__restrict__ r, cpx<double> *__restrict__ v,
                                                    cpx<double> *__restrict__ vp, cpx<double> *__restrict__ d1,
                                                    cpx<double> *__restrict__ d2, const QState *st, const int *due,
                                                    const int *active, size_t n, size_t rs)
{
    const int rhs = blockIdx.y;
    if (!due[rhs] || !active[rhs]) return;
    const size_t o = (size_t)rhs * rs;
    const double s = 1.0 / sqrt(st[rhs].rr_true);
    Q_LOOP(n)
    {
        const cpx<double> a = r[o + e];
        v[o + e] = {a.re * s, a.im * s};
        vp[o + e] = {0.0, 0.0};
        d1[o + e] = {0.0, 0.0};
        d2[o + e] = {0.0, 0.0};
    }
}

// ------------------------------------------------------------------ host

namespace {

struct QPlan {
    size_t H, RS2;
    char *x, *buf[3], *d[2], *o, *b, *r, *q, *o64;  // half fields (rhs stride H)
    char *bfull, *dfull, *efull;                       // HRW_SYS_D_EO (rhs stride 2 H)
    QState *st;
    int *active;  // [0, MAX_RHS) active, [MAX_RHS, 2 MAX_RHS) due
    double *coef_k, *coef_k2, *coef_mk, *scal, *part;
    int nb, pstride;
};

void plan_qmr(Arena &ar, const Geom &g, int nr, int n_rhs, int sys, QPlan &P)
{
    P.H = spinor_elems(g, nr);
    P.RS2 = 2 * P.H;
    const size_t hb = P.H * n_rhs * 16;
    P.x = (char *)ar.take(hb);
    for (auto &p : P.buf) p = (char *)ar.take(hb);
    for (auto &p : P.d) p = (char *)ar.take(hb);
    P.o = (char *)ar.take(hb);
    P.b = (char *)ar.take(hb);
    P.r = (char *)ar.take(hb);
    P.q = (char *)ar.take(hb);
    P.o64 = (char *)ar.take(hb);
    P.bfull = P.dfull = P.efull = nullptr;
    if (sys == HRW_SYS_D_EO) {
        P.bfull = (char *)ar.take(2 * hb);
        P.dfull = (char *)ar.take(2 * hb);
        P.efull = (char *)ar.take(2 * hb);
    }
    P.st = (QState *)ar.take(sizeof(QState) * MAX_RHS);
    P.active = (int *)ar.take(sizeof(int) * 2 * MAX_RHS);
    P.coef_k = (double *)ar.take(sizeof(double) * MAX_RHS);
    P.coef_k2 = (double *)ar.take(sizeof(double) * MAX_RHS);
    P.coef_mk = (double *)ar.take(sizeof(double) * MAX_RHS);
    P.scal = (double *)ar.take(sizeof(double) * 2 * MAX_RHS);
    P.nb = vec_grid(sys == HRW_SYS_D_EO ? 2 * P.H : P.H);
    P.pstride = 2 * P.nb;
    P.part = (double *)ar.take(sizeof(double) * (size_t)P.pstride * n_rhs);
}

struct QRun {
    const hrw_gauge *g;
    QPlan *P;
    Phases ph;
    int n;
    hipStream_t st;
    int nbh;
    int nr;
    double tol;
};

// out = D_hat in (FP64 half fields, rhs stride H)
int q_dhat(QRun &R, const void *in, void *odd, void *out, const int *run)
{
    HopCall a;
    a.dt = 0;
    a.n_rhs = R.n;
    a.rstride = R.P->H;
    a.run = run;
    a.parity = 1;
    a.epi = EPI_PLAIN;
    a.in[0] = in;
    a.out[1] = odd;
    int rc = run_hop(R.g, R.ph, a, R.st);
    if (rc) return rc;
    HopCall b = a;
    b.parity = 0;
    b.epi = EPI_AXPY;
    b.in[0] = nullptr;
    b.out[1] = nullptr;
    b.in[1] = odd;
    b.self[0] = in;
    b.out[0] = out;
    b.coef = R.P->coef_k2;
    return run_hop(R.g, R.ph, b, R.st);
}

// true residual r = b - D_hat x of the systems in due, then start / check
int q_check(QRun &R, int first, int record_only, int *host)
{
    QPlan &P = *R.P;
    const int *due = P.active + MAX_RHS;
    const dim3 grid(R.nbh, R.n);
    int rc = q_dhat(R, P.x, P.o64, P.q, due);
    if (rc) return rc;
    q_resid_kernel<<<grid, WG, 0, R.st>>>((const cpx<double> *)P.b, (const cpx<double> *)P.q, (cpx<double> *)P.r,
                                          due, P.H, P.H, R.nr, P.part, P.pstride);
    HRW_HIP(hipGetLastError());
    q_start_kernel<<<R.n, WG, 0, R.st>>>(P.st, P.active, due, P.part, P.pstride, R.nbh, R.tol, first, record_only,
                                         host);
    HRW_HIP(hipGetLastError());
    return HRW_OK;
}

}  // namespace

int qmr_g5_solve(const hrw_gauge *g, const hrw_solve_params *prm, int n_rhs, const double *kappa, const double *b_in,
                 double *x_out, hrw_solve_result *res, void *ws, size_t ws_bytes, hipStream_t st)
{
    const auto t0 = std::chrono::steady_clock::now();
    Arena ar(ws, ws_bytes);
    QPlan P;
    plan_qmr(ar, g->g, g->nr, n_rhs, prm->system, P);
    if (!ar.fits()) return fail(HRW_ENOMEM, "workspace too small: need %zu bytes, got %zu", ar.off + 256, ws_bytes);
    QRun R{g, &P, make_phases(prm->theta), n_rhs, st, vec_grid(P.H), g->nr, prm->tol};
    int rc;
    double kv[MAX_RHS], k2[MAX_RHS], mk[MAX_RHS];
    for (int j = 0; j < n_rhs; ++j) {
        kv[j] = kappa[j];
        k2[j] = kappa[j] * kappa[j];
        mk[j] = -kappa[j];
    }
    HRW_HIP(launch_zero(ar.base, ar.off, st));
    if ((rc = set_device_doubles(P.coef_k, kv, n_rhs, st))) return rc;
    if ((rc = set_device_doubles(P.coef_k2, k2, n_rhs, st))) return rc;
    if ((rc = set_device_doubles(P.coef_mk, mk, n_rhs, st))) return rc;
    const size_t H = P.H;
    if (prm->system == HRW_SYS_DHAT_EO) {
        HRW_HIP(launch_pack_spinor(0, g->nr, g->g, false, 0, n_rhs, b_in, P.b, nullptr, H, st));
    } else {
        // b'_e = b_e + kappa H_eo b_o
        HRW_HIP(launch_pack_spinor(0, g->nr, g->g, true, 0, n_rhs, b_in, P.bfull, P.bfull + H * 16, P.RS2, st));
        HopCall c;
        c.dt = 0;
        c.n_rhs = n_rhs;
        c.rstride = P.RS2;
        c.parity = 0;
        c.epi = EPI_AXPY;
        c.coef = P.coef_mk;
        c.in[1] = P.bfull + H * 16;
        c.self[0] = P.bfull;
        c.out[0] = P.dfull;
        if ((rc = run_hop(g, R.ph, c, st))) return rc;
        HRW_HIP(hipMemcpy2DAsync(P.b, H * 16, P.dfull, P.RS2 * 16, H * 16, n_rhs, hipMemcpyDeviceToDevice, st));
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
    // start: x = 0, so r = b (the check computes it as b - D_hat 0)
    int *due = P.active + MAX_RHS;
    const dim3 grid(R.nbh, n_rhs);
    // buffer roles: v, vp, w and d1, d2 rotate by pointer exchange
    char *v = P.buf[0], *vp = P.buf[1], *w = P.buf[2], *d1 = P.d[0], *d2 = P.d[1];
    auto seed = [&]() -> int {
        q_seed_kernel<<<grid, WG, 0, st>>>((const cpx<double> *)P.r, (cpx<double> *)v, (cpx<double> *)vp,
                                           (cpx<double> *)d1, (cpx<double> *)d2, P.st, due, P.active, H, H);
        HRW_HIP(hipGetLastError());
        return HRW_OK;
    };
    q_mark_kernel<<<1, 64, 0, st>>>(P.st, due, n_rhs, 1);
    HRW_HIP(hipGetLastError());
    // the first check sets |b|^2 and tol^2 |b|^2 and starts every system with a nonzero finite b
    if ((rc = q_check(R, 1, 0, hf.dev)) || (rc = seed())) return rc;
    HRW_HIP(hipStreamSynchronize(st));
    auto any = [&](int val) {
        for (int j = 0; j < n_rhs; ++j)
            if (hf.host[j] == val) return true;
        return false;
    };
    long long enq = 0;
    for (;;) {
        const long long e0 = enq;
        while (any(1)) {
            if ((rc = q_dhat(R, v, P.o, w, P.active))) return rc;
            q_jdot_kernel<<<grid, WG, 0, st>>>((const cpx<double> *)v, (const cpx<double> *)w, P.active, H, H, R.nr,
                                               P.part, P.pstride);
            HRW_HIP(hipGetLastError());
            q_alpha_kernel<<<n_rhs, WG, 0, st>>>(P.st, P.active, P.part, P.pstride, R.nbh);
            HRW_HIP(hipGetLastError());
            q_lanczos_kernel<<<grid, WG, 0, st>>>((cpx<double> *)w, (const cpx<double> *)v, (const cpx<double> *)vp,
                                                  P.st, P.active, H, H, R.nr, P.part, P.pstride);
            HRW_HIP(hipGetLastError());
            q_rot_kernel<<<n_rhs, WG, 0, st>>>(P.st, P.active, P.part, P.pstride, R.nbh, prm->max_iter, hf.dev);
            HRW_HIP(hipGetLastError());
            q_update_kernel<<<grid, WG, 0, st>>>((const cpx<double> *)v, (const cpx<double> *)d1, (cpx<double> *)d2,
                                                 (cpx<double> *)P.x, (cpx<double> *)w, P.st, H, H);
            HRW_HIP(hipGetLastError());
            // v_{n-1} <- v_n, v_n <- w (scaled), w <- old v_{n-1}; d2 holds the new direction
            char *t = vp;
            vp = v;
            v = w;
            w = t;
            std::swap(d1, d2);
            HRW_HIP(hipEventRecord(ev[enq % 3], st));
            ++enq;
            if (enq - e0 >= 2) {
                HRW_HIP(hipEventSynchronize(ev[(enq - 2) % 3]));
                if (any(2)) break;
            }
        }
        HRW_HIP(hipStreamSynchronize(st));
        if (any(2)) {
            q_mark_kernel<<<1, 64, 0, st>>>(P.st, due, n_rhs, 0);
            HRW_HIP(hipGetLastError());
            if ((rc = q_check(R, 0, 0, hf.dev)) || (rc = seed())) return rc;
            HRW_HIP(hipStreamSynchronize(st));
            continue;
        }
        if (!any(1)) break;
    }
    // final FP64 residual of every system (recorded, no decision)
    q_mark_kernel<<<1, 64, 0, st>>>(P.st, due, n_rhs, 1);
    HRW_HIP(hipGetLastError());
    if ((rc = q_check(R, 0, 1, nullptr))) return rc;
    if (prm->system == HRW_SYS_DHAT_EO) {
        HRW_HIP(launch_unpack_spinor(0, g->nr, g->g, false, 0, n_rhs, P.x, nullptr, H, x_out, st));
    } else {
        HRW_HIP(hipMemcpy2DAsync(P.dfull, P.RS2 * 16, P.x, H * 16, H * 16, n_rhs, hipMemcpyDeviceToDevice, st));
        HopCall c;
        c.dt = 0;
        c.n_rhs = n_rhs;
        c.rstride = P.RS2;
        c.parity = 1;
        c.epi = EPI_AXPY;
        c.coef = P.coef_mk;
        c.in[0] = P.dfull;
        c.self[1] = P.bfull + H * 16;
        c.out[1] = P.dfull + H * 16;
        if ((rc = run_hop(g, R.ph, c, st))) return rc;
        HRW_HIP(launch_unpack_spinor(0, g->nr, g->g, true, 0, n_rhs, P.dfull, P.dfull + H * 16, P.RS2, x_out, st));
        HopCall d;
        d.dt = 0;
        d.n_rhs = n_rhs;
        d.rstride = P.RS2;
        d.parity = -1;
        d.epi = EPI_AXPY;
        d.coef = P.coef_k;
        for (int q = 0; q < 2; ++q) {
            d.in[q] = P.dfull + q * H * 16;
            d.self[q] = P.dfull + q * H * 16;
            d.out[q] = P.efull + q * H * 16;
        }
        if ((rc = run_hop(g, R.ph, d, st))) return rc;
        const int nb2 = vec_grid(2 * H);
        HRW_HIP(launch_residual<double>((const cpx<double> *)P.bfull, (const cpx<double> *)P.efull,
                                        (cpx<double> *)P.dfull, 2 * H, P.RS2, n_rhs, P.part, P.pstride, nb2, st));
        HRW_HIP(launch_sum_partials(P.part, P.pstride, nb2, n_rhs, P.scal, st));
        HRW_HIP(launch_norm2<double>((const cpx<double> *)P.bfull, 2 * H, P.RS2, n_rhs, P.part, P.pstride, nb2, st));
        HRW_HIP(launch_sum_partials(P.part, P.pstride, nb2, n_rhs, P.scal + MAX_RHS, st));
    }
    std::vector<QState> hs(n_rhs);
    HRW_HIP(hipMemcpyAsync(hs.data(), P.st, sizeof(QState) * n_rhs, hipMemcpyDeviceToHost, st));
    double dres[2 * MAX_RHS] = {0};
    if (prm->system == HRW_SYS_D_EO)
        HRW_HIP(hipMemcpyAsync(dres, P.scal, sizeof(double) * 2 * MAX_RHS, hipMemcpyDeviceToHost, st));
    HRW_HIP(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int overall = HRW_OK;
    for (int j = 0; j < n_rhs; ++j) {
        const QState &c = hs[j];
        hrw_solve_result &o = res[j];
        memset(&o, 0, sizeof o);
        o.iters = c.iters;
        o.restarts = c.restarts;
        o.true_rel_resid = c.bb > 0 ? sqrt(c.rr_true / c.bb) : 0.0;
        o.recursive_rel_resid = c.bb > 0 ? fabs(c.tau) / sqrt(c.bb) : 0.0;
        o.d_rel_resid = dres[MAX_RHS + j] > 0 ? sqrt(dres[j] / dres[MAX_RHS + j]) : 0.0;
        o.seconds = secs;
        o.status = c.status == CG_DONE ? HRW_OK : c.status == CG_BREAKDOWN ? HRW_EBREAKDOWN : HRW_NOT_CONVERGED;
        if (o.status == HRW_EBREAKDOWN) overall = HRW_EBREAKDOWN;
        else if (o.status == HRW_NOT_CONVERGED && overall == HRW_OK) overall = HRW_NOT_CONVERGED;
    }
    if (timing().on) timing_harvest();
    return overall;
}

}  // namespace hrw
