// Host engine of libhrw: resident represented gauge fields, operator applies
// and the conjugate-gradient driver (arXiv 2405.19294, Sec. 3.1 operator and
// even/odd preconditioning, Sec. 3.3 CG).
//
// All device memory belongs to the caller: the engine lays its packed fields,
// partial sums and scalars out in the caller's workspace with a bump
// allocator, and the same planner answers the workspace-size queries.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <chrono>

#include "engine.h"

namespace hrw {

// ------------------------------------------------------------------ errors

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}
void clear_error() { g_err[0] = 0; }
const char *last_error() { return g_err; }

// ------------------------------------------------------------------ timing

Timing &timing()
{
    static Timing t;
    return t;
}

// timing events carry no system-scope fence: they only feed hipEventElapsedTime,
// and the fence (an L2 writeback and invalidate) cost ~4 us per record
static hipError_t timing_event(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

bool timed_begin(hipStream_t st, hipEvent_t *ev, int kc)
{
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.on) return false;
    if (t.seen[kc]++ % t.every) return false;
    if (t.pool.empty()) {
        hipEvent_t e;
        if (timing_event(&e) != hipSuccess) return false;
        t.pool.push_back(e);
    }
    *ev = t.pool.back();
    t.pool.pop_back();
    if (hipEventRecord(*ev, st) != hipSuccess) {
        t.pool.push_back(*ev);
        return false;
    }
    return true;
}

void timed_end(hipStream_t st, hipEvent_t start, int kc, int kc2, double bytes)
{
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    hipEvent_t e;
    if (t.pool.empty()) {
        if (timing_event(&e) != hipSuccess) {
            t.pool.push_back(start);
            return;
        }
    } else {
        e = t.pool.back();
        t.pool.pop_back();
    }
    (void)hipEventRecord(e, st);
    t.pending.push_back({start, e, kc, kc2, bytes});
}

int timing_harvest()
{
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    for (auto &p : t.pending) {
        hipError_t e = hipEventSynchronize(p.b);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return fail(HRW_EDEVICE, "timing event: %s", hipGetErrorString(e));
        t.launches[p.kc] += 1;
        t.ms[p.kc] += ms;
        t.bytes[p.kc] += p.bytes;
        if (p.kc2 >= 0) {
            t.launches[p.kc2] += 1;
            t.ms[p.kc2] += ms;
            t.bytes[p.kc2] += p.bytes;
        }
        t.pool.push_back(p.a);
        t.pool.push_back(p.b);
    }
    t.pending.clear();
    return HRW_OK;
}

// ------------------------------------------------------------------ small helpers

Phases make_phases(const double theta[4])
{
    Phases p;
    for (int m = 0; m < 4; ++m) {
        const double t = theta ? theta[m] : 0.0;
        p.re[m] = cos(t);
        p.im[m] = sin(t);
    }
    return p;
}

double hop_bytes(const Geom &g, int nr, int dt, int parity, int epi, int n_rhs, int fused_nc, bool two_rows)
{
    const double sites = (double)g.half * (parity < 0 ? 2 : 1);
    const double cb = (double)dtype_cbytes(dt);
    // the fused representation map streams the N x N fundamental links; the
    // SU(3) two-row hop reads 6 of the 9 entries of each link
    const double links = 8.0 * (fused_nc ? fused_nc * fused_nc : two_rows ? 6 : nr * nr) * cb;
    const double sp = 4.0 * nr * cb;
    double per = sp;  // neighbour spinors (each input spinor once)
    if (epi == EPI_PLAIN) per += sp;            // out
    else if (epi == EPI_AXPY) per += 2 * sp;    // self + out
    else per += 3 * sp;                         // self and r read; r written
    // the multi-source kernel reads each link once for all sources
    const double link_reads = !fused_nc && hop_uses_mrhs(nr, dt, n_rhs) ? 1.0 : (double)n_rhs;
    return (per * n_rhs + links * link_reads) * sites;
}

int run_hop(const hrw_gauge *g, const Phases &ph, const HopCall &c, hipStream_t st)
{
    if (!g->blocks[c.dt][0]) return fail(HRW_EUNSUPPORTED, "gauge field has no links stored in dtype %d", c.dt);
    // single-source launches of a field that keeps its fundamental links build U_R in the hop;
    // the multi-source kernel keeps its LDS copy of the stored U_R
    const int fused_nc =
        (g->fblocks[c.dt][0] && hop_fused_pays(g->nr, c.dt) && !hop_uses_mrhs(g->nr, c.dt, c.n_rhs)) ? g->nc : 0;
    // SU(3) fundamental fields flagged special unitary: single-source hops read two rows per link
    const bool two_rows = !fused_nc && (g->mask & HRW_STORE_SU3_TWO_ROWS) && !hop_uses_mrhs(g->nr, c.dt, c.n_rhs);
    hipEvent_t ev;
    const bool tm = timed_begin(st, &ev, KC_HOP_PLAIN + c.epi);
    hipError_t err = hipErrorInvalidValue;
    dispatch_dtype(c.dt, [&](auto sv) {
        typedef decltype(sv) S;
        HopArgs<S> a;
        memset(&a, 0, sizeof a);
        a.g = g->g;
        a.parity = c.parity;
        a.n_rhs = c.n_rhs;
        a.rstride = c.rstride;
        for (int q = 0; q < 2; ++q) {
            a.gauge[q] = (const cpx<S> *)(fused_nc ? g->fblocks[c.dt][q] : g->blocks[c.dt][q]);
            a.in[q] = (const cpx<S> *)c.in[q];
            a.out[q] = (cpx<S> *)c.out[q];
            a.self[q] = (const cpx<S> *)c.self[q];
            a.r[q] = (cpx<S> *)c.r[q];
            a.x[q] = (cpx<S> *)c.x[q];
            a.p[q] = (const cpx<S> *)c.p[q];
        }
        for (int m = 0; m < 4; ++m) {
            a.ph_re[m] = ph.re[m];
            a.ph_im[m] = ph.im[m];
        }
        a.coef = c.coef;
        a.alpha = c.alpha;
        a.active = c.active;
        a.run = c.run;
        a.partial = c.partial;
        a.pstride = c.pstride;
        a.red_cs = c.red_cs;
        a.red_partial = c.red_partial;
        a.red_alpha = c.red_alpha;
        a.red_pstride = c.red_pstride;
        a.red_nparts = c.red_nparts;
        a.red_n = c.red_n;
        err = fused_nc   ? launch_hop_fused<S>(g->nc, g->rep, c.dagger, c.epi, a, st)
              : two_rows ? launch_hop_su3<S>(c.dagger, c.epi, a, st)
                         : launch_hop<S>(g->nr, c.dagger, c.epi, a, st);
    });
    if (err != hipSuccess) return fail(HRW_EDEVICE, "hop launch failed: %s", hipGetErrorString(err));
    if (tm)
        timed_end(st, ev, KC_HOP, KC_HOP_PLAIN + c.epi,
                  hop_bytes(g->g, g->nr, c.dt, c.parity, c.epi, c.n_rhs, fused_nc, two_rows));
    return HRW_OK;
}

struct DoubleArg {
    double v[MAX_RHS];
};
__global__ void set_doubles_kernel(double *dst, DoubleArg a, int n)
{
    if ((int)threadIdx.x < n) dst[threadIdx.x] = a.v[threadIdx.x];
}

int set_device_doubles(double *dst, const double *vals, int n, hipStream_t st)
{
    if (n > MAX_RHS) return fail(HRW_EINVAL, "too many values");
    DoubleArg a;
    memset(&a, 0, sizeof a);
    for (int k = 0; k < n; ++k) a.v[k] = vals[k];
    set_doubles_kernel<<<1, 64, 0, st>>>(dst, a, n);
    HRW_HIP(hipGetLastError());
    return HRW_OK;
}

// pool of pinned, device-mapped host slots for convergence flags
static std::mutex g_flags_mu;
static int *g_flags_host = nullptr;
static int *g_flags_dev = nullptr;
static std::vector<int> g_flags_free;
constexpr int FLAG_SLOTS = 64;

int host_flags_acquire(HostFlags *f)
{
    std::lock_guard<std::mutex> lk(g_flags_mu);
    if (!g_flags_host) {
        void *p = nullptr;
        HRW_HIP(hipHostMalloc(&p, sizeof(int) * FLAG_SLOTS * MAX_RHS, hipHostMallocMapped));
        void *d = nullptr;
        HRW_HIP(hipHostGetDevicePointer(&d, p, 0));
        g_flags_host = (int *)p;
        g_flags_dev = (int *)d;
        for (int s = FLAG_SLOTS - 1; s >= 0; --s) g_flags_free.push_back(s);
    }
    if (g_flags_free.empty()) return fail(HRW_ENOMEM, "too many concurrent solves");
    f->slot = g_flags_free.back();
    g_flags_free.pop_back();
    f->host = g_flags_host + f->slot * MAX_RHS;
    f->dev = g_flags_dev + f->slot * MAX_RHS;
    return HRW_OK;
}

void host_flags_release(HostFlags *f)
{
    if (f->slot < 0) return;
    std::lock_guard<std::mutex> lk(g_flags_mu);
    g_flags_free.push_back(f->slot);
    f->slot = -1;
}

// ------------------------------------------------------------------ sizes

int gauge_storage_bytes(const Geom &g, int nc, int nr, unsigned mask, size_t *bytes)
{
    Arena ar(nullptr, 0);
    for (int d = 0; d < 4; ++d)
        if (mask & (1u << d))
            for (int q = 0; q < 2; ++q) ar.take(gauge_block_elems(g, nr) * dtype_cbytes(d));
    if (mask & HRW_STORE_FUND_HOP)
        for (int d = 0; d < 4; ++d)
            if (mask & (1u << d))
                for (int q = 0; q < 2; ++q) ar.take(gauge_block_elems(g, nc) * dtype_cbytes(d));
    if (mask & HRW_STORE_SU3_TWO_ROWS) ar.take(sizeof(unsigned long long));  // special-unitarity check
    *bytes = ar.off + 256;
    return HRW_OK;
}

// per-rhs stride of packed fields with `halves` halves each
static size_t half_elems(const Geom &g, int nr) { return spinor_elems(g, nr); }

static int partial_stride(const Geom &g, int nr)
{
    const int a = 2 * hop_groups(g);
    const int b = vec_grid(2 * half_elems(g, nr));
    return a > b ? a : b;
}

struct ApplyPlan {
    void *f[4];   // four full-size (two-half) fields, n_rhs each
    double *coef;
    double *partial;
};

static void plan_apply(Arena &ar, const Geom &g, int nr, int n_rhs, ApplyPlan &pl)
{
    const size_t H = half_elems(g, nr);
    for (int k = 0; k < 4; ++k) pl.f[k] = ar.take(2 * H * n_rhs * 16);
    pl.coef = (double *)ar.take(sizeof(double) * MAX_RHS);
    pl.partial = (double *)ar.take(sizeof(double) * (size_t)partial_stride(g, nr) * n_rhs);
}

int apply_workspace(const Geom &g, int nr, int n_rhs, size_t *bytes)
{
    Arena ar(nullptr, 0);
    ApplyPlan pl;
    plan_apply(ar, g, nr, n_rhs, pl);
    *bytes = ar.off + 256;
    return HRW_OK;
}

// ------------------------------------------------------------------ operator applies

static int check_ws(const Arena &ar, size_t ws_bytes)
{
    if (!ar.fits()) return fail(HRW_ENOMEM, "workspace too small: need %zu bytes, got %zu", ar.off, ws_bytes);
    return HRW_OK;
}

int dw_apply(const hrw_gauge *g, double kappa, const double theta[4], int dt, int n_rhs, int dagger,
             const double *in, double *out, void *ws, size_t ws_bytes, hipStream_t st)
{
    Arena ar(ws, ws_bytes);
    ApplyPlan pl;
    plan_apply(ar, g->g, g->nr, n_rhs, pl);
    int rc = check_ws(ar, ws_bytes);
    if (rc) return rc;
    const size_t H = half_elems(g->g, g->nr);
    const size_t cb = dtype_cbytes(dt);
    char *fi = (char *)pl.f[0], *fo = (char *)pl.f[1];
    HRW_HIP(launch_pack_spinor(dt, g->nr, g->g, true, 0, n_rhs, in, fi, fi + H * cb, 2 * H, st));
    double k[MAX_RHS];
    for (int j = 0; j < n_rhs; ++j) k[j] = kappa;
    rc = set_device_doubles(pl.coef, k, n_rhs, st);
    if (rc) return rc;
    HopCall c;
    c.dt = dt;
    c.parity = -1;
    c.dagger = dagger != 0;
    c.epi = EPI_AXPY;
    c.n_rhs = n_rhs;
    c.rstride = 2 * H;
    for (int q = 0; q < 2; ++q) {
        c.in[q] = fi + q * H * cb;
        c.self[q] = fi + q * H * cb;
        c.out[q] = fo + q * H * cb;
    }
    c.coef = pl.coef;
    rc = run_hop(g, make_phases(theta), c, st);
    if (rc) return rc;
    HRW_HIP(launch_unpack_spinor(dt, g->nr, g->g, true, 0, n_rhs, fo, fo + H * cb, 2 * H, out, st));
    return HRW_OK;
}

int hop_eo_apply(const hrw_gauge *g, int out_parity, const double theta[4], int dt, int n_rhs,
                 int dagger, const double *in, double *out, void *ws, size_t ws_bytes, hipStream_t st)
{
    Arena ar(ws, ws_bytes);
    ApplyPlan pl;
    plan_apply(ar, g->g, g->nr, n_rhs, pl);
    int rc = check_ws(ar, ws_bytes);
    if (rc) return rc;
    const size_t H = half_elems(g->g, g->nr);
    const int ip = 1 - out_parity;
    HRW_HIP(launch_pack_spinor(dt, g->nr, g->g, false, ip, n_rhs, in, ip == 0 ? pl.f[0] : nullptr,
                               ip == 1 ? pl.f[0] : nullptr, H, st));
    HopCall c;
    c.dt = dt;
    c.parity = out_parity;
    c.dagger = dagger != 0;
    c.epi = EPI_PLAIN;
    c.n_rhs = n_rhs;
    c.rstride = H;
    c.in[ip] = pl.f[0];
    c.out[out_parity] = pl.f[1];
    rc = run_hop(g, make_phases(theta), c, st);
    if (rc) return rc;
    HRW_HIP(launch_unpack_spinor(dt, g->nr, g->g, false, out_parity, n_rhs,
                                 out_parity == 0 ? pl.f[1] : nullptr, out_parity == 1 ? pl.f[1] : nullptr,
                                 H, out, st));
    return HRW_OK;
}

// D_hat on caller-provided device buffers: f0 (packed input), f1 (odd
// intermediate), f2 (packed output), each n_rhs half fields of dtype dt, and
// coef (MAX_RHS doubles).  Every entry these kernels read is written first in
// the same call, so the buffers need no clearing between calls.
static int deo_apply_on(const hrw_gauge *g, const double *kappa, const double theta[4], int dt, int n_rhs,
                        int dagger, const double *in, double *out, void *f0, void *f1, void *f2, double *coef,
                        hipStream_t st)
{
    const size_t H = half_elems(g->g, g->nr);
    HRW_HIP(launch_pack_spinor(dt, g->nr, g->g, false, 0, n_rhs, in, f0, nullptr, H, st));
    double k2[MAX_RHS];
    for (int j = 0; j < n_rhs; ++j) k2[j] = kappa[j] * kappa[j];
    int rc = set_device_doubles(coef, k2, n_rhs, st);
    if (rc) return rc;
    const Phases ph = make_phases(theta);
    HopCall c;
    c.dt = dt;
    c.dagger = dagger != 0;
    c.n_rhs = n_rhs;
    c.rstride = H;
    c.parity = 1;
    c.epi = EPI_PLAIN;
    c.in[0] = f0;
    c.out[1] = f1;
    rc = run_hop(g, ph, c, st);
    if (rc) return rc;
    HopCall d;
    d.dt = dt;
    d.dagger = dagger != 0;
    d.n_rhs = n_rhs;
    d.rstride = H;
    d.parity = 0;
    d.epi = EPI_AXPY;
    d.in[1] = f1;
    d.self[0] = f0;
    d.out[0] = f2;
    d.coef = coef;
    rc = run_hop(g, ph, d, st);
    if (rc) return rc;
    HRW_HIP(launch_unpack_spinor(dt, g->nr, g->g, false, 0, n_rhs, f2, nullptr, H, out, st));
    return HRW_OK;
}

int deo_apply(const hrw_gauge *g, const double *kappa, const double theta[4], int dt, int n_rhs,
              int dagger, const double *in, double *out, void *ws, size_t ws_bytes, hipStream_t st)
{
    Arena ar(ws, ws_bytes);
    ApplyPlan pl;
    plan_apply(ar, g->g, g->nr, n_rhs, pl);
    int rc = check_ws(ar, ws_bytes);
    if (rc) return rc;
    return deo_apply_on(g, kappa, theta, dt, n_rhs, dagger, in, out, pl.f[0], pl.f[1], pl.f[2], pl.coef, st);
}

// the compact plan of the allocation-free D_hat: three half fields of dtype dt
// per source and the coefficients, nothing else
static void plan_deo_compact(Arena &ar, const Geom &g, int nr, int dt, int n_rhs, void *f[3], double **coef)
{
    const size_t bytes = half_elems(g, nr) * n_rhs * dtype_cbytes(dt);
    for (int k = 0; k < 3; ++k) f[k] = ar.take(bytes);
    *coef = (double *)ar.take(sizeof(double) * MAX_RHS);
}

size_t deo_compact_bytes(const hrw_gauge *g, int dt, int n_rhs)
{
    Arena ar(nullptr, 0);
    void *f[3];
    double *coef;
    plan_deo_compact(ar, g->g, g->nr, dt, n_rhs, f, &coef);
    return ar.off;
}

int deo_apply_compact(const hrw_gauge *g, const double *kappa, const double theta[4], int dt, int n_rhs,
                      int dagger, const double *in, double *out, void *buf, size_t buf_bytes, hipStream_t st)
{
    Arena ar(buf, buf_bytes);
    void *f[3];
    double *coef;
    plan_deo_compact(ar, g->g, g->nr, dt, n_rhs, f, &coef);
    int rc = check_ws(ar, buf_bytes);
    if (rc) return rc;
    return deo_apply_on(g, kappa, theta, dt, n_rhs, dagger, in, out, f[0], f[1], f[2], coef, st);
}

// ------------------------------------------------------------------ CG

// A packed field: n_rhs slots of `two ? 2 : 1` halves, rhs stride RS elements.
struct Fld {
    char *base = nullptr;
    int dt = 0;
    size_t H = 0;
    bool two = false;
    void *h(int q) const { return base + (two ? (size_t)q * H * dtype_cbytes(dt) : 0); }
};

struct CgPlan {
    int sys;          // hrw_system
    bool mixed;
    int dl;           // inner dtype
    size_t H, RS;     // half elems, rhs stride
    // inner-precision fields
    Fld x, r, p, s, t, u;
    // FP64 fields (b always; x, r and temps for the FP64 operator in mixed mode)
    Fld b, x64, r64, s64, t64, u64, q64;
    // CGNR extras (FP64, two halves): full source, scratch
    Fld bfull, dfull;
    CgState *cs;
    double *alpha, *beta, *coef_k, *coef_k2, *coef_mk, *scal;
    int *active;
    double *pa, *pb;
    int pstride;
};

static Fld take_fld(Arena &ar, int dt, size_t H, bool two, size_t RS, int n_rhs)
{
    Fld f;
    f.dt = dt;
    f.H = H;
    f.two = two;
    f.base = (char *)ar.take(RS * n_rhs * dtype_cbytes(dt));
    return f;
}

static int plan_cg(Arena &ar, const Geom &g, int nr, int n_rhs, const hrw_solve_params *prm, CgPlan &pl)
{
    pl.sys = prm->system;
    pl.dl = prm->inner_dtype;
    pl.mixed = pl.dl != 0;
    pl.H = half_elems(g, nr);
    const bool full = pl.sys == HRW_SYS_DDAG_D_FULL;
    const bool cgnr = pl.sys == HRW_SYS_D_CGNR_EO;
    const bool two = full || cgnr;  // fields carry both parities
    pl.RS = two ? 2 * pl.H : pl.H;
    const size_t H = pl.H, RS = pl.RS;
    // e/o systems keep odd temporaries in their own half-size fields
    auto mk = [&](int dt, bool tw) { return take_fld(ar, dt, H, tw, RS, n_rhs); };
    pl.b = mk(0, two);
    const int di = pl.dl;
    pl.x = mk(di, two);
    pl.r = mk(di, two);
    pl.p = mk(di, two);
    pl.s = mk(di, two);
    if (!full) {
        // odd temporaries: use odd halves of two-half fields in CGNR, own fields otherwise
        pl.t = mk(di, two);
        pl.u = mk(di, two);
    }
    // FP64 true residual and operator output: scratch of the checks, so a check
    // never touches the state of systems that are still iterating
    pl.r64 = mk(0, two);
    pl.q64 = mk(0, two);
    if (pl.mixed) {
        pl.x64 = mk(0, two);
        pl.s64 = mk(0, two);
        if (!full) {
            pl.t64 = mk(0, two);
            pl.u64 = mk(0, two);
        }
    }
    if (cgnr) {
        pl.bfull = mk(0, true);
        pl.dfull = mk(0, true);
    }
    pl.cs = (CgState *)ar.take(sizeof(CgState) * MAX_RHS);
    pl.alpha = (double *)ar.take(sizeof(double) * MAX_RHS);
    pl.beta = (double *)ar.take(sizeof(double) * MAX_RHS);
    pl.coef_k = (double *)ar.take(sizeof(double) * MAX_RHS);
    pl.coef_k2 = (double *)ar.take(sizeof(double) * MAX_RHS);
    pl.coef_mk = (double *)ar.take(sizeof(double) * MAX_RHS);
    pl.scal = (double *)ar.take(sizeof(double) * 4 * MAX_RHS);
    pl.active = (int *)ar.take(sizeof(int) * 3 * MAX_RHS);  // active, due, advanced flags
    pl.pstride = partial_stride(g, nr);
    pl.pa = (double *)ar.take(sizeof(double) * (size_t)pl.pstride * n_rhs);
    pl.pb = (double *)ar.take(sizeof(double) * (size_t)pl.pstride * n_rhs);
    return HRW_OK;
}

int cg_workspace(const Geom &g, int nr, int n_rhs, const hrw_solve_params *p, size_t *bytes)
{
    Arena ar(nullptr, 0);
    CgPlan pl;
    plan_cg(ar, g, nr, n_rhs, p, pl);
    *bytes = ar.off + 256;
    return HRW_OK;
}

struct CgRun {
    const hrw_gauge *g;
    CgPlan *pl;
    Phases ph;
    int n_rhs;
    hipStream_t st;
    bool full() const { return pl->sys == HRW_SYS_DDAG_D_FULL; }
    int nparts_hop() const { return (full() ? 2 : 1) * hop_groups(g->g); }
    size_t elems() const { return full() ? 2 * pl->H : pl->H; }  // active elements per rhs
};

// q = A x with A = D^+ D (full) or D_hat^+ D_hat (e/o); fields share dtype.
static int apply_A(CgRun &R, const Fld &x, const Fld &s, const Fld &t, const Fld &u, const Fld &q)
{
    CgPlan &P = *R.pl;
    HopCall c;
    c.dt = x.dt;
    c.n_rhs = R.n_rhs;
    c.rstride = P.RS;
    int rc;
    if (R.full()) {
        c.parity = -1;
        c.epi = EPI_AXPY;
        c.coef = P.coef_k;
        for (int k = 0; k < 2; ++k) {
            c.in[k] = x.h(k);
            c.self[k] = x.h(k);
            c.out[k] = s.h(k);
        }
        if ((rc = run_hop(R.g, R.ph, c, R.st))) return rc;
        c.dagger = true;
        for (int k = 0; k < 2; ++k) {
            c.in[k] = s.h(k);
            c.self[k] = s.h(k);
            c.out[k] = q.h(k);
        }
        return run_hop(R.g, R.ph, c, R.st);
    }
    HopCall a = c;
    a.parity = 1;
    a.epi = EPI_PLAIN;
    a.in[0] = x.h(0);
    a.out[1] = t.h(1);
    if ((rc = run_hop(R.g, R.ph, a, R.st))) return rc;
    HopCall b = c;
    b.parity = 0;
    b.epi = EPI_AXPY;
    b.coef = P.coef_k2;
    b.in[1] = t.h(1);
    b.self[0] = x.h(0);
    b.out[0] = s.h(0);
    if ((rc = run_hop(R.g, R.ph, b, R.st))) return rc;
    a.dagger = true;
    a.in[0] = s.h(0);
    a.out[1] = u.h(1);
    if ((rc = run_hop(R.g, R.ph, a, R.st))) return rc;
    b.dagger = true;
    b.in[1] = u.h(1);
    b.self[0] = s.h(0);
    b.out[0] = q.h(0);
    return run_hop(R.g, R.ph, b, R.st);
}

// one CG iteration on the inner fields
static int cg_iteration(CgRun &R, int max_iter, ReliableSchedule sched, int *host_active)
{
    CgPlan &P = *R.pl;
    const int dt = P.dl;
    HopCall c;
    c.dt = dt;
    c.n_rhs = R.n_rhs;
    c.rstride = P.RS;
    c.run = P.active;  // systems that are not iterating skip every hop of the iteration
    int rc;
    // q = A p: D p (its |.|^2 partials give <p, A p>), then D^+ of it with the CG update of r
    if (R.full()) {
        HopCall a = c;
        a.parity = -1;
        a.epi = EPI_AXPY;
        a.coef = P.coef_k;
        a.partial = P.pa;
        a.pstride = P.pstride;
        for (int k = 0; k < 2; ++k) {
            a.in[k] = P.p.h(k);
            a.self[k] = P.p.h(k);
            a.out[k] = P.s.h(k);
        }
        if ((rc = run_hop(R.g, R.ph, a, R.st))) return rc;
        HRW_HIP(launch_cg_alpha(P.cs, P.pa, P.pstride, R.nparts_hop(), R.n_rhs, P.alpha, R.st));
        HopCall b = c;
        b.parity = -1;
        b.dagger = true;
        b.epi = EPI_CG;
        b.coef = P.coef_k;
        for (int k = 0; k < 2; ++k) {
            b.in[k] = P.s.h(k);
            b.self[k] = P.s.h(k);
            b.r[k] = P.r.h(k);
        }
        b.alpha = P.alpha;
        b.active = P.active;
        b.partial = P.pb;
        b.pstride = P.pstride;
        if ((rc = run_hop(R.g, R.ph, b, R.st))) return rc;
    } else {
        HopCall a = c;
        a.parity = 1;
        a.epi = EPI_PLAIN;
        a.in[0] = P.p.h(0);
        a.out[1] = P.t.h(1);
        if ((rc = run_hop(R.g, R.ph, a, R.st))) return rc;
        HopCall b = c;
        b.parity = 0;
        b.epi = EPI_AXPY;
        b.coef = P.coef_k2;
        b.in[1] = P.t.h(1);
        b.self[0] = P.p.h(0);
        b.out[0] = P.s.h(0);
        b.partial = P.pa;
        b.pstride = P.pstride;
        if ((rc = run_hop(R.g, R.ph, b, R.st))) return rc;
        // the first hop of D_hat^+ carries the alpha step (the second stage of the
        // <p, A p> reduction): no launch of its own, and alpha is set before the
        // CG hop that needs it
        HopCall d = c;
        d.parity = 1;
        d.dagger = true;
        d.epi = EPI_PLAIN;
        d.in[0] = P.s.h(0);
        d.out[1] = P.u.h(1);
        d.red_cs = P.cs;
        d.red_partial = P.pa;
        d.red_alpha = P.alpha;
        d.red_pstride = P.pstride;
        d.red_nparts = R.nparts_hop();
        d.red_n = R.n_rhs;
        if ((rc = run_hop(R.g, R.ph, d, R.st))) return rc;
        HopCall e = c;
        e.parity = 0;
        e.dagger = true;
        e.epi = EPI_CG;
        e.coef = P.coef_k2;
        e.in[1] = P.u.h(1);
        e.self[0] = P.s.h(0);
        e.r[0] = P.r.h(0);
        e.alpha = P.alpha;
        e.active = P.active;
        e.partial = P.pb;
        e.pstride = P.pstride;
        if ((rc = run_hop(R.g, R.ph, e, R.st))) return rc;
    }
    int *advanced = P.active + 2 * MAX_RHS;
    HRW_HIP(launch_cg_beta(P.cs, P.pb, P.pstride, R.nparts_hop(), R.n_rhs, max_iter, sched, P.beta, P.active,
                           advanced, host_active, R.st));
    // x += alpha p and p = r + beta p in one pass for the systems that took this step
    int err = HRW_OK;
    dispatch_dtype(dt, [&](auto sv) {
        typedef decltype(sv) S;
        if (launch_cg_xp<S>((const cpx<S> *)P.r.h(0), (cpx<S> *)P.p.h(0), (cpx<S> *)P.x.h(0), P.alpha, P.beta,
                            advanced, R.elems(), P.RS, R.n_rhs, R.st) != hipSuccess)
            err = fail(HRW_EDEVICE, "x/p update launch failed");
    });
    return err;
}

// r64 = b - A x64 in FP64 with |r64|^2 partials in pb (plain mode uses the inner fields)
static int true_residual(CgRun &R, const Fld &x, const Fld &r, const Fld &s, const Fld &t, const Fld &u,
                         const Fld &q)
{
    CgPlan &P = *R.pl;
    int rc = apply_A(R, x, s, t, u, q);
    if (rc) return rc;
    const int nb = vec_grid(R.elems());
    HRW_HIP(launch_residual<double>((const cpx<double> *)P.b.h(0), (const cpx<double> *)q.h(0),
                                    (cpx<double> *)r.h(0), R.elems(), P.RS, R.n_rhs, P.pb, P.pstride, nb,
                                    R.st));
    return HRW_OK;
}

// CgState flags -> host after a true-residual check
__global__ void flags_to_host_kernel(const int *active, int *host, int n)
{
    if ((int)threadIdx.x < n) host[threadIdx.x] = active[threadIdx.x];
}

// due[rhs] = 1 for the systems a reliable pass must treat (all of them when `all`)
__global__ void mark_due_kernel(const CgState *cs, int *due, int n, int all)
{
    const int rhs = threadIdx.x;
    if (rhs < n) due[rhs] = all || cs[rhs].status == CG_UPDATE_DUE || cs[rhs].status == CG_RECURSIVE_DONE;
}

// Decision after an FP64 true residual: a due system that meets the
// tolerance is done; otherwise it resumes from the true residual (keeping
// its search direction in mixed precision; plain CG restarts with p = r).
// `record_all` also stores the true residual of systems that are not due
// (the final pass, after every system was folded).
__global__ void __launch_bounds__(WG) cg_reliable_kernel(CgState *cs, const double *partial, int pstride,
                                                          int nparts, const int *due, int *active_out,
                                                          int max_restarts, int record_all, double scale_numer)
{
    __shared__ double sh[WG / 64];
    const int rhs = blockIdx.x;
    double s = strided_sum(partial + (size_t)rhs * pstride, threadIdx.x, nparts, blockDim.x);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double rt = 0;
        for (int k = 0; k < WG / 64; ++k) rt += sh[k];
        CgState c = cs[rhs];
        c.scale_prev = c.scale;
        if (record_all) c.rr_true = rt;
        if (due[rhs] && (c.status == CG_UPDATE_DUE || c.status == CG_RECURSIVE_DONE)) {
            c.rr_true = rt;
            c.updates += 1;
            c.since = 0;
            if (rt <= c.tol2) {
                c.status = CG_DONE;
                c.active = 0;
            } else if (!(rt == rt) || isinf(rt)) {
                c.status = CG_BREAKDOWN;
                c.active = 0;
            } else {
                if (c.status == CG_RECURSIVE_DONE) c.restarts += 1;
                if (c.restarts > max_restarts) {
                    c.status = CG_MAXITER;
                    c.active = 0;
                } else {
                    c.status = CG_RUNNING;
                    c.active = 1;
                    c.scale = scale_numer > 0 ? sqrt(scale_numer / rt) : 1.0;
                    c.rr = rt * c.scale * c.scale;
                    c.rr_last = c.rr;
                }
            }
        }
        cs[rhs] = c;
        active_out[rhs] = c.active;
    }
}

// host flags: 1 running, 2 waiting for a reliable update, 0 otherwise
static bool any_running(const int *host, int n)
{
    for (int j = 0; j < n; ++j)
        if (host[j] == 1) return true;
    return false;
}
static bool any_due(const int *host, int n)
{
    for (int j = 0; j < n; ++j)
        if (host[j] == 2) return true;
    return false;
}

// ------------------------------------------------------------------ sessions

// A view of the plan restricted to slots [slot, slot + n): every field base and
// per-system array is offset, so the routines above run on that range alone.
static CgPlan plan_view(const CgPlan &P, int slot)
{
    CgPlan v = P;
    auto off = [&](Fld &f) {
        if (f.base) f.base += (size_t)slot * P.RS * dtype_cbytes(f.dt);
    };
    for (Fld *f : {&v.x, &v.r, &v.p, &v.s, &v.t, &v.u, &v.b, &v.x64, &v.r64, &v.s64, &v.t64, &v.u64, &v.q64,
                   &v.bfull, &v.dfull})
        off(*f);
    v.cs += slot;
    v.alpha += slot;
    v.beta += slot;
    v.coef_k += slot;
    v.coef_k2 += slot;
    v.coef_mk += slot;
    v.scal += slot;
    v.active += slot;
    v.pa += (size_t)slot * P.pstride;
    v.pb += (size_t)slot * P.pstride;
    return v;
}

__global__ void mark_range_kernel(int *due, int n, int lo, int hi)
{
    const int j = threadIdx.x;
    if (j < n) due[j] = j >= lo && j < hi;
}

// a free slot: inactive, never due, excluded from the running count
__global__ void free_slots_kernel(CgState *cs, int *active, int n)
{
    const int j = threadIdx.x;
    if (j < n) {
        CgState c;
        memset(&c, 0, sizeof c);
        c.status = CG_DONE;
        c.scale = 1.0;
        c.scale_prev = 1.0;
        cs[j] = c;
        active[j] = 0;
    }
}

}  // namespace hrw

struct hrw_cg_session {
    const hrw_gauge *g;
    hrw_solve_params prm;
    int n_slots;
    hipStream_t st;
    hrw::CgPlan P;
    hrw::Phases ph;
    hrw::HostFlags hf;
    hipEvent_t ev[3];
    long long enq;
    hrw::ReliableSchedule sched;
    double scale_numer;
    size_t E;
    int nbv;
    int used[hrw::MAX_RHS];          // 1 while a slot holds a request
    double kappa[hrw::MAX_RHS];
    hrw::CgState host_state[hrw::MAX_RHS];
    std::chrono::steady_clock::time_point t_load[hrw::MAX_RHS];
};

namespace hrw {

static int hi_used(const hrw_cg_session *s)
{
    int h = 0;
    for (int j = 0; j < s->n_slots; ++j)
        if (s->used[j]) h = j + 1;
    return h;
}

static CgRun run_of(hrw_cg_session *s, CgPlan &P, int n)
{
    return CgRun{s->g, &P, s->ph, n, s->st};
}

int session_create(const hrw_gauge *g, const hrw_solve_params *prm, int n_slots, void *ws, size_t ws_bytes,
                   hipStream_t st, hrw_cg_session **out)
{
    Arena ar(ws, ws_bytes);
    CgPlan P;
    plan_cg(ar, g->g, g->nr, n_slots, prm, P);
    int rc = check_ws(ar, ws_bytes);
    if (rc) return rc;
    if (!g->blocks[P.dl][0] || !g->blocks[0][0])
        return fail(HRW_EUNSUPPORTED, "gauge field lacks FP64 links or links in the inner dtype");
    hrw_cg_session *s = new hrw_cg_session;
    s->g = g;
    s->prm = *prm;
    s->n_slots = n_slots;
    s->st = st;
    s->P = P;
    s->ph = make_phases(prm->theta);
    s->enq = 0;
    for (auto &e : s->ev) e = nullptr;
    s->hf = HostFlags();
    s->sched.every = P.mixed ? (prm->reliable_every > 0 ? prm->reliable_every : 50) : 0;
    s->sched.delta2 = P.mixed ? prm->reliable_delta * prm->reliable_delta : 0.0;
    CgRun R = run_of(s, s->P, n_slots);
    s->E = R.elems();
    s->nbv = vec_grid(s->E);
    // FP16 storage keeps each system at RMS ~1 (its range ends near 6e-8); CG is
    // linear, so the inner recursion runs on scaled vectors
    s->scale_numer = P.dl == 3 ? 2.0 * (double)s->E : 0.0;
    for (int j = 0; j < MAX_RHS; ++j) {
        s->used[j] = 0;
        s->kappa[j] = 0;
        memset(&s->host_state[j], 0, sizeof(CgState));
    }
    auto cleanup = [&](int code) {
        for (auto &e : s->ev)
            if (e) (void)hipEventDestroy(e);
        host_flags_release(&s->hf);
        delete s;
        return code;
    };
    if ((rc = host_flags_acquire(&s->hf))) return cleanup(rc);
    for (auto &e : s->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return cleanup(fail(HRW_EDEVICE, "event creation failed"));
    // padding lanes (a half lattice ending in a partial 64-site block) start at zero and so stay
    // finite in the reductions that sweep whole blocks; every other entry is written before it
    // is read (x and x64 are cleared when a system is loaded)
    if (g->g.half % BLK && launch_zero(ar.base, ar.off, st) != hipSuccess)
        return cleanup(fail(HRW_EDEVICE, "workspace clear failed"));
    free_slots_kernel<<<1, 64, 0, st>>>(P.cs, P.active, n_slots);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(HRW_EDEVICE, "slot init failed"));
    for (int j = 0; j < n_slots; ++j) s->hf.host[j] = 0;
    *out = s;
    return HRW_OK;
}

int session_destroy(hrw_cg_session *s)
{
    if (!s) return HRW_OK;
    (void)hipStreamSynchronize(s->st);
    for (auto &e : s->ev)
        if (e) (void)hipEventDestroy(e);
    host_flags_release(&s->hf);
    delete s;
    return HRW_OK;
}

// Load n systems (stacked canonical sources b, one kappa each) into slots
// [slot, slot + n): pack, Schur prologue (CGNR), |b|^2, state and r = p = b.
int session_load(hrw_cg_session *s, int slot, int n, const double *kappa, const double *b_in)
{
    if (slot < 0 || n < 1 || slot + n > s->n_slots) return fail(HRW_EINVAL, "slot range outside the session");
    for (int j = slot; j < slot + n; ++j)
        if (s->used[j]) return fail(HRW_EINVAL, "slot %d is in use", j);
    const hrw_gauge *g = s->g;
    const hipStream_t st = s->st;
    CgPlan V = plan_view(s->P, slot);
    CgRun R = run_of(s, V, n);
    const int nr = g->nr;
    int rc;
    double kv[MAX_RHS], k2[MAX_RHS], mk[MAX_RHS];
    for (int j = 0; j < n; ++j) {
        kv[j] = kappa[j];
        k2[j] = kappa[j] * kappa[j];
        mk[j] = -kappa[j];
        s->kappa[slot + j] = kappa[j];
    }
    if ((rc = set_device_doubles(V.coef_k, kv, n, st))) return rc;
    if ((rc = set_device_doubles(V.coef_k2, k2, n, st))) return rc;
    if ((rc = set_device_doubles(V.coef_mk, mk, n, st))) return rc;
    // fresh solution and residual state for these slots
    for (Fld *f : {&V.x, &V.x64}) {
        if (!f->base) continue;
        HRW_HIP(launch_zero(f->base, (size_t)n * V.RS * dtype_cbytes(f->dt), st));
    }
    if (V.sys == HRW_SYS_DDAG_D_EO) {
        HRW_HIP(launch_pack_spinor(0, nr, g->g, false, 0, n, b_in, V.b.h(0), nullptr, V.RS, st));
    } else if (V.sys == HRW_SYS_DDAG_D_FULL) {
        HRW_HIP(launch_pack_spinor(0, nr, g->g, true, 0, n, b_in, V.b.h(0), V.b.h(1), V.RS, st));
    } else {
        // b'_e = b_e + kappa H_eo b_o, then eta = D_hat^+ b'_e
        HRW_HIP(launch_pack_spinor(0, nr, g->g, true, 0, n, b_in, V.bfull.h(0), V.bfull.h(1), V.RS, st));
        HopCall c;
        c.dt = 0;
        c.n_rhs = n;
        c.rstride = V.RS;
        c.parity = 0;
        c.epi = EPI_AXPY;
        c.coef = V.coef_mk;
        c.in[1] = V.bfull.h(1);
        c.self[0] = V.bfull.h(0);
        c.out[0] = V.dfull.h(0);
        if ((rc = run_hop(g, s->ph, c, st))) return rc;
        HopCall a;
        a.dt = 0;
        a.n_rhs = n;
        a.rstride = V.RS;
        a.parity = 1;
        a.dagger = true;
        a.epi = EPI_PLAIN;
        a.in[0] = V.dfull.h(0);
        a.out[1] = V.dfull.h(1);
        if ((rc = run_hop(g, s->ph, a, st))) return rc;
        HopCall d = a;
        d.parity = 0;
        d.epi = EPI_AXPY;
        d.coef = V.coef_k2;
        d.in[1] = V.dfull.h(1);
        d.self[0] = V.dfull.h(0);
        d.out[0] = V.b.h(0);
        if ((rc = run_hop(g, s->ph, d, st))) return rc;
    }
    const size_t E = s->E;
    HRW_HIP(launch_norm2<double>((const cpx<double> *)V.b.h(0), E, V.RS, n, V.pa, V.pstride, s->nbv, st));
    HRW_HIP(launch_cg_init(V.cs, V.pa, V.pstride, s->nbv, n, s->prm.tol, s->scale_numer, V.active, st));
    if (V.mixed) {
        HRW_HIP(launch_zero(V.x.base, (size_t)n * V.RS * dtype_cbytes(V.dl), st));
        HRW_HIP(launch_seed(V.dl, (const double *)V.b.base, V.r.base, V.p.base, V.cs, E, V.RS, n, st));
    } else {
        HRW_HIP(launch_copy<double>((const cpx<double> *)V.b.base, (cpx<double> *)V.r.base, (size_t)n * V.RS, st));
        HRW_HIP(launch_copy<double>((const cpx<double> *)V.b.base, (cpx<double> *)V.p.base, (size_t)n * V.RS, st));
    }
    HRW_HIP(hipStreamSynchronize(st));
    const auto now = std::chrono::steady_clock::now();
    for (int j = slot; j < slot + n; ++j) {
        s->used[j] = 1;
        s->t_load[j] = now;
        s->hf.host[j] = 1;
    }
    (void)R;
    return HRW_OK;
}

// One reliable pass (plain CG: true-residual check) over the slots [0, n) that are due.
static int reliable_pass(hrw_cg_session *s, int n)
{
    CgPlan &P = s->P;
    CgRun R = run_of(s, P, n);
    const hipStream_t st = s->st;
    const int max_restarts = 20;
    int rc;
    mark_due_kernel<<<1, 64, 0, st>>>(P.cs, P.active + MAX_RHS, n, 0);
    HRW_HIP(hipGetLastError());
    const int *due = P.active + MAX_RHS;
    if (P.mixed) {
        // x64 += x_lo; x_lo = 0; r64 = b - A64 x64; decide; p_lo += r64 - r_lo; r_lo = r64
        HRW_HIP(launch_fold(P.dl, P.x.base, (double *)P.x64.base, due, P.cs, s->E, P.RS, n, st));
        if ((rc = true_residual(R, P.x64, P.r64, P.s64, P.t64, P.u64, P.q64))) return rc;
        cg_reliable_kernel<<<n, WG, 0, st>>>(P.cs, P.pb, P.pstride, s->nbv, due, P.active, max_restarts, 0,
                                             s->scale_numer);
        HRW_HIP(hipGetLastError());
        HRW_HIP(launch_reseed(P.dl, (const double *)P.r64.base, P.r.base, P.p.base, due, P.cs, s->E, P.RS, n, st));
    } else {
        // the iteration's temporaries are free between iterations; r64, q64 are scratch
        if ((rc = true_residual(R, P.x, P.r64, P.s, P.t, P.u, P.q64))) return rc;
        cg_reliable_kernel<<<n, WG, 0, st>>>(P.cs, P.pb, P.pstride, s->nbv, due, P.active, max_restarts, 0, 0.0);
        HRW_HIP(hipGetLastError());
        // re-activated systems restart from their true residual: r = p = r64
        HRW_HIP(launch_restart((const double *)P.r64.h(0), (double *)P.r.h(0), (double *)P.p.h(0), due, P.active,
                               s->E, P.RS, n, st));
    }
    flags_to_host_kernel<<<1, 64, 0, st>>>(P.active, s->hf.dev, n);
    HRW_HIP(hipGetLastError());
    HRW_HIP(hipStreamSynchronize(st));
    return HRW_OK;
}

static int refresh_states(hrw_cg_session *s)
{
    HRW_HIP(hipMemcpyAsync(s->host_state, s->P.cs, sizeof(CgState) * s->n_slots, hipMemcpyDeviceToHost, s->st));
    HRW_HIP(hipStreamSynchronize(s->st));
    return HRW_OK;
}

// Advance every loaded slot by up to max_iters CG iterations (stopping early
// when nothing runs), with the reliable passes that fall due.  *running
// receives the number of slots still iterating.
int session_step(hrw_cg_session *s, int max_iters, int *running)
{
    const int n = hi_used(s);
    int rc;
    auto count = [&]() {
        int c = 0;
        for (int j = 0; j < n; ++j) c += s->used[j] && s->hf.host[j] != 0;
        return c;
    };
    if (n == 0 || (!any_running(s->hf.host, n) && !any_due(s->hf.host, n))) {
        if (running) *running = 0;
        return refresh_states(s);
    }
    CgRun R = run_of(s, s->P, n);
    const int max_iter = s->prm.max_iter > 0 ? s->prm.max_iter : 1;
    int done_iters = 0;
    while (done_iters < max_iters) {
        // iterate until nothing runs, some slot waits for its reliable update, or the budget is spent
        bool need_pass = false;
        int k = 0;
        const long long e0 = s->enq;
        for (; done_iters + k < max_iters; ++k) {
            if (!any_running(s->hf.host, n)) break;
            if ((rc = cg_iteration(R, max_iter, s->sched, s->hf.dev))) return rc;
            HRW_HIP(hipEventRecord(s->ev[s->enq % 3], s->st));
            ++s->enq;
            if (s->enq - e0 >= 2) {
                HRW_HIP(hipEventSynchronize(s->ev[(s->enq - 2) % 3]));
                if (!any_running(s->hf.host, n) || any_due(s->hf.host, n)) {
                    ++k;
                    break;
                }
            }
        }
        done_iters += k;
        HRW_HIP(hipStreamSynchronize(s->st));
        need_pass = any_due(s->hf.host, n) || !any_running(s->hf.host, n);
        if (need_pass) {
            if ((rc = reliable_pass(s, n))) return rc;
        }
        if (!any_running(s->hf.host, n) || k == 0) break;
    }
    if ((rc = refresh_states(s))) return rc;
    if (running) *running = count();
    return HRW_OK;
}

int session_slot_state(hrw_cg_session *s, int *state)
{
    for (int j = 0; j < s->n_slots; ++j) {
        if (!s->used[j]) state[j] = 0;
        else state[j] = (s->hf.host[j] != 0) ? 1 : 2;
    }
    return HRW_OK;
}

// Read slots [slot, slot + n): fold, FP64 residual, (CGNR) reconstruction and
// |b - D x|, unpack into x_out, fill res, and free the slots.
int session_read(hrw_cg_session *s, int slot, int n, double *x_out, hrw_solve_result *res)
{
    if (slot < 0 || n < 1 || slot + n > s->n_slots) return fail(HRW_EINVAL, "slot range outside the session");
    for (int j = slot; j < slot + n; ++j)
        if (!s->used[j]) return fail(HRW_EINVAL, "slot %d holds no request", j);
    const hrw_gauge *g = s->g;
    const hipStream_t st = s->st;
    CgPlan V = plan_view(s->P, slot);
    CgRun R = run_of(s, V, n);
    const int nr = g->nr;
    const size_t H = V.H;
    int rc;
    mark_range_kernel<<<1, 64, 0, st>>>(V.active + MAX_RHS, n, 0, n);
    HRW_HIP(hipGetLastError());
    const int *due = V.active + MAX_RHS;
    // A slot that finished (CG_DONE) got there through an FP64 true-residual check of its
    // current solution (or has b = 0) and has not moved since: its recorded residual is
    // current.  Only when some read slot stopped otherwise is the check run again.
    if ((rc = refresh_states(s))) return rc;
    bool all_done = true;
    for (int j = slot; j < slot + n; ++j) all_done = all_done && s->host_state[j].status == CG_DONE;
    if (V.mixed) HRW_HIP(launch_fold(V.dl, V.x.base, (double *)V.x64.base, due, V.cs, s->E, V.RS, n, st));
    if (!all_done) {
        if (V.mixed) {
            if ((rc = true_residual(R, V.x64, V.r64, V.s64, V.t64, V.u64, V.q64))) return rc;
        } else {
            if ((rc = true_residual(R, V.x, V.r64, V.s, V.t, V.u, V.q64))) return rc;
        }
        // record the FP64 residual of every read slot without changing decisions
        cg_reliable_kernel<<<n, WG, 0, st>>>(V.cs, V.pb, V.pstride, s->nbv, due, V.active, 0, 1, 0.0);
        HRW_HIP(hipGetLastError());
    }
    const Fld &X = V.mixed ? V.x64 : V.x;
    if (V.sys == HRW_SYS_DDAG_D_EO) {
        HRW_HIP(launch_unpack_spinor(0, nr, g->g, false, 0, n, X.h(0), nullptr, V.RS, x_out, st));
    } else if (V.sys == HRW_SYS_DDAG_D_FULL) {
        HRW_HIP(launch_unpack_spinor(0, nr, g->g, true, 0, n, X.h(0), X.h(1), V.RS, x_out, st));
    } else {
        // x_o = b_o + kappa H_oe x_e; then |b - D x| over the full lattice
        HopCall c;
        c.dt = 0;
        c.n_rhs = n;
        c.rstride = V.RS;
        c.parity = 1;
        c.epi = EPI_AXPY;
        c.coef = V.coef_mk;
        c.in[0] = X.h(0);
        c.self[1] = V.bfull.h(1);
        c.out[1] = X.h(1);
        if ((rc = run_hop(g, s->ph, c, st))) return rc;
        HRW_HIP(launch_unpack_spinor(0, nr, g->g, true, 0, n, X.h(0), X.h(1), V.RS, x_out, st));
        HopCall d;
        d.dt = 0;
        d.n_rhs = n;
        d.rstride = V.RS;
        d.parity = -1;
        d.epi = EPI_AXPY;
        d.coef = V.coef_k;
        for (int k = 0; k < 2; ++k) {
            d.in[k] = X.h(k);
            d.self[k] = X.h(k);
            d.out[k] = V.dfull.h(k);
        }
        if ((rc = run_hop(g, s->ph, d, st))) return rc;
        const int nb2 = vec_grid(2 * H);
        HRW_HIP(launch_residual<double>((const cpx<double> *)V.bfull.h(0), (const cpx<double> *)V.dfull.h(0),
                                        (cpx<double> *)V.q64.h(0), 2 * H, V.RS, n, V.pa, V.pstride, nb2, st));
        HRW_HIP(launch_sum_partials(V.pa, V.pstride, nb2, n, V.scal, st));
        HRW_HIP(launch_norm2<double>((const cpx<double> *)V.bfull.h(0), 2 * H, V.RS, n, V.pb, V.pstride, nb2, st));
        HRW_HIP(launch_sum_partials(V.pb, V.pstride, nb2, n, V.scal + MAX_RHS, st));
    }
    std::vector<CgState> hs(n);
    HRW_HIP(hipMemcpyAsync(hs.data(), V.cs, sizeof(CgState) * n, hipMemcpyDeviceToHost, st));
    double dres[2 * MAX_RHS] = {0};
    if (V.sys == HRW_SYS_D_CGNR_EO) {
        HRW_HIP(hipMemcpyAsync(dres, V.scal, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        HRW_HIP(hipMemcpyAsync(dres + MAX_RHS, V.scal + MAX_RHS, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    }
    // the slots are free again: inactive and never due
    free_slots_kernel<<<1, 64, 0, st>>>(V.cs, V.active, n);
    HRW_HIP(hipGetLastError());
    HRW_HIP(hipStreamSynchronize(st));
    const auto now = std::chrono::steady_clock::now();
    int overall = HRW_OK;
    for (int j = 0; j < n; ++j) {
        const CgState &c = hs[j];
        hrw_solve_result &o = res[j];
        o.iters = c.iters;
        o.reliable_updates = V.mixed ? c.updates : 0;
        o.restarts = c.restarts;
        o.true_rel_resid = c.rr0 > 0 ? sqrt(c.rr_true / c.rr0) : 0.0;
        o.recursive_rel_resid = c.rr0 > 0 ? sqrt(c.rr / (c.rr0 * c.scale * c.scale)) : 0.0;
        o.d_rel_resid = (V.sys == HRW_SYS_D_CGNR_EO && dres[MAX_RHS + j] > 0) ? sqrt(dres[j] / dres[MAX_RHS + j])
                                                                            : 0.0;
        o.seconds = std::chrono::duration<double>(now - s->t_load[slot + j]).count();
        o.status = c.status == CG_DONE ? HRW_OK : c.status == CG_BREAKDOWN ? HRW_EBREAKDOWN : HRW_NOT_CONVERGED;
        if (o.status == HRW_EBREAKDOWN) overall = HRW_EBREAKDOWN;
        else if (o.status == HRW_NOT_CONVERGED && overall == HRW_OK) overall = HRW_NOT_CONVERGED;
        s->used[slot + j] = 0;
        s->hf.host[slot + j] = 0;
    }
    if (timing().on) timing_harvest();
    return overall;
}

int cg_solve(const hrw_gauge *g, const hrw_solve_params *prm, int n_rhs, const double *kappa,
             const double *b_in, double *x_out, hrw_solve_result *res, void *ws, size_t ws_bytes,
             hipStream_t st)
{
    hrw_cg_session *s = nullptr;
    int rc = session_create(g, prm, n_rhs, ws, ws_bytes, st, &s);
    if (rc) return rc;
    struct Close {
        hrw_cg_session *s;
        ~Close() { session_destroy(s); }
    } close{s};
    if ((rc = session_load(s, 0, n_rhs, kappa, b_in))) return rc;
    int running = 1;
    while (running > 0)
        if ((rc = session_step(s, 1 << 30, &running))) return rc;
    return session_read(s, 0, n_rhs, x_out, res);
}

}  // namespace hrw
