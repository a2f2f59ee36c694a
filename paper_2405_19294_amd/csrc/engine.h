// Host-side engine of libhrw: resident gauge fields, workspace planning,
// operator applies and the CG driver.  Internal to the library.
#pragma once

#include <mutex>
#include <string>
#include <vector>

#include "../../include/hrw.h"
#include "kernels.h"

struct hrw_gauge {
    int dims[4];
    int nc, rep, nr;
    unsigned mask;
    hrw::Geom g;
    void *blocks[4][2];  // [dtype][output parity] packed hopping blocks (or null)
    void *fblocks[4][2]; // fundamental links in the hopping layout for the fused representation map (or null)
};

// resident clover term of one gauge field (blocks of A and A^-1 per parity)
struct hrw_clover {
    const hrw_gauge *g;
    double kappa, csw;
    unsigned mask;
    void *a[2][2], *inv[2][2];  // [F64 / F32][parity]
};

namespace hrw {

// error reporting (thread-local message)
int fail(int code, const char *fmt, ...);
void clear_error();

#define HRW_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return ::hrw::fail(HRW_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// bump allocator over a caller buffer; with base == nullptr it only measures
struct Arena {
    char *base;
    size_t cap, off;
    // the base is rounded up to 256 bytes; sizes reported to callers carry 256 bytes of slack
    Arena(void *b, size_t c) : base(nullptr), cap(0), off(0)
    {
        if (b) {
            const size_t a = ((size_t)b + 255) & ~(size_t)255;
            const size_t lost = a - (size_t)b;
            base = (char *)a;
            cap = c > lost ? c - lost : 0;
        }
    }
    void *take(size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
    bool fits() const { return off <= cap; }
};

// ------------------------------------------------------------------ timing

struct Timing {
    std::mutex mu;
    bool on = false;
    int every = 1;                  // time one launch in `every` of each class
    long long seen[KC_COUNT] = {};  // launches of each class since enabling
    struct Pending {
        hipEvent_t a, b;
        int kc, kc2;  // kc2: second class credited (-1 = none)
        double bytes;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    long long launches[KC_COUNT] = {};
    double ms[KC_COUNT] = {};
    double bytes[KC_COUNT] = {};
};
Timing &timing();
// record a start event for a launch of class kc (returns false when timing
// is off or this launch is not one of the sampled ones)
bool timed_begin(hipStream_t st, hipEvent_t *ev, int kc);
void timed_end(hipStream_t st, hipEvent_t start, int kc, int kc2, double bytes);
int timing_harvest();

// ------------------------------------------------------------------ operator plumbing

struct Phases {
    double re[4], im[4];
};
Phases make_phases(const double theta[4]);

// algorithmic bytes of one hop launch (min-traffic model)
double hop_bytes(const Geom &g, int nr, int dt, int parity, int epi, int n_rhs, int fused_nc = 0,
                 bool two_rows = false);

// generic hop launch with timing, dtype-erased pointers
struct HopCall {
    int dt = 0;
    int parity = 0;
    bool dagger = false;
    int epi = EPI_PLAIN;
    int n_rhs = 1;
    size_t rstride = 0;
    const void *in[2] = {nullptr, nullptr};
    void *out[2] = {nullptr, nullptr};
    const void *self[2] = {nullptr, nullptr};
    void *r[2] = {nullptr, nullptr};
    void *x[2] = {nullptr, nullptr};
    const void *p[2] = {nullptr, nullptr};
    const double *coef = nullptr;
    const double *alpha = nullptr;
    const int *active = nullptr;
    const int *run = nullptr;  // per rhs: skip sources whose system is not iterating
    double *partial = nullptr;
    int pstride = 0;
    // the CG alpha step on the side of a plain-epilogue launch (see HopArgs)
    CgState *red_cs = nullptr;
    const double *red_partial = nullptr;
    double *red_alpha = nullptr;
    int red_pstride = 0, red_nparts = 0, red_n = 0;
};
int run_hop(const hrw_gauge *g, const Phases &ph, const HopCall &c, hipStream_t st);

// write host values into a device double / int array (by-value kernel argument)
int set_device_doubles(double *dst, const double *vals, int n, hipStream_t st);

// pinned, device-visible host flags for convergence polling
struct HostFlags {
    int *host = nullptr;
    int *dev = nullptr;
    int slot = -1;
};
int host_flags_acquire(HostFlags *f);
void host_flags_release(HostFlags *f);

// ------------------------------------------------------------------ engine entry points

int gauge_storage_bytes(const Geom &g, int nc, int nr, unsigned mask, size_t *bytes);
int apply_workspace(const Geom &g, int nr, int n_rhs, size_t *bytes);
int cg_workspace(const Geom &g, int nr, int n_rhs, const hrw_solve_params *p, size_t *bytes);

int dw_apply(const hrw_gauge *g, double kappa, const double theta[4], int dt, int n_rhs, int dagger,
             const double *in, double *out, void *ws, size_t ws_bytes, hipStream_t st);
int hop_eo_apply(const hrw_gauge *g, int out_parity, const double theta[4], int dt, int n_rhs,
                 int dagger, const double *in, double *out, void *ws, size_t ws_bytes, hipStream_t st);
int deo_apply(const hrw_gauge *g, const double *kappa, const double theta[4], int dt, int n_rhs,
              int dagger, const double *in, double *out, void *ws, size_t ws_bytes, hipStream_t st);
// D_hat in a caller-provided buffer laid out by the compact plan (three half
// fields of dtype dt per source and the coefficients); deo_compact_bytes is
// what that plan needs from a 256-byte aligned base
size_t deo_compact_bytes(const hrw_gauge *g, int dt, int n_rhs);
int deo_apply_compact(const hrw_gauge *g, const double *kappa, const double theta[4], int dt, int n_rhs,
                      int dagger, const double *in, double *out, void *buf, size_t buf_bytes, hipStream_t st);
int cg_solve(const hrw_gauge *g, const hrw_solve_params *p, int n_rhs, const double *kappa,
             const double *b, double *x, hrw_solve_result *res, void *ws, size_t ws_bytes,
             hipStream_t st);
int bicg_workspace(const Geom &g, int nr, int n_rhs, const hrw_solve_params *p, size_t *bytes, bool clover = false);
int bicgstab_solve(const hrw_gauge *g, const hrw_solve_params *p, int n_rhs, const double *kappa,
                   const double *b, double *x, hrw_solve_result *res, void *ws, size_t ws_bytes,
                   hipStream_t st, const hrw_clover *cl = nullptr);
int qmr_g5_solve(const hrw_gauge *g, const hrw_solve_params *p, int n_rhs, const double *kappa, const double *b,
                 double *x, hrw_solve_result *res, void *ws, size_t ws_bytes, hipStream_t st);
int clover_storage_bytes(const hrw_gauge *g, unsigned mask, size_t *bytes);
int clover_create(const hrw_gauge *g, double kappa, double csw, unsigned mask, void *storage, size_t storage_bytes,
                  hipStream_t st, hrw_clover **out);
hipError_t launch_clover_mul(int dt, int nr, const Geom &g, const void *bm, const void *in, void *out, int n_rhs,
                             size_t rstride, hipStream_t st);
int dsw_apply(const hrw_clover *c, const double theta[4], int dt, int n_rhs, int dagger, const double *in,
              double *out, void *ws, size_t ws_bytes, hipStream_t st);
int dsw_eo_apply(const hrw_clover *c, const double theta[4], int dt, int n_rhs, int dagger, const double *in,
                 double *out, void *ws, size_t ws_bytes, hipStream_t st);
int dsw_eo_packed(const hrw_clover *c, const Phases &ph, int dt, int n_rhs, bool dagger, size_t rs, const void *in_e,
                  void *t, void *w, void *u, void *out_e, const double *coef_k2, const int *run, hipStream_t st);
int session_create(const hrw_gauge *g, const hrw_solve_params *prm, int n_slots, void *ws, size_t ws_bytes,
                   hipStream_t st, hrw_cg_session **out);
int session_destroy(hrw_cg_session *s);
int session_load(hrw_cg_session *s, int slot, int n, const double *kappa, const double *b);
int session_step(hrw_cg_session *s, int max_iters, int *running);
int session_slot_state(hrw_cg_session *s, int *state);
int session_read(hrw_cg_session *s, int slot, int n, double *x, hrw_solve_result *res);

}  // namespace hrw
