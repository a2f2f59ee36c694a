// extern "C" entry points of libhrw (declared in include/hrw.h).  Each call
// validates its arguments before enqueueing anything and reports failures
// through a status code plus a thread-local message.
#include <string.h>

#include <exception>
#include <mutex>
#include <new>

#include "engine.h"

namespace hrw {
const char *last_error();
}

using namespace hrw;

namespace {

int rep_dim_of(int nc, int rep)
{
    switch (rep) {
    case HRW_REP_FUND: return nc;
    case HRW_REP_ADJ: return nc * nc - 1;
    case HRW_REP_SYM: return nc * (nc + 1) / 2;
    case HRW_REP_ASYM: return nc * (nc - 1) / 2;
    }
    return -1;
}

int check_lattice(const int dims[4])
{
    if (!dims) return fail(HRW_EINVAL, "dims is null");
    long long v = 1;
    for (int m = 0; m < 4; ++m) {
        if (dims[m] < 2 || dims[m] % 2) return fail(HRW_EINVAL, "extent dims[%d] = %d must be even and >= 2", m, dims[m]);
        v *= dims[m];
    }
    if (v / 2 > (1LL << 30)) return fail(HRW_EINVAL, "lattice too large");
    return HRW_OK;
}

int check_group(int nc, int rep, int *nr)
{
    if (nc < 2 || rep < 0 || rep > 3) return fail(HRW_EINVAL, "bad nc %d or rep %d", nc, rep);
    if (nc > 4) return fail(HRW_EUNSUPPORTED, "nc = %d not built (2..4)", nc);
    const int r = rep_dim_of(nc, rep);
    if (r < 2 || !nr_supported(r)) return fail(HRW_EUNSUPPORTED, "representation dimension %d has no kernels", r);
    *nr = r;
    return HRW_OK;
}

int check_dtype(int dt)
{
    if (dt < 0 || dt > 3) return fail(HRW_EINVAL, "bad dtype %d", dt);
    return HRW_OK;
}

int check_storage_mask(int nc, int rep, unsigned mask)
{
    if (!(mask & 0xf) || (mask & ~0x3fu)) return fail(HRW_EINVAL, "bad storage mask 0x%x", mask);
    if ((mask & HRW_STORE_FUND_HOP) && !hop_fused_supported(nc, rep))
        return fail(HRW_EUNSUPPORTED, "the fused representation map is built for SU(2) adj/sym, SU(3) sym, SU(4) asym");
    if ((mask & HRW_STORE_SU3_TWO_ROWS) && !(nc == 3 && rep == HRW_REP_FUND))
        return fail(HRW_EUNSUPPORTED, "two-row links are for SU(3) fundamental fields");
    return HRW_OK;
}

int check_rhs(int n)
{
    if (n < 1 || n > MAX_RHS) return fail(HRW_EINVAL, "n_rhs = %d outside 1..%d", n, MAX_RHS);
    return HRW_OK;
}

template <class F>
int guarded(F &&f)
{
    clear_error();
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return fail(HRW_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(HRW_EDEVICE, "internal error: %s", e.what());
    } catch (...) {
        return fail(HRW_EDEVICE, "internal error");
    }
}

// Device scratch of hrw_deo_apply_noalloc: a file-scope array, so that entry
// point never allocates.  Each GPU the library runs on holds its own copy from
// module load until the process ends.  Host code must not use the array's name
// as a device address (it is a host-side stand-in); it uses the address
// hipGetSymbolAddress returns for the current device instead.
static __device__ __align__(256) unsigned char scratch[HRW_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];

// the current device's address of `scratch`, looked up on its first use on that device
int scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HRW_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(HRW_EDEVICE, "device %d outside 0..%d", dev, MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HRW_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HRW_OK;
}

}  // namespace

extern "C" {

const char *hrw_last_error(void) { return last_error(); }

const char *hrw_version(void) { return "hrw 0.1 gfx950"; }

int hrw_rep_dim(int nc, int rep, int *n_r)
{
    return guarded([&] {
        if (!n_r) return fail(HRW_EINVAL, "n_r is null");
        if (nc < 2 || rep < 0 || rep > 3) return fail(HRW_EINVAL, "bad nc %d or rep %d", nc, rep);
        *n_r = rep_dim_of(nc, rep);
        return HRW_OK;
    });
}

int hrw_rep_map(int nc, int rep, long long n_links, const double *u_f, double *u_r, void *stream)
{
    return guarded([&] {
        if (nc < 2 || rep < 0 || rep > 3 || n_links < 0) return fail(HRW_EINVAL, "bad arguments");
        if (nc > 4) return fail(HRW_EUNSUPPORTED, "nc = %d not built (2..4)", nc);
        if (rep_dim_of(nc, rep) < 2) return fail(HRW_EUNSUPPORTED, "trivial representation");
        if (n_links > 0 && (!u_f || !u_r)) return fail(HRW_EINVAL, "null field pointer");
        HRW_HIP(launch_rep_map(nc, rep, n_links, u_f, u_r, (hipStream_t)stream));
        return HRW_OK;
    });
}

int hrw_gauge_storage_size(const int dims[4], int nc, int rep, unsigned storage_mask, size_t *bytes)
{
    return guarded([&] {
        int nr, rc;
        if ((rc = check_lattice(dims)) || (rc = check_group(nc, rep, &nr))) return rc;
        if (!bytes || (rc = check_storage_mask(nc, rep, storage_mask))) return rc ? rc : fail(HRW_EINVAL, "null output");
        return gauge_storage_bytes(make_geom(dims), nc, nr, storage_mask, bytes);
    });
}

int hrw_gauge_create(const int dims[4], int nc, int rep, const double *u_f, unsigned storage_mask, void *storage,
                     size_t storage_bytes, void *stream, hrw_gauge **out)
{
    return guarded([&] {
        int nr, rc;
        if ((rc = check_lattice(dims)) || (rc = check_group(nc, rep, &nr))) return rc;
        if (!u_f || !storage || !out) return fail(HRW_EINVAL, "null pointer");
        if ((rc = check_storage_mask(nc, rep, storage_mask))) return rc;
        const Geom g = make_geom(dims);
        size_t need;
        gauge_storage_bytes(g, nc, nr, storage_mask, &need);
        if (storage_bytes < need) return fail(HRW_ENOMEM, "storage too small: need %zu bytes", need);
        hrw_gauge *h = new hrw_gauge;
        memset(h, 0, sizeof *h);
        for (int m = 0; m < 4; ++m) h->dims[m] = dims[m];
        h->nc = nc;
        h->rep = rep;
        h->nr = nr;
        h->mask = storage_mask;
        h->g = g;
        Arena ar(storage, storage_bytes);
        for (int d = 0; d < 4; ++d)
            if (storage_mask & (1u << d))
                for (int q = 0; q < 2; ++q) h->blocks[d][q] = ar.take(gauge_block_elems(g, nr) * dtype_cbytes(d));
        if (storage_mask & HRW_STORE_FUND_HOP)
            for (int d = 0; d < 4; ++d)
                if (storage_mask & (1u << d))
                    for (int q = 0; q < 2; ++q) h->fblocks[d][q] = ar.take(gauge_block_elems(g, nc) * dtype_cbytes(d));
        unsigned long long *defect =
            (storage_mask & HRW_STORE_SU3_TWO_ROWS) ? (unsigned long long *)ar.take(sizeof(unsigned long long)) : nullptr;
        // two-row links: the hops rebuild row 2 as conj(row 0 x row 1), exact only for special
        // unitary links, so the packing kernel also measures the links' defect (one host sync)
        hipError_t e = launch_gauge_pack(nc, rep, nr, g, u_f, h->blocks, (hipStream_t)stream, defect);
        // the fundamental links in the same hopping layout (representation map = identity)
        if (e == hipSuccess && (storage_mask & HRW_STORE_FUND_HOP))
            e = launch_gauge_pack(nc, HRW_REP_FUND, nc, g, u_f, h->fblocks, (hipStream_t)stream);
        unsigned long long bits = 0;
        if (e == hipSuccess && defect) {
            e = hipMemcpyAsync(&bits, defect, sizeof bits, hipMemcpyDeviceToHost, (hipStream_t)stream);
            if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
        }
        if (e != hipSuccess) {
            delete h;
            return fail(HRW_EDEVICE, "gauge packing failed: %s", hipGetErrorString(e));
        }
        if (defect) {
            double d;
            memcpy(&d, &bits, sizeof d);
            // FP64 storage: the rebuilt row must match to well below the 1e-13 operator tolerance;
            // otherwise a few units of the most precise stored format
            const double tol = (storage_mask & HRW_STORE_F64)   ? 1e-12
                               : (storage_mask & HRW_STORE_F32) ? 4.0 * 0x1p-24
                               : (storage_mask & HRW_STORE_F16) ? 4.0 * 0x1p-11
                                                                : 4.0 * 0x1p-8;
            if (!(d <= tol)) {
                delete h;
                return fail(HRW_EINVAL,
                            "two-row storage needs special unitary links: max |u_2 - conj(u_0 x u_1)| = %.3e > %.1e",
                            d, tol);
            }
        }
        *out = h;
        return HRW_OK;
    });
}

int hrw_gauge_destroy(hrw_gauge *g)
{
    delete g;
    return HRW_OK;
}

int hrw_gauge_info(const hrw_gauge *g, int dims[4], int *nc, int *rep, int *n_r, unsigned *storage_mask)
{
    if (!g) return fail(HRW_EINVAL, "null gauge");
    if (dims)
        for (int m = 0; m < 4; ++m) dims[m] = g->dims[m];
    if (nc) *nc = g->nc;
    if (rep) *rep = g->rep;
    if (n_r) *n_r = g->nr;
    if (storage_mask) *storage_mask = g->mask;
    return HRW_OK;
}

static int check_params(const hrw_solve_params *p)
{
    if (!p) return fail(HRW_EINVAL, "params is null");
    if (!(p->tol > 0) || p->max_iter < 1) return fail(HRW_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (p->system < 0 || p->system > 4) return fail(HRW_EINVAL, "bad system %d", p->system);
    if (p->inner_dtype < 0 || p->inner_dtype > 3) return fail(HRW_EINVAL, "bad inner dtype %d", p->inner_dtype);
    if (p->reliable_every < 0) return fail(HRW_EINVAL, "reliable_every must be >= 0");
    if (!(p->reliable_delta >= 0 && p->reliable_delta < 1)) return fail(HRW_EINVAL, "reliable_delta must be in [0, 1)");
    return HRW_OK;
}

int hrw_workspace_size(const int dims[4], int nc, int rep, int n_rhs, const hrw_solve_params *params, size_t *bytes)
{
    return guarded([&] {
        int nr, rc;
        if ((rc = check_lattice(dims)) || (rc = check_group(nc, rep, &nr)) || (rc = check_rhs(n_rhs))) return rc;
        if (!bytes) return fail(HRW_EINVAL, "bytes is null");
        const Geom g = make_geom(dims);
        if (!params) return apply_workspace(g, nr, n_rhs, bytes);
        if ((rc = check_params(params))) return rc;
        if (params->system >= HRW_SYS_DHAT_EO) return bicg_workspace(g, nr, n_rhs, params, bytes);
        return cg_workspace(g, nr, n_rhs, params, bytes);
    });
}

static int check_apply(const hrw_gauge *g, int dt, int n_rhs, const void *in, const void *out)
{
    int rc;
    if (!g) return fail(HRW_EINVAL, "null gauge");
    if ((rc = check_dtype(dt)) || (rc = check_rhs(n_rhs))) return rc;
    if (!in || !out) return fail(HRW_EINVAL, "null field pointer");
    if (in == out) return fail(HRW_EINVAL, "in and out must not overlap");
    if (!g->blocks[dt][0]) return fail(HRW_EUNSUPPORTED, "gauge field has no links stored in dtype %d", dt);
    return HRW_OK;
}

int hrw_dw_apply(const hrw_gauge *g, double kappa, const double theta[4], int dtype, int n_rhs, int dagger,
                 const double *in, double *out, void *workspace, size_t ws_bytes, void *stream)
{
    return guarded([&] {
        int rc;
        if ((rc = check_apply(g, dtype, n_rhs, in, out))) return rc;
        if (!workspace) return fail(HRW_EINVAL, "null workspace");
        return dw_apply(g, kappa, theta, dtype, n_rhs, dagger, in, out, workspace, ws_bytes, (hipStream_t)stream);
    });
}

int hrw_hop_eo(const hrw_gauge *g, int out_parity, const double theta[4], int dtype, int n_rhs, int dagger,
               const double *in_half, double *out_half, void *workspace, size_t ws_bytes, void *stream)
{
    return guarded([&] {
        int rc;
        if ((rc = check_apply(g, dtype, n_rhs, in_half, out_half))) return rc;
        if (out_parity != 0 && out_parity != 1) return fail(HRW_EINVAL, "out_parity must be 0 or 1");
        if (!workspace) return fail(HRW_EINVAL, "null workspace");
        return hop_eo_apply(g, out_parity, theta, dtype, n_rhs, dagger, in_half, out_half, workspace, ws_bytes,
                            (hipStream_t)stream);
    });
}

int hrw_deo_apply(const hrw_gauge *g, const double *kappa_per_rhs, const double theta[4], int dtype, int n_rhs,
                  int dagger, const double *in_e, double *out_e, void *workspace, size_t ws_bytes, void *stream)
{
    return guarded([&] {
        int rc;
        if ((rc = check_apply(g, dtype, n_rhs, in_e, out_e))) return rc;
        if (!kappa_per_rhs || !workspace) return fail(HRW_EINVAL, "null kappa or workspace");
        return deo_apply(g, kappa_per_rhs, theta, dtype, n_rhs, dagger, in_e, out_e, workspace, ws_bytes,
                         (hipStream_t)stream);
    });
}

int hrw_deo_apply_noalloc(const hrw_gauge *g, const double *kappa_per_rhs, const double theta[4], int dtype,
                          int n_rhs, int dagger, const double *in_e, double *out_e, void *stream)
{
    return guarded([&] {
        int rc;
        if ((rc = check_apply(g, dtype, n_rhs, in_e, out_e))) return rc;
        if (!kappa_per_rhs) return fail(HRW_EINVAL, "null kappa");
        const size_t need = deo_compact_bytes(g, dtype, n_rhs);
        if (need > HRW_NOALLOC_SCRATCH_BYTES)
            return fail(HRW_ENOMEM, "needs %zu bytes of scratch, the static scratch holds %zu", need,
                        (size_t)HRW_NOALLOC_SCRATCH_BYTES);
        void *buf = nullptr;
        if ((rc = scratch_address(&buf))) return rc;
        return deo_apply_compact(g, kappa_per_rhs, theta, dtype, n_rhs, dagger, in_e, out_e, buf,
                                 HRW_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream);
    });
}

int hrw_cg_solve(const hrw_gauge *g, const hrw_solve_params *params, int n_rhs, const double *kappa_per_rhs,
                 const double *b, double *x, hrw_solve_result *res, void *workspace, size_t ws_bytes, void *stream)
{
    return guarded([&] {
        int rc;
        if (!g) return fail(HRW_EINVAL, "null gauge");
        if ((rc = check_params(params)) || (rc = check_rhs(n_rhs))) return rc;
        if (params->system > HRW_SYS_D_CGNR_EO) return fail(HRW_EINVAL, "CG solves systems 0-2 (normal equations)");
        if (!kappa_per_rhs || !b || !x || !res || !workspace) return fail(HRW_EINVAL, "null pointer");
        if (b == x) return fail(HRW_EINVAL, "b and x must not overlap");
        if (!g->blocks[0][0]) return fail(HRW_EUNSUPPORTED, "CG needs FP64 links (HRW_STORE_F64)");
        if (!g->blocks[params->inner_dtype][0]) return fail(HRW_EUNSUPPORTED, "gauge field lacks links in the inner dtype");
        return cg_solve(g, params, n_rhs, kappa_per_rhs, b, x, res, workspace, ws_bytes, (hipStream_t)stream);
    });
}

static int check_bicg_params(const hrw_solve_params *params, int n_rhs)
{
    int rc;
    if ((rc = check_params(params)) || (rc = check_rhs(n_rhs))) return rc;
    if (params->system != HRW_SYS_DHAT_EO && params->system != HRW_SYS_D_EO)
        return fail(HRW_EINVAL, "BiCGstab solves HRW_SYS_DHAT_EO or HRW_SYS_D_EO, got system %d", params->system);
    if (params->inner_dtype == HRW_F16)
        return fail(HRW_EUNSUPPORTED, "BiCGstab runs with FP64, FP32 or BF16 inner fields");
    return HRW_OK;
}

int hrw_bicgstab_solve(const hrw_gauge *g, const hrw_solve_params *params, int n_rhs, const double *kappa_per_rhs,
                       const double *b, double *x, hrw_solve_result *res, void *workspace, size_t ws_bytes,
                       void *stream)
{
    return guarded([&] {
        int rc;
        if (!g) return fail(HRW_EINVAL, "null gauge");
        if ((rc = check_bicg_params(params, n_rhs))) return rc;
        if (!kappa_per_rhs || !b || !x || !res || !workspace) return fail(HRW_EINVAL, "null pointer");
        if (b == x) return fail(HRW_EINVAL, "b and x must not overlap");
        if (!g->blocks[0][0]) return fail(HRW_EUNSUPPORTED, "BiCGstab needs FP64 links (HRW_STORE_F64)");
        if (!g->blocks[params->inner_dtype][0]) return fail(HRW_EUNSUPPORTED, "gauge field lacks links in the inner dtype");
        return bicgstab_solve(g, params, n_rhs, kappa_per_rhs, b, x, res, workspace, ws_bytes, (hipStream_t)stream);
    });
}

int hrw_qmr_g5_solve(const hrw_gauge *g, const hrw_solve_params *params, int n_rhs, const double *kappa_per_rhs,
                     const double *b, double *x, hrw_solve_result *res, void *workspace, size_t ws_bytes,
                     void *stream)
{
    return guarded([&] {
        int rc;
        if (!g) return fail(HRW_EINVAL, "null gauge");
        if ((rc = check_bicg_params(params, n_rhs))) return rc;
        if (params->inner_dtype != HRW_F64) return fail(HRW_EUNSUPPORTED, "QMR-g5 runs in FP64");
        if (!kappa_per_rhs || !b || !x || !res || !workspace) return fail(HRW_EINVAL, "null pointer");
        if (b == x) return fail(HRW_EINVAL, "b and x must not overlap");
        if (!g->blocks[0][0]) return fail(HRW_EUNSUPPORTED, "QMR-g5 needs FP64 links (HRW_STORE_F64)");
        return qmr_g5_solve(g, params, n_rhs, kappa_per_rhs, b, x, res, workspace, ws_bytes, (hipStream_t)stream);
    });
}

int hrw_clover_storage_size(const hrw_gauge *g, unsigned storage_mask, size_t *bytes)
{
    return guarded([&] {
        if (!g || !bytes) return fail(HRW_EINVAL, "null pointer");
        if (!(storage_mask & 3u) || (storage_mask & ~3u)) return fail(HRW_EINVAL, "clover storage mask: F64 and/or F32");
        return clover_storage_bytes(g, storage_mask, bytes);
    });
}

int hrw_clover_create(const hrw_gauge *g, double kappa, double csw, unsigned storage_mask, void *storage,
                      size_t storage_bytes, void *stream, hrw_clover **out)
{
    return guarded([&] {
        if (!g || !storage || !out) return fail(HRW_EINVAL, "null pointer");
        if (!(storage_mask & 3u) || (storage_mask & ~3u)) return fail(HRW_EINVAL, "clover storage mask: F64 and/or F32");
        if (!(kappa == kappa) || !(csw == csw)) return fail(HRW_EINVAL, "kappa and c_sw must be finite");
        if (!g->blocks[0][0]) return fail(HRW_EUNSUPPORTED, "the clover term is built from FP64 links (HRW_STORE_F64)");
        return clover_create(g, kappa, csw, storage_mask, storage, storage_bytes, (hipStream_t)stream, out);
    });
}

int hrw_clover_destroy(hrw_clover *c)
{
    delete c;
    return HRW_OK;
}

static int check_clover_apply(const hrw_clover *c, int dt, int n_rhs, const void *in, const void *out, const void *ws)
{
    int rc;
    if (!c) return fail(HRW_EINVAL, "null clover");
    if ((rc = check_apply(c->g, dt, n_rhs, in, out))) return rc;
    if (!ws) return fail(HRW_EINVAL, "null workspace");
    if (dt > 1 || !c->a[dt][0]) return fail(HRW_EUNSUPPORTED, "clover blocks not stored in dtype %d", dt);
    return HRW_OK;
}

int hrw_dsw_apply(const hrw_clover *c, const double theta[4], int dtype, int n_rhs, int dagger, const double *in,
                  double *out, void *workspace, size_t ws_bytes, void *stream)
{
    return guarded([&] {
        int rc;
        if ((rc = check_clover_apply(c, dtype, n_rhs, in, out, workspace))) return rc;
        return dsw_apply(c, theta, dtype, n_rhs, dagger, in, out, workspace, ws_bytes, (hipStream_t)stream);
    });
}

int hrw_dsw_eo_apply(const hrw_clover *c, const double theta[4], int dtype, int n_rhs, int dagger,
                     const double *in_e, double *out_e, void *workspace, size_t ws_bytes, void *stream)
{
    return guarded([&] {
        int rc;
        if ((rc = check_clover_apply(c, dtype, n_rhs, in_e, out_e, workspace))) return rc;
        return dsw_eo_apply(c, theta, dtype, n_rhs, dagger, in_e, out_e, workspace, ws_bytes, (hipStream_t)stream);
    });
}

int hrw_clover_workspace_size(const hrw_clover *c, int n_rhs, const hrw_solve_params *params, size_t *bytes)
{
    return guarded([&] {
        int rc;
        if (!c || !bytes) return fail(HRW_EINVAL, "null pointer");
        if ((rc = check_bicg_params(params, n_rhs))) return rc;
        return bicg_workspace(c->g->g, c->g->nr, n_rhs, params, bytes, true);
    });
}

int hrw_clover_bicgstab_solve(const hrw_clover *c, const hrw_solve_params *params, int n_rhs, const double *b,
                              double *x, hrw_solve_result *res, void *workspace, size_t ws_bytes, void *stream)
{
    return guarded([&] {
        int rc;
        if (!c) return fail(HRW_EINVAL, "null clover");
        if ((rc = check_bicg_params(params, n_rhs))) return rc;
        if (!b || !x || !res || !workspace) return fail(HRW_EINVAL, "null pointer");
        if (b == x) return fail(HRW_EINVAL, "b and x must not overlap");
        const int dl = params->inner_dtype;
        if (dl > HRW_F32) return fail(HRW_EUNSUPPORTED, "clover BiCGstab runs with FP64 or FP32 inner fields");
        if (!c->g->blocks[dl][0] || !c->a[dl][0] || !c->a[0][0])
            return fail(HRW_EUNSUPPORTED, "links and clover blocks needed in FP64 and in the inner dtype");
        double k[MAX_RHS];
        for (int j = 0; j < n_rhs; ++j) k[j] = c->kappa;
        return bicgstab_solve(c->g, params, n_rhs, k, b, x, res, workspace, ws_bytes, (hipStream_t)stream, c);
    });
}

int hrw_cg_session_create(const hrw_gauge *g, const hrw_solve_params *params, int n_slots, void *workspace,
                          size_t ws_bytes, void *stream, hrw_cg_session **out)
{
    return guarded([&] {
        int rc;
        if (!g || !out || !workspace) return fail(HRW_EINVAL, "null pointer");
        if ((rc = check_params(params)) || (rc = check_rhs(n_slots))) return rc;
        if (params->system > HRW_SYS_D_CGNR_EO) return fail(HRW_EINVAL, "CG solves systems 0-2 (normal equations)");
        if (!g->blocks[0][0]) return fail(HRW_EUNSUPPORTED, "CG needs FP64 links (HRW_STORE_F64)");
        if (!g->blocks[params->inner_dtype][0]) return fail(HRW_EUNSUPPORTED, "gauge field lacks links in the inner dtype");
        return session_create(g, params, n_slots, workspace, ws_bytes, (hipStream_t)stream, out);
    });
}

int hrw_cg_session_load(hrw_cg_session *s, int slot, int n, const double *kappa, const double *b)
{
    return guarded([&] {
        if (!s || !kappa || !b) return fail(HRW_EINVAL, "null pointer");
        return session_load(s, slot, n, kappa, b);
    });
}

int hrw_cg_session_step(hrw_cg_session *s, int max_iters, int *running)
{
    return guarded([&] {
        if (!s || max_iters < 1) return fail(HRW_EINVAL, "null session or max_iters < 1");
        return session_step(s, max_iters, running);
    });
}

int hrw_cg_session_slots(hrw_cg_session *s, int *state)
{
    return guarded([&] {
        if (!s || !state) return fail(HRW_EINVAL, "null pointer");
        return session_slot_state(s, state);
    });
}

int hrw_cg_session_read(hrw_cg_session *s, int slot, int n, double *x, hrw_solve_result *res)
{
    return guarded([&] {
        if (!s || !x || !res) return fail(HRW_EINVAL, "null pointer");
        return session_read(s, slot, n, x, res);
    });
}

int hrw_cg_session_destroy(hrw_cg_session *s)
{
    return guarded([&] { return session_destroy(s); });
}

int hrw_timing_enable(int on)
{
    Timing &t = timing();
    timing_harvest();
    std::lock_guard<std::mutex> lk(t.mu);
    t.on = on > 0;
    t.every = on > 1 ? on : 1;
    for (int k = 0; k < KC_COUNT; ++k) {
        t.seen[k] = 0;
        t.launches[k] = 0;
        t.ms[k] = 0;
        t.bytes[k] = 0;
    }
    return HRW_OK;
}

int hrw_timing_read(int kernel_class, long long *launches, double *total_ms, double *bytes)
{
    if (kernel_class < 0 || kernel_class >= KC_COUNT) return fail(HRW_EINVAL, "unknown kernel class");
    int rc = timing_harvest();
    if (rc) return rc;
    Timing &t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    if (launches) *launches = t.launches[kernel_class];
    if (total_ms) *total_ms = t.ms[kernel_class];
    if (bytes) *bytes = t.bytes[kernel_class];
    return HRW_OK;
}

}  // extern "C"
