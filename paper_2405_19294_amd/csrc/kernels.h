// Launch wrappers of libhrw's device kernels (internal to the library).
#pragma once

#include <type_traits>

#include "hrw_internal.h"

namespace hrw {

// ------------------------------------------------------------------ dispatch

// Colour dimensions N_R with compiled hopping kernels.
inline bool nr_supported(int nr) { return nr == 2 || nr == 3 || nr == 4 || nr == 6 || nr == 8; }

template <class F>
inline bool dispatch_nr(int nr, F &&f)
{
    switch (nr) {
    case 2: f(std::integral_constant<int, 2>{}); return true;
    case 3: f(std::integral_constant<int, 3>{}); return true;
    case 4: f(std::integral_constant<int, 4>{}); return true;
    case 6: f(std::integral_constant<int, 6>{}); return true;
    case 8: f(std::integral_constant<int, 8>{}); return true;
    }
    return false;
}

// dtype ids follow enum hrw_dtype
template <class F>
inline bool dispatch_dtype(int dt, F &&f)
{
    switch (dt) {
    case 0: f(double{}); return true;
    case 1: f(float{}); return true;
    case 2: f(bf16_t{}); return true;
    case 3: f(f16_t{}); return true;
    }
    return false;
}

inline size_t dtype_cbytes(int dt)  // bytes of one complex number
{
    return dt == 0 ? 16 : dt == 1 ? 8 : 4;
}

// ------------------------------------------------------------------ hopping kernel

enum Epilogue {
    EPI_PLAIN = 0,  // out = H in
    EPI_AXPY = 1,   // out = self - c H in              (+ optional |out|^2 partials)
    EPI_CG = 2      // q = self - c H in; r -= alpha q; |r|^2 partials (x moves in launch_cg_xp)
};

struct CgState;

// Pointers are per parity: index 0 / 1 = the half field of that parity.
template <class S>
struct HopArgs {
    Geom g;
    int parity;        // output parity, or -1 for both parities in one launch
    int grid_half;     // blocks per parity when parity == -1
    int n_rhs;
    int pad_;
    size_t rstride;    // complex elements between right-hand sides of one field
    const cpx<S> *gauge[2];  // hopping block for output parity 0 / 1
    const cpx<S> *in[2];     // input halves (read at parity 1 - output parity)
    cpx<S> *out[2];
    const cpx<S> *self[2];
    cpx<S> *r[2];
    cpx<S> *x[2];
    const cpx<S> *p[2];
    double ph_re[4], ph_im[4];  // exp(i theta_mu)
    const double *coef;          // device, per rhs: c of the epilogue
    const double *alpha;         // device, per rhs (EPI_CG)
    const int *active;           // device, per rhs: 0 = frozen (EPI_CG leaves r, x)
    const int *run;              // device, per rhs, or null: 0 = skip this source entirely
                                 // (no loads, stores or partial; its outputs keep old values)
    double *partial;             // per-block partial norms, [rhs * pstride + block]
    int pstride;
    int tile_ts;                 // workgroups per time slice (0 = no tiling)
    int tile_c;                  // workgroups per spatial chunk of the walk
    int tile_p;                  // multi-source walk: x1-planes per chunk (<= 1: the chunk is c consecutive workgroups)
    int tile_b;                  // multi-source walk: workgroups per x1-plane of a time slice
    int ngroups;                 // 16-site partial-sum groups per parity
    // the CG alpha step run on the side of a plain-epilogue launch (null: none):
    // red_n systems, their partials of <p, A p> and state, alpha written per system
    CgState *red_cs;
    const double *red_partial;
    double *red_alpha;
    int red_pstride;
    int red_nparts;
    int red_n;
    int stage;                   // one-thread-per-site kernels: stage the input in LDS (see stage_input)
};

// Launch the hopping kernel.  kc_bytes receives the algorithmic bytes.
template <class S>
hipError_t launch_hop(int nr, bool dagger, int epi, const HopArgs<S> &a, hipStream_t st);

// Hopping kernel with the representation map fused in: a.gauge holds the
// fundamental links (packed like the N x N fundamental hopping blocks) and
// each thread builds the rows of U_R it needs in registers, so the link
// stream shrinks by N^2 / N_R^2.  Built for the representations whose rows
// are cheap closed forms: SU(2) adjoint and symmetric, SU(3) symmetric,
// SU(4) antisymmetric.
constexpr bool hop_fused_supported(int nc, int rep)
{
    return (nc == 2 && (rep == 1 || rep == 2)) || (nc == 3 && rep == 2) || (nc == 4 && rep == 3);
}
template <class S>
hipError_t launch_hop_fused(int nc, int rep, bool dagger, int epi, const HopArgs<S> &a, hipStream_t st);
// SU(3) fundamental hop reading two rows of each link (third row rebuilt)
template <class S>
hipError_t launch_hop_su3(bool dagger, int epi, const HopArgs<S> &a, hipStream_t st);

// Whether a single-source hop of a field that keeps its fundamental links
// builds U_R in registers.  Building a row costs about as much arithmetic as
// applying it, so the fused hop does roughly twice the arithmetic of the
// stored-U_R hop.  Measured on MI355X (D_hat, SU(2) adj and SU(4) asym 24^3x48,
// SU(3) sym 32^4): 1.2-1.8x faster in FP64 and 1.3-1.9x in FP32 storage;
// with 16-bit storage the links are already small against the arithmetic and
// only N_R <= 4 still gains (N_R = 6 in FP16: 7% slower), so 16-bit N_R = 6
// hops read the stored U_R.
constexpr bool hop_fused_pays(int nr, int dt) { return dt <= 1 || nr <= 4; }

// Colour rows each thread of the hopping kernel owns (threads per site =
// N_R / rows): the colour-parallel split keeps the registers of the larger
// representations below the spill point (zero scratch for every instance,
// 2-6 waves per SIMD).  FP64 registers are twice as wide, so FP64 splits
// earlier.  Measured at SU(3) sym 32^4 FP32: one thread per site (6 rows)
// beats two threads of 3 rows, 274 vs 321 us per D_hat hop.
constexpr int hop_rows(int nr, int dt)
{
    return dt == 0 ? (nr == 4 ? 2 : nr == 6 ? 3 : nr == 8 ? 1 : nr) : (nr == 8 ? 4 : nr);
}
constexpr int HOP_MAX_G = 8;  // largest threads-per-site of any instance
constexpr int PG_SITES = 16;  // sites per FP64 partial-sum group of the hopping kernels
constexpr int MR_SITES = 16;  // sites per workgroup of the multi-source hopping kernel
constexpr int MR_MAX_THREADS = 256;  // largest multi-source workgroup

// Smallest thread count of a multi-source workgroup with `sites` sites and g
// row threads per site: a whole number of wavefronts and of (site, row group)
// sets, so that every round of items keeps the same site per thread.
inline int mr_unit(int g, int sites) { return sites * g > 64 ? sites * g : 64; }

// Threads of a multi-source workgroup for n_rhs sources.  The sites x g x
// n_rhs (source, site, row group) items run in rounds of `threads` (a
// multiple of mr_unit); the choice maximises blocks_per_cu(threads) x items
// per round, i.e. the busy lanes a CU holds on average.  Ties go to the
// larger workgroup.
template <class F>
inline int mr_threads(int g, int n_rhs, F blocks_per_cu, int sites = MR_SITES)
{
    const long items = (long)sites * g * n_rhs;
    const int unit = mr_unit(g, sites);
    int best = MR_MAX_THREADS;
    double best_score = -1;
    for (int t = MR_MAX_THREADS; t >= unit; t -= 64) {
        if (t % unit) continue;
        const long rounds = (items + t - 1) / t;
        const double score = (double)blocks_per_cu(t) * (double)items / (double)rounds;
        if (score > best_score) {
            best_score = score;
            best = t;
        }
    }
    return best;
}

// Fewest sources for which the multi-source kernel beats one single-source
// launch row per source (measured at 32^4: N_R <= 4 from 3 sources; N_R >= 6
// from 4 in FP64 and from 6 in 32-bit storage, whose single-source kernel is
// relatively faster).
constexpr int mrhs_min_sources(int nr, int dt) { return nr < 6 ? 3 : (dt == 0 ? 4 : 6); }

// Whether a launch with n_rhs sources runs the multi-source kernel (links
// shared through LDS); else one grid row per source re-reads the links.
constexpr bool hop_uses_mrhs(int nr, int dt, int n_rhs)
{
    return n_rhs >= mrhs_min_sources(nr, dt) && (nr / hop_rows(nr, dt)) * MR_SITES <= WG / 2;
}

// Partial sums per parity written by one hopping launch: one per 16-site
// group and source, in the same order for any number of sources, so a
// batched solve reduces exactly like a single one.
inline int hop_groups(const Geom &g) { return (g.half + PG_SITES - 1) / PG_SITES; }

// Blocks per parity of one hop launch (also the number of partials it writes).
inline int hop_grid(const Geom &g, int tps) { return (int)(((long long)g.half * tps + WG - 1) / WG); }
inline int hop_grid_for(const Geom &g, int nr, int dt) { return hop_grid(g, nr / hop_rows(nr, dt)); }

// ------------------------------------------------------------------ layout kernels

// canonical FP64 spinor field(s) -> packed halves.  full: canonical full
// lattice ([rhs][V][4][nr]); otherwise canonical half field of parity `parity`
// ([rhs][V/2][4][nr]).  dst[q] = packed half of parity q (rhs stride rstride).
hipError_t launch_pack_spinor(int dt, int nr, const Geom &g, bool full, int parity, int n_rhs,
                              const double *src, void *dst0, void *dst1, size_t rstride,
                              hipStream_t st);
hipError_t launch_unpack_spinor(int dt, int nr, const Geom &g, bool full, int parity, int n_rhs,
                                const void *src0, const void *src1, size_t rstride, double *dst,
                                hipStream_t st);

// representation map, canonical in and out
hipError_t launch_rep_map(int nc, int rep, long long n_links, const double *uf, double *ur,
                          hipStream_t st);

// fused representation map + packing into the hopping blocks of every dtype in
// mask; blocks[dt][q] = packed block for output parity q (or null).  defect
// (SU(3) fundamental only, else null): receives max |u_2 - conj(u_0 x u_1)|
// over the links, as the bit pattern of a double (cleared first).
hipError_t launch_gauge_pack(int nc, int rep, int nr, const Geom &g, const double *uf,
                             void *const blocks[4][2], hipStream_t st, unsigned long long *defect = nullptr);

// ------------------------------------------------------------------ vector kernels

// all operate on n_rhs fields of `halves` consecutive packed halves each
hipError_t launch_zero(void *dst, size_t bytes, hipStream_t st);
// dst = src (same dtype)
template <class S>
hipError_t launch_copy(const cpx<S> *src, cpx<S> *dst, size_t elems, hipStream_t st);
// dst(Sd) = src(Ss) converted, elementwise over elems complex numbers
hipError_t launch_convert(int dt_src, const void *src, int dt_dst, void *dst, size_t elems,
                          hipStream_t st);

// per-block partials of |a|^2 over n_rhs fields of elems complex each
template <class S>
hipError_t launch_norm2(const cpx<S> *a, size_t elems, size_t rstride, int n_rhs,
                        double *partial, int pstride, int nblocks, hipStream_t st);
// r = b - q, partials of |r|^2
template <class S>
hipError_t launch_residual(const cpx<S> *b, const cpx<S> *q, cpx<S> *r, size_t elems,
                           size_t rstride, int n_rhs, double *partial, int pstride,
                           int nblocks, hipStream_t st);
// p = r + beta p for active rhs
template <class S>
hipError_t launch_xpay(const cpx<S> *r, cpx<S> *p, const double *beta, const int *active,
                       size_t elems, size_t rstride, int n_rhs, hipStream_t st);
// the end of a CG iteration for the rhs with advanced[rhs] != 0:
// x += alpha p, then p = r + beta p (one pass over x, p and r)
template <class S>
hipError_t launch_cg_xp(const cpx<S> *r, cpx<S> *p, cpx<S> *x, const double *alpha, const double *beta,
                        const int *advanced, size_t elems, size_t rstride, int n_rhs, hipStream_t st);
// y += a x  with a per rhs (device), x and y possibly of different dtypes
hipError_t launch_axpy_mixed(int dt_x, const void *x, int dt_y, void *y, const double *a,
                             size_t elems, size_t rstride_x, size_t rstride_y, int n_rhs,
                             hipStream_t st);

// blocks the vector kernels use for `elems` complex numbers per rhs
int vec_grid(size_t elems);

// ------------------------------------------------------------------ CG scalars

struct CgState {      // per right-hand side, device
    double rr;        // |r|^2 (recursive)
    double rr0;       // |b|^2
    double pap;       // <p, A p> = |D p|^2
    double alpha, beta;
    double tol2;      // tol^2 * rr0
    double rr_true;   // last true |r|^2
    double rr_last;   // |r|^2 right after the last reliable update
    double scale;     // inner fields hold scale * (true vectors); 1 unless FP16 storage
    double scale_prev;// scale before the last reliable decision (used by the reseed)
    int status;       // see CgStatus
    int iters;
    int active;       // 1 while the recursion advances
    int restarts;     // re-activations after the recursion had converged
    int updates;      // FP64 true-residual evaluations (reliable updates)
    int since;        // iterations since the last reliable update
};

enum CgStatus { CG_RUNNING = 0, CG_RECURSIVE_DONE = 1, CG_BREAKDOWN = 2, CG_DONE = 3,
                CG_MAXITER = 4, CG_UPDATE_DUE = 5 };

// Reliable-update schedule of one right-hand side: due after `every`
// iterations of its own (0 = never) or once |r| fell below delta |r_last|
// (delta = 0: off).  Each system keeps its own schedule, so its arithmetic
// does not depend on which other systems share the batch.
struct ReliableSchedule {
    int every;
    double delta2;
};

// reduce partials of pap, set alpha (breakdown check)
hipError_t launch_cg_alpha(CgState *st_, const double *partial, int pstride, int nparts,
                           int n_rhs, double *alpha_out, hipStream_t st);
// reduce partials of |r|^2, set beta, advance iteration, recursive convergence;
// host_active (host-mapped, may be null) receives each rhs' active flag
// advanced_out[rhs] = 1 for the systems that took this iteration's step: they
// still complete it with p = r + beta p, even when this kernel stops them.
hipError_t launch_cg_beta(CgState *st_, const double *partial, int pstride, int nparts,
                          int n_rhs, int max_iter, ReliableSchedule sched, double *beta_out,
                          int *active_out, int *advanced_out, int *host_active, hipStream_t st);
// mixed precision, per rhs with due[rhs] != 0: x64 += x_lo / scale, x_lo = 0
hipError_t launch_fold(int dt_lo, void *x_lo, double *x64, const int *due, const CgState *cs,
                       size_t elems, size_t rstride, int n_rhs, hipStream_t st);
// mixed precision, per rhs with due[rhs] != 0 (true vectors: v = v_lo / scale):
// p += r64 - r, then r = r64, both stored in the new scale.  Shifting p by the
// residual correction keeps p = r + beta p_prev valid for the replaced residual.
hipError_t launch_reseed(int dt_lo, const double *r64, void *r_lo, void *p_lo, const int *due,
                         const CgState *cs, size_t elems, size_t rstride, int n_rhs, hipStream_t st);
// initialise: rr0 = sum(partials), status running; scale_numer > 0 picks
// scale = sqrt(scale_numer / rr0) (inner fields of RMS ~1), else scale = 1;
// the recursion's rr is kept in scaled units
hipError_t launch_cg_init(CgState *st_, const double *partial, int pstride, int nparts,
                          int n_rhs, double tol, double scale_numer, int *active_out, hipStream_t st);
// plain CG: r = p = r64 for the systems with due[rhs] && active[rhs]
hipError_t launch_restart(const double *r64, double *r, double *p, const int *due, const int *active,
                          size_t elems, size_t rstride, int n_rhs, hipStream_t st);
// mixed precision start: r_lo = p_lo = round(scale * b)
hipError_t launch_seed(int dt_lo, const double *b64, void *r_lo, void *p_lo, const CgState *cs,
                       size_t elems, size_t rstride, int n_rhs, hipStream_t st);
// plain sum of partials into out[rhs]
hipError_t launch_sum_partials(const double *partial, int pstride, int nparts, int n_rhs,
                               double *out, hipStream_t st);

}  // namespace hrw
