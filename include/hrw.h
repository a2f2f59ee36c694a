/*
 * hrw.h - C ABI of libhrw, the MI355X (gfx950) library for the Wilson-Dirac
 * operator with fermions in a representation R of SU(N), its even/odd
 * (Schur) form and conjugate-gradient inversion of D^dagger D.
 *
 * Method: arXiv 2405.19294, Sec. 3.1 (Wilson-Dirac operator in single and
 * double precision for general higher representations of SU(N_c), with
 * even/odd preconditioning), Sec. 3.1.2 (spinors carry N_f = N_R colour
 * components, links are N_R x N_R matrices), Sec. 3.2 (site-wise linear
 * algebra and reductions) and Sec. 3.3 (CG).
 *
 * Conventions (the paper leaves them open; these readings are binding):
 *   - Lattice extents dims[0..3]; dims[0] is time; site index lexicographic
 *     with x3 fastest.  Every extent must be even and >= 2 for every call,
 *     the full-lattice ones included: the library keeps every field, and the
 *     hopping blocks of the links, split by parity (Sec. 3.1, even/odd
 *     preconditioning), and a site's index within its parity is its
 *     lexicographic index halved only when all extents are even.  Odd
 *     extents are HRW_EINVAL.
 *   - Euclidean chiral gamma basis, gamma_5 = g0 g1 g2 g3 = diag(1,1,-1,-1):
 *       g0 = [[0,-1],[-1,0]],  gk = [[0,-i s_k],[i s_k,0]]  (2x2 blocks).
 *   - (H psi)(x) = sum_mu ph+_mu(x) (1 - g_mu) U_mu(x) psi(x+mu)
 *                       + ph-_mu(x) (1 + g_mu) U_mu(x-mu)^+ psi(x-mu),
 *     D_W = 1 - kappa H (Wilson r = 1).  ph+_mu(x) = exp(i theta_mu) if
 *     x_mu = N_mu - 1, ph-_mu(x) = exp(-i theta_mu) if x_mu = 0, else 1.
 *     Phases are applied on wrap-crossing hops, never stored in U, so one
 *     resident gauge field serves every theta.  theta = (pi,0,0,0) is
 *     antiperiodic time.
 *   - Even sites: x0+x1+x2+x3 even.  H_eo maps odd to even sites, H_oe even
 *     to odd.  D_hat = 1 - kappa^2 H_eo H_oe acts on even sites.
 *   - Representation bases: adjoint generators T^a = generalised Gell-Mann / 2
 *     (symmetric off-diagonal pairs j<k, antisymmetric pairs j<k, then the
 *     diagonal ones), (U_adj)_ab = 2 Re Tr(T^a U T^b U^+); two-index
 *     symmetric / antisymmetric bases e_(jk) over lexicographic pairs
 *     (j<=k / j<k), normalised to Tr(e^+ e) = 1, acted on by M -> U M U^T.
 *
 * Canonical layout (every pointer argument below, unless stated otherwise):
 *   - interleaved complex FP64 (re, im);
 *   - spinor field [site][spin 4][colour N_R]; n_rhs fields are stacked
 *     [rhs][site][spin][colour];
 *   - gauge field [site][mu 4][row][col], U_mu(x) joins x to x+mu;
 *   - half-parity fields list that parity's sites in lexicographic order.
 * Spin components are those of the chiral basis (g_5 = diag(1, 1, -1, -1)).
 * The library converts to its own device layout internally, and to a spin
 * basis in which g_0 is diagonal (per colour q_s = psi_s - psi_{s+2},
 * q_{s+2} = psi_s + psi_{s+2}); results come back in the chiral basis, so the
 * conversion adds one FP64 rounding each way and, for FP32/16-bit storage,
 * the storage rounding applies to q.
 *
 * Ownership: every field, storage and workspace pointer is device memory owned
 * by the caller (the Python binding takes it from torch).  The library
 * allocates no device memory.  A gauge handle owns only a small host struct;
 * the represented links live in the caller's storage until
 * hrw_gauge_destroy.  Calls are ordered on the caller's HIP stream (NULL =
 * default stream) and return after enqueueing, except hrw_cg_solve, which
 * returns when the solve is complete.
 *
 * Errors: every call returns an int status.  Arguments are validated before
 * anything is enqueued; on a negative status nothing was enqueued (except
 * HRW_EDEVICE, which reports a failed HIP call) and hrw_last_error() returns
 * a message for the calling thread.
 *
 * Environment (read at each hopping-kernel launch):
 *   HRW_TUNE=0       use the occupancy model for the multi-source kernel's
 *                    launch shape instead of timing the candidates (16 or 32
 *                    sites per workgroup x threads x walk chunk and the
 *                    x1-planes it spans) on the first
 *                    plain-epilogue launch of each (sources, extents);
 *                    results are bitwise the same either way;
 *   HRW_TUNE_CACHE   file of tuned launch shapes (JSON, keyed by architecture,
 *                    N_R, row split, storage type, sources and
 *                    ceil(log2(sites per parity))), read before tuning and
 *                    updated after; default $HOME/.cache/hrw/tune.json, an
 *                    empty value keeps the shapes in memory only;
 *   HRW_HOP_STAGE=1  single-source hops with 32-bit or 16-bit storage and
 *                    N_R <= 4 stage their input in LDS and read the x3 and x2
 *                    neighbours from there (slower on MI355X, hence off by
 *                    default); results are bitwise the same either way;
 *   HRW_MRHS_SITES=16|32  pin the multi-source workgroup to that many sites
 *                    (occupancy-model threads, no tuning; bitwise the same
 *                    results);
 *   HRW_MRHS_PLANES=1|2|4|8  pin the x1-planes per chunk of the multi-source
 *                    walk (the order workgroups visit the lattice; bitwise
 *                    the same results);
 *   HRW_MRHS_MFMA=1  run FP32 N_R = 6 launches with >= 6 sources on the
 *                    matrix-core multi-source kernel (results differ from the
 *                    default vector kernel only by FP32 rounding; slower on
 *                    MI355X).
 */
#ifndef HRW_H
#define HRW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define HRW_OK 0
#define HRW_NOT_CONVERGED 1 /* result written, tolerance not reached */
#define HRW_EINVAL (-1)       /* null pointer, bad extent, bad enum value */
#define HRW_EUNSUPPORTED (-2) /* N_c / representation / dtype combination not built */
#define HRW_ENOMEM (-3)       /* storage or workspace smaller than required */
#define HRW_EDEVICE (-4)      /* a HIP call failed */
#define HRW_EBREAKDOWN (-5)   /* CG breakdown: non-finite value or Re<p,Ap> <= 0 */

/* ---------------------------------------------------------------- enums */
enum hrw_rep { HRW_REP_FUND = 0, HRW_REP_ADJ = 1, HRW_REP_SYM = 2, HRW_REP_ASYM = 3 };

/* Precision of link/spinor storage; arithmetic is FP64 for HRW_F64 and FP32
 * for the others (FP32 accumulation for the 16-bit storage formats). */
enum hrw_dtype { HRW_F64 = 0, HRW_F32 = 1, HRW_BF16 = 2, HRW_F16 = 3 };

/* storage_mask bits for hrw_gauge_create: which link precisions to keep */
#define HRW_STORE_F64 (1u << HRW_F64)
#define HRW_STORE_F32 (1u << HRW_F32)
#define HRW_STORE_BF16 (1u << HRW_BF16)
#define HRW_STORE_F16 (1u << HRW_F16)
/* Also keep the fundamental links, in the hopping layout of every precision in
 * the mask, and let single-source hops build the rows of U_R from them in
 * registers (the representation map fused into the hop: the link stream
 * shrinks by N^2 / N_R^2 for extra arithmetic).  Built for SU(2) adjoint and
 * symmetric, SU(3) symmetric and SU(4) antisymmetric; HRW_EUNSUPPORTED for
 * the others.  Results agree with the stored-U_R path to rounding (U_R is
 * evaluated in the arithmetic precision of the hop).  Multi-source launches,
 * and 16-bit-storage hops with N_R = 6 (where the extra arithmetic outweighs
 * the saved bytes), keep using the stored U_R; so on such a field a system's
 * result depends, at rounding level, on how many systems share its launches
 * (the batched == single bitwise guarantee of the solvers and sessions holds
 * only without this flag).  Sec. 3.1.2 (the represented link is built from
 * the fundamental one). */
#define HRW_STORE_FUND_HOP (1u << 4)

/* Storage flag for SU(3) fundamental fields whose links are special unitary:
 * single-source hops read only the first two rows of each link and rebuild
 * the third as conj(u_0 x u_1), 2/3 of the link bytes (the classic two-row
 * compression of SU(3) links; the paper stores full links, Sec. 3.1).  The
 * storage itself keeps all three rows (plus 8 bytes for the check below);
 * multi-source launches read the stored rows.  Because a link that is not
 * special unitary would enter the hops through its rebuilt row,
 * hrw_gauge_create measures max |u_2 - conj(u_0 x u_1)| over all links of
 * u_f (one reduction and a host synchronisation of the stream) and returns
 * HRW_EINVAL when it exceeds 1e-12 with FP64 storage in the mask, else 4
 * units of the most precise stored format.  HRW_EUNSUPPORTED for other
 * groups or representations.  Single-source and batched results differ at
 * rounding level, as for HRW_STORE_FUND_HOP. */
#define HRW_STORE_SU3_TWO_ROWS (1u << 5)

/* Linear systems: 0-2 for hrw_cg_solve (Hermitian positive definite normal
 * equations), 3-4 for hrw_bicgstab_solve (the operator itself). */
enum hrw_system {
    HRW_SYS_DDAG_D_FULL = 0, /* D^+ D x = b on the full lattice                       */
    HRW_SYS_DDAG_D_EO = 1,   /* D_hat^+ D_hat x_e = b_e on the even sites (half field) */
    HRW_SYS_D_CGNR_EO = 2,   /* D x = b on the full lattice via the even/odd Schur
                                complement, CG on its normal equations, and
                                reconstruction of the odd sites                     */
    HRW_SYS_DHAT_EO = 3,     /* D_hat x_e = b_e on the even sites (half field)      */
    HRW_SYS_D_EO = 4         /* D x = b on the full lattice via the even/odd Schur
                                complement (BiCGstab on D_hat) and reconstruction   */
};

typedef struct hrw_gauge hrw_gauge; /* opaque resident represented gauge field */

typedef struct {
    double tol;            /* stop when the FP64 true relative residual <= tol   */
    int max_iter;          /* iteration cap (per right-hand side)                */
    int system;            /* enum hrw_system                                     */
    int inner_dtype;       /* HRW_F64: plain FP64 CG; F32/BF16/F16: mixed precision
                              with FP64 reliable updates                          */
    int reliable_every;    /* iterations between FP64 reliable updates (mixed)   */
    double reliable_delta; /* also update when |r| fell by this factor since the
                              last update (0 = off)                               */
    double theta[4];       /* boundary phases                                     */
} hrw_solve_params;

typedef struct {
    int status;                 /* HRW_OK, HRW_NOT_CONVERGED or HRW_EBREAKDOWN        */
    int iters;                  /* CG iterations performed                            */
    int reliable_updates;       /* FP64 reliable updates (mixed precision)            */
    int restarts;               /* restarts after a failed true-residual check        */
    double true_rel_resid;      /* |b - A x| / |b| recomputed in FP64 at exit         */
    double recursive_rel_resid; /* the iterated residual at exit                      */
    double d_rel_resid;         /* HRW_SYS_D_CGNR_EO: |b - D x| / |b| in FP64, else 0 */
    double seconds;             /* wall time of the whole call                        */
} hrw_solve_result;

/* ---------------------------------------------------------------- calls */

/* Last error message of the calling thread ("" if none). */
const char *hrw_last_error(void);

/* Library version string. */
const char *hrw_version(void);

/* Dimension N_R of representation rep of SU(nc): N, N^2-1, N(N+1)/2, N(N-1)/2.
 * Sec. 3.1.2 (spinor ~ N_f, link ~ N_f^2).  EINVAL for nc < 2 or bad rep. */
int hrw_rep_dim(int nc, int rep, int *n_r);

/* Stateless representation map U_F -> U_R for n_links links (Sec. 3.1:
 * fermions in general higher representations; the link each fermion sees is
 * the represented one).  u_f: device [n_links][nc][nc] complex FP64;
 * u_r: device [n_links][N_R][N_R] complex FP64 (caller-allocated, must not
 * overlap u_f).  Supported nc: 2, 3, 4.  Enqueued on stream. */
int hrw_rep_map(int nc, int rep, long long n_links, const double *u_f, double *u_r,
                void *stream);

/* Bytes of device storage hrw_gauge_create needs for the given links.
 * The resident field keeps, per requested precision, each link twice (once
 * per parity's hopping block) in the library's device layout. */
int hrw_gauge_storage_size(const int dims[4], int nc, int rep, unsigned storage_mask,
                           size_t *bytes);

/* Build a resident represented gauge field from fundamental links u_f
 * (device, canonical [V][4][nc][nc] complex FP64): the links U_R the fermions
 * of representation R hop with (Sec. 3.1; Sec. 3.1.2 for their N_R x N_R
 * size), kept on the device for every later operator and solve (the paper's
 * fields are likewise resident in GPU memory, Sec. 2.1).  The representation map
 * runs on the device in FP64 and the result is rounded once (ties to even)
 * into each precision in storage_mask (must include HRW_STORE_F64 whenever
 * FP64 operators or solves will be used).  storage: caller-owned device
 * memory of at least hrw_gauge_storage_size bytes, alive until destroy.
 * The flag bits HRW_STORE_FUND_HOP and HRW_STORE_SU3_TWO_ROWS select how
 * single-source hops read the links (see their definitions); a mask with
 * unknown bits is HRW_EINVAL, a flag the group or representation does not
 * support is HRW_EUNSUPPORTED.  On success *out receives the handle. */
int hrw_gauge_create(const int dims[4], int nc, int rep, const double *u_f,
                     unsigned storage_mask, void *storage, size_t storage_bytes, void *stream,
                     hrw_gauge **out);

/* Free the host struct (the caller frees the storage). NULL is accepted. */
int hrw_gauge_destroy(hrw_gauge *g);

/* Representation dimension and lattice of a handle. */
int hrw_gauge_info(const hrw_gauge *g, int dims[4], int *nc, int *rep, int *n_r,
                   unsigned *storage_mask);

/* Workspace bytes for the operator applies (params == NULL) or for
 * hrw_cg_solve with these params, for n_rhs right-hand sides: the packed
 * fields of the Sec. 3.3 CG (x, r, p, A p and the temporaries of the two
 * D_hat applications per iteration, Sec. 3.1), the low-precision copies of
 * a mixed solve and the partial sums of the Sec. 3.2 reductions.  This is
 * also the per-request device footprint the serving loop admits by.
 * bytes receives the size; EINVAL / EUNSUPPORTED as hrw_gauge_create. */
int hrw_workspace_size(const int dims[4], int nc, int rep, int n_rhs,
                       const hrw_solve_params *params, size_t *bytes);

/* out = D_W in (dagger = 0) or D_W^+ in (dagger = 1), D_W = 1 - kappa H
 * (Sec. 3.1), for n_rhs stacked full-lattice fields, computed with links and
 * spinors stored in dtype (inputs are rounded once to dtype, in the storage
 * spin basis described with the canonical layout: with 16-bit storage
 * |psi_s| + |psi_{s+2}| must lie within the format's range; FP32
 * accumulation below FP64).  in/out: device canonical FP64, must not overlap.
 * theta: host double[4]. */
int hrw_dw_apply(const hrw_gauge *g, double kappa, const double theta[4], int dtype, int n_rhs,
                 int dagger, const double *in, double *out, void *workspace, size_t ws_bytes,
                 void *stream);

/* Off-diagonal hopping block: out_parity = 0 gives H_eo (odd -> even), 1 gives
 * H_oe (even -> odd); dagger = 1 gives the corresponding block of H^+
 * (Sec. 3.1, even/odd preconditioning).  in_half / out_half: device canonical
 * half-parity fields, n_rhs stacked. */
int hrw_hop_eo(const hrw_gauge *g, int out_parity, const double theta[4], int dtype, int n_rhs,
               int dagger, const double *in_half, double *out_half, void *workspace,
               size_t ws_bytes, void *stream);

/* out_e = D_hat in_e, D_hat = 1 - kappa^2 H_eo H_oe on even sites (dagger: the
 * adjoint, 1 - kappa^2 (H^+)_eo (H^+)_oe): the even/odd preconditioned
 * operator of Sec. 3.1, the Schur complement of D on the even sites.
 * kappa_per_rhs: host double[n_rhs].  in_e / out_e: device canonical even
 * half fields, n_rhs stacked, must not overlap.  workspace: at least
 * hrw_workspace_size(..., n_rhs, NULL) bytes (holds the packed fields and the
 * odd intermediate H_oe in_e).  Enqueued on stream; EINVAL / ENOMEM on bad
 * arguments, nothing enqueued. */
int hrw_deo_apply(const hrw_gauge *g, const double *kappa_per_rhs, const double theta[4],
                  int dtype, int n_rhs, int dagger, const double *in_e, double *out_e,
                  void *workspace, size_t ws_bytes, void *stream);

/* Bytes of the static device scratch behind hrw_deo_apply_noalloc (320 MiB:
 * D_hat of one FP64 source at 32^4 with N_R = 3, 302 MB, fits). */
#define HRW_NOALLOC_SCRATCH_BYTES (320ull << 20)

/* hrw_deo_apply without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same D_hat, computed by the same
 * kernels bit for bit, with its temporaries (three packed half fields of
 * dtype per source and the coefficients) in a file-scope device array of
 * HRW_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The call allocates nothing and calls no
 * allocating routine.  It needs three buffers of n_rhs P bytes and 512
 * bytes of coefficients, each rounded up to 256 bytes, P = (V/2 rounded up
 * to 64 sites) x 4 N_R x (16, 8, 4, 4 bytes for F64, F32, BF16, F16); a call
 * needing more than HRW_NOALLOC_SCRATCH_BYTES is HRW_ENOMEM, nothing enqueued.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (two streams, two host threads) race and corrupt each other's results;
 * serialise them.  Nothing needs clearing between calls (every scratch entry
 * a call reads it writes first).  Other arguments, errors and stream
 * ordering as hrw_deo_apply. */
int hrw_deo_apply_noalloc(const hrw_gauge *g, const double *kappa_per_rhs, const double theta[4],
                          int dtype, int n_rhs, int dagger, const double *in_e, double *out_e,
                          void *stream);

/* Conjugate gradient (Sec. 3.3) for n_rhs independent systems sharing the
 * gauge field, each with its own kappa (host double[n_rhs]).  b and x are
 * device canonical fields: half-parity (even) for HRW_SYS_DDAG_D_EO, full
 * lattice otherwise.  x = 0 is the start vector; the loop stops each system
 * on its FP64 true relative residual.  res: host array of n_rhs results.
 * Returns HRW_OK when every system converged, HRW_NOT_CONVERGED if any hit
 * max_iter, HRW_EBREAKDOWN if any broke down (others are still solved). */
int hrw_cg_solve(const hrw_gauge *g, const hrw_solve_params *params, int n_rhs,
                 const double *kappa_per_rhs, const double *b, double *x, hrw_solve_result *res,
                 void *workspace, size_t ws_bytes, void *stream);

/* Stabilised bi-conjugate gradient (BiCGstab, van der Vorst 1992; one of the
 * inverters of Sec. 3.3) on D_hat itself (HRW_SYS_DHAT_EO: b, x are even half
 * fields) or for D x = b through the even/odd Schur complement
 * (HRW_SYS_D_EO: b, x full-lattice fields; b'_e = b_e + kappa H_eo b_o,
 * D_hat x_e = b'_e, x_o = b_o + kappa H_oe x_e; res.d_rel_resid receives
 * |b - D x| / |b|).  n_rhs independent systems share the gauge field, each
 * with its own kappa (host double[n_rhs]).  x = 0 is the start vector, the
 * starting residual is the shadow vector, and each system stops on its FP64
 * true relative residual |b_e - D_hat x_e| / |b_e| <= tol.  inner_dtype
 * HRW_F64 runs plain FP64 (the true residual is checked at recursive
 * convergence; above tol the iteration starts again from it); HRW_F32 (or
 * HRW_BF16: BF16 storage, FP32 arithmetic) runs the recurrences on the
 * low-precision fields with FP64 reliable updates (reliable_every,
 * reliable_delta, and at recursive convergence), the solution accumulating in
 * FP64.  A vanished coefficient (rho, <r0, D_hat p> or omega) also starts
 * again; more than 100 new starts end as HRW_EBREAKDOWN.  res.iters counts
 * BiCGstab iterations (two D_hat applications each).  Workspace:
 * hrw_workspace_size with the same params.  Returns as hrw_cg_solve;
 * EUNSUPPORTED for FP16 inner storage, EINVAL for systems 0-2. */
int hrw_bicgstab_solve(const hrw_gauge *g, const hrw_solve_params *params, int n_rhs,
                       const double *kappa_per_rhs, const double *b, double *x, hrw_solve_result *res,
                       void *workspace, size_t ws_bytes, void *stream);

/* QMR on the g5-symmetric Lanczos process (QMR-g5, one of the inverters of
 * Sec. 3.3) for the same systems as hrw_bicgstab_solve (HRW_SYS_DHAT_EO,
 * HRW_SYS_D_EO), in FP64 (inner_dtype HRW_F64; others HRW_EUNSUPPORTED).
 * D_hat^+ = g5 D_hat g5, so the Lanczos process takes one D_hat application
 * per iteration (res.iters counts them) and its coefficients are real; the
 * iterate minimises the quasi-residual.  When sqrt(k + 1) x quasi-residual
 * (k steps since the last start: a bound on the true residual) reaches tol
 * (or a Lanczos coefficient vanishes) the FP64 true residual is computed;
 * above tol the process starts again from it (res.restarts).  Workspace:
 * hrw_workspace_size with the same params (the BiCGstab size covers it). */
int hrw_qmr_g5_solve(const hrw_gauge *g, const hrw_solve_params *params, int n_rhs, const double *kappa_per_rhs,
                     const double *b, double *x, hrw_solve_result *res, void *workspace, size_t ws_bytes,
                     void *stream);

/* ---------------------------------------------------------------- clover term
 * Sheikholeslami-Wohlert improvement (Sec. 3.1): D_sw = A - kappa H with the
 * site-local A(x) = 1 - kappa c_sw sum_{mu<nu} g_mu g_nu (x) F_mu,nu(x), F the
 * clover average (Q - Q^+)/8 of the four plaquette leaves of the mu-nu plane
 * at x built from the represented links (this is the kappa normalisation of
 * 1 + c_sw (i/4) sigma_mu,nu F_mu,nu).  A is Hermitian and block-diagonal in
 * the chiral basis; the handle keeps the two (2 N_R)^2 blocks of A and of
 * A^-1 per site, built once on the device in FP64 (and rounded to FP32 when
 * HRW_STORE_F32 is in the mask), for one (kappa, c_sw).  It references the
 * gauge field, which must stay alive, and holds no device memory of its own. */
typedef struct hrw_clover hrw_clover;

/* Bytes of caller storage for a clover term (mask: HRW_STORE_F64 and/or HRW_STORE_F32). */
int hrw_clover_storage_size(const hrw_gauge *g, unsigned storage_mask, size_t *bytes);

/* Build A and A^-1 from g's FP64 links (g needs HRW_STORE_F64).  A singular block
 * (not possible for small kappa c_sw) leaves non-finite entries in A^-1. */
int hrw_clover_create(const hrw_gauge *g, double kappa, double csw, unsigned storage_mask, void *storage,
                      size_t storage_bytes, void *stream, hrw_clover **out);
int hrw_clover_destroy(hrw_clover *c);

/* out = D_sw in on the full lattice (dagger: A - kappa H^+ = D_sw^+), canonical
 * fields as hrw_dw_apply; dtype F64 or F32 (the clover blocks and the links must
 * be stored in it); workspace: hrw_workspace_size with params = NULL. */
int hrw_dsw_apply(const hrw_clover *c, const double theta[4], int dtype, int n_rhs, int dagger,
                  const double *in, double *out, void *workspace, size_t ws_bytes, void *stream);

/* out_e = D_hat_sw in_e = A_ee in_e - kappa^2 H_eo A_oo^-1 H_oe in_e on even half
 * fields (dagger: with the H^+ blocks, = D_hat_sw^+); as hrw_dsw_apply otherwise. */
int hrw_dsw_eo_apply(const hrw_clover *c, const double theta[4], int dtype, int n_rhs, int dagger,
                     const double *in_e, double *out_e, void *workspace, size_t ws_bytes, void *stream);

/* BiCGstab with the clover term: D_hat_sw x_e = b_e (HRW_SYS_DHAT_EO) or D_sw x = b
 * through the Schur complement (HRW_SYS_D_EO: b'_e = b_e + kappa H_eo A_oo^-1 b_o,
 * D_hat_sw x_e = b'_e, x_o = A_oo^-1 (b_o + kappa H_oe x_e), res.d_rel_resid =
 * |b - D_sw x| / |b|), for the kappa the clover term was built with; otherwise as
 * hrw_bicgstab_solve (HRW_F32 inner fields need FP32 clover blocks and links).
 * Workspace: hrw_clover_workspace_size. */
int hrw_clover_workspace_size(const hrw_clover *c, int n_rhs, const hrw_solve_params *params, size_t *bytes);
int hrw_clover_bicgstab_solve(const hrw_clover *c, const hrw_solve_params *params, int n_rhs, const double *b,
                              double *x, hrw_solve_result *res, void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- solver sessions
 * A session is a CG solver with n_slots slots (n_slots <= 64) that share one
 * resident gauge field, one set of parameters and one caller workspace
 * (hrw_workspace_size with n_rhs = n_slots).  Systems are loaded into free
 * slots and read out when finished at any step boundary, while the other
 * slots keep iterating: this is the continuous-batching engine of the serving
 * loop.  Each slot runs its own recurrence (own kappa, alpha, beta, reliable-
 * update schedule and convergence test), so a system's result does not depend
 * on what else shares the session; hrw_cg_solve is create + load + step until
 * done + read.  A session belongs to one host thread at a time; sessions on
 * different streams may run concurrently.  Sec. 3.3 (CG), Sec. 3.1. */
typedef struct hrw_cg_session hrw_cg_session;

/* Create a session on `stream`; the workspace must stay alive until destroy. */
int hrw_cg_session_create(const hrw_gauge *g, const hrw_solve_params *params, int n_slots,
                          void *workspace, size_t ws_bytes, void *stream, hrw_cg_session **out);

/* Load n systems into the free slots [slot, slot + n): b is n stacked canonical
 * device fields (even half for HRW_SYS_DDAG_D_EO, full lattice otherwise),
 * kappa a host double[n].  Synchronous: returns when the slots are set up. */
int hrw_cg_session_load(hrw_cg_session *s, int slot, int n, const double *kappa, const double *b);

/* Advance every loaded slot by up to max_iters CG iterations (with the FP64
 * reliable updates / true-residual checks that fall due); *running receives
 * the number of slots still iterating.  Returns after the work is complete. */
int hrw_cg_session_step(hrw_cg_session *s, int max_iters, int *running);

/* state[n_slots]: 0 free, 1 iterating, 2 finished (ready to read). */
int hrw_cg_session_slots(hrw_cg_session *s, int *state);

/* Read the finished (or stopped) slots [slot, slot + n): FP64 true residual,
 * odd-site reconstruction for HRW_SYS_D_CGNR_EO, solution into x (n stacked
 * canonical device fields), results into res[n] (seconds = time since load);
 * the slots become free.  Returns the worst status as hrw_cg_solve does. */
int hrw_cg_session_read(hrw_cg_session *s, int slot, int n, double *x, hrw_solve_result *res);

/* Destroy the host part of a session (NULL accepted); the caller frees the workspace. */
int hrw_cg_session_destroy(hrw_cg_session *s);

/* ---------------------------------------------------------------- timing
 * Optional per-kernel timing with HIP events recorded on the launch stream
 * around hopping-kernel launches.  hrw_timing_enable(n) with n >= 1 clears
 * the counters and times one launch in n of each epilogue class (the 1st,
 * (n+1)-th, ... since the call; n = 1: every launch), n <= 0 turns timing
 * off; hrw_timing_read fills, for kernel class k, the count of timed
 * launches, their summed event time in ms and summed algorithmic bytes
 * (min-traffic model: every link, neighbour spinor and epilogue operand
 * counted once per launch), so time / launches is the average duration of
 * the sampled launches.  Classes: 0 = all hopping launches; 3, 4, 5 =
 * hopping launches with the plain (out = H in), axpy (out = self - c H in)
 * and fused CG-update epilogues; 1, 2 are reserved (always zero).  EINVAL for
 * an unknown class.  Each timed launch adds two event records on its stream
 * (a few microseconds each on MI355X); an odd n alternates between launches
 * that repeat in pairs. */
int hrw_timing_enable(int on);
int hrw_timing_read(int kernel_class, long long *launches, double *total_ms, double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* HRW_H */
