// Clover (Sheikholeslami-Wohlert) improvement of the Wilson operator, one of
// the operator features of arXiv 2405.19294 Sec. 3.1, for fermions in the
// representation R:
//   D_sw = A - kappa H,  A(x) = 1 - kappa c_sw sum_{mu<nu} g_mu g_nu (x) F_mu,nu(x)
// (the kappa normalisation of 1 + c_sw (i/4) sigma.F), F = (Q - Q^+)/8 with Q
// the four plaquette leaves of the mu-nu plane at x built from the
// represented links.  In the chiral basis g_mu g_nu is block-diagonal: on
// the upper (spins 0, 1) and lower (spins 2, 3) pair it is s i sigma_m, with
//   (0,k): upper -i sigma_k, lower +i sigma_k;  (1,2): i sigma_3;
//   (1,3): -i sigma_2;  (2,3): i sigma_1 (both pairs),
// so A = diag(A_0, A_1), each a (2 N_R) x (2 N_R) Hermitian block
//   A_chi = [[1 - kc i G3, -kc (i G1 + G2)], [-kc (i G1 - G2), 1 + kc i G3]],
//   G1 = s F01 + F23, G2 = s F02 - F13, G3 = s F03 + F12, s = -1 (chi = 0), +1 (chi = 1),
// kc = kappa c_sw.
//
// The blocks and their inverses are built once per (gauge field, kappa, c_sw)
// by a setup kernel in FP64 (Gauss-Jordan with partial pivoting per block)
// and kept resident in the site-blocked layout, in FP64 and optionally FP32.
// Both are Hermitian, so a block of size M = 2 N_R is stored as M^2 / 2
// complex slots: the M real diagonal entries in pairs (slot r/2, real part for
// even r, imaginary part for odd r) followed by the strictly upper triangle
// row by row; the site-local multiply reads every slot once and uses it for
// both (r, c) and (c, r).
// The operator applies compose the existing hopping kernels with a site-local
// block multiply:
//   D_sw psi      = (A psi) - kappa H psi                    (axpy epilogue, self = A psi)
//   D_hat_sw psi_e = A_ee psi_e - kappa^2 H_eo A_oo^-1 H_oe psi_e,
// the Schur complement of D_sw on the even sites.
#include <math.h>
#include <string.h>

#include "engine.h"

namespace hrw {

struct Z {
    double re, im;
};
__device__ inline Z zmul(Z a, Z b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Z zmulc(Z a, Z b) { return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im}; }  // a conj(b)

// elements of one packed clover block field: per site 2 chirality blocks of (2 N_R)^2 / 2 slots
inline size_t clover_elems(const Geom &g, int nr) { return (size_t)g.nblk * BLK * (2 * nr) * (2 * nr); }

// slot of the upper entry (r, c), r < c, of a packed Hermitian M x M block
__host__ __device__ constexpr int herm_slot(int m, int r, int c) { return m / 2 + r * m - r * (r + 1) / 2 + (c - r - 1); }

template <int NR>
__device__ inline void fetch_link(const Geom &g, const cpx<double> *const blk[2], int y0, int y1, int y2, int y3,
                                  int mu, Z (&u)[NR][NR])
{
    int y[4] = {y0, y1, y2, y3};
    for (int m = 0; m < 4; ++m) y[m] = (y[m] % g.d[m] + g.d[m]) % g.d[m];
    const int qy = (y[0] + y[1] + y[2] + y[3]) & 1;
    const int iy = eo_index(g, y);
    const cpx<double> *b = blk[qy];
    // forward slot mu of the hopping block of the site's own parity holds U_mu(y)
    for (int r = 0; r < NR; ++r)
        for (int c = 0; c < NR; ++c) {
            const cpx<double> v = b[lay(iy, mu * NR * NR + r * NR + c, 8 * NR * NR)];
            u[r][c] = {v.re, v.im};
        }
}

// acc = acc * (u or u^+)
template <int NR>
__device__ inline void right_mul(Z (&acc)[NR][NR], const Z (&u)[NR][NR], bool dag)
{
    Z t[NR][NR];
    for (int r = 0; r < NR; ++r)
        for (int c = 0; c < NR; ++c) {
            Z s = {0, 0};
            for (int k = 0; k < NR; ++k) {
                const Z p = dag ? zmulc(acc[r][k], u[c][k]) : zmul(acc[r][k], u[k][c]);
                s.re += p.re;
                s.im += p.im;
            }
            t[r][c] = s;
        }
    for (int r = 0; r < NR; ++r)
        for (int c = 0; c < NR; ++c) acc[r][c] = t[r][c];
}

// F_mu,nu(x) = (Q - Q^+) / 8 from the four leaves at x
template <int NR>
__device__ void clover_leaf_f(const Geom &g, const cpx<double> *const blk[2], const int (&x)[4], int mu, int nu,
                              Z (&f)[NR][NR])
{
    int e[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    e[0][mu] = 1;
    e[1][nu] = 1;
    // each leaf: four links (offset in units of mu, nu; direction; dagger)
    struct Step {
        int a, b, dir, dag;
    };
    const Step leaves[4][4] = {
        {{0, 0, 0, 0}, {1, 0, 1, 0}, {0, 1, 0, 1}, {0, 0, 1, 1}},      // U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
        {{0, 0, 1, 0}, {-1, 1, 0, 1}, {-1, 0, 1, 1}, {-1, 0, 0, 0}},   // U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu)
        {{-1, 0, 0, 1}, {-1, -1, 1, 1}, {-1, -1, 0, 0}, {0, -1, 1, 0}},  // U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
        {{0, -1, 1, 1}, {0, -1, 0, 0}, {1, -1, 1, 0}, {0, 0, 0, 1}}};  // U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
    Z q[NR][NR];
    for (int r = 0; r < NR; ++r)
        for (int c = 0; c < NR; ++c) q[r][c] = {0, 0};
    for (int l = 0; l < 4; ++l) {
        Z acc[NR][NR];
        for (int r = 0; r < NR; ++r)
            for (int c = 0; c < NR; ++c) acc[r][c] = {r == c ? 1.0 : 0.0, 0.0};
        for (int k = 0; k < 4; ++k) {
            const Step st = leaves[l][k];
            Z u[NR][NR];
            fetch_link<NR>(g, blk, x[0] + st.a * e[0][0] + st.b * e[1][0], x[1] + st.a * e[0][1] + st.b * e[1][1],
                           x[2] + st.a * e[0][2] + st.b * e[1][2], x[3] + st.a * e[0][3] + st.b * e[1][3],
                           st.dir == 0 ? mu : nu, u);
            right_mul<NR>(acc, u, st.dag != 0);
        }
        for (int r = 0; r < NR; ++r)
            for (int c = 0; c < NR; ++c) {
                q[r][c].re += acc[r][c].re;
                q[r][c].im += acc[r][c].im;
            }
    }
    for (int r = 0; r < NR; ++r)
        for (int c = 0; c < NR; ++c)
            f[r][c] = {(q[r][c].re - q[c][r].re) / 8.0, (q[r][c].im + q[c][r].im) / 8.0};
}

struct CloverOut {
    cpx<double> *a64[2], *inv64[2];  // per parity
    cpx<float> *a32[2], *inv32[2];   // optional
};

// upper triangle and real diagonal of a Hermitian block, in FP64 and (if p32) FP32
template <int M>
__device__ inline void store_packed(cpx<double> *p64, cpx<float> *p32, int i, int chi, const Z (&a)[M][M])
{
    constexpr int BS = M * M / 2;
    for (int r = 0; r < M; r += 2) {
        const size_t o = lay(i, chi * BS + r / 2, 2 * BS);
        p64[o] = {a[r][r].re, a[r + 1][r + 1].re};
        if (p32) p32[o] = {(float)a[r][r].re, (float)a[r + 1][r + 1].re};
    }
    for (int r = 0; r < M; ++r)
        for (int c = r + 1; c < M; ++c) {
            const size_t o = lay(i, chi * BS + herm_slot(M, r, c), 2 * BS);
            p64[o] = {a[r][c].re, a[r][c].im};
            if (p32) p32[o] = {(float)a[r][c].re, (float)a[r][c].im};
        }
}

// One thread per site: the two chirality blocks of A and of A^-1.
template <int NR>
__global__ void __launch_bounds__(64) clover_build_kernel(Geom g, const cpx<double> *blk0, const cpx<double> *blk1,
                                                          double kc, CloverOut out)
{
    constexpr int M = 2 * NR;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * g.half) return;
    const int q = t >= g.half ? 1 : 0;
    const int i = t - q * g.half;
    const cpx<double> *const blk[2] = {blk0, blk1};
    int x[4];
    eo_coords(g, q, i, x);
    Z f[6][NR][NR];
    {
        int p = 0;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) clover_leaf_f<NR>(g, blk, x, mu, nu, f[p++]);
    }
    // plane order: 01, 02, 03, 12, 13, 23
    for (int chi = 0; chi < 2; ++chi) {
        const double s = chi == 0 ? -1.0 : 1.0;
        Z a[M][M], inv[M][M];
        for (int r = 0; r < NR; ++r)
            for (int c = 0; c < NR; ++c) {
                const Z g1 = {s * f[0][r][c].re + f[5][r][c].re, s * f[0][r][c].im + f[5][r][c].im};
                const Z g2 = {s * f[1][r][c].re - f[4][r][c].re, s * f[1][r][c].im - f[4][r][c].im};
                const Z g3 = {s * f[2][r][c].re + f[3][r][c].re, s * f[2][r][c].im + f[3][r][c].im};
                const double dl = r == c ? 1.0 : 0.0;
                // i z = (-z.im, z.re)
                a[r][c] = {dl + kc * g3.im, -kc * g3.re};                        // 1 - kc i G3
                a[NR + r][NR + c] = {dl - kc * g3.im, kc * g3.re};               // 1 + kc i G3
                a[r][NR + c] = {-kc * (-g1.im + g2.re), -kc * (g1.re + g2.im)};  // -kc (i G1 + G2)
                a[NR + r][c] = {-kc * (-g1.im - g2.re), -kc * (g1.re - g2.im)};  // -kc (i G1 - G2)
            }
        store_packed(out.a64[q], out.a32[q], i, chi, a);
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) inv[r][c] = {r == c ? 1.0 : 0.0, 0.0};
        // Gauss-Jordan elimination with partial pivoting
        for (int c = 0; c < M; ++c) {
            int piv = c;
            double best = a[c][c].re * a[c][c].re + a[c][c].im * a[c][c].im;
            for (int r = c + 1; r < M; ++r) {
                const double m2 = a[r][c].re * a[r][c].re + a[r][c].im * a[r][c].im;
                if (m2 > best) {
                    best = m2;
                    piv = r;
                }
            }
            if (piv != c)
                for (int k = 0; k < M; ++k) {
                    const Z t1 = a[c][k], t2 = inv[c][k];
                    a[c][k] = a[piv][k];
                    inv[c][k] = inv[piv][k];
                    a[piv][k] = t1;
                    inv[piv][k] = t2;
                }
            const Z d = a[c][c];
            const double dn = d.re * d.re + d.im * d.im;  // 0 only for a singular block (then inf/NaN follow)
            const Z di = {d.re / dn, -d.im / dn};
            for (int k = 0; k < M; ++k) {
                a[c][k] = zmul(a[c][k], di);
                inv[c][k] = zmul(inv[c][k], di);
            }
            for (int r = 0; r < M; ++r) {
                if (r == c) continue;
                const Z fct = a[r][c];
                for (int k = 0; k < M; ++k) {
                    const Z p = zmul(fct, a[c][k]), p2 = zmul(fct, inv[c][k]);
                    a[r][k].re -= p.re;
                    a[r][k].im -= p.im;
                    inv[r][k].re -= p2.re;
                    inv[r][k].im -= p2.im;
                }
            }
        }
        store_packed(out.inv64[q], out.inv32[q], i, chi, inv);
    }
}

// out = B in on the sites of one parity, B a packed block field (A or A^-1)
// whose two blocks act on the chiral halves (spins 0, 1 and 2, 3) of the
// chiral basis; blockIdx.y = rhs, one thread per site.  The fields are held in
// the hopping kernels' storage basis (q_s = psi_s - psi_{s+2}, q_{s+2} =
// psi_s + psi_{s+2}), so the thread forms the chiral halves u = (q_s +
// q_{s+2}) / 2 and d = (q_{s+2} - q_s) / 2, multiplies u by the first block
// and d by the second, and returns (B u - B d, B u + B d) in the same basis.
template <class S, int NR>
__device__ __forceinline__ void block_mul(const cpx<S> *__restrict__ blk, int i, int chi,
                                          const typename acc_of<S>::type (&vr)[2 * NR],
                                          const typename acc_of<S>::type (&vi)[2 * NR],
                                          typename acc_of<S>::type (&sr)[2 * NR],
                                          typename acc_of<S>::type (&si)[2 * NR])
{
    typedef typename acc_of<S>::type A;
    constexpr int M = 2 * NR;
    constexpr int BS = M * M / 2;
    // diagonal (real)
#pragma unroll
    for (int r = 0; r < M; r += 2) {
        A d0, d1;
        load_c(blk + lay(i, chi * BS + r / 2, 2 * BS), d0, d1);
        sr[r] = d0 * vr[r];
        si[r] = d0 * vi[r];
        sr[r + 1] = d1 * vr[r + 1];
        si[r + 1] = d1 * vi[r + 1];
    }
    // each upper slot m = B(r, c) serves out_r += m v_c and out_c += conj(m) v_r
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
        for (int c = r + 1; c < M; ++c) {
            A mr, mi;
            load_c(blk + lay(i, chi * BS + herm_slot(M, r, c), 2 * BS), mr, mi);
            sr[r] = fmac(mr, vr[c], sr[r]);
            sr[r] = fmac(-mi, vi[c], sr[r]);
            si[r] = fmac(mr, vi[c], si[r]);
            si[r] = fmac(mi, vr[c], si[r]);
            sr[c] = fmac(mr, vr[r], sr[c]);
            sr[c] = fmac(mi, vi[r], sr[c]);
            si[c] = fmac(mr, vi[r], si[c]);
            si[c] = fmac(-mi, vr[r], si[c]);
        }
}

template <class S, int NR>
__global__ void __launch_bounds__(WG) clover_mul_kernel(const cpx<S> *__restrict__ bm, const cpx<S> *__restrict__ in,
                                                        cpx<S> *__restrict__ out, int half, size_t rstride)
{
    typedef typename acc_of<S>::type A;
    constexpr int M = 2 * NR;
    constexpr int NC = 4 * NR;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= half) return;
    const size_t ro = (size_t)blockIdx.y * rstride;
    A ur[M], ui[M], dr[M], di[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        A ar, ai, br, bi;
        load_c(in + ro + lay(i, c, NC), ar, ai);
        load_c(in + ro + lay(i, M + c, NC), br, bi);
        ur[c] = (ar + br) * (A)0.5;
        ui[c] = (ai + bi) * (A)0.5;
        dr[c] = (br - ar) * (A)0.5;
        di[c] = (bi - ai) * (A)0.5;
    }
    A pr[M], pi[M], mr[M], mi[M];
    block_mul<S, NR>(bm, i, 0, ur, ui, pr, pi);
    block_mul<S, NR>(bm, i, 1, dr, di, mr, mi);
#pragma unroll
    for (int c = 0; c < M; ++c) {
        store_c(out + ro + lay(i, c, NC), pr[c] - mr[c], pi[c] - mi[c]);
        store_c(out + ro + lay(i, M + c, NC), pr[c] + mr[c], pi[c] + mi[c]);
    }
}

hipError_t launch_clover_mul(int dt, int nr, const Geom &g, const void *bm, const void *in, void *out, int n_rhs,
                             size_t rstride, hipStream_t st)
{
    const dim3 grid((unsigned)((g.half + WG - 1) / WG), (unsigned)n_rhs, 1);
    bool ok = false;
    dispatch_nr(nr, [&](auto nrc) {
        constexpr int NR = decltype(nrc)::value;
        if (dt == 0) {
            clover_mul_kernel<double, NR><<<grid, WG, 0, st>>>((const cpx<double> *)bm, (const cpx<double> *)in,
                                                               (cpx<double> *)out, g.half, rstride);
            ok = true;
        } else if (dt == 1) {
            clover_mul_kernel<float, NR><<<grid, WG, 0, st>>>((const cpx<float> *)bm, (const cpx<float> *)in,
                                                              (cpx<float> *)out, g.half, rstride);
            ok = true;
        }
    });
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------ host

int clover_storage_bytes(const hrw_gauge *g, unsigned mask, size_t *bytes)
{
    Arena ar(nullptr, 0);
    for (int d = 0; d < 2; ++d)
        if (mask & (1u << d))
            for (int k = 0; k < 4; ++k) ar.take(clover_elems(g->g, g->nr) * dtype_cbytes(d));
    *bytes = ar.off + 256;
    return HRW_OK;
}

int clover_create(const hrw_gauge *g, double kappa, double csw, unsigned mask, void *storage, size_t storage_bytes,
                  hipStream_t st, hrw_clover **out)
{
    size_t need;
    clover_storage_bytes(g, mask, &need);
    if (storage_bytes < need) return fail(HRW_ENOMEM, "clover storage too small: need %zu bytes", need);
    hrw_clover *c = new hrw_clover;
    memset(c, 0, sizeof *c);
    c->g = g;
    c->kappa = kappa;
    c->csw = csw;
    c->mask = mask;
    Arena ar(storage, storage_bytes);
    for (int d = 0; d < 2; ++d)
        if (mask & (1u << d))
            for (int q = 0; q < 2; ++q) {
                c->a[d][q] = ar.take(clover_elems(g->g, g->nr) * dtype_cbytes(d));
                c->inv[d][q] = ar.take(clover_elems(g->g, g->nr) * dtype_cbytes(d));
            }
    CloverOut o;
    memset(&o, 0, sizeof o);
    for (int q = 0; q < 2; ++q) {
        o.a64[q] = (cpx<double> *)c->a[0][q];
        o.inv64[q] = (cpx<double> *)c->inv[0][q];
        o.a32[q] = (cpx<float> *)c->a[1][q];
        o.inv32[q] = (cpx<float> *)c->inv[1][q];
    }
    // the padding lanes of the block fields stay zero
    hipError_t e = launch_zero(storage, ar.off, st);
    const unsigned blocks = (unsigned)((2LL * g->g.half + 63) / 64);
    bool ok = e == hipSuccess && dispatch_nr(g->nr, [&](auto nrc) {
        constexpr int NR = decltype(nrc)::value;
        clover_build_kernel<NR><<<blocks, 64, 0, st>>>(g->g, (const cpx<double> *)g->blocks[0][0],
                                                       (const cpx<double> *)g->blocks[0][1], kappa * csw, o);
    });
    if (e == hipSuccess) e = ok ? hipGetLastError() : hipErrorInvalidValue;
    if (e != hipSuccess) {
        delete c;
        return fail(HRW_EDEVICE, "clover setup failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return HRW_OK;
}

static int check_clover_ws(const Geom &g, int nr, int n_rhs, size_t ws_bytes)
{
    size_t need;
    apply_workspace(g, nr, n_rhs, &need);
    if (ws_bytes < need) return fail(HRW_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, ws_bytes);
    return HRW_OK;
}

// workspace: the four two-half fields of the operator applies (hrw_workspace_size with params = NULL)
static void clover_fields(void *ws, const Geom &g, int nr, int n_rhs, char *f[4], double **coef)
{
    Arena ar(ws, (size_t)-1);
    const size_t H = spinor_elems(g, nr);
    for (int k = 0; k < 4; ++k) f[k] = (char *)ar.take(2 * H * n_rhs * 16);
    *coef = (double *)ar.take(sizeof(double) * MAX_RHS);
}

int dsw_apply(const hrw_clover *c, const double theta[4], int dt, int n_rhs, int dagger, const double *in,
              double *out, void *ws, size_t ws_bytes, hipStream_t st)
{
    const hrw_gauge *g = c->g;
    int rc = check_clover_ws(g->g, g->nr, n_rhs, ws_bytes);
    if (rc) return rc;
    char *f[4];
    double *coef;
    clover_fields(ws, g->g, g->nr, n_rhs, f, &coef);
    const size_t H = spinor_elems(g->g, g->nr);
    const size_t cb = dtype_cbytes(dt);
    HRW_HIP(launch_pack_spinor(dt, g->nr, g->g, true, 0, n_rhs, in, f[0], f[0] + H * cb, 2 * H, st));
    // u = A psi on both parities
    for (int q = 0; q < 2; ++q)
        HRW_HIP(launch_clover_mul(dt, g->nr, g->g, c->a[dt][q], f[0] + q * H * cb, f[1] + q * H * cb, n_rhs, 2 * H,
                                  st));
    double k[MAX_RHS];
    for (int j = 0; j < n_rhs; ++j) k[j] = c->kappa;
    if ((rc = set_device_doubles(coef, k, n_rhs, st))) return rc;
    HopCall h;
    h.dt = dt;
    h.parity = -1;
    h.dagger = dagger != 0;
    h.epi = EPI_AXPY;
    h.n_rhs = n_rhs;
    h.rstride = 2 * H;
    for (int q = 0; q < 2; ++q) {
        h.in[q] = f[0] + q * H * cb;
        h.self[q] = f[1] + q * H * cb;
        h.out[q] = f[2] + q * H * cb;
    }
    h.coef = coef;
    if ((rc = run_hop(g, make_phases(theta), h, st))) return rc;
    HRW_HIP(launch_unpack_spinor(dt, g->nr, g->g, true, 0, n_rhs, f[2], f[2] + H * cb, 2 * H, out, st));
    return HRW_OK;
}

// out_e = A_ee in_e - kappa^2 H_eo A_oo^-1 H_oe in_e on packed half fields (rhs stride rs) of dtype dt;
// t, w: odd temporaries, u: even temporary
int dsw_eo_packed(const hrw_clover *c, const Phases &ph, int dt, int n_rhs, bool dagger, size_t rs, const void *in_e,
                  void *t, void *w, void *u, void *out_e, const double *coef_k2, const int *run, hipStream_t st)
{
    const hrw_gauge *g = c->g;
    HopCall a;
    a.dt = dt;
    a.dagger = dagger;
    a.n_rhs = n_rhs;
    a.rstride = rs;
    a.run = run;
    a.parity = 1;
    a.epi = EPI_PLAIN;
    a.in[0] = in_e;
    a.out[1] = t;
    int rc = run_hop(g, ph, a, st);
    if (rc) return rc;
    HRW_HIP(launch_clover_mul(dt, g->nr, g->g, c->inv[dt][1], t, w, n_rhs, rs, st));
    HRW_HIP(launch_clover_mul(dt, g->nr, g->g, c->a[dt][0], in_e, u, n_rhs, rs, st));
    HopCall b = a;
    b.parity = 0;
    b.epi = EPI_AXPY;
    b.in[0] = nullptr;
    b.out[1] = nullptr;
    b.in[1] = w;
    b.self[0] = u;
    b.out[0] = out_e;
    b.coef = coef_k2;
    return run_hop(g, ph, b, st);
}

int dsw_eo_apply(const hrw_clover *c, const double theta[4], int dt, int n_rhs, int dagger, const double *in,
                 double *out, void *ws, size_t ws_bytes, hipStream_t st)
{
    const hrw_gauge *g = c->g;
    int rc = check_clover_ws(g->g, g->nr, n_rhs, ws_bytes);
    if (rc) return rc;
    char *f[4];
    double *coef;
    clover_fields(ws, g->g, g->nr, n_rhs, f, &coef);
    const size_t H = spinor_elems(g->g, g->nr);
    const size_t cb = dtype_cbytes(dt);
    HRW_HIP(launch_pack_spinor(dt, g->nr, g->g, false, 0, n_rhs, in, f[0], nullptr, H, st));
    double k2[MAX_RHS];
    for (int j = 0; j < n_rhs; ++j) k2[j] = c->kappa * c->kappa;
    if ((rc = set_device_doubles(coef, k2, n_rhs, st))) return rc;
    // half fields with rhs stride H: in f0, t f1, w f1 + n H, u f2, out f3
    if ((rc = dsw_eo_packed(c, make_phases(theta), dt, n_rhs, dagger != 0, H, f[0], f[1], f[1] + (size_t)n_rhs * H * cb,
                            f[2], f[3], coef, nullptr, st)))
        return rc;
    HRW_HIP(launch_unpack_spinor(dt, g->nr, g->g, false, 0, n_rhs, f[3], nullptr, H, out, st));
    return HRW_OK;
}

}  // namespace hrw
