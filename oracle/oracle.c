/*
 * Plain FP64 CPU oracle for the Wilson-Dirac operator with fermions in a
 * representation R of SU(N), its even/odd (Schur) form, conjugate-gradient
 * inversion of D^dagger D and BiCGstab inversion of D.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the GPU
 * library shares no code, header, table or helper with it.
 *
 * Sources of each definition (arXiv 2405.19294):
 *   - the operator is the Wilson-Dirac operator in single/double precision for
 *     any N_c and higher representations, with even/odd preconditioning
 *     (Sec. 3.1); the spinor carries ~N_f colour components and the
 *     represented link is an N_f x N_f matrix (Sec. 3.1.2);
 *   - the inverters are CG, BiCGstab and QMR-g5 (Sec. 3.3); inner products and
 *     norms are global reductions (Sec. 3.2).
 * The paper prints no formula for D, the gamma basis, the representation
 * bases or the boundary-phase placement; the readings fixed here are:
 *   - Euclidean chiral gamma basis, gamma_5 = g0 g1 g2 g3 = diag(1,1,-1,-1);
 *   - (H psi)(x) = sum_mu [ ph+_mu(x) (1 - g_mu) U_mu(x) psi(x+mu)
 *                         + ph-_mu(x) (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ],
 *     D = 1 - kappa H (Wilson r = 1);
 *   - ph+_mu(x) = exp(i theta_mu) when x_mu = N_mu - 1, ph-_mu(x) =
 *     exp(-i theta_mu) when x_mu = 0, else 1; phases are never folded into U;
 *   - adjoint generators T^a = generalised Gell-Mann / 2 (symmetric
 *     off-diagonal, antisymmetric off-diagonal, diagonal), (U_A)_ab =
 *     2 Re Tr(T^a U T^b U^+); two-index bases e_(jk) with M -> U M U^T and
 *     (U_R)_ab = Tr(e_a^+ U e_b U^T);
 *   - even sites have x0+x1+x2+x3 even; D_hat = 1 - kappa^2 H_eo H_oe.
 * Gamma matrices are multiplied as literal 4x4 matrices (no spin
 * projection), and the even/odd blocks are taken by masking the full hop, so
 * that nothing in here mirrors the GPU kernels' structure.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_NOT_CONVERGED 1
#define ORC_BREAKDOWN (-5)

enum { REP_FUND = 0, REP_ADJ = 1, REP_SYM = 2, REP_ASYM = 3 };

/* ------------------------------------------------------------------ lattice */

static long vol(const int d[4]) { return (long)d[0] * d[1] * d[2] * d[3]; }

static void coords(const int d[4], long s, int x[4])
{
    x[3] = (int)(s % d[3]);
    s /= d[3];
    x[2] = (int)(s % d[2]);
    s /= d[2];
    x[1] = (int)(s % d[1]);
    x[0] = (int)(s / d[1]);
}

static long index_of(const int d[4], const int x[4])
{
    return (((long)x[0] * d[1] + x[1]) * d[2] + x[2]) * d[3] + x[3];
}

static int parity_of(const int x[4]) { return (x[0] + x[1] + x[2] + x[3]) & 1; }

/* ------------------------------------------------------------------ gamma */

static cplx G[5][4][4];
static int gamma_ready = 0;

static void init_gamma(void)
{
    if (gamma_ready) return;
    memset(G, 0, sizeof G);
    /* g0 = [[0,-1],[-1,0]] in 2x2 blocks */
    G[0][0][2] = -1; G[0][1][3] = -1; G[0][2][0] = -1; G[0][3][1] = -1;
    /* gk = [[0, -i sigma_k], [i sigma_k, 0]] */
    G[1][0][3] = -I; G[1][1][2] = -I; G[1][2][1] = I; G[1][3][0] = I;
    G[2][0][3] = -1; G[2][1][2] = 1; G[2][2][1] = 1; G[2][3][0] = -1;
    G[3][0][2] = -I; G[3][1][3] = I; G[3][2][0] = I; G[3][3][1] = -I;
    /* g5 = g0 g1 g2 g3, computed by matrix products */
    cplx a[4][4], b[4][4];
    memcpy(a, G[0], sizeof a);
    for (int m = 1; m < 4; ++m) {
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                cplx s = 0;
                for (int k = 0; k < 4; ++k) s += a[i][k] * G[m][k][j];
                b[i][j] = s;
            }
        memcpy(a, b, sizeof a);
    }
    memcpy(G[4], a, sizeof a);
    gamma_ready = 1;
}

/* Copy gamma matrix m (0..3, 4 = gamma_5) out, row-major complex. */
void orc_gamma(int m, double *out)
{
    init_gamma();
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            out[2 * (4 * i + j)] = creal(G[m][i][j]);
            out[2 * (4 * i + j) + 1] = cimag(G[m][i][j]);
        }
}

/* ------------------------------------------------------------------ rep map */

int orc_rep_dim(int nc, int rep)
{
    if (nc < 1) return -1;
    switch (rep) {
    case REP_FUND: return nc;
    case REP_ADJ: return nc * nc - 1;
    case REP_SYM: return nc * (nc + 1) / 2;
    case REP_ASYM: return nc * (nc - 1) / 2;
    }
    return -1;
}

/* dense N x N helpers */
static void mm(int n, const cplx *a, const cplx *b, cplx *c)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cplx s = 0;
            for (int k = 0; k < n; ++k) s += a[i * n + k] * b[k * n + j];
            c[i * n + j] = s;
        }
}

static void dagger(int n, const cplx *a, cplx *c)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) c[i * n + j] = conj(a[j * n + i]);
}

static void transpose(int n, const cplx *a, cplx *c)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) c[i * n + j] = a[j * n + i];
}

static cplx trace(int n, const cplx *a)
{
    cplx s = 0;
    for (int i = 0; i < n; ++i) s += a[i * n + i];
    return s;
}

/* Basis matrices of the representation space, each N x N; returns count. */
static int build_basis(int n, int rep, cplx *basis /* [nr][n*n] */)
{
    int a = 0;
    const int nn = n * n;
    if (rep == REP_ADJ) {
        /* generalised Gell-Mann matrices divided by 2 */
        for (int j = 0; j < n; ++j)
            for (int k = j + 1; k < n; ++k) {
                cplx *t = basis + (long)a * nn;
                memset(t, 0, sizeof(cplx) * nn);
                t[j * n + k] = 0.5;
                t[k * n + j] = 0.5;
                ++a;
            }
        for (int j = 0; j < n; ++j)
            for (int k = j + 1; k < n; ++k) {
                cplx *t = basis + (long)a * nn;
                memset(t, 0, sizeof(cplx) * nn);
                t[j * n + k] = -0.5 * I;
                t[k * n + j] = 0.5 * I;
                ++a;
            }
        for (int l = 1; l < n; ++l) {
            cplx *t = basis + (long)a * nn;
            memset(t, 0, sizeof(cplx) * nn);
            const double c = 1.0 / sqrt(2.0 * l * (l + 1));
            for (int m = 0; m < l; ++m) t[m * n + m] = c;
            t[l * n + l] = -l * c;
            ++a;
        }
    } else if (rep == REP_SYM) {
        for (int j = 0; j < n; ++j)
            for (int k = j; k < n; ++k) {
                cplx *e = basis + (long)a * nn;
                memset(e, 0, sizeof(cplx) * nn);
                if (j == k) {
                    e[j * n + j] = 1.0;
                } else {
                    e[j * n + k] = M_SQRT1_2;
                    e[k * n + j] = M_SQRT1_2;
                }
                ++a;
            }
    } else if (rep == REP_ASYM) {
        for (int j = 0; j < n; ++j)
            for (int k = j + 1; k < n; ++k) {
                cplx *e = basis + (long)a * nn;
                memset(e, 0, sizeof(cplx) * nn);
                e[j * n + k] = M_SQRT1_2;
                e[k * n + j] = -M_SQRT1_2;
                ++a;
            }
    }
    return a;
}

/* One link U (N x N) -> U_R (nr x nr) by the trace definitions. */
static void rep_one(int n, int rep, int nr, const cplx *basis, const cplx *u, cplx *ur,
                    cplx *w1, cplx *w2, cplx *w3)
{
    const int nn = n * n;
    if (rep == REP_FUND) {
        memcpy(ur, u, sizeof(cplx) * nn);
        return;
    }
    if (rep == REP_ADJ) {
        cplx ud[64];
        dagger(n, u, ud);
        for (int b = 0; b < nr; ++b) {
            mm(n, u, basis + (long)b * nn, w1);  /* U T^b */
            mm(n, w1, ud, w2);                   /* U T^b U^+ */
            for (int a = 0; a < nr; ++a) {
                mm(n, basis + (long)a * nn, w2, w3);
                ur[a * nr + b] = 2.0 * creal(trace(n, w3));
            }
        }
        return;
    }
    /* two-index: M -> U M U^T, (U_R)_ab = Tr(e_a^+ U e_b U^T) */
    cplx ut[64], ed[64];
    transpose(n, u, ut);
    for (int b = 0; b < nr; ++b) {
        mm(n, u, basis + (long)b * nn, w1);
        mm(n, w1, ut, w2);
        for (int a = 0; a < nr; ++a) {
            dagger(n, basis + (long)a * nn, ed);
            mm(n, ed, w2, w3);
            ur[a * nr + b] = trace(n, w3);
        }
    }
}

/* u_f: n_links x N x N complex; u_r: n_links x nr x nr complex. */
int orc_rep_map(int nc, int rep, long n_links, const double *u_f, double *u_r)
{
    const int nr = orc_rep_dim(nc, rep);
    if (nr < 1 || nc > 8 || n_links < 0 || !u_f || !u_r) return ORC_EINVAL;
    const int nn = nc * nc;
    cplx *basis = (cplx *)malloc(sizeof(cplx) * (size_t)(nr > 0 ? nr : 1) * nn);
    build_basis(nc, rep, basis);
    const cplx *uf = (const cplx *)u_f;
    cplx *ur = (cplx *)u_r;
#pragma omp parallel
    {
        cplx w1[64], w2[64], w3[64];
#pragma omp for schedule(static)
        for (long l = 0; l < n_links; ++l)
            rep_one(nc, rep, nr, basis, uf + l * nn, ur + l * (long)nr * nr, w1, w2, w3);
    }
    free(basis);
    return ORC_OK;
}

/* Basis matrices for the tests (nr x N x N complex). */
int orc_rep_basis(int nc, int rep, double *out)
{
    if (rep == REP_FUND || orc_rep_dim(nc, rep) < 1) return ORC_EINVAL;
    build_basis(nc, rep, (cplx *)out);
    return ORC_OK;
}

/* ------------------------------------------------------------------ hop */

/* Hopping term H (sign = +1) or its adjoint H^+ (sign = -1) on the full
 * lattice.  u: [V][4][nr][nr], in/out: [V][4][nr]. */
static void hop_full(const int d[4], int nr, const cplx *u, const double theta[4], int sign,
                     const cplx *in, cplx *out)
{
    init_gamma();
    const long v = vol(d);
    const int sp = 4 * nr;
    const long ls = (long)nr * nr;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < v; ++s) {
        int x[4];
        coords(d, s, x);
        cplx acc[4 * 16];
        cplx t[4 * 16];
        for (int i = 0; i < sp; ++i) acc[i] = 0;
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = 0; dir < 2; ++dir) {
                int y[4] = {x[0], x[1], x[2], x[3]};
                cplx ph = 1.0;
                const cplx *link;
                int adj;
                if (dir == 0) { /* forward: U_mu(x) psi(x+mu), projector (1 - sign g_mu) */
                    y[mu] = (x[mu] + 1) % d[mu];
                    if (x[mu] == d[mu] - 1) ph = cexp(I * theta[mu]);
                    link = u + (s * 4 + mu) * ls;
                    adj = 0;
                } else { /* backward: U_mu(x-mu)^+ psi(x-mu), projector (1 + sign g_mu) */
                    y[mu] = (x[mu] + d[mu] - 1) % d[mu];
                    if (x[mu] == 0) ph = cexp(-I * theta[mu]);
                    link = u + (index_of(d, y) * 4 + mu) * ls;
                    adj = 1;
                }
                const cplx *src = in + index_of(d, y) * sp;
                /* t[spin][a] = sum_b link(a,b) src[spin][b] (or the adjoint) */
                for (int al = 0; al < 4; ++al)
                    for (int a = 0; a < nr; ++a) {
                        cplx z = 0;
                        for (int b = 0; b < nr; ++b) {
                            cplx l = adj ? conj(link[b * nr + a]) : link[a * nr + b];
                            z += l * src[al * nr + b];
                        }
                        t[al * nr + a] = z;
                    }
                const double gs = (dir == 0 ? -1.0 : 1.0) * sign;
                for (int al = 0; al < 4; ++al)
                    for (int a = 0; a < nr; ++a) {
                        cplx z = t[al * nr + a];
                        for (int be = 0; be < 4; ++be) z += gs * G[mu][al][be] * t[be * nr + a];
                        acc[al * nr + a] += ph * z;
                    }
            }
        }
        for (int i = 0; i < sp; ++i) out[s * sp + i] = acc[i];
    }
}

static int check_dims(const int d[4], int nr)
{
    if (!d || nr < 1 || nr > 16) return 0;
    for (int m = 0; m < 4; ++m)
        if (d[m] < 2) return 0;
    return 1;
}

int orc_hop(const int *dims, int nr, const double *u, const double *theta, int dagger_,
            const double *in, double *out)
{
    if (!check_dims(dims, nr) || !u || !in || !out) return ORC_EINVAL;
    const double zero[4] = {0, 0, 0, 0};
    hop_full(dims, nr, (const cplx *)u, theta ? theta : zero, dagger_ ? -1 : 1,
             (const cplx *)in, (cplx *)out);
    return ORC_OK;
}

/* D psi = psi - kappa H psi (dagger: psi - kappa H^+ psi). */
int orc_dw(const int *dims, int nr, const double *u, double kappa, const double *theta,
           int dagger_, const double *in, double *out)
{
    if (!check_dims(dims, nr) || !u || !in || !out || in == out) return ORC_EINVAL;
    int rc = orc_hop(dims, nr, u, theta, dagger_, in, out);
    if (rc) return rc;
    const long n = vol(dims) * 4 * nr;
    const cplx *a = (const cplx *)in;
    cplx *b = (cplx *)out;
    for (long i = 0; i < n; ++i) b[i] = a[i] - kappa * b[i];
    return ORC_OK;
}

/* ------------------------------------------------------------------ even/odd */

/* Half-parity fields list the sites of one parity in lexicographic order. */
static long half_count(const int d[4], int p)
{
    long c = 0;
    const long v = vol(d);
    for (long s = 0; s < v; ++s) {
        int x[4];
        coords(d, s, x);
        c += parity_of(x) == p;
    }
    return c;
}

static void embed(const int d[4], int nr, int p, const cplx *half, cplx *full)
{
    const long v = vol(d);
    const int sp = 4 * nr;
    long k = 0;
    for (long s = 0; s < v; ++s) {
        int x[4];
        coords(d, s, x);
        if (parity_of(x) == p) {
            memcpy(full + s * sp, half + k * sp, sizeof(cplx) * sp);
            ++k;
        } else {
            memset(full + s * sp, 0, sizeof(cplx) * sp);
        }
    }
}

static void extract(const int d[4], int nr, int p, const cplx *full, cplx *half)
{
    const long v = vol(d);
    const int sp = 4 * nr;
    long k = 0;
    for (long s = 0; s < v; ++s) {
        int x[4];
        coords(d, s, x);
        if (parity_of(x) == p) {
            memcpy(half + k * sp, full + s * sp, sizeof(cplx) * sp);
            ++k;
        }
    }
}

static int even_dims(const int d[4])
{
    for (int m = 0; m < 4; ++m)
        if (d[m] % 2) return 0;
    return 1;
}

/* Block of H (or H^+) mapping parity 1-out_parity to out_parity. */
int orc_hop_eo(const int *dims, int nr, const double *u, const double *theta, int dagger_,
               int out_parity, const double *in_half, double *out_half)
{
    if (!check_dims(dims, nr) || !even_dims(dims) || (out_parity & ~1) || !u || !in_half ||
        !out_half)
        return ORC_EINVAL;
    const long v = vol(dims);
    const size_t bytes = sizeof(cplx) * (size_t)v * 4 * nr;
    cplx *a = (cplx *)malloc(bytes), *b = (cplx *)malloc(bytes);
    embed(dims, nr, 1 - out_parity, (const cplx *)in_half, a);
    const double zero[4] = {0, 0, 0, 0};
    hop_full(dims, nr, (const cplx *)u, theta ? theta : zero, dagger_ ? -1 : 1, a, b);
    extract(dims, nr, out_parity, b, (cplx *)out_half);
    free(a);
    free(b);
    return ORC_OK;
}

/* D_hat psi_e = psi_e - kappa^2 H_eo H_oe psi_e (dagger: with H^+ blocks). */
int orc_deo(const int *dims, int nr, const double *u, double kappa, const double *theta,
            int dagger_, const double *in_e, double *out_e)
{
    if (!check_dims(dims, nr) || !even_dims(dims) || !in_e || !out_e || in_e == out_e)
        return ORC_EINVAL;
    const long h = vol(dims) / 2;
    cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)h * 4 * nr);
    int rc = orc_hop_eo(dims, nr, u, theta, dagger_, 1, in_e, (double *)t);
    if (!rc) rc = orc_hop_eo(dims, nr, u, theta, dagger_, 0, (const double *)t, out_e);
    free(t);
    if (rc) return rc;
    const long n = h * 4 * nr;
    const cplx *a = (const cplx *)in_e;
    cplx *b = (cplx *)out_e;
    for (long i = 0; i < n; ++i) b[i] = a[i] - kappa * kappa * b[i];
    return ORC_OK;
}

int orc_parity_count(const int *dims, int parity) { return (int)half_count(dims, parity & 1); }

/* ------------------------------------------------------------------ clover */

/*
 * Sheikholeslami-Wohlert (clover) term, one of the operator improvements of
 * Sec. 3.1.  In the kappa normalisation of D = 1 - kappa H the improved
 * operator is D_sw = A - kappa H with the site-local
 *   A(x) = 1 - kappa c_sw sum_{mu<nu} (g_mu g_nu) (x) F_mu,nu(x),
 * which is (1/(4+m0)) times 1 + c_sw (i/4) sigma_mu,nu F_mu,nu summed over all
 * mu, nu with sigma_mu,nu = (i/2)[g_mu, g_nu].  F is the clover average in the
 * representation R: F = (Q - Q^+)/8, Q the sum of the four plaquette leaves in
 * the mu-nu plane that start and end at x, built from the represented links.
 * The boundary phases of the fermion field do not enter F.
 */

/* U_mu at x (periodic) */
static const cplx *link_at(const int d[4], int nr, const cplx *u, const int x[4], int mu)
{
    int y[4];
    for (int m = 0; m < 4; ++m) y[m] = ((x[m] % d[m]) + d[m]) % d[m];
    return u + (index_of(d, y) * 4 + mu) * (long)nr * nr;
}

/* out = M0' M1' M2' M3', Mk' = Mk or Mk^+ */
static void path4(int n, const cplx *const m[4], const int dag[4], cplx *out)
{
    cplx *t = (cplx *)malloc(sizeof(cplx) * n * n), *a = (cplx *)malloc(sizeof(cplx) * n * n),
         *b = (cplx *)malloc(sizeof(cplx) * n * n);
    for (int i = 0; i < n * n; ++i) a[i] = 0;
    for (int i = 0; i < n; ++i) a[i * n + i] = 1;
    for (int k = 0; k < 4; ++k) {
        if (dag[k]) dagger(n, m[k], t);
        else memcpy(t, m[k], sizeof(cplx) * n * n);
        mm(n, a, t, b);
        memcpy(a, b, sizeof(cplx) * n * n);
    }
    memcpy(out, a, sizeof(cplx) * n * n);
    free(t);
    free(a);
    free(b);
}

/* F_mu,nu(x) (nr x nr) from the four leaves */
static void clover_f(const int d[4], int nr, const cplx *u, const int x[4], int mu, int nu, cplx *f)
{
    const long n2 = (long)nr * nr;
    cplx *q = (cplx *)calloc(n2, sizeof(cplx)), *leaf = (cplx *)malloc(sizeof(cplx) * n2);
    int xm[4], xn[4], xmn[4], xpm_mn[4], xmm_pn[4];
    for (int k = 0; k < 4; ++k) xm[k] = xn[k] = xmn[k] = xpm_mn[k] = xmm_pn[k] = x[k];
    /* shifted sites: x+mu, x+nu, x-mu, x-nu, x-mu-nu, x+mu-nu, x-mu+nu */
    int xpm[4], xpn[4];
    for (int k = 0; k < 4; ++k) xpm[k] = xpn[k] = x[k];
    xpm[mu] += 1;
    xpn[nu] += 1;
    xm[mu] -= 1;
    xn[nu] -= 1;
    xmn[mu] -= 1;
    xmn[nu] -= 1;
    xpm_mn[mu] += 1;
    xpm_mn[nu] -= 1;
    xmm_pn[mu] -= 1;
    xmm_pn[nu] += 1;
    {   /* U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ */
        const cplx *m[4] = {link_at(d, nr, u, x, mu), link_at(d, nr, u, xpm, nu), link_at(d, nr, u, xpn, mu),
                            link_at(d, nr, u, x, nu)};
        const int dg[4] = {0, 0, 1, 1};
        path4(nr, m, dg, leaf);
        for (long i = 0; i < n2; ++i) q[i] += leaf[i];
    }
    {   /* U_nu(x) U_mu(x-mu+nu)^+ U_nu(x-mu)^+ U_mu(x-mu) */
        const cplx *m[4] = {link_at(d, nr, u, x, nu), link_at(d, nr, u, xmm_pn, mu), link_at(d, nr, u, xm, nu),
                            link_at(d, nr, u, xm, mu)};
        const int dg[4] = {0, 1, 1, 0};
        path4(nr, m, dg, leaf);
        for (long i = 0; i < n2; ++i) q[i] += leaf[i];
    }
    {   /* U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu) */
        const cplx *m[4] = {link_at(d, nr, u, xm, mu), link_at(d, nr, u, xmn, nu), link_at(d, nr, u, xmn, mu),
                            link_at(d, nr, u, xn, nu)};
        const int dg[4] = {1, 1, 0, 0};
        path4(nr, m, dg, leaf);
        for (long i = 0; i < n2; ++i) q[i] += leaf[i];
    }
    {   /* U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+ */
        const cplx *m[4] = {link_at(d, nr, u, xn, nu), link_at(d, nr, u, xn, mu), link_at(d, nr, u, xpm_mn, nu),
                            link_at(d, nr, u, x, mu)};
        const int dg[4] = {1, 0, 0, 1};
        path4(nr, m, dg, leaf);
        for (long i = 0; i < n2; ++i) q[i] += leaf[i];
    }
    for (int a = 0; a < nr; ++a)
        for (int b = 0; b < nr; ++b) f[a * nr + b] = (q[a * nr + b] - conj(q[b * nr + a])) / 8.0;
    free(q);
    free(leaf);
}

/* A(x) as a (4 nr) x (4 nr) matrix, index spin * nr + colour, for every site: a_out [V][4nr][4nr] */
int orc_clover(const int *dims, int nr, const double *u, double kappa, double csw, double *a_out)
{
    if (!check_dims(dims, nr) || !u || !a_out) return ORC_EINVAL;
    init_gamma();
    const long v = vol(dims);
    const int sp = 4 * nr;
    const long n2 = (long)nr * nr;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < v; ++s) {
        int x[4];
        coords(dims, s, x);
        cplx *a = (cplx *)a_out + s * sp * sp;
        for (int i = 0; i < sp * sp; ++i) a[i] = 0;
        for (int i = 0; i < sp; ++i) a[i * sp + i] = 1;
        cplx *f = (cplx *)malloc(sizeof(cplx) * n2);
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                clover_f(dims, nr, (const cplx *)u, x, mu, nu, f);
                cplx gg[4][4];
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) {
                        cplx z = 0;
                        for (int k = 0; k < 4; ++k) z += G[mu][i][k] * G[nu][k][j];
                        gg[i][j] = z;
                    }
                for (int al = 0; al < 4; ++al)
                    for (int be = 0; be < 4; ++be) {
                        if (gg[al][be] == 0) continue;
                        for (int p = 0; p < nr; ++p)
                            for (int q = 0; q < nr; ++q)
                                a[(al * nr + p) * sp + be * nr + q] -= kappa * csw * gg[al][be] * f[p * nr + q];
                    }
            }
        free(f);
    }
    return ORC_OK;
}

/* Solve m x = b (n unknowns) by Gaussian elimination with partial pivoting; m, b overwritten. */
static int dense_solve(int n, cplx *m, cplx *b)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (cabs(m[r * n + c]) > cabs(m[piv * n + c])) piv = r;
        if (m[piv * n + c] == 0) return ORC_BREAKDOWN;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                cplx t = m[c * n + k];
                m[c * n + k] = m[piv * n + k];
                m[piv * n + k] = t;
            }
            cplx t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            const cplx l = m[r * n + c] / m[c * n + c];
            for (int k = c; k < n; ++k) m[r * n + k] -= l * m[c * n + k];
            b[r] -= l * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        cplx z = b[r];
        for (int k = r + 1; k < n; ++k) z -= m[r * n + k] * b[k];
        b[r] = z / m[r * n + r];
    }
    return ORC_OK;
}

/* A (inverse = 0) or A^-1 (inverse = 1) on the sites of one parity (half fields). */
int orc_clover_apply(const int *dims, int nr, const double *u, double kappa, double csw, int parity,
                     int inverse, const double *in_half, double *out_half)
{
    if (!check_dims(dims, nr) || !even_dims(dims) || (parity & ~1) || !u || !in_half || !out_half)
        return ORC_EINVAL;
    const long v = vol(dims);
    const int sp = 4 * nr;
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)v * sp * sp);
    int rc = orc_clover(dims, nr, u, kappa, csw, (double *)a);
    long k = 0;
    cplx *m = (cplx *)malloc(sizeof(cplx) * sp * sp);
    for (long s = 0; s < v && rc == ORC_OK; ++s) {
        int x[4];
        coords(dims, s, x);
        if (parity_of(x) != parity) continue;
        const cplx *in = (const cplx *)in_half + k * sp;
        cplx *out = (cplx *)out_half + k * sp;
        const cplx *as = a + s * sp * sp;
        if (inverse) {
            memcpy(m, as, sizeof(cplx) * sp * sp);
            memcpy(out, in, sizeof(cplx) * sp);
            rc = dense_solve(sp, m, out);
        } else {
            for (int i = 0; i < sp; ++i) {
                cplx z = 0;
                for (int j = 0; j < sp; ++j) z += as[i * sp + j] * in[j];
                out[i] = z;
            }
        }
        ++k;
    }
    free(m);
    free(a);
    return rc;
}

/* D_sw psi = A psi - kappa H psi (dagger: A psi - kappa H^+ psi; A is Hermitian). */
int orc_dsw(const int *dims, int nr, const double *u, double kappa, double csw, const double *theta,
            int dagger_, const double *in, double *out)
{
    if (!check_dims(dims, nr) || !u || !in || !out || in == out) return ORC_EINVAL;
    const long v = vol(dims);
    const int sp = 4 * nr;
    cplx *a = (cplx *)malloc(sizeof(cplx) * (size_t)v * sp * sp);
    int rc = orc_clover(dims, nr, u, kappa, csw, (double *)a);
    if (!rc) rc = orc_hop(dims, nr, u, theta, dagger_, in, out);
    if (!rc) {
        const cplx *pin = (const cplx *)in;
        cplx *po = (cplx *)out;
        for (long s = 0; s < v; ++s)
            for (int i = 0; i < sp; ++i) {
                cplx z = 0;
                for (int j = 0; j < sp; ++j) z += a[s * sp * sp + i * sp + j] * pin[s * sp + j];
                po[s * sp + i] = z - kappa * po[s * sp + i];
            }
    }
    free(a);
    return rc;
}

/* D_hat_sw psi_e = A_ee psi_e - kappa^2 H_eo A_oo^-1 H_oe psi_e (dagger: with H^+ blocks),
 * the Schur complement of D_sw on the even sites. */
int orc_dsw_eo(const int *dims, int nr, const double *u, double kappa, double csw, const double *theta,
               int dagger_, const double *in_e, double *out_e)
{
    if (!check_dims(dims, nr) || !even_dims(dims) || !in_e || !out_e || in_e == out_e) return ORC_EINVAL;
    const long h = vol(dims) / 2;
    const size_t bytes = sizeof(cplx) * (size_t)h * 4 * nr;
    cplx *t = (cplx *)malloc(bytes), *w = (cplx *)malloc(bytes), *ae = (cplx *)malloc(bytes);
    int rc = orc_hop_eo(dims, nr, u, theta, dagger_, 1, in_e, (double *)t);
    if (!rc) rc = orc_clover_apply(dims, nr, u, kappa, csw, 1, 1, (const double *)t, (double *)w);
    if (!rc) rc = orc_hop_eo(dims, nr, u, theta, dagger_, 0, (const double *)w, out_e);
    if (!rc) rc = orc_clover_apply(dims, nr, u, kappa, csw, 0, 0, in_e, (double *)ae);
    if (!rc) {
        const long n = h * 4 * nr;
        cplx *b = (cplx *)out_e;
        for (long i = 0; i < n; ++i) b[i] = ae[i] - kappa * kappa * b[i];
    }
    free(t);
    free(w);
    free(ae);
    return rc;
}

/* ------------------------------------------------------------------ CG */

typedef struct {
    const int *dims;
    int nr;
    const double *u;
    double kappa;
    const double *theta;
    int system; /* CG: 0 D^+D full lattice, 1 D_hat^+ D_hat on even sites;
                   BiCGstab: 0 D, 1 D_hat, 2 D_sw, 3 D_hat_sw */
    cplx *tmp;
    double csw;
} op_ctx;

static void apply_normal(op_ctx *c, const cplx *in, cplx *out)
{
    if (c->system == 0) {
        orc_dw(c->dims, c->nr, c->u, c->kappa, c->theta, 0, (const double *)in, (double *)c->tmp);
        orc_dw(c->dims, c->nr, c->u, c->kappa, c->theta, 1, (const double *)c->tmp, (double *)out);
    } else {
        orc_deo(c->dims, c->nr, c->u, c->kappa, c->theta, 0, (const double *)in, (double *)c->tmp);
        orc_deo(c->dims, c->nr, c->u, c->kappa, c->theta, 1, (const double *)c->tmp, (double *)out);
    }
}

static double norm2(long n, const cplx *a)
{
    double s = 0;
    for (long i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

static double re_dot(long n, const cplx *a, const cplx *b)
{
    double s = 0;
    for (long i = 0; i < n; ++i) s += creal(conj(a[i]) * b[i]);
    return s;
}

/*
 * Conjugate gradient (Hestenes-Stiefel) for A x = eta, A = D^+D (system 0) or
 * D_hat^+ D_hat on the even sites (system 1), starting from x = 0.  The loop
 * stops when the recursive residual reaches tol; the true residual eta - A x
 * is then recomputed and, if still above tol, CG restarts from it.
 * alpha/beta (length max_iter, may be NULL) receive the coefficients for the
 * Lanczos condition-number estimate.  info[0] = iterations, info[1] = true
 * relative residual, info[2] = restarts.
 */
int orc_cg(const int *dims, int nr, const double *u, double kappa, const double *theta,
           int system, const double *eta, double *x_out, double tol, int max_iter,
           double *alpha_hist, double *beta_hist, double *info)
{
    if (!check_dims(dims, nr) || (system != 0 && system != 1) || !eta || !x_out)
        return ORC_EINVAL;
    if (system == 1 && !even_dims(dims)) return ORC_EINVAL;
    const long sites = system == 0 ? vol(dims) : vol(dims) / 2;
    const long n = sites * 4 * nr;
    const size_t bytes = sizeof(cplx) * (size_t)n;
    op_ctx c = {dims, nr, u, kappa, theta, system, (cplx *)malloc(bytes), 0.0};
    cplx *x = (cplx *)x_out, *r = (cplx *)malloc(bytes), *p = (cplx *)malloc(bytes),
         *q = (cplx *)malloc(bytes);
    const cplx *b = (const cplx *)eta;
    memset(x, 0, bytes);
    memcpy(r, b, bytes);
    memcpy(p, b, bytes);
    const double bb = norm2(n, b);
    double rr = bb;
    int it = 0, restarts = 0, status = ORC_NOT_CONVERGED;
    double true_rel = bb > 0 ? 1.0 : 0.0;
    if (bb == 0) status = ORC_OK;
    while (status == ORC_NOT_CONVERGED && it < max_iter) {
        apply_normal(&c, p, q);
        const double pq = re_dot(n, p, q);
        if (!(pq > 0) || !isfinite(pq)) {
            status = ORC_BREAKDOWN;
            break;
        }
        const double a = rr / pq;
        for (long i = 0; i < n; ++i) {
            x[i] += a * p[i];
            r[i] -= a * q[i];
        }
        const double rr_new = norm2(n, r);
        const double bt = rr_new / rr;
        if (alpha_hist) alpha_hist[it] = a;
        if (beta_hist) beta_hist[it] = bt;
        ++it;
        if (sqrt(rr_new / bb) <= tol) {
            apply_normal(&c, x, q);
            for (long i = 0; i < n; ++i) r[i] = b[i] - q[i];
            rr = norm2(n, r);
            true_rel = sqrt(rr / bb);
            if (true_rel <= tol) {
                status = ORC_OK;
                break;
            }
            memcpy(p, r, bytes);
            ++restarts;
            continue;
        }
        for (long i = 0; i < n; ++i) p[i] = r[i] + bt * p[i];
        rr = rr_new;
    }
    if (status == ORC_NOT_CONVERGED) {
        apply_normal(&c, x, q);
        for (long i = 0; i < n; ++i) r[i] = b[i] - q[i];
        true_rel = sqrt(norm2(n, r) / bb);
    }
    if (info) {
        info[0] = it;
        info[1] = true_rel;
        info[2] = restarts;
    }
    free(c.tmp);
    free(r);
    free(p);
    free(q);
    return status;
}

/* ------------------------------------------------------------------ mixed-precision CG */

/*
 * CG with reliable updates (Clark et al., "Solving lattice QCD systems of
 * equations using mixed precision solvers on GPUs", Comput. Phys. Commun. 181
 * (2010) 1517), emulated on the CPU.  The paper's CG (Sec. 3.3) runs in one
 * precision; this is the mixed-precision form of it: the iteration runs on
 * fields stored in a low-precision format with single-precision arithmetic,
 * and every so often the solution is folded into an FP64 accumulator and the
 * residual is recomputed in FP64 from it.
 *
 * Emulation of the low precision:
 *   - arithmetic of the inner iteration (the operator, the vector updates) is
 *     C float arithmetic; the links are the FP64 links rounded once to the
 *     storage format;
 *   - every field the iteration stores (x, r, p and the operator's
 *     intermediate fields) is rounded to the storage format after each float
 *     result: binary32 leaves float values as they are, bfloat16 and binary16
 *     round them to nearest even;
 *   - inner products and norms accumulate the float values in FP64; alpha and
 *     beta are FP64 and enter the float updates rounded to float;
 *   - |r|^2 is taken from the float residual before it is stored.
 * With fmt = ORC_FMT_F64 the inner iteration is plain FP64 arithmetic; with
 * reliable updates off it is then the same computation as orc_cg.
 *
 * Reliable-update step (the readings this build fixes where the method is
 * stated loosely): a system is due after `every` of its own iterations
 * (0: never), when |r| fell below delta |r| at the last update (delta = 0:
 * never), or when its recursion meets tol.  A due system first completes its
 * iteration (p = r + beta p), then in FP64
 *     x64 += x_lo / s,  x_lo = 0,  r64 = eta - A x64;
 * if |r64| <= tol |eta| it stops; otherwise p_lo = s' (p_lo / s + (r64 -
 * r_lo / s)) and r_lo = s' r64, so p = r + beta p_prev still holds for the
 * replaced residual, and beta at the next iteration uses |r64|^2.  The inner
 * fields hold s times the true vectors: s = 1, except for binary16 storage
 * where s = sqrt(2 n / |r|^2) (n complex entries) is chosen at the start and
 * at every update so that the stored entries have RMS 1 (binary16 ends near
 * 6e-8); CG is linear, so alpha and beta do not depend on s.  A system whose
 * recursion met tol but whose FP64 residual did not is counted as a restart;
 * more than 20 restarts end the solve.
 *
 * system: 0 = D^+D on the full lattice, 1 = D_hat^+ D_hat on the even sites.
 * fmt: ORC_FMT_F64 (-1), 0 = binary32, 1 = bfloat16, 2 = binary16.
 * info: [0] iterations, [1] final FP64 true relative residual, [2] restarts,
 * [3] reliable updates (FP64 true-residual evaluations).
 * log (may be NULL, log_cap entries of 3 doubles): per update, the iteration
 * count at which it ran, its cause (1: every, 2: delta, 3: recursion met tol)
 * and |r64| / |eta|.
 * drop (may be NULL, max_iter entries): per iteration, |r|^2 / |r|^2 at the
 * last update (the quantity the delta trigger compares with delta^2).
 */
#define ORC_FMT_F64 (-1)

static double round_to_format(double x, int p, int emin, double maxfin);
static int fmt_params(int fmt, int *p, int *emin, double *maxfin);

/* one stored real: the value rounded to the storage format */
static double store_real(int fmt, double v)
{
    int p, emin;
    double maxfin;
    if (fmt == ORC_FMT_F64 || fmt_params(fmt, &p, &emin, &maxfin)) return v;
    return round_to_format(v, p, emin, maxfin);
}

static cplx store_c(int fmt, double re, double im) { return store_real(fmt, re) + I * store_real(fmt, im); }

/* float-arithmetic hop (H or H^+) on the full lattice: the hop_full sums in float */
typedef float complex fcplx;
static void hop_full_f(const int d[4], int nr, const fcplx *u, const double theta[4], int sign, const fcplx *in,
                       fcplx *out)
{
    init_gamma();
    const long v = vol(d);
    const int sp = 4 * nr;
    const long ls = (long)nr * nr;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < v; ++s) {
        int x[4];
        coords(d, s, x);
        fcplx acc[4 * 16];
        fcplx t[4 * 16];
        for (int i = 0; i < sp; ++i) acc[i] = 0;
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = 0; dir < 2; ++dir) {
                int y[4] = {x[0], x[1], x[2], x[3]};
                fcplx ph = 1.0f;
                const fcplx *link;
                int adj;
                if (dir == 0) {
                    y[mu] = (x[mu] + 1) % d[mu];
                    if (x[mu] == d[mu] - 1) ph = (float)cos(theta[mu]) + I * (float)sin(theta[mu]);
                    link = u + (s * 4 + mu) * ls;
                    adj = 0;
                } else {
                    y[mu] = (x[mu] + d[mu] - 1) % d[mu];
                    if (x[mu] == 0) ph = (float)cos(theta[mu]) - I * (float)sin(theta[mu]);
                    link = u + (index_of(d, y) * 4 + mu) * ls;
                    adj = 1;
                }
                const fcplx *src = in + index_of(d, y) * sp;
                for (int al = 0; al < 4; ++al)
                    for (int a = 0; a < nr; ++a) {
                        fcplx z = 0;
                        for (int b = 0; b < nr; ++b) {
                            fcplx l = adj ? conjf(link[b * nr + a]) : link[a * nr + b];
                            z += l * src[al * nr + b];
                        }
                        t[al * nr + a] = z;
                    }
                const float gs = (dir == 0 ? -1.0f : 1.0f) * (float)sign;
                for (int al = 0; al < 4; ++al)
                    for (int a = 0; a < nr; ++a) {
                        fcplx z = t[al * nr + a];
                        for (int be = 0; be < 4; ++be) z += gs * (fcplx)G[mu][al][be] * t[be * nr + a];
                        acc[al * nr + a] += ph * z;
                    }
            }
        }
        for (int i = 0; i < sp; ++i) out[s * sp + i] = acc[i];
    }
}

typedef struct {
    const int *dims;
    int nr, system, fmt;
    const double *theta;
    double kappa;
    const cplx *u64;   /* FP64 links */
    fcplx *ulo;        /* links rounded to the storage format, as floats */
    fcplx *fa, *fb;    /* full-lattice float scratch */
    cplx *da;          /* full-lattice double scratch */
    cplx *t1, *t2;     /* inner-field scratch (one system) */
    long n;            /* complex entries of one system's field */
} mixed_ctx;

/* float hop of a field given by its stored values (full lattice, or the
 * out_parity block from parity 1 - out_parity); out holds float values */
static void lo_hop(mixed_ctx *m, int dag, int out_parity, const cplx *in, cplx *out)
{
    const long v = vol(m->dims);
    const long nf = v * 4 * m->nr;
    if (m->system == 0) {
        for (long i = 0; i < nf; ++i) m->fa[i] = (float)creal(in[i]) + I * (float)cimag(in[i]);
    } else {
        embed(m->dims, m->nr, 1 - out_parity, in, m->da);
        for (long i = 0; i < nf; ++i) m->fa[i] = (float)creal(m->da[i]) + I * (float)cimag(m->da[i]);
    }
    hop_full_f(m->dims, m->nr, m->ulo, m->theta, dag ? -1 : 1, m->fa, m->fb);
    if (m->system == 0) {
        for (long i = 0; i < nf; ++i) out[i] = crealf(m->fb[i]) + I * cimagf(m->fb[i]);
    } else {
        for (long i = 0; i < nf; ++i) m->da[i] = crealf(m->fb[i]) + I * cimagf(m->fb[i]);
        extract(m->dims, m->nr, out_parity, m->da, out);
    }
}

/* out = in - c * hop(in) in float, c rounded to float; store: round to the format */
static void lo_axpy_hop(mixed_ctx *m, int dag, const cplx *in, cplx *out, int store)
{
    const float c = (float)(m->system == 0 ? m->kappa : m->kappa * m->kappa);
    if (m->system == 0) {
        lo_hop(m, dag, 0, in, m->t1);
    } else {
        lo_hop(m, dag, 1, in, m->t2);
        for (long i = 0; i < m->n; ++i) m->t2[i] = store_c(m->fmt, creal(m->t2[i]), cimag(m->t2[i]));
        lo_hop(m, dag, 0, m->t2, m->t1);
    }
    for (long i = 0; i < m->n; ++i) {
        const float re = (float)creal(in[i]) - c * (float)creal(m->t1[i]);
        const float im = (float)cimag(in[i]) - c * (float)cimag(m->t1[i]);
        out[i] = store ? store_c(m->fmt, re, im) : (double)re + I * (double)im;
    }
}

/* q = A p in the inner precision (D p stored, D^+ of it in float) */
static void lo_apply_normal(mixed_ctx *m, const cplx *p, cplx *s, cplx *q)
{
    lo_axpy_hop(m, 0, p, s, 1);
    lo_axpy_hop(m, 1, s, q, 0);
}

static int mixed_mutation = 0; /* planted mistakes for the pin tests; 0 = none */

void orc_set_mixed_mutation(int k) { mixed_mutation = k; }

int orc_cg_mixed(const int *dims, int nr, const double *u, double kappa, const double *theta, int system,
                 const double *eta, double *x_out, double tol, int max_iter, int fmt, int every, double delta,
                 double *info, double *log, int log_cap, double *drop)
{
    int fp, fe;
    double fm;
    if (!check_dims(dims, nr) || (system != 0 && system != 1) || !eta || !x_out || max_iter < 1)
        return ORC_EINVAL;
    if (fmt != ORC_FMT_F64 && fmt_params(fmt, &fp, &fe, &fm)) return ORC_EINVAL;
    if (system == 1 && !even_dims(dims)) return ORC_EINVAL;
    const long v = vol(dims);
    const long n = (system == 0 ? v : v / 2) * 4 * nr;
    const long nf = v * 4 * nr;
    const size_t bytes = sizeof(cplx) * (size_t)n;
    const int lo = fmt != ORC_FMT_F64;
    mixed_ctx m = {dims, nr, system, fmt, theta, kappa, (const cplx *)u, NULL, NULL, NULL, NULL, NULL, NULL, n};
    op_ctx c64 = {dims, nr, u, kappa, theta, system, (cplx *)malloc(bytes), 0.0};
    cplx *x64 = (cplx *)x_out, *x = (cplx *)calloc(n, sizeof(cplx)), *r = (cplx *)malloc(bytes),
         *p = (cplx *)malloc(bytes), *q = (cplx *)malloc(bytes), *s = (cplx *)malloc(bytes),
         *r64 = (cplx *)malloc(bytes);
    if (lo) {
        const long nl = v * 4 * (long)nr * nr;
        m.ulo = (fcplx *)malloc(sizeof(fcplx) * nl);
        for (long i = 0; i < nl; ++i) {
            const cplx z = store_c(fmt, creal(m.u64[i]), cimag(m.u64[i]));
            m.ulo[i] = (float)creal(z) + I * (float)cimag(z);
        }
        m.fa = (fcplx *)malloc(sizeof(fcplx) * nf);
        m.fb = (fcplx *)malloc(sizeof(fcplx) * nf);
        m.da = (cplx *)malloc(sizeof(cplx) * nf);
        m.t1 = (cplx *)malloc(bytes);
        m.t2 = (cplx *)malloc(bytes);
    }
    const cplx *b = (const cplx *)eta;
    memset(x64, 0, bytes);
    const double bb = norm2(n, b);
    /* inner fields hold sc times the true vectors (binary16: RMS 1) */
    double sc = (fmt == 2 && bb > 0 && isfinite(bb) && mixed_mutation != 6) ? sqrt(2.0 * (double)n / bb) : 1.0;
    for (long i = 0; i < n; ++i) {
        r[i] = store_c(fmt, sc * creal(b[i]), sc * cimag(b[i]));
        p[i] = r[i];
    }
    double rr = bb * sc * sc, rr_last = rr;
    int it = 0, since = 0, restarts = 0, updates = 0, nlog = 0;
    int status = bb > 0 ? ORC_NOT_CONVERGED : ORC_OK;
    double true_rel = bb > 0 ? 1.0 : 0.0;
    if (!isfinite(bb)) status = ORC_BREAKDOWN;
    while (status == ORC_NOT_CONVERGED) {
        /* q = A p, alpha = |r|^2 / <p, q> */
        if (lo) lo_apply_normal(&m, p, s, q);
        else apply_normal(&c64, p, q);
        const double pq = re_dot(n, p, q);
        if (!(pq > 0) || !isfinite(pq)) {
            status = ORC_BREAKDOWN;
            break;
        }
        const double a = rr / pq;
        double rr_new;
        if (lo) {
            const float af = (float)a;
            rr_new = 0;
            for (long i = 0; i < n; ++i) {
                const float xr = (float)creal(x[i]) + af * (float)creal(p[i]);
                const float xi = (float)cimag(x[i]) + af * (float)cimag(p[i]);
                const float rr_ = (float)creal(r[i]) - af * (float)creal(q[i]);
                const float ri = (float)cimag(r[i]) - af * (float)cimag(q[i]);
                x[i] = store_c(fmt, xr, xi);
                r[i] = store_c(fmt, rr_, ri);
                rr_new += (double)rr_ * rr_ + (double)ri * ri;
            }
        } else {
            for (long i = 0; i < n; ++i) {
                x[i] += a * p[i];
                r[i] -= a * q[i];
            }
            rr_new = norm2(n, r);
        }
        const double bt = rr_new / rr;
        ++it;
        ++since;
        rr = rr_new;
        if (drop) drop[it - 1] = rr_new / rr_last;
        int cause = 0;
        if (!isfinite(rr_new)) {
            status = ORC_BREAKDOWN;
            break;
        } else if (sqrt(rr_new / (bb * sc * sc)) <= tol) {
            cause = 3;
        } else if (it >= max_iter) {
            break;
        } else if (every > 0 && since >= every + (mixed_mutation == 5)) {
            cause = 1;
        } else if (delta > 0 && rr_new < delta * delta * rr_last) {
            cause = 2;
        }
        /* p = r + beta p (also for a system that is now due) */
        if (lo) {
            const float bf = (float)bt;
            for (long i = 0; i < n; ++i)
                p[i] = store_c(fmt, (float)creal(r[i]) + bf * (float)creal(p[i]),
                               (float)cimag(r[i]) + bf * (float)cimag(p[i]));
        } else {
            for (long i = 0; i < n; ++i) p[i] = r[i] + bt * p[i];
        }
        if (!cause) continue;
        if (cause == 3 && mixed_mutation == 4) { /* planted: trust the recursion */
            for (long i = 0; i < n; ++i) x64[i] += x[i] / sc;
            status = ORC_OK;
            break;
        }
        /* reliable update: fold x_lo into x64, FP64 true residual */
        const double inv = 1.0 / sc;
        for (long i = 0; i < n; ++i) {
            const double fr = mixed_mutation == 2 ? 1.0 : inv;
            x64[i] = creal(x64[i]) + creal(x[i]) * fr + I * (cimag(x64[i]) + cimag(x[i]) * fr);
            if (mixed_mutation == 3) x64[i] = store_c(0, creal(x64[i]), cimag(x64[i]));
            if (mixed_mutation != 1) x[i] = 0;
        }
        if (mixed_mutation == 7 && lo) lo_apply_normal(&m, x64, s, q);
        else apply_normal(&c64, x64, q);
        for (long i = 0; i < n; ++i) r64[i] = b[i] - q[i];
        const double rt = norm2(n, r64);
        ++updates;
        since = 0;
        true_rel = sqrt(rt / bb);
        if (log && nlog < log_cap) {
            log[3 * nlog] = it;
            log[3 * nlog + 1] = cause;
            log[3 * nlog + 2] = true_rel;
            ++nlog;
        }
        if (true_rel <= tol) {
            status = ORC_OK;
            break;
        }
        if (!isfinite(rt)) {
            status = ORC_BREAKDOWN;
            break;
        }
        if (cause == 3 && ++restarts > 20) break;
        /* resume from the true residual: keep p = r + beta p_prev valid */
        const double sn = (fmt == 2 && mixed_mutation != 6) ? sqrt(2.0 * (double)n / rt) : 1.0;
        const double rsc = mixed_mutation == 8 ? 1.0 : sn;
        for (long i = 0; i < n; ++i) {
            const cplx ro = r[i] * inv, po = p[i] * inv;
            r[i] = store_c(fmt, rsc * creal(r64[i]), rsc * cimag(r64[i]));
            const cplx pn = po + (r64[i] - ro);
            p[i] = store_c(fmt, sn * creal(pn), sn * cimag(pn));
        }
        sc = sn;
        rr = rt * sc * sc;
        rr_last = rr;
    }
    if (status == ORC_NOT_CONVERGED || status == ORC_BREAKDOWN) {
        for (long i = 0; i < n; ++i) x64[i] += x[i] / sc;
        apply_normal(&c64, x64, q);
        for (long i = 0; i < n; ++i) r64[i] = b[i] - q[i];
        true_rel = bb > 0 ? sqrt(norm2(n, r64) / bb) : 0.0;
    } else if (mixed_mutation == 4) {
        apply_normal(&c64, x64, q);
        for (long i = 0; i < n; ++i) r64[i] = b[i] - q[i];
        true_rel = sqrt(norm2(n, r64) / bb);
    }
    if (info) {
        info[0] = it;
        info[1] = true_rel;
        info[2] = restarts;
        info[3] = updates;
        info[4] = nlog;
    }
    free(c64.tmp);
    free(x);
    free(r);
    free(p);
    free(q);
    free(s);
    free(r64);
    if (lo) {
        free(m.ulo);
        free(m.fa);
        free(m.fb);
        free(m.da);
        free(m.t1);
        free(m.t2);
    }
    return status;
}

/* ------------------------------------------------------------------ BiCGstab */

/* D (system 0, full lattice) or D_hat (system 1, even sites) applied to in. */
static void apply_op(op_ctx *c, const cplx *in, cplx *out)
{
    if (c->system == 0)
        orc_dw(c->dims, c->nr, c->u, c->kappa, c->theta, 0, (const double *)in, (double *)out);
    else if (c->system == 1)
        orc_deo(c->dims, c->nr, c->u, c->kappa, c->theta, 0, (const double *)in, (double *)out);
    else if (c->system == 2)
        orc_dsw(c->dims, c->nr, c->u, c->kappa, c->csw, c->theta, 0, (const double *)in, (double *)out);
    else
        orc_dsw_eo(c->dims, c->nr, c->u, c->kappa, c->csw, c->theta, 0, (const double *)in, (double *)out);
}

/* <a, b> = sum_i conj(a_i) b_i */
static cplx cdot(long n, const cplx *a, const cplx *b)
{
    cplx s = 0;
    for (long i = 0; i < n; ++i) s += conj(a[i]) * b[i];
    return s;
}

static int cfinite(cplx z) { return isfinite(creal(z)) && isfinite(cimag(z)); }

/*
 * Stabilised bi-conjugate gradient (van der Vorst, SIAM J. Sci. Stat. Comput.
 * 13 (1992) 631, one of the inverters of Sec. 3.3) for D x = b on the full
 * lattice (system 0) or D_hat x_e = b_e on the even sites (system 1), from
 * x = 0 with the shadow residual r0 equal to the starting residual.  Each
 * iteration is a Bi-CG step followed by a one-dimensional minimal-residual
 * step:
 *   p = r + (rho / rho_old)(alpha / omega)(p - omega v)   (p = r after a start)
 *   v = A p,  alpha = rho / <r0, v>,  s = r - alpha v
 *   t = A s,  omega = <t, s> / |t|^2  (0 when t = 0),  x += alpha p + omega s
 *   r = s - omega t,  rho_old = rho,  rho = <r0, r>
 * with <a, b> = sum conj(a) b.  When |r| <= tol |b| the true residual b - A x
 * is recomputed; if it is still above tol, or a coefficient is not finite
 * (rho, <r0, v> or omega vanished), the iteration starts again from the true
 * residual, which also becomes the new shadow vector.  info[0] = iterations,
 * info[1] = true relative residual, info[2] = restarts.
 */
static int bicgstab_run(op_ctx c, const double *b_in, double *x_out, double tol, int max_iter, double *info);

int orc_bicgstab(const int *dims, int nr, const double *u, double kappa, const double *theta,
                 int system, const double *b_in, double *x_out, double tol, int max_iter,
                 double *info)
{
    if (!check_dims(dims, nr) || (system != 0 && system != 1) || !b_in || !x_out)
        return ORC_EINVAL;
    if (system == 1 && !even_dims(dims)) return ORC_EINVAL;
    op_ctx c = {dims, nr, u, kappa, theta, system, NULL, 0.0};
    return bicgstab_run(c, b_in, x_out, tol, max_iter, info);
}

/* The same method for the clover-improved D_sw (system 0) or its Schur complement D_hat_sw (1). */
int orc_bicgstab_sw(const int *dims, int nr, const double *u, double kappa, double csw, const double *theta,
                    int system, const double *b_in, double *x_out, double tol, int max_iter, double *info)
{
    if (!check_dims(dims, nr) || (system != 0 && system != 1) || !b_in || !x_out)
        return ORC_EINVAL;
    if (system == 1 && !even_dims(dims)) return ORC_EINVAL;
    op_ctx c = {dims, nr, u, kappa, theta, system + 2, NULL, csw};
    return bicgstab_run(c, b_in, x_out, tol, max_iter, info);
}

static int bicgstab_run(op_ctx c, const double *b_in, double *x_out, double tol, int max_iter, double *info)
{
    const int *dims = c.dims;
    const int nr = c.nr;
    const long sites = (c.system == 0 || c.system == 2) ? vol(dims) : vol(dims) / 2;
    const long n = sites * 4 * nr;
    const size_t bytes = sizeof(cplx) * (size_t)n;
    cplx *x = (cplx *)x_out;
    cplx *r = (cplx *)malloc(bytes), *r0 = (cplx *)malloc(bytes), *p = (cplx *)malloc(bytes),
         *v = (cplx *)malloc(bytes), *s = (cplx *)malloc(bytes), *t = (cplx *)malloc(bytes);
    const cplx *b = (const cplx *)b_in;
    memset(x, 0, bytes);
    memcpy(r, b, bytes);
    memcpy(r0, b, bytes);
    memset(p, 0, bytes);
    memset(v, 0, bytes);
    const double bb = norm2(n, b);
    const double tol2 = tol * tol * bb;
    cplx rho = bb, rho_old = 1, alpha = 1, omega = 1;
    int it = 0, restarts = 0, fresh = 1, status = ORC_NOT_CONVERGED;
    double rr_true = bb;
    if (!isfinite(bb)) status = ORC_BREAKDOWN;
    else if (bb == 0) status = ORC_OK;
    while (status == ORC_NOT_CONVERGED && it < max_iter) {
        int restart = 0;
        if (fresh) {
            memcpy(p, r, bytes);
        } else {
            const cplx beta = (rho / rho_old) * (alpha / omega);
            if (!cfinite(beta) || omega == 0 || rho_old == 0) {
                restart = 1;
            } else {
                for (long i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            }
        }
        if (!restart) {
            fresh = 0;
            apply_op(&c, p, v);
            const cplx rv = cdot(n, r0, v);
            alpha = rho / rv;
            if (rv == 0 || !cfinite(alpha)) restart = 1;
        }
        if (!restart) {
            for (long i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
            apply_op(&c, s, t);
            const double tt = norm2(n, t);
            omega = tt > 0 ? cdot(n, t, s) / tt : 0;
            for (long i = 0; i < n; ++i) {
                x[i] += alpha * p[i] + omega * s[i];
                r[i] = s[i] - omega * t[i];
            }
            ++it;
            rho_old = rho;
            rho = cdot(n, r0, r);
            if (norm2(n, r) > tol2) continue;
        }
        /* recursive convergence or breakdown: check the true residual */
        apply_op(&c, x, t);
        for (long i = 0; i < n; ++i) r[i] = b[i] - t[i];
        rr_true = norm2(n, r);
        if (!isfinite(rr_true)) {
            status = ORC_BREAKDOWN;
            break;
        }
        if (rr_true <= tol2) {
            status = ORC_OK;
            break;
        }
        if (++restarts > 100) {
            status = ORC_BREAKDOWN;
            break;
        }
        memcpy(r0, r, bytes);
        rho = rr_true;
        fresh = 1;
    }
    if (status == ORC_NOT_CONVERGED) {
        apply_op(&c, x, t);
        for (long i = 0; i < n; ++i) r[i] = b[i] - t[i];
        rr_true = norm2(n, r);
    }
    if (info) {
        info[0] = it;
        info[1] = bb > 0 ? sqrt(rr_true / bb) : 0.0;
        info[2] = restarts;
    }
    free(r);
    free(r0);
    free(p);
    free(v);
    free(s);
    free(t);
    return status;
}

/* ------------------------------------------------------------------ QMR-g5 */

/* out = g5 in on n_sites sites (literal 4x4 product with gamma_5) */
static void g5_apply(long n_sites, int nr, const cplx *in, cplx *out)
{
    init_gamma();
    for (long s = 0; s < n_sites; ++s)
        for (int al = 0; al < 4; ++al)
            for (int a = 0; a < nr; ++a) {
                cplx z = 0;
                for (int be = 0; be < 4; ++be) z += G[4][al][be] * in[(s * 4 + be) * nr + a];
                out[(s * 4 + al) * nr + a] = z;
            }
}

/* [a, b] = <a, g5 b> = sum conj(a) (g5 b) */
static cplx g5_dot(long n_sites, int nr, const cplx *a, const cplx *b, cplx *tmp)
{
    g5_apply(n_sites, nr, b, tmp);
    return cdot(n_sites * 4 * nr, a, tmp);
}

/*
 * QMR on the g5-symmetric Lanczos process (the QMR-g5 inverter of Sec. 3.3):
 * D and D_hat satisfy A^+ = g5 A g5, so A is self-adjoint in the indefinite
 * form [a, b] = <a, g5 b> and the two-sided Lanczos process needs one product
 * with A per step.  With v_1 = r_0 / |r_0|, delta_n = [v_n, v_n]:
 *   alpha_n = [v_n, A v_n] / delta_n,   beta_n = rho_n delta_n / delta_{n-1}  (beta_1 = 0)
 *   w = A v_n - alpha_n v_n - beta_n v_{n-1},  rho_{n+1} = |w|,  v_{n+1} = w / rho_{n+1}
 * so that A V_n = V_{n+1} T_n with T_n real tridiagonal ((n+1) x n).  The
 * iterate x_n = x_0 + V_n y_n minimises the quasi-residual |rho_1 e_1 - T_n y|,
 * updated with Givens rotations and three-term direction vectors; the true
 * residual satisfies |r_n| <= sqrt(k + 1) |quasi-residual| after k steps from
 * the last start.  When that bound reaches tol |b| (or [v, v] or rho vanishes)
 * the true residual is recomputed; above tol the process starts again from it.
 * (Stopping on the quasi-residual alone can stall: a start from a residual at
 * rounding level has [v, v] near zero, the Lanczos step is then almost empty
 * and the quasi-residual still passes.)  system 0: D on
 * the full lattice, 1: D_hat on the even sites.  info as orc_bicgstab.
 */
int orc_qmr_g5(const int *dims, int nr, const double *u, double kappa, const double *theta, int system,
               const double *b_in, double *x_out, double tol, int max_iter, double *info)
{
    if (!check_dims(dims, nr) || (system != 0 && system != 1) || !b_in || !x_out) return ORC_EINVAL;
    if (system == 1 && !even_dims(dims)) return ORC_EINVAL;
    op_ctx c = {dims, nr, u, kappa, theta, system, NULL, 0.0};
    const long sites = system == 0 ? vol(dims) : vol(dims) / 2;
    const long n = sites * 4 * nr;
    const size_t bytes = sizeof(cplx) * (size_t)n;
    cplx *x = (cplx *)x_out;
    cplx *r = (cplx *)malloc(bytes), *v = (cplx *)malloc(bytes), *vp = (cplx *)malloc(bytes),
         *w = (cplx *)malloc(bytes), *d1 = (cplx *)malloc(bytes), *d2 = (cplx *)malloc(bytes),
         *tmp = (cplx *)malloc(bytes);
    const cplx *b = (const cplx *)b_in;
    memset(x, 0, bytes);
    memcpy(r, b, bytes);
    const double bb = norm2(n, b);
    int it = 0, restarts = 0, status = ORC_NOT_CONVERGED;
    double rr_true = bb;
    if (!isfinite(bb)) status = ORC_BREAKDOWN;
    else if (bb == 0) status = ORC_OK;
    while (status == ORC_NOT_CONVERGED && it < max_iter) {
        /* start (or start again) from the residual r */
        const double rho1 = sqrt(norm2(n, r));
        for (long i = 0; i < n; ++i) {
            v[i] = r[i] / rho1;
            vp[i] = 0;
            d1[i] = 0;
            d2[i] = 0;
        }
        double delta = creal(g5_dot(sites, nr, v, v, tmp));
        double beta = 0;
        double c1 = 1, s1 = 0, c2 = 1, s2 = 0; /* rotations G_{n-1}, G_{n-2} */
        double tau = rho1;                     /* rotated right-hand side, current row */
        int check = 0, k = 0;                  /* k: steps since this start */
        while (it < max_iter) {
            if (delta == 0 || !isfinite(delta)) {
                check = 1;
                break;
            }
            apply_op(&c, v, w);
            const double alpha = creal(g5_dot(sites, nr, v, w, tmp)) / delta;
            for (long i = 0; i < n; ++i) w[i] -= alpha * v[i] + beta * vp[i];
            const double rho_next = sqrt(norm2(n, w));
            /* column n of T: beta (row n-1), alpha (row n), rho_next (row n+1) */
            const double e = s2 * beta;
            const double f0 = c2 * beta;
            const double f = c1 * f0 + s1 * alpha;
            const double g0 = -s1 * f0 + c1 * alpha;
            const double rr = sqrt(g0 * g0 + rho_next * rho_next);
            const double cn = g0 / rr, sn = rho_next / rr;
            for (long i = 0; i < n; ++i) {
                const cplx dn = (v[i] - f * d1[i] - e * d2[i]) / rr;
                d2[i] = d1[i];
                d1[i] = dn;
                x[i] += cn * tau * dn;
            }
            tau = -sn * tau;
            ++it;
            ++k;
            c2 = c1;
            s2 = s1;
            c1 = cn;
            s1 = sn;
            if ((k + 1) * tau * tau <= tol * tol * bb || rho_next == 0 || !isfinite(rho_next)) {
                check = 1;
                break;
            }
            /* next Lanczos vector */
            for (long i = 0; i < n; ++i) {
                vp[i] = v[i];
                v[i] = w[i] / rho_next;
            }
            const double delta_next = creal(g5_dot(sites, nr, v, v, tmp));
            beta = rho_next * delta_next / delta;
            delta = delta_next;
        }
        if (!check) break; /* max_iter */
        apply_op(&c, x, tmp);
        for (long i = 0; i < n; ++i) r[i] = b[i] - tmp[i];
        rr_true = norm2(n, r);
        if (!isfinite(rr_true)) {
            status = ORC_BREAKDOWN;
            break;
        }
        if (rr_true <= tol * tol * bb) {
            status = ORC_OK;
            break;
        }
        if (++restarts > 100) {
            status = ORC_BREAKDOWN;
            break;
        }
    }
    if (status == ORC_NOT_CONVERGED) {
        apply_op(&c, x, tmp);
        for (long i = 0; i < n; ++i) r[i] = b[i] - tmp[i];
        rr_true = norm2(n, r);
    }
    if (info) {
        info[0] = it;
        info[1] = bb > 0 ? sqrt(rr_true / bb) : 0.0;
        info[2] = restarts;
    }
    free(r);
    free(v);
    free(vp);
    free(w);
    free(d1);
    free(d2);
    free(tmp);
    return status;
}

/* ------------------------------------------------------------------ 16-bit rounding */

/*
 * Round a double to the nearest value of a binary floating-point format with
 * p significand bits and smallest normal exponent emin (ties to even), by
 * scaling to an integer: x = m 2^e with 0.5 <= |m| < 1, quantum
 * 2^(max(e, emin + 1) - p).  Values beyond the largest finite number go to
 * infinity as IEEE round-to-nearest prescribes.
 */
static double round_to_format(double x, int p, int emin, double maxfin)
{
    if (x == 0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);
    if (e < emin + 1) e = emin + 1;
    const double q = ldexp(1.0, e - p);
    const double r = nearbyint(x / q) * q; /* default rounding mode: ties to even */
    if (fabs(r) > maxfin) return copysign(INFINITY, x);
    return r;
}

/* fmt: 0 = IEEE binary32, 1 = bfloat16, 2 = IEEE binary16: significand bits,
 * smallest normal exponent and largest finite value (nonzero: unknown fmt) */
static int fmt_params(int fmt, int *p, int *emin, double *maxfin)
{
    switch (fmt) {
    case 0: *p = 24; *emin = -126; *maxfin = ldexp(2.0 - ldexp(1.0, -23), 127); return 0;
    case 1: *p = 8; *emin = -126; *maxfin = ldexp(2.0 - ldexp(1.0, -7), 127); return 0;
    case 2: *p = 11; *emin = -14; *maxfin = 65504.0; return 0;
    }
    return 1;
}

/* Round n doubles in place to format fmt (as fmt_params). */
int orc_round(int fmt, long n, double *a)
{
    int p, emin;
    double maxfin;
    if (fmt_params(fmt, &p, &emin, &maxfin)) return ORC_EINVAL;
    for (long i = 0; i < n; ++i) a[i] = round_to_format(a[i], p, emin, maxfin);
    return ORC_OK;
}

/* Threads the OpenMP loops above use. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
