/* Test driver for the oracle under AddressSanitizer / UndefinedBehaviorSanitizer
 * (test infrastructure only: built and run by tests/test_sanitizers.py on the CPU).
 * Calls every entry point of oracle.c on tiny lattices, including the argument
 * errors, and checks that the results are finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_rep_dim(int nc, int rep);
int orc_rep_map(int nc, int rep, long n_links, const double *u_f, double *u_r);
int orc_rep_basis(int nc, int rep, double *out);
int orc_hop(const int *dims, int nr, const double *u, const double *theta, int dagger_, const double *in, double *out);
int orc_dw(const int *dims, int nr, const double *u, double kappa, const double *theta, int dagger_, const double *in,
           double *out);
int orc_hop_eo(const int *dims, int nr, const double *u, const double *theta, int dagger_, int out_parity,
               const double *in_half, double *out_half);
int orc_deo(const int *dims, int nr, const double *u, double kappa, const double *theta, int dagger_,
            const double *in_e, double *out_e);
int orc_clover(const int *dims, int nr, const double *u, double kappa, double csw, double *a_out);
int orc_clover_apply(const int *dims, int nr, const double *u, double kappa, double csw, int parity, int inverse,
                     const double *in, double *out);
int orc_dsw(const int *dims, int nr, const double *u, double kappa, double csw, const double *theta, int dagger_,
            const double *in, double *out);
int orc_dsw_eo(const int *dims, int nr, const double *u, double kappa, double csw, const double *theta, int dagger_,
               const double *in_e, double *out_e);
int orc_cg(const int *dims, int nr, const double *u, double kappa, const double *theta, int system, const double *eta,
           double *x_out, double tol, int max_iter, double *alpha_hist, double *beta_hist, double *info);
int orc_cg_mixed(const int *dims, int nr, const double *u, double kappa, const double *theta, int system,
                 const double *eta, double *x_out, double tol, int max_iter, int fmt, int every, double delta,
                 double *info, double *log, int log_cap, double *drop);
int orc_bicgstab(const int *dims, int nr, const double *u, double kappa, const double *theta, int system,
                 const double *b_in, double *x_out, double tol, int max_iter, double *info);
int orc_bicgstab_sw(const int *dims, int nr, const double *u, double kappa, double csw, const double *theta,
                    int system, const double *b_in, double *x_out, double tol, int max_iter, double *info);
int orc_qmr_g5(const int *dims, int nr, const double *u, double kappa, const double *theta, int system,
               const double *b_in, double *x_out, double tol, int max_iter, double *info);
int orc_round(int fmt, long n, double *a);

static unsigned long long state = 88172645463325252ull;
static double rnd(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}

static int finite_all(const double *a, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

static int run(int nc, int rep, const int dims[4])
{
    const int nr = orc_rep_dim(nc, rep);
    const long v = (long)dims[0] * dims[1] * dims[2] * dims[3];
    const long nf = 2L * v * 4 * nc * nc, nu = 2L * v * 4 * nr * nr, ns = 2L * v * 4 * nr;
    double *uf = calloc(nf, sizeof(double)), *ur = calloc(nu, sizeof(double));
    double *in = calloc(ns, sizeof(double)), *out = calloc(ns, sizeof(double)), *tmp = calloc(ns, sizeof(double));
    double *a = calloc((size_t)v * 2 * (4 * nr) * (4 * nr), sizeof(double));
    double *basis = calloc(2L * nr * nc * nc * 4 + 64, sizeof(double));
    const double theta[4] = {3.14159265358979, 0.3, -0.2, 0.1};
    double info[8], alpha[400], beta[400], log[3 * 500], drop[400];
    /* unitary links: diagonal phases are enough for memory checking */
    for (long l = 0; l < v * 4; ++l)
        for (int i = 0; i < nc; ++i) {
            const double ph = 3.0 * rnd();
            uf[2 * ((l * nc + i) * nc + i)] = cos(ph);
            uf[2 * ((l * nc + i) * nc + i) + 1] = sin(ph);
        }
    for (long i = 0; i < ns; ++i) in[i] = rnd();
    CHECK(orc_rep_map(nc, rep, v * 4, uf, ur) == 0 && finite_all(ur, nu));
    (void)orc_rep_basis(nc, rep, basis);
    CHECK(orc_hop(dims, nr, ur, theta, 0, in, out) == 0 && finite_all(out, ns));
    CHECK(orc_dw(dims, nr, ur, 0.12, theta, 1, in, out) == 0 && finite_all(out, ns));
    CHECK(orc_dw(dims, nr, ur, 0.12, theta, 0, in, in) != 0); /* in == out is refused */
    CHECK(orc_hop_eo(dims, nr, ur, theta, 0, 1, in, out) == 0 && finite_all(out, ns / 2));
    CHECK(orc_deo(dims, nr, ur, 0.12, theta, 1, in, out) == 0 && finite_all(out, ns / 2));
    CHECK(orc_clover(dims, nr, ur, 0.12, 1.1, a) == 0);
    CHECK(orc_clover_apply(dims, nr, ur, 0.12, 1.1, 1, 1, in, out) == 0 && finite_all(out, ns / 2));
    CHECK(orc_dsw(dims, nr, ur, 0.12, 1.1, theta, 1, in, out) == 0 && finite_all(out, ns));
    CHECK(orc_dsw_eo(dims, nr, ur, 0.12, 1.1, theta, 0, in, out) == 0 && finite_all(out, ns / 2));
    CHECK(orc_cg(dims, nr, ur, 0.12, theta, 1, in, out, 1e-10, 400, alpha, beta, info) == 0);
    CHECK(orc_cg(dims, nr, ur, 0.12, theta, 0, in, out, 1e-10, 400, alpha, beta, info) == 0);
    for (int fmt = -1; fmt < 3; ++fmt)
        CHECK(orc_cg_mixed(dims, nr, ur, 0.12, theta, 1, in, out, 1e-10, 400, fmt, 20, 1e-2, info, log, 500, drop) == 0);
    CHECK(orc_bicgstab(dims, nr, ur, 0.12, theta, 1, in, out, 1e-10, 400, info) == 0);
    CHECK(orc_bicgstab_sw(dims, nr, ur, 0.12, 1.1, theta, 0, in, out, 1e-10, 400, info) == 0);
    CHECK(orc_qmr_g5(dims, nr, ur, 0.12, theta, 1, in, out, 1e-10, 400, info) == 0);
    memcpy(tmp, in, ns * sizeof(double));
    for (int fmt = 0; fmt < 3; ++fmt) CHECK(orc_round(fmt, ns, tmp) == 0 && finite_all(tmp, ns));
    /* argument errors */
    const int bad[4] = {3, 2, 2, 2};
    CHECK(orc_deo(bad, nr, ur, 0.12, theta, 0, in, out) != 0);
    CHECK(orc_hop(dims, nr, NULL, theta, 0, in, out) != 0);
    free(uf); free(ur); free(in); free(out); free(tmp); free(a); free(basis);
    return 0;
}

int main(void)
{
    const int d1[4] = {2, 2, 2, 4}, d2[4] = {2, 4, 2, 2};
    if (run(2, 0, d1) || run(2, 1, d2) || run(3, 0, d1) || run(3, 2, d2) || run(4, 3, d1)) return 1;
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
