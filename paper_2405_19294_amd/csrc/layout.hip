// Layout conversion and the representation map (arXiv 2405.19294, Sec. 3.1:
// fermions in general higher representations of SU(N_c); Sec. 2.1: the GPU
// wants component-blocked fields rather than the CPU's site-by-site order).
//
// Representation map, evaluated entry by entry from closed forms:
//   two-index antisymmetric, basis e_[jk] = (E_jk - E_kj)/sqrt2 (j<k):
//       (U_A)_{[jk],[lm]} = U_jl U_km - U_jm U_kl
//   two-index symmetric, e_(jk) = c_jk (E_jk + E_kj), c = 1/sqrt2 (j<k), 1/2 (j=k):
//       (U_S)_{(jk),(lm)} = 2 c_jk c_lm (U_jl U_km + U_jm U_kl)
//   adjoint, T^a = generalised Gell-Mann / 2:  column b of U_adj is obtained
//       from M = U T^b U^+ = sum of outer products of columns of U, and
//       (U_adj)_ab = 2 Re Tr(T^a M) read off from the few entries of T^a.
#include "kernels.h"

namespace hrw {

// ------------------------------------------------------------------ spinor packing

template <class S>
__global__ void __launch_bounds__(WG) pack_spinor_kernel(Geom g, int nr, bool full, int parity,
                                                          int n_rhs, const double *__restrict__ src,
                                                          cpx<S> *dst0, cpx<S> *dst1, size_t rstride)
{
    // one thread per destination element (rhs, parity q, padded site i, component k),
    // ordered as the destination layout so the stores are contiguous
    const int nc = 4 * nr;
    const size_t per_half = (size_t)g.nblk * BLK * nc;
    const int nq = full ? 2 : 1;
    const size_t total = per_half * nq * n_rhs;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t e = t % per_half;
        const size_t qr = t / per_half;
        const int q = full ? (int)(qr % 2) : parity;
        const int rhs = (int)(full ? qr / 2 : qr);
        const int lane = (int)(e % BLK);
        const size_t bk = e / BLK;
        const int k = (int)(bk % nc);
        const int i = (int)(bk / nc) * BLK + lane;
        cpx<S> v;
        if (i < g.half) {
            size_t sbase;  // the site's first canonical component
            if (full) {
                int x[4];
                eo_coords(g, q, i, x);
                const size_t lex = (((size_t)x[0] * g.d[1] + x[1]) * g.d[2] + x[2]) * g.d[3] + x[3];
                sbase = ((size_t)rhs * 2 * g.half + lex) * nc;
            } else {
                sbase = ((size_t)rhs * g.half + i) * nc;
            }
            // storage basis: q_s = psi_s - psi_{s+2}, q_{s+2} = psi_s + psi_{s+2}
            const int sp = k / nr, c = k - sp * nr;
            const size_t up = sbase + (size_t)(sp & 1) * nr + c, dn = up + 2 * nr;
            const double sg = sp < 2 ? -1.0 : 1.0;
            v.re = conv<S>::from_f64(src[2 * up] + sg * src[2 * dn]);
            v.im = conv<S>::from_f64(src[2 * up + 1] + sg * src[2 * dn + 1]);
        } else {
            v.re = conv<S>::from_f64(0.0);
            v.im = conv<S>::from_f64(0.0);
        }
        cpx<S> *dst = (q == 0 ? dst0 : dst1) + (size_t)rhs * rstride;
        dst[e] = v;
    }
}

template <class S>
__global__ void __launch_bounds__(WG) unpack_spinor_kernel(Geom g, int nr, bool full, int parity,
                                                            int n_rhs, const cpx<S> *src0,
                                                            const cpx<S> *src1, size_t rstride,
                                                            double *__restrict__ dst)
{
    // one thread per canonical destination element (rhs, site, component)
    typedef typename acc_of<S>::type A;
    const int nc = 4 * nr;
    const size_t nsites = full ? (size_t)2 * g.half : (size_t)g.half;
    const size_t total = nsites * nc * n_rhs;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(t % nc);
        const size_t sr = t / nc;
        const size_t site = sr % nsites;
        const int rhs = (int)(sr / nsites);
        int q, i;
        if (full) {
            size_t s = site;
            int x[4];
            x[3] = (int)(s % g.d[3]); s /= g.d[3];
            x[2] = (int)(s % g.d[2]); s /= g.d[2];
            x[1] = (int)(s % g.d[1]);
            x[0] = (int)(s / g.d[1]);
            q = (x[0] + x[1] + x[2] + x[3]) & 1;
            i = (int)(site >> 1);
        } else {
            q = parity;
            i = (int)site;
        }
        const cpx<S> *src = (q == 0 ? src0 : src1) + (size_t)rhs * rstride;
        // chiral basis: psi_s = (q_s + q_{s+2}) / 2, psi_{s+2} = (q_{s+2} - q_s) / 2, in FP64
        const int sp = k / nr, c = k - sp * nr;
        const int ka = (sp & 1) * nr + c, kb = ka + 2 * nr;
        A ar, ai, br, bi;
        load_c(src + lay(i, ka, nc), ar, ai);
        load_c(src + lay(i, kb, nc), br, bi);
        const double sg = sp < 2 ? 1.0 : -1.0;
        dst[2 * t] = ((double)br + sg * (double)ar) * 0.5;
        dst[2 * t + 1] = ((double)bi + sg * (double)ai) * 0.5;
    }
}

static int stream_grid(size_t total)
{
    size_t b = (total + WG - 1) / WG;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_pack_spinor(int dt, int nr, const Geom &g, bool full, int parity, int n_rhs,
                              const double *src, void *dst0, void *dst1, size_t rstride,
                              hipStream_t st)
{
    const size_t total = (size_t)g.nblk * BLK * 4 * nr * (full ? 2 : 1) * n_rhs;
    bool ok = dispatch_dtype(dt, [&](auto sv) {
        typedef decltype(sv) S;
        pack_spinor_kernel<S><<<stream_grid(total), WG, 0, st>>>(
            g, nr, full, parity, n_rhs, src, (cpx<S> *)dst0, (cpx<S> *)dst1, rstride);
    });
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(int dt, int nr, const Geom &g, bool full, int parity, int n_rhs,
                                const void *src0, const void *src1, size_t rstride, double *dst,
                                hipStream_t st)
{
    const size_t total = (size_t)g.half * (full ? 2 : 1) * 4 * nr * n_rhs;
    bool ok = dispatch_dtype(dt, [&](auto sv) {
        typedef decltype(sv) S;
        unpack_spinor_kernel<S><<<stream_grid(total), WG, 0, st>>>(
            g, nr, full, parity, n_rhs, (const cpx<S> *)src0, (const cpx<S> *)src1, rstride, dst);
    });
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------ representation map

struct C64 {
    double re, im;
};
__device__ inline C64 cmul(C64 a, C64 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline C64 cmulc(C64 a, C64 b) { return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im}; }  // a conj(b)
__device__ inline C64 cadd(C64 a, C64 b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline C64 csub(C64 a, C64 b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline C64 cscale(C64 a, double s) { return {a.re * s, a.im * s}; }

// q-th pair (j<k) in lexicographic order, or (j<=k) when with_diag
__device__ inline void nth_pair(int n, int q, bool with_diag, int &j, int &k)
{
    for (j = 0; j < n; ++j) {
        const int cnt = with_diag ? n - j : n - j - 1;
        if (q < cnt) {
            k = with_diag ? j + q : j + 1 + q;
            return;
        }
        q -= cnt;
    }
    j = k = 0;
}

// column b of U_R, written to col[0..nr)
template <int N, int REP>
__device__ void rep_column(const C64 (&u)[N][N], int b, C64 *col)
{
    constexpr int NR = REP == 0 ? N : REP == 1 ? N * N - 1 : REP == 2 ? N * (N + 1) / 2 : N * (N - 1) / 2;
    if (REP == 0) {
        #pragma unroll
        for (int a = 0; a < NR; ++a) col[a] = u[a][b];
    } else if (REP == 3) {
        int l, m;
        nth_pair(N, b, false, l, m);
        #pragma unroll
        for (int a = 0; a < NR; ++a) {
            int j, k;
            nth_pair(N, a, false, j, k);
            col[a] = csub(cmul(u[j][l], u[k][m]), cmul(u[j][m], u[k][l]));
        }
    } else if (REP == 2) {
        int l, m;
        nth_pair(N, b, true, l, m);
        const double clm = l == m ? 0.5 : M_SQRT1_2;
        #pragma unroll
        for (int a = 0; a < NR; ++a) {
            int j, k;
            nth_pair(N, a, true, j, k);
            const double cjk = j == k ? 0.5 : M_SQRT1_2;
            col[a] = cscale(cadd(cmul(u[j][l], u[k][m]), cmul(u[j][m], u[k][l])), 2.0 * cjk * clm);
        }
    } else {
        // adjoint: M = U T^b U^+ from outer products u_j u_k^+ of columns of U
        constexpr int NP = N * (N - 1) / 2;
        C64 mm[N][N];
        if (b < 2 * NP) {
            int j, k;
            nth_pair(N, b < NP ? b : b - NP, false, j, k);
            #pragma unroll
            for (int r = 0; r < N; ++r)
                #pragma unroll
                for (int c = 0; c < N; ++c) {
                    const C64 jk = cmulc(u[r][j], u[c][k]);  // (u_j u_k^+)_rc
                    const C64 kj = cmulc(u[r][k], u[c][j]);
                    if (b < NP) {  // T = (E_jk + E_kj)/2
                        mm[r][c] = cscale(cadd(jk, kj), 0.5);
                    } else {       // T = (-i E_jk + i E_kj)/2
                        const C64 dlt = csub(kj, jk);       // i (kj - jk) / 2
                        mm[r][c] = {-0.5 * dlt.im, 0.5 * dlt.re};
                    }
                }
        } else {
            const int l = b - 2 * NP + 1;
            const double cl = 1.0 / sqrt(2.0 * l * (l + 1));
            #pragma unroll
            for (int r = 0; r < N; ++r)
                #pragma unroll
                for (int c = 0; c < N; ++c) {
                    C64 s = {0, 0};
                    #pragma unroll
                    for (int m = 0; m < l; ++m) s = cadd(s, cmulc(u[r][m], u[c][m]));
                    s = csub(s, cscale(cmulc(u[r][l], u[c][l]), (double)l));
                    mm[r][c] = cscale(s, cl);
                }
        }
        #pragma unroll
        for (int a = 0; a < NR; ++a) {
            double v;
            if (a < NP) {
                int j, k;
                nth_pair(N, a, false, j, k);
                v = mm[j][k].re + mm[k][j].re;
            } else if (a < 2 * NP) {
                int j, k;
                nth_pair(N, a - NP, false, j, k);
                v = mm[k][j].im - mm[j][k].im;
            } else {
                const int l = a - 2 * NP + 1;
                const double cl = 1.0 / sqrt(2.0 * l * (l + 1));
                double s = 0;
                #pragma unroll
                for (int m = 0; m < l; ++m) s += mm[m][m].re;
                v = 2.0 * cl * (s - l * mm[l][l].re);
            }
            col[a] = {v, 0.0};
        }
    }
}

template <int N>
__device__ inline void load_link(const double *p, C64 (&u)[N][N])
{
    #pragma unroll
    for (int r = 0; r < N; ++r)
        #pragma unroll
        for (int c = 0; c < N; ++c) u[r][c] = {p[2 * (r * N + c)], p[2 * (r * N + c) + 1]};
}

template <int N, int REP>
__global__ void __launch_bounds__(WG) rep_map_kernel(long long n_links, const double *__restrict__ uf,
                                                      double *__restrict__ ur)
{
    constexpr int NR = REP == 0 ? N : REP == 1 ? N * N - 1 : REP == 2 ? N * (N + 1) / 2 : N * (N - 1) / 2;
    const long long l = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_links) return;
    C64 u[N][N];
    load_link<N>(uf + l * 2 * N * N, u);
    C64 col[NR];
    double *o = ur + l * 2 * NR * NR;
    #pragma unroll
    for (int b = 0; b < NR; ++b) {
        rep_column<N, REP>(u, b, col);
        #pragma unroll
        for (int a = 0; a < NR; ++a) {
            o[2 * (a * NR + b)] = col[a].re;
            o[2 * (a * NR + b) + 1] = col[a].im;
        }
    }
}

template <class F>
static bool dispatch_rep(int nc, int rep, F &&f)
{
#define HRW_REP_CASE(N_, R_)                                                      \
    if (nc == N_ && rep == R_) {                                                  \
        f(std::integral_constant<int, N_>{}, std::integral_constant<int, R_>{}); \
        return true;                                                              \
    }
    HRW_REP_CASE(2, 0) HRW_REP_CASE(2, 1) HRW_REP_CASE(2, 2)
    HRW_REP_CASE(3, 0) HRW_REP_CASE(3, 1) HRW_REP_CASE(3, 2) HRW_REP_CASE(3, 3)
    HRW_REP_CASE(4, 0) HRW_REP_CASE(4, 1) HRW_REP_CASE(4, 2) HRW_REP_CASE(4, 3)
#undef HRW_REP_CASE
    return false;
}

hipError_t launch_rep_map(int nc, int rep, long long n_links, const double *uf, double *ur,
                          hipStream_t st)
{
    if (n_links == 0) return hipSuccess;
    const long long blocks = (n_links + WG - 1) / WG;
    bool ok = dispatch_rep(nc, rep, [&](auto nv, auto rv) {
        rep_map_kernel<decltype(nv)::value, decltype(rv)::value><<<(unsigned)blocks, WG, 0, st>>>(n_links, uf, ur);
    });
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------ gauge packing

struct GaugeBlocks {
    void *p[4][2];  // [dtype][output parity]
};

template <class S>
__device__ inline void put_link(void *blk, size_t off, C64 v)
{
    cpx<S> w;
    w.re = conv<S>::from_f64(v.re);
    w.im = conv<S>::from_f64(v.im);
    ((cpx<S> *)blk)[off] = w;
}

__device__ inline void put_all(const GaugeBlocks &gb, int q, size_t off, C64 v)
{
    if (gb.p[0][q]) put_link<double>(gb.p[0][q], off, v);
    if (gb.p[1][q]) put_link<float>(gb.p[1][q], off, v);
    if (gb.p[2][q]) put_link<bf16_t>(gb.p[2][q], off, v);
    if (gb.p[3][q]) put_link<f16_t>(gb.p[3][q], off, v);
}

// Largest deviation of an SU(3) link from special unitarity as the two-row hops
// see it: max over links and entries of |u_2c - conj(u_0a u_1b - u_0b u_1a)|,
// (a, b) = (c+1, c+2) mod 3.  For a unitary U this is |1 - det U| times the
// modulus of a row entry, so it catches both non-unitary and U(3) links.  Each
// wavefront folds its maximum into *out with an integer atomic max (the bit
// patterns of non-negative doubles order like the numbers; NaN compares
// larger than any finite value).
__device__ inline double su3_link_defect(const C64 (&u)[3][3])
{
    double m = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        const C64 x = csub(cmul(u[0][a], u[1][b]), cmul(u[0][b], u[1][a]));
        const double dr = u[2][c].re - x.re, di = u[2][c].im + x.im;
        const double d = sqrt(dr * dr + di * di);
        m = (d > m || d != d) ? d : m;
    }
    return m;
}

// fold a thread's value into *out: wavefront max, then one atomic per wavefront
// (every lane of the wavefront must call it)
__device__ inline void fold_defect(double m, unsigned long long *out)
{
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_down(m, off, 64);
        m = (o > m || o != o) ? o : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// one thread per (site, mu): U_R(x, mu) goes to the forward slot of x and, as
// U_R^+, to the backward slot of x + mu
template <int N, int REP>
__global__ void __launch_bounds__(WG) gauge_pack_kernel(Geom g, const double *__restrict__ uf,
                                                         GaugeBlocks gb, unsigned long long *defect)
{
    constexpr int NR = REP == 0 ? N : REP == 1 ? N * N - 1 : REP == 2 ? N * (N + 1) / 2 : N * (N - 1) / 2;
    constexpr int GC = 8 * NR * NR;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long v = 2LL * g.half;
    if constexpr (N == 3 && REP == 0) {
        // special-unitarity check of the fundamental SU(3) links (two-row storage), on the
        // links this kernel reads anyway; before the bounds return: every lane folds
        if (defect) {
            double m = 0;
            if (t < 4 * v) {
                C64 u[3][3];
                load_link<3>(uf + t * 18, u);
                m = su3_link_defect(u);
            }
            fold_defect(m, defect);
        }
    }
    if (t >= 4 * v) return;
    const long long s = t >> 2;
    const int mu = (int)(t & 3);
    int x[4];
    long long r = s;
    x[3] = (int)(r % g.d[3]); r /= g.d[3];
    x[2] = (int)(r % g.d[2]); r /= g.d[2];
    x[1] = (int)(r % g.d[1]);
    x[0] = (int)(r / g.d[1]);
    const int q = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int i = (int)(s >> 1);
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (x[mu] + 1) % g.d[mu];
    const int j = eo_index(g, y);  // y has parity 1 - q
    C64 u[N][N];
    load_link<N>(uf + (s * 4 + mu) * 2 * N * N, u);
    C64 col[NR];
    #pragma unroll
    for (int b = 0; b < NR; ++b) {
        rep_column<N, REP>(u, b, col);
        #pragma unroll
        for (int a = 0; a < NR; ++a) {
            // forward slot of x: direction mu, entry (a, b)
            put_all(gb, q, lay(i, mu * NR * NR + a * NR + b, GC), col[a]);
            // backward slot of x + mu: direction 4 + mu, entry (b, a) of U_R^+
            put_all(gb, 1 - q, lay(j, (4 + mu) * NR * NR + b * NR + a, GC), {col[a].re, -col[a].im});
        }
    }
}

hipError_t launch_gauge_pack(int nc, int rep, int nr, const Geom &g, const double *uf,
                             void *const blocks[4][2], hipStream_t st, unsigned long long *defect)
{
    if (defect && !(nc == 3 && rep == 0)) return hipErrorInvalidValue;
    if (defect) {
        hipError_t e = launch_zero(defect, sizeof *defect, st);
        if (e != hipSuccess) return e;
    }
    GaugeBlocks gb;
    for (int d = 0; d < 4; ++d)
        for (int q = 0; q < 2; ++q) gb.p[d][q] = blocks[d][q];
    // zero the padding lanes first so every stored word is defined (the packing below writes
    // every entry of every site, so a half lattice of whole 64-site blocks has nothing to clear)
    for (int d = 0; d < 4; ++d)
        for (int q = 0; q < 2; ++q)
            if (gb.p[d][q] && g.half % BLK) {
                const size_t bytes = gauge_block_elems(g, nr) * dtype_cbytes(d);
                hipError_t e = launch_zero(gb.p[d][q], bytes, st);
                if (e != hipSuccess) return e;
            }
    const long long total = 8LL * g.half;
    const long long blocks_ = (total + WG - 1) / WG;
    bool ok = dispatch_rep(nc, rep, [&](auto nv, auto rv) {
        constexpr int N = decltype(nv)::value, REP = decltype(rv)::value;
        constexpr int NR = REP == 0 ? N : REP == 1 ? N * N - 1 : REP == 2 ? N * (N + 1) / 2 : N * (N - 1) / 2;
        // only representations with hopping kernels are ever packed (SU(4) adjoint
        // and symmetric, N_R = 15 and 10, are not)
        if constexpr (NR <= 8) gauge_pack_kernel<N, REP><<<(unsigned)blocks_, WG, 0, st>>>(g, uf, gb, defect);
    });
    if (!nr_supported(nr)) return hipErrorInvalidValue;
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace hrw
