// Wilson hopping kernel for the even/odd blocks of H (arXiv 2405.19294,
// Sec. 3.1), one thread per output site.
//
// Per output site x and direction mu the thread
//   1. loads the neighbour spinor psi(x +- mu) (4 N_R complex, coalesced
//      across the wavefront by the site-blocked layout; 2 N_R along mu = 0,
//      see the spin basis below),
//   2. projects it to a half-spinor h = (1 -+ g_mu) psi, which has only two
//      independent spin components (the same half-spinor trick the paper
//      uses to halve its messages, Sec. 2.2),
//   3. applies the boundary phase when the hop wraps,
//   4. multiplies both components by the N_R x N_R link (forward: U_mu(x),
//      backward: the stored U_mu(x - mu)^+), streaming the link from HBM,
//   5. reconstructs the other two spin components and accumulates.
// The epilogue is fused: out = H in, out = self - c H in (with |out|^2
// partials), or the CG update r -= alpha (self - c H in) with |r|^2
// partials.  Partials are reduced per workgroup in a fixed order, so
// the result is bitwise reproducible.
//
// Spin basis.  Device fields hold q = T psi, psi in the chiral basis and T
// acting on the spin pairs (s, s + 2) of each colour as
//   q_s = psi_s - psi_{s+2},  q_{s+2} = psi_s + psi_{s+2}   (s = 0, 1),
// the packing and unpacking kernels applying T and T^-1.  T is sqrt(2) times a
// unitary map, so the operator on q is the unitary transform of D: g_1..g_3
// keep their chiral form and g_0 becomes diag(1, 1, -1, -1).  The two
// projections along mu = 0 then take one half of the spinor each: (1 - g_0) q
// = 2 (0, 0, q2, q3) and (1 + g_0) q = 2 (q0, q1, 0, 0).  A hop along mu = 0
// reads 2 N_R of the neighbour's 4 N_R components and adds to two output spin
// components only; mu = 0 is the slowest lattice index, whose neighbours lie
// a whole time slice away and are the most expensive reads of the hop.
//
// Spin projection with s = -1 for (1 - g_mu) and s = +1 for (1 + g_mu);
// q = (p0, p1 | p2, p3) by spin, g = U h:
//   mu = 0: s = -1: h0 = 2 p2, h1 = 2 p3; out2 += g0, out3 += g1
//           s = +1: h0 = 2 p0, h1 = 2 p1; out0 += g0, out1 += g1
//   mu = 1: h0 = p0 - s i p3,  h1 = p1 - s i p2;  out2 += s i g1, out3 += s i g0
//   mu = 2: h0 = p0 - s p3,    h1 = p1 + s p2;    out2 += s g1,   out3 += -s g0
//   mu = 3: h0 = p0 - s i p2,  h1 = p1 + s i p3;  out2 += s i g0, out3 += -s i g1
// (for mu > 0 out0 += g0, out1 += g1 as well).  The forward hop of H uses
// s = -1 and the backward hop s = +1; H^+ swaps them.
#pragma once

#include <stdlib.h>

#include <stdio.h>
#include <sys/stat.h>
#include <unistd.h>

#include <array>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "cg_reduce.h"
#include "kernels.h"

namespace hrw {

__device__ inline double wave_block_sum(double v, double *sh)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += sh[k];
    return r;
}

// first of the two spin components a mu = 0 hop with projector sign SG reads
// and writes: (1 - g_0) keeps spins 2, 3 and (1 + g_0) spins 0, 1
template <int SG> constexpr int t_half() { return SG < 0 ? 2 : 0; }

template <int MU, int SG, class A, int NR>
__device__ __forceinline__ void project(const A (&pr)[4][NR], const A (&pi)[4][NR], A (&hr)[2][NR],
                                        A (&hi)[2][NR])
{
    const A s = (A)SG;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        if (MU == 0) {  // only spins B, B + 1 were loaded (t_half)
            constexpr int B = t_half<SG>();
            hr[0][c] = 2 * pr[B][c]; hi[0][c] = 2 * pi[B][c];
            hr[1][c] = 2 * pr[B + 1][c]; hi[1][c] = 2 * pi[B + 1][c];
        } else if (MU == 1) {  // - s i p3, - s i p2 :  i z = (-zi, zr)
            hr[0][c] = pr[0][c] + s * pi[3][c]; hi[0][c] = pi[0][c] - s * pr[3][c];
            hr[1][c] = pr[1][c] + s * pi[2][c]; hi[1][c] = pi[1][c] - s * pr[2][c];
        } else if (MU == 2) {
            hr[0][c] = pr[0][c] - s * pr[3][c]; hi[0][c] = pi[0][c] - s * pi[3][c];
            hr[1][c] = pr[1][c] + s * pr[2][c]; hi[1][c] = pi[1][c] + s * pi[2][c];
        } else {  // h0 = p0 - s i p2, h1 = p1 + s i p3
            hr[0][c] = pr[0][c] + s * pi[2][c]; hi[0][c] = pi[0][c] - s * pr[2][c];
            hr[1][c] = pr[1][c] - s * pi[3][c]; hi[1][c] = pi[1][c] + s * pr[3][c];
        }
    }
}

template <int MU, int SG, class A, int NR>
__device__ __forceinline__ void reconstruct(const A (&gr)[2][NR], const A (&gi)[2][NR], A (&ar)[4][NR],
                                            A (&ai)[4][NR])
{
    const A s = (A)SG;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        if (MU == 0) {
            constexpr int B = t_half<SG>();
            ar[B][c] += gr[0][c]; ai[B][c] += gi[0][c];
            ar[B + 1][c] += gr[1][c]; ai[B + 1][c] += gi[1][c];
            continue;
        }
        ar[0][c] += gr[0][c]; ai[0][c] += gi[0][c];
        ar[1][c] += gr[1][c]; ai[1][c] += gi[1][c];
        if (MU == 1) {  // out2 += s i g1, out3 += s i g0
            ar[2][c] -= s * gi[1][c]; ai[2][c] += s * gr[1][c];
            ar[3][c] -= s * gi[0][c]; ai[3][c] += s * gr[0][c];
        } else if (MU == 2) {  // out2 += s g1, out3 += -s g0
            ar[2][c] += s * gr[1][c]; ai[2][c] += s * gi[1][c];
            ar[3][c] -= s * gr[0][c]; ai[3][c] -= s * gi[0][c];
        } else {  // out2 += s i g0, out3 += -s i g1
            ar[2][c] -= s * gi[0][c]; ai[2][c] += s * gr[0][c];
            ar[3][c] += s * gi[1][c]; ai[3][c] -= s * gr[1][c];
        }
    }
}

// reconstruction for one colour row (the same table as reconstruct)
template <int MU, int SG, class A>
__device__ __forceinline__ void reconstruct_row(A g0r, A g0i, A g1r, A g1i, A &a0r, A &a0i, A &a1r, A &a1i,
                                                A &a2r, A &a2i, A &a3r, A &a3i)
{
    const A s = (A)SG;
    if (MU == 0) {
        if (t_half<SG>() == 0) {
            a0r += g0r; a0i += g0i;
            a1r += g1r; a1i += g1i;
        } else {
            a2r += g0r; a2i += g0i;
            a3r += g1r; a3i += g1i;
        }
        return;
    }
    a0r += g0r; a0i += g0i;
    a1r += g1r; a1i += g1i;
    if (MU == 1) {
        a2r -= s * g1i; a2i += s * g1r;
        a3r -= s * g0i; a3i += s * g0r;
    } else if (MU == 2) {
        a2r += s * g1r; a2i += s * g1i;
        a3r -= s * g0r; a3i -= s * g0i;
    } else {
        a2r -= s * g0i; a2i += s * g0r;
        a3r += s * g1i; a3i -= s * g1r;
    }
}

// g = U h for one link row (ur, ui) and both half-spinor components, as
// chains of fused multiply-adds (four per complex product)
template <class A, int NR>
__device__ __forceinline__ void link_row(const A (&ur)[NR], const A (&ui)[NR], const A (&hr)[2][NR],
                                         const A (&hi)[2][NR], A &s0r, A &s0i, A &s1r, A &s1i)
{
    s0r = ur[0] * hr[0][0]; s0i = ur[0] * hi[0][0];
    s1r = ur[0] * hr[1][0]; s1i = ur[0] * hi[1][0];
    s0r = fmac(-ui[0], hi[0][0], s0r); s0i = fmac(ui[0], hr[0][0], s0i);
    s1r = fmac(-ui[0], hi[1][0], s1r); s1i = fmac(ui[0], hr[1][0], s1i);
#pragma unroll
    for (int c = 1; c < NR; ++c) {
        s0r = fmac(ur[c], hr[0][c], s0r); s0r = fmac(-ui[c], hi[0][c], s0r);
        s0i = fmac(ur[c], hi[0][c], s0i); s0i = fmac(ui[c], hr[0][c], s0i);
        s1r = fmac(ur[c], hr[1][c], s1r); s1r = fmac(-ui[c], hi[1][c], s1r);
        s1i = fmac(ur[c], hi[1][c], s1i); s1i = fmac(ui[c], hr[1][c], s1i);
    }
}

// Where a thread reads its links from: the packed field in HBM (streamed past
// L2, each link is read once per launch) or a workgroup's LDS copy (the
// multi-source kernel).  The arithmetic is the same either way.
template <class S, int NR>
struct GlobalLinks {
    static constexpr bool ROWWISE = false;  // all rows' loads issued up front (HBM latency)
    static constexpr bool FUSED = false;
    static constexpr bool REAL = false;
    static constexpr int NF = 1;
    static constexpr int REPID = 0;
    static constexpr bool RECON = false;
    const cpx<S> *__restrict__ g;
    int i;
    __device__ __forceinline__ void load(int comp, typename acc_of<S>::type &re,
                                         typename acc_of<S>::type &im) const
    {
        load_c_nt(g + lay(i, comp, 8 * NR * NR), re, im);
    }
};

// SU(3) fundamental links in HBM of which only the first two rows are read:
// the rows of a special unitary 3 x 3 matrix satisfy u_2 = conj(u_0 x u_1),
// so the third row is rebuilt in registers and 2/3 of the link bytes cross
// HBM.  The stored blocks keep all three rows (other kernels read them).
template <class S>
struct Su3Links {
    static constexpr bool ROWWISE = false;
    static constexpr bool FUSED = false;
    static constexpr bool REAL = false;
    static constexpr int NF = 1;
    static constexpr int REPID = 0;
    static constexpr bool RECON = true;
    const cpx<S> *__restrict__ g;
    int i;
    __device__ __forceinline__ void load(int comp, typename acc_of<S>::type &re,
                                         typename acc_of<S>::type &im) const
    {
        load_c_nt(g + lay(i, comp, 8 * 9), re, im);
    }
};

template <class S, int NS = MR_SITES>
struct LdsLinks {
    static constexpr bool ROWWISE = true;  // one row at a time: fewer live registers
    static constexpr bool FUSED = false;
    static constexpr bool REAL = false;
    static constexpr int NF = 1;
    static constexpr int REPID = 0;
    static constexpr bool RECON = false;
    const cpx<S> *l;  // [comp][NS sites]
    int s;
    __device__ __forceinline__ void load(int comp, typename acc_of<S>::type &re,
                                         typename acc_of<S>::type &im) const
    {
        load_c(l + comp * NS + s, re, im);
    }
};

// Fundamental links in HBM (the N x N hopping blocks: U(x) forward, U(x - mu)^+
// backward) and the rows of U_R built from them in registers: the
// representation map fused into the hop.  R(U^+) = R(U)^+ for a unitary U, so
// the backward slots need no separate formula.
template <class S, int N, int REP>
struct RepLinks {
    static constexpr bool ROWWISE = true;
    static constexpr bool FUSED = true;
    static constexpr bool REAL = REP == 1;  // the adjoint representation is real
    static constexpr int NF = N;
    static constexpr int REPID = REP;
    static constexpr bool RECON = false;
    const cpx<S> *__restrict__ g;
    int i;
    template <class A>
    __device__ __forceinline__ void load_fund(int dd, A (&fr)[N][N], A (&fi)[N][N]) const
    {
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int c = 0; c < N; ++c) load_c_nt(g + lay(i, dd * N * N + r * N + c, 8 * N * N), fr[r][c], fi[r][c]);
    }
};

// (j, k) of the q-th index pair in lexicographic order: j <= k with the
// diagonal (symmetric basis), j < k without it (antisymmetric basis)
__host__ __device__ constexpr int pair_j(int n, bool diag, int q)
{
    int j = 0;
    while (q >= (diag ? n - j : n - j - 1)) {
        q -= diag ? n - j : n - j - 1;
        ++j;
    }
    return j;
}
__host__ __device__ constexpr int pair_k(int n, bool diag, int q)
{
    int j = 0;
    while (q >= (diag ? n - j : n - j - 1)) {
        q -= diag ? n - j : n - j - 1;
        ++j;
    }
    return diag ? j + q : j + 1 + q;
}

// Row a of U_R from the fundamental link u = (fr, fi).
//   antisymmetric, basis (E_jk - E_kj)/sqrt2:  (U_R)_(jk),(lm) = u_jl u_km - u_jm u_kl
//   symmetric, basis E_jj and (E_jk + E_kj)/sqrt2:
//       (U_R)_(jk),(lm) = (u_jl u_km + u_jm u_kl) 2 c_jk c_lm,  c = 1/2 on the diagonal, 1/sqrt2 off it
//   SU(2) adjoint, T^a = sigma_a / 2:  (U_R)_ab = (1/2) Re Tr(sigma_a u sigma_b u^+), i.e. the Pauli
//       components of W = u^+ sigma_a u:  (Re w01, -Im w01, w00)
// The rows j, k of u are picked with selects, so a row index that differs
// between the lanes of a wavefront costs no dynamic register indexing.
template <int N, int REP, int NR, class A>
__device__ __forceinline__ void rep_row(const A (&fr)[N][N], const A (&fi)[N][N], int a, A (&lr)[NR],
                                        A (&li)[NR])
{
    if constexpr (REP == 1) {
        static_assert(N == 2 && NR == 3, "fused adjoint row: SU(2) only");
        // z = conj(u00) u10, and the (0, 1) entry of W for each sigma_a
        const A zr = fr[0][0] * fr[1][0] + fi[0][0] * fi[1][0];
        const A zi = fr[0][0] * fi[1][0] - fi[0][0] * fr[1][0];
        A w00, w01r, w01i;
        if (a == 0) {  // sigma_1: w01 = conj(u00) u11 + conj(u10) u01
            w00 = zr + zr;
            w01r = fr[0][0] * fr[1][1] + fi[0][0] * fi[1][1] + fr[1][0] * fr[0][1] + fi[1][0] * fi[0][1];
            w01i = fr[0][0] * fi[1][1] - fi[0][0] * fr[1][1] + fr[1][0] * fi[0][1] - fi[1][0] * fr[0][1];
        } else if (a == 1) {  // sigma_2: w01 = -i conj(u00) u11 + i conj(u10) u01
            w00 = zi + zi;
            const A ar = fr[0][0] * fr[1][1] + fi[0][0] * fi[1][1], ai = fr[0][0] * fi[1][1] - fi[0][0] * fr[1][1];
            const A br = fr[1][0] * fr[0][1] + fi[1][0] * fi[0][1], bi = fr[1][0] * fi[0][1] - fi[1][0] * fr[0][1];
            w01r = ai - bi;
            w01i = br - ar;
        } else {  // sigma_3: w01 = conj(u00) u01 - conj(u10) u11
            w00 = fr[0][0] * fr[0][0] + fi[0][0] * fi[0][0] - fr[1][0] * fr[1][0] - fi[1][0] * fi[1][0];
            w01r = fr[0][0] * fr[0][1] + fi[0][0] * fi[0][1] - fr[1][0] * fr[1][1] - fi[1][0] * fi[1][1];
            w01i = fr[0][0] * fi[0][1] - fi[0][0] * fr[0][1] - fr[1][0] * fi[1][1] + fi[1][0] * fr[1][1];
        }
        lr[0] = w01r;
        lr[1] = -w01i;
        lr[2] = w00;
        li[0] = li[1] = li[2] = (A)0;
    } else {
        constexpr bool DIAG = REP == 2;
        int q = a, j = 0, k = 0;
#pragma unroll
        for (int jj = 0; jj < N; ++jj) {
            const int cnt = DIAG ? N - jj : N - jj - 1;
            if (q >= 0 && q < cnt) {
                j = jj;
                k = DIAG ? jj + q : jj + 1 + q;
            }
            q -= cnt;
        }
        A ujr[N], uji[N], ukr[N], uki[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            ujr[c] = fr[0][c];
            uji[c] = fi[0][c];
            ukr[c] = fr[0][c];
            uki[c] = fi[0][c];
        }
#pragma unroll
        for (int t = 1; t < N; ++t)
#pragma unroll
            for (int c = 0; c < N; ++c) {
                ujr[c] = j == t ? fr[t][c] : ujr[c];
                uji[c] = j == t ? fi[t][c] : uji[c];
                ukr[c] = k == t ? fr[t][c] : ukr[c];
                uki[c] = k == t ? fi[t][c] : uki[c];
            }
        const A cj = DIAG ? (j == k ? (A)1 : (A)M_SQRT2) : (A)1;  // 2 c_jk
#pragma unroll
        for (int b = 0; b < NR; ++b) {
            const int l = pair_j(N, DIAG, b), m = pair_k(N, DIAG, b);
            const A pr = ujr[l] * ukr[m] - uji[l] * uki[m], pi = ujr[l] * uki[m] + uji[l] * ukr[m];
            const A qr = ujr[m] * ukr[l] - uji[m] * uki[l], qi = ujr[m] * uki[l] + uji[m] * ukr[l];
            if (DIAG) {
                const A f = cj * (l == m ? (A)0.5 : (A)M_SQRT1_2);
                lr[b] = f * (pr + qr);
                li[b] = f * (pi + qi);
            } else {
                lr[b] = pr - qr;
                li[b] = pi - qi;
            }
        }
    }
}

// g = U h for a real link row
template <class A, int NR>
__device__ __forceinline__ void link_row_real(const A (&ur)[NR], const A (&hr)[2][NR], const A (&hi)[2][NR],
                                              A &s0r, A &s0i, A &s1r, A &s1i)
{
    s0r = ur[0] * hr[0][0];
    s0i = ur[0] * hi[0][0];
    s1r = ur[0] * hr[1][0];
    s1i = ur[0] * hi[1][0];
#pragma unroll
    for (int c = 1; c < NR; ++c) {
        s0r = fmac(ur[c], hr[0][c], s0r);
        s0i = fmac(ur[c], hi[0][c], s0i);
        s1r = fmac(ur[c], hr[1][c], s1r);
        s1i = fmac(ur[c], hi[1][c], s1i);
    }
}

// third row of a special unitary 3 x 3 matrix from its first two:
// u_2c = conj(u_0a u_1b - u_0b u_1a) with (a, b) = (c+1, c+2) mod 3
template <class A, int RS, int NR>
__device__ __forceinline__ void su3_third_row(A (&ur)[RS][NR], A (&ui)[RS][NR])
{
    static_assert(RS == 3 && NR == 3, "SU(3) fundamental rows");
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        const A re = (ur[0][a] * ur[1][b] - ui[0][a] * ui[1][b]) - (ur[0][b] * ur[1][a] - ui[0][b] * ui[1][a]);
        const A im = (ur[0][a] * ui[1][b] + ui[0][a] * ur[1][b]) - (ur[0][b] * ui[1][a] + ui[0][b] * ur[1][a]);
        ur[2][c] = re;
        ui[2][c] = -im;
    }
}

// The input spinors a workgroup stages in LDS: the half-sites lo .. lo + n - 1
// of the input half field (its own sites and one x3 line before and after),
// component-major ([comp][n]).  A neighbour inside that range is read from LDS,
// any other from global memory.  l == nullptr: nothing staged.
template <class S>
struct Stage {
    const cpx<S> *l;
    int lo, n;
};

// one direction (forward or backward) of one mu, for colour rows r0 .. r0+RS-1
template <int MU, int DIR, bool DAG, int NR, int RS, class S, class LS, bool STG>
__device__ __forceinline__ void hop_dir(const HopArgs<S> &a, const cpx<S> *__restrict__ in,
                                        const LS &links, int r0, const int (&x)[4],
                                        typename acc_of<S>::type (&ar)[4][RS],
                                        typename acc_of<S>::type (&ai)[4][RS], const Stage<S> &stg)
{
    typedef typename acc_of<S>::type A;
    constexpr int NC = 4 * NR;
    // projector sign: forward (1 - g) for H, backward (1 + g); H^+ swaps
    constexpr int SG = (DIR == 0) ? (DAG ? 1 : -1) : (DAG ? -1 : 1);
    int y[4] = {x[0], x[1], x[2], x[3]};
    bool wrap;
    if (DIR == 0) {
        y[MU] = x[MU] + 1;
        wrap = y[MU] == a.g.d[MU];
        if (wrap) y[MU] = 0;
    } else {
        y[MU] = x[MU] - 1;
        wrap = y[MU] < 0;
        if (wrap) y[MU] = a.g.d[MU] - 1;
    }
    const int j = eo_index(a.g, y);
    A pr[4][NR], pi[4][NR];
    // the staged path is a separate instance: its range check and second load
    // path cost the unstaged FP64 hop 7% even when nothing was staged
    // spins this hop reads: all four, or along mu = 0 the half its projector keeps
    constexpr int S0 = MU == 0 ? t_half<SG>() : 0, S1 = MU == 0 ? S0 + 2 : 4;
    bool staged = false;
    if constexpr (STG) {
        const int k = j - stg.lo;
        staged = (unsigned)k < (unsigned)stg.n;
        if (staged) {
#pragma unroll
            for (int sp = S0; sp < S1; ++sp)
#pragma unroll
                for (int c = 0; c < NR; ++c) load_c(stg.l + (sp * NR + c) * stg.n + k, pr[sp][c], pi[sp][c]);
        }
    }
    if (!staged) {
#pragma unroll
        for (int sp = S0; sp < S1; ++sp)
#pragma unroll
            for (int c = 0; c < NR; ++c) load_c(in + lay(j, sp * NR + c, NC), pr[sp][c], pi[sp][c]);
    }
    constexpr int DD = MU + 4 * DIR;
    // links from HBM: every row's loads are issued together with the spinor's,
    // before any arithmetic waits on them (unused when links come from LDS)
    A ur[LS::ROWWISE ? 1 : RS][NR], ui[LS::ROWWISE ? 1 : RS][NR];
    if constexpr (!LS::ROWWISE) {
        // rows read from memory (two of an SU(3) link when its third row is rebuilt)
        constexpr int RL = LS::RECON ? 2 : RS;
#pragma unroll
        for (int r = 0; r < RL; ++r)
#pragma unroll
            for (int c = 0; c < NR; ++c) links.load(DD * NR * NR + (r0 + r) * NR + c, ur[r][c], ui[r][c]);
    }
    // fundamental link of this direction (fused representation map)
    A fr[LS::NF][LS::NF], fi[LS::NF][LS::NF];
    if constexpr (LS::FUSED) links.load_fund(DD, fr, fi);
    A hr[2][NR], hi[2][NR];
    project<MU, SG>(pr, pi, hr, hi);
    if (wrap) {
        const A cr = (A)a.ph_re[MU];
        const A ci = DIR == 0 ? (A)a.ph_im[MU] : -(A)a.ph_im[MU];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                const A tr = hr[k][c] * cr - hi[k][c] * ci;
                const A ti = hr[k][c] * ci + hi[k][c] * cr;
                hr[k][c] = tr;
                hi[k][c] = ti;
            }
    }
    if constexpr (LS::ROWWISE) {
        // links from LDS (or built from the fundamental link): one row at a time
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            A lr[NR], li[NR];
            if constexpr (LS::FUSED) {
                rep_row<LS::NF, LS::REPID>(fr, fi, r0 + r, lr, li);
            } else {
#pragma unroll
                for (int c = 0; c < NR; ++c) links.load(DD * NR * NR + (r0 + r) * NR + c, lr[c], li[c]);
            }
            A s0r, s0i, s1r, s1i;
            if constexpr (LS::REAL) link_row_real(lr, hr, hi, s0r, s0i, s1r, s1i);
            else link_row(lr, li, hr, hi, s0r, s0i, s1r, s1i);
            reconstruct_row<MU, SG>(s0r, s0i, s1r, s1i, ar[0][r], ai[0][r], ar[1][r], ai[1][r], ar[2][r],
                                    ai[2][r], ar[3][r], ai[3][r]);
        }
    } else {
        if constexpr (LS::RECON) su3_third_row(ur, ui);
        A gr[2][RS], gi[2][RS];
#pragma unroll
        for (int r = 0; r < RS; ++r) link_row(ur[r], ui[r], hr, hi, gr[0][r], gi[0][r], gr[1][r], gi[1][r]);
        reconstruct<MU, SG>(gr, gi, ar, ai);
    }
    // Materialise the accumulators here.  Without this the optimiser sinks
    // every direction's "acc += g" to the end of the kernel, keeping all eight
    // directions' products live at once (256 VGPRs and spills even for N_R=2).
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < RS; ++c) asm volatile("" : "+v"(ar[sp][c]), "+v"(ai[sp][c]));
}

// XCD-aware block order: the dispatcher deals workgroups to the 8 XCDs round
// robin; renumber them so that each XCD walks one contiguous slab of the
// lattice and neighbour spinors are found in its own L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    if (n % 8) return b;
    return (b % 8) * (n / 8) + b / 8;
}

// Time-tiled walk: the slab an XCD owns is traversed chunk by chunk, each
// spatial chunk of C workgroups through every time slice before the next, so
// the +-t neighbours of a block are touched C workgroups apart instead of a
// whole time slice apart (which exceeds an XCD's L2 at 32^4).
__device__ __forceinline__ int tile_remap(int L, int n, int ts, int c)
{
    if (ts <= 0 || c <= 0) return L;
    const int T = n / ts;
    const int ch = L / (c * T);
    const int rem = L - ch * c * T;
    const int t = rem / c;
    const int w = rem - t * c;
    return t * ts + ch * c + w;
}

// The multi-source walk: a chunk is a block of p x1-planes by c / p
// consecutive workgroups of each plane (B workgroups per plane), walked
// through every time slice like tile_remap's; p <= 1 is tile_remap.  With one
// 16-site line per workgroup the x1 neighbours of a line are B workgroups
// apart, so flat chunks put them in another chunk, a whole walk through the
// time slices away.
__device__ __forceinline__ int tile_remap_planes(int L, int n, int ts, int c, int p, int B)
{
    if (p <= 1 || ts <= 0 || c <= 0) return tile_remap(L, n, ts, c);
    const int T = n / ts;
    const int q = c / p;
    const int ch = L / (c * T);
    const int rem = L - ch * c * T;
    const int t = rem / c;
    const int w = rem - t * c;
    const int per_row = B / q;  // chunks side by side in one band of p planes
    const int cha = ch / per_row, chb = ch - cha * per_row;
    return t * ts + (cha * p + w / q) * B + chb * q + w % q;
}

// FP64 sum over the 16*G lanes (16 sites x G row threads) of one partial-sum
// group, in a fixed tree; the result is valid in the group's first lane.
// Groups wider than a wavefront (G = 8) combine their two halves through LDS.
template <int G>
__device__ __forceinline__ double group_sum(double v, double *sh)
{
    constexpr int SEG = PG_SITES * G;
    constexpr int W = SEG < 64 ? SEG : 64;
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_down(v, off, W);
    if (SEG > 64) {
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) sh[w] = v;
        __syncthreads();
        if ((threadIdx.x & (SEG - 1)) == 0)
            for (int k = 1; k < SEG / 64; ++k) v += sh[w + k];
        __syncthreads();
    }
    return v;
}

// the per-site body shared by both kernels: hop of site i for one source,
// then the epilogue; returns this thread's |.|^2 contribution
template <int NR, int RS, class S, bool DAG, int EPI, class LS, bool STG = false>
__device__ __forceinline__ double site_hop(const HopArgs<S> &a, int parity, int i, int r0, int rhs,
                                           const LS &links, const Stage<S> &stg = Stage<S>{nullptr, 0, 0})
{
    typedef typename acc_of<S>::type A;
    constexpr int NC = 4 * NR;
    const size_t roff = (size_t)rhs * a.rstride;
    double nrm = 0;
    int x[4];
    eo_coords(a.g, parity, i, x);
    const cpx<S> *__restrict__ in = a.in[1 - parity] + roff;
    A ar[4][RS], ai[4][RS];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < RS; ++c) ar[sp][c] = ai[sp][c] = 0;
    hop_dir<0, 0, DAG, NR, RS, S, LS, STG>(a, in, links, r0, x, ar, ai, stg);
    hop_dir<0, 1, DAG, NR, RS, S, LS, STG>(a, in, links, r0, x, ar, ai, stg);
    hop_dir<1, 0, DAG, NR, RS, S, LS, STG>(a, in, links, r0, x, ar, ai, stg);
    hop_dir<1, 1, DAG, NR, RS, S, LS, STG>(a, in, links, r0, x, ar, ai, stg);
    hop_dir<2, 0, DAG, NR, RS, S, LS, STG>(a, in, links, r0, x, ar, ai, stg);
    hop_dir<2, 1, DAG, NR, RS, S, LS, STG>(a, in, links, r0, x, ar, ai, stg);
    hop_dir<3, 0, DAG, NR, RS, S, LS, STG>(a, in, links, r0, x, ar, ai, stg);
    hop_dir<3, 1, DAG, NR, RS, S, LS, STG>(a, in, links, r0, x, ar, ai, stg);
    if (EPI == EPI_PLAIN) {
        cpx<S> *out = a.out[parity] + roff;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < RS; ++c) store_c_nt(out + lay(i, sp * NR + r0 + c, NC), ar[sp][c], ai[sp][c]);
    } else {
        const A cf = (A)a.coef[rhs];
        const cpx<S> *self = a.self[parity] + roff;
        if (EPI == EPI_AXPY) {
            cpx<S> *out = a.out[parity] + roff;
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int c = 0; c < RS; ++c) {
                    const size_t o = lay(i, sp * NR + r0 + c, NC);
                    A sr, si;
                    load_c_nt(self + o, sr, si);
                    const A vr = sr - cf * ar[sp][c], vi = si - cf * ai[sp][c];
                    store_c_nt(out + o, vr, vi);
                    nrm += (double)vr * (double)vr + (double)vi * (double)vi;
                }
        } else {  // EPI_CG: r -= alpha q (x += alpha p follows in launch_cg_xp)
            cpx<S> *r = a.r[parity] + roff;
            const bool act = a.active[rhs] != 0;
            const A al = (A)a.alpha[rhs];
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int c = 0; c < RS; ++c) {
                    const size_t o = lay(i, sp * NR + r0 + c, NC);
                    A sr, si, rr_, ri;
                    load_c_nt(self + o, sr, si);
                    load_c_nt(r + o, rr_, ri);
                    if (act) {
                        const A qr = sr - cf * ar[sp][c], qi = si - cf * ai[sp][c];
                        rr_ -= al * qr;
                        ri -= al * qi;
                        store_c_nt(r + o, rr_, ri);
                    }
                    nrm += (double)rr_ * (double)rr_ + (double)ri * (double)ri;
                }
        }
    }
    return nrm;
}

// Stage the input spinors of a one-thread-per-site workgroup (sites i0 ..
// i0 + WG - 1) in LDS: the half-sites from one x3 line (a.g.n3h sites) before
// i0 to one line after the workgroup's last site, clipped to the half field.
// They hold every x3 neighbour of the workgroup's sites and, away from the
// periodic wrap in x2, every x2 neighbour (one line apart), so six of a
// site's eight neighbour reads usually come from LDS.  Called by every thread
// (it synchronises the workgroup); a.stage == 0 stages nothing.
template <int NR, class S>
__device__ __forceinline__ Stage<S> stage_input(const HopArgs<S> &a, const cpx<S> *__restrict__ in, int i0,
                                                cpx<S> *lds)
{
    constexpr int NC = 4 * NR;
    if (!a.stage) return Stage<S>{nullptr, 0, 0};
    const int lo = max(i0 - a.g.n3h, 0);
    const int hi = min(i0 + WG + a.g.n3h, a.g.half);
    const int n = hi - lo;
    for (int e = threadIdx.x; e < NC * n; e += WG) {
        const int comp = e / n, k = e - comp * n;
        lds[e] = in[lay(lo + k, comp, NC)];
    }
    __syncthreads();
    return Stage<S>{lds, lo, n};
}

template <int NR, int RS, class S, bool DAG, int EPI, bool STG = false>
__global__ void __launch_bounds__(WG) hop_kernel(const HopArgs<S> a)
{
    constexpr int G = NR / RS;  // threads per site, each owning RS colour rows
    __shared__ double sh[WG / 64];
    int parity = a.parity, bx = blockIdx.x;
    if (parity < 0) {
        parity = bx >= a.grid_half;
        if (parity) bx -= a.grid_half;
    }
    bx = tile_remap(xcd_remap(bx, a.grid_half), a.grid_half, a.tile_ts, a.tile_c);
    const int rhs = blockIdx.y;
    if (EPI == EPI_PLAIN) hop_alpha_on_the_side(a, sh);
    if (a.run && !a.run[rhs]) return;  // whole workgroup: one source
    const int gid = bx * WG + threadIdx.x;
    const int i = gid / G;
    const int r0 = (gid - i * G) * RS;
    double nrm = 0;
    Stage<S> stg{nullptr, 0, 0};
    if constexpr (STG && G == 1) {
        extern __shared__ __align__(16) unsigned char stage_raw[];
        stg = stage_input<NR>(a, a.in[1 - parity] + (size_t)rhs * a.rstride, bx * WG, (cpx<S> *)stage_raw);
    }
    if (i < a.g.half) {
        GlobalLinks<S, NR> links{a.gauge[parity], i};
        nrm = site_hop<NR, RS, S, DAG, EPI, GlobalLinks<S, NR>, STG && G == 1>(a, parity, i, r0, rhs, links, stg);
    }
    if (EPI != EPI_PLAIN && a.partial) {
        const double t = group_sum<G>(nrm, sh);
        const int grp = i / PG_SITES;
        if ((threadIdx.x & (PG_SITES * G - 1)) == 0 && grp < a.ngroups)
            a.partial[(size_t)rhs * a.pstride + (a.parity < 0 ? parity * a.ngroups : 0) + grp] = t;
    }
}

// The single-source kernel with the representation map fused in (RepLinks):
// a.gauge[q] holds the fundamental hopping blocks of output parity q.
template <int N, int REP, int NR, int RS, class S, bool DAG, int EPI, bool STG = false>
__global__ void __launch_bounds__(WG) hop_fused_kernel(const HopArgs<S> a)
{
    constexpr int G = NR / RS;
    __shared__ double sh[WG / 64];
    int parity = a.parity, bx = blockIdx.x;
    if (parity < 0) {
        parity = bx >= a.grid_half;
        if (parity) bx -= a.grid_half;
    }
    bx = tile_remap(xcd_remap(bx, a.grid_half), a.grid_half, a.tile_ts, a.tile_c);
    const int rhs = blockIdx.y;
    if (EPI == EPI_PLAIN) hop_alpha_on_the_side(a, sh);
    if (a.run && !a.run[rhs]) return;
    const int gid = bx * WG + threadIdx.x;
    const int i = gid / G;
    const int r0 = (gid - i * G) * RS;
    double nrm = 0;
    Stage<S> stg{nullptr, 0, 0};
    if constexpr (STG && G == 1) {
        extern __shared__ __align__(16) unsigned char stage_raw[];
        stg = stage_input<NR>(a, a.in[1 - parity] + (size_t)rhs * a.rstride, bx * WG, (cpx<S> *)stage_raw);
    }
    if (i < a.g.half) {
        RepLinks<S, N, REP> links{a.gauge[parity], i};
        nrm = site_hop<NR, RS, S, DAG, EPI, RepLinks<S, N, REP>, STG && G == 1>(a, parity, i, r0, rhs, links, stg);
    }
    if (EPI != EPI_PLAIN && a.partial) {
        const double t = group_sum<G>(nrm, sh);
        const int grp = i / PG_SITES;
        if ((threadIdx.x & (PG_SITES * G - 1)) == 0 && grp < a.ngroups)
            a.partial[(size_t)rhs * a.pstride + (a.parity < 0 ? parity * a.ngroups : 0) + grp] = t;
    }
}

// The single-source kernel for SU(3) fundamental links read as two rows per
// link (Su3Links); one thread per site, as hop_kernel at N_R = 3.
template <class S, bool DAG, int EPI, bool STG = false>
__global__ void __launch_bounds__(WG) hop_su3_kernel(const HopArgs<S> a)
{
    __shared__ double sh[WG / 64];
    int parity = a.parity, bx = blockIdx.x;
    if (parity < 0) {
        parity = bx >= a.grid_half;
        if (parity) bx -= a.grid_half;
    }
    bx = tile_remap(xcd_remap(bx, a.grid_half), a.grid_half, a.tile_ts, a.tile_c);
    const int rhs = blockIdx.y;
    if (EPI == EPI_PLAIN) hop_alpha_on_the_side(a, sh);
    if (a.run && !a.run[rhs]) return;
    const int i = bx * WG + threadIdx.x;
    double nrm = 0;
    Stage<S> stg{nullptr, 0, 0};
    if constexpr (STG) {
        extern __shared__ __align__(16) unsigned char stage_raw[];
        stg = stage_input<3>(a, a.in[1 - parity] + (size_t)rhs * a.rstride, bx * WG, (cpx<S> *)stage_raw);
    }
    if (i < a.g.half) {
        Su3Links<S> links{a.gauge[parity], i};
        nrm = site_hop<3, 3, S, DAG, EPI, Su3Links<S>, STG>(a, parity, i, 0, rhs, links, stg);
    }
    if (EPI != EPI_PLAIN && a.partial) {
        const double t = group_sum<1>(nrm, sh);
        const int grp = i / PG_SITES;
        if ((threadIdx.x & (PG_SITES - 1)) == 0 && grp < a.ngroups)
            a.partial[(size_t)rhs * a.pstride + (a.parity < 0 ? parity * a.ngroups : 0) + grp] = t;
    }
}

// Multi-source kernel: a workgroup owns MRS sites (16 or 32: one or two
// partial-sum groups) and every source.  It copies the sites' links (all 8
// directions) into LDS once, then its threads run the per-site hop reading
// links from LDS: each link crosses HBM once per launch however many sources
// there are.  The workgroup has as many threads as (source, site, row group)
// items, up to MR_MAX_THREADS per round (a whole number of MRS x G items, see
// mr_threads and MrTuner), so a round is never partly idle.  Thread t keeps
// its site and row group in every round; only the source advances.  The site
// count changes neither the per-site arithmetic nor the 16-site partial sums,
// so results are bitwise the same for either.
// Waves per SIMD the instance is compiled for: 32-bit N_R <= 6 fits three
// (168 VGPRs), except the fused CG update at N_R = 6, whose epilogue operands
// (self, r, x, p for 4 N_R components) need more registers: at three waves it
// spilled 28-164 bytes per lane, so it is compiled for two; so are the
// 32-site N_R = 6 workgroups, whose 74 KB of links allow two per CU anyway.
template <class S, int NR, int EPI, int MRS>
struct MRW { static constexpr int value = NR < 6 || (NR == 6 && EPI != EPI_CG && MRS == 16) ? 3 : 2; };
template <int NR, int EPI, int MRS> struct MRW<double, NR, EPI, MRS> { static constexpr int value = 2; };

template <int NR, int RS, class S, bool DAG, int EPI, int MRS = MR_SITES>
__global__ void __launch_bounds__(MR_MAX_THREADS) __attribute__((amdgpu_waves_per_eu(MRW<S, NR, EPI, MRS>::value)))
hop_mrhs_kernel(const HopArgs<S> a)
{
    static_assert(MRS % PG_SITES == 0, "whole partial-sum groups per workgroup");
    constexpr int G = NR / RS;
    constexpr int GC = 8 * NR * NR;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<S> *lk = (cpx<S> *)smem_raw;
    __shared__ double sh[MR_MAX_THREADS / 64];
    const int nt = blockDim.x;  // a multiple of 64 and of MRS * G
    int parity = a.parity, bx = blockIdx.x;
    if (parity < 0) {
        parity = bx >= a.grid_half;
        if (parity) bx -= a.grid_half;
    }
    // the remapped index is uniform over the workgroup: held in a scalar register (kept in a
    // vector register it tipped the 16-site FP32 axpy instances into 12-28 B of spill)
    bx = __builtin_amdgcn_readfirstlane(
        tile_remap_planes(xcd_remap(bx, a.grid_half), a.grid_half, a.tile_ts, a.tile_c, a.tile_p, a.tile_b));
    if (EPI == EPI_PLAIN) hop_alpha_on_the_side(a, sh);
    const int i0 = bx * MRS;
    const cpx<S> *__restrict__ gauge = a.gauge[parity];
    for (int e = threadIdx.x; e < GC * MRS; e += nt) {
        const int comp = e / MRS, s = e - comp * MRS;
        const int i = i0 + s;
        cpx<S> v;
        if (i < a.g.half) {
            typename acc_of<S>::type re, im;
            load_c_nt(gauge + lay(i, comp, GC), re, im);
            v.re = conv<S>::from_acc(re);
            v.im = conv<S>::from_acc(im);
        } else {
            v.re = conv<S>::from_acc(0);
            v.im = conv<S>::from_acc(0);
        }
        lk[e] = v;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int rg = t % G;
    const int s = (t / G) % MRS;
    const int i = i0 + s;
    LdsLinks<S, MRS> links{lk, s};
    const int items = MRS * G * a.n_rhs;
    for (int e0 = 0; e0 < items; e0 += nt) {
        const int rhs = (e0 + t) / (MRS * G);
        const bool live = rhs < a.n_rhs && (!a.run || a.run[rhs]);
        double nrm = 0;
        if (i < a.g.half && live) nrm = site_hop<NR, RS, S, DAG, EPI>(a, parity, i, rg * RS, rhs, links);
        if (EPI != EPI_PLAIN && a.partial) {
            const double tt = group_sum<G>(nrm, sh);
            const int grp = bx * (MRS / PG_SITES) + s / PG_SITES;
            if ((t & (PG_SITES * G - 1)) == 0 && live && grp < a.ngroups)
                a.partial[(size_t)rhs * a.pstride + (a.parity < 0 ? parity * a.ngroups : 0) + grp] = tt;
        }
    }
}

// Tiling of the work order (see tile_remap); disabled unless every time slice
// holds a whole number of workgroups.
inline void hop_tiling(const Geom &g, int sites_per_wg, int *ts, int *c, int cmax = 16)
{
    *ts = 0;
    *c = 0;
    const long long per_slice = (long long)g.half / g.d[0];  // sites per time slice
    if ((long long)g.half % g.d[0] || per_slice % sites_per_wg) return;
    const int n = (int)(per_slice / sites_per_wg);
    if (n < 2) return;
    int best = 1;
    for (int k = 1; k <= cmax && k <= n; ++k)
        if (n % k == 0) best = k;
    *ts = n;
    *c = best;
}

// x1-plane blocking of the multi-source walk (tile_remap_planes): p planes per
// chunk, set only where the chunk tiles whole planes of every time slice;
// otherwise both stay 0 (the flat chunk)
inline void hop_tiling_planes(const Geom &g, int sites_per_wg, int p, int ts, int c, int *tp, int *tb)
{
    *tp = 0;
    *tb = 0;
    if (p <= 1 || ts <= 0 || c <= 0 || c % p) return;
    const long long plane = (long long)g.d[2] * g.d[3] / 2;  // half-sites of one x1-plane of a time slice
    if (plane % sites_per_wg) return;
    const int B = (int)(plane / sites_per_wg);
    const int q = c / p;
    if (B % q || ts % B || (ts / B) % p) return;
    *tp = p;
    *tb = B;
}

// HRW_MRHS_PLANES=1, 2, 4 or 8 pins the x1-planes per chunk of the
// multi-source walk over the tuned choice: for tests and experiments
inline int mr_planes_env()
{
    const char *e = getenv("HRW_MRHS_PLANES");
    if (!e) return 0;
    const int v = atoi(e);
    return v == 1 || v == 2 || v == 4 || v == 8 ? v : 0;
}

// enum hrw_dtype of a storage type (0 FP64, 1 FP32, 2 BF16, 3 FP16)
template <class S> constexpr int dtype_id() { return 1; }
template <> constexpr int dtype_id<double>() { return 0; }
template <> constexpr int dtype_id<bf16_t>() { return 2; }
template <> constexpr int dtype_id<f16_t>() { return 3; }

// Workgroup size of one multi-source kernel instance for n_rhs sources, from
// the runtime's occupancy figure for each candidate size (queried once per
// instance and size; lds is fixed per instance).
template <int NR, int RS, class S, bool D, int E, int MRS>
int mr_block(int n_rhs, size_t lds)
{
    static int occ[MR_MAX_THREADS / 64 + 1] = {};
    static std::mutex mu;
    auto blocks_per_cu = [&](int t) {
        std::lock_guard<std::mutex> lock(mu);
        int &o = occ[t / 64];
        if (!o) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, hop_mrhs_kernel<NR, RS, S, D, E, MRS>, t, lds) !=
                    hipSuccess || nb < 1)
                nb = 1;
            o = nb;
        }
        return o;
    };
    return mr_threads(NR / RS, n_rhs, blocks_per_cu, MRS);
}

template <int NR, class S>
constexpr size_t mr_lds(int sites) { return sizeof(cpx<S>) * 8 * NR * NR * (size_t)sites; }

// Whether the 32-site workgroup is built for an instance: two partial-sum
// groups of G row threads must fit a round (32 G <= 128) and its links the LDS.
template <int NR, int RS, class S>
constexpr bool mr_has32() { return 32 * (NR / RS) <= WG / 2 && mr_lds<NR, S>(32) <= 160 * 1024; }

// ------------------------------------------------------------ launch-shape tuning
//
// Launch shape of the multi-source kernel: sites per workgroup (16 or 32),
// threads per workgroup and the spatial chunk of the time-tiled walk (its
// width and the x1-planes it spans, tile_remap_planes).  None
// changes any result (the partial sums are per 16-site group, the per-source
// arithmetic is fixed), so the shape is picked by timing.  On the first
// plain-epilogue launch of each (instance family, sources, lattice extents)
// every candidate runs twice on the caller's stream and the fastest is kept
// for every epilogue of that key for the life of the process, and written to
// a cache file (JSON, keyed by architecture, N_R, row split, storage type,
// sources and volume class = ceil(log2(sites per parity))) that later
// processes read before tuning.  The file is $HRW_TUNE_CACHE, else
// $HOME/.cache/hrw/tune.json; HRW_TUNE_CACHE set to an empty string keeps
// the choices in memory only.  Until a key is tuned (or with HRW_TUNE=0, or
// while the stream is being captured into a graph) the occupancy model
// (mr_block, 16 sites), chunk 16 and MR_PLANES planes are used.
struct MrShape {
    int threads;
    int cmax;    // chunk limit handed to hop_tiling (the chunk itself follows the launch's geometry)
    int sites;   // sites per workgroup: 16 or 32
    int planes = 1;  // x1-planes per chunk of the walk (tile_remap_planes; 1: flat chunks)
};

// the untuned walk: chunks of 16 workgroups over 4 x1-planes (at SU(3) sym
// 32^4 with 24 sources the plain hop took 2229 us against 2531 us with flat
// chunks; 2 planes 2340 us, 8 planes 2232 us)
constexpr int MR_PLANES = 4;

inline bool mr_tuning_enabled()
{
    const char *e = getenv("HRW_TUNE");
    return !(e && e[0] == '0');
}

// The persistent part of the tuner: one JSON file shared by every instance
// family, an object whose entries are  "key": {"threads": T, "cmax": C,
// "sites": S, "planes": P, "us": U}  (written one per line; an entry without
// "planes" has flat chunks).
struct TuneCache {
    std::mutex mu;
    bool loaded = false;
    std::map<std::string, std::pair<MrShape, double>> entries;

    static std::string path()
    {
        const char *e = getenv("HRW_TUNE_CACHE");
        if (e) return std::string(e);
        const char *h = getenv("HOME");
        if (!h || !h[0]) return std::string();
        return std::string(h) + "/.cache/hrw/tune.json";
    }

    // entries of an object of objects  {"key": {"threads": T, "cmax": C, "sites": S, "planes": P,
    // "us": U}, ...} in any JSON layout; entries with unusable values are skipped
    void read_file(const std::string &p, std::map<std::string, std::pair<MrShape, double>> &into)
    {
        FILE *f = fopen(p.c_str(), "r");
        if (!f) return;
        std::string text;
        char buf[4096];
        size_t n;
        while ((n = fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (1u << 22)) text.append(buf, n);
        fclose(f);
        auto field = [](const std::string &obj, const char *name, double *v) {
            const size_t k = obj.find(std::string("\"") + name + "\"");
            if (k == std::string::npos) return false;
            const size_t c = obj.find(':', k);
            return c != std::string::npos && sscanf(obj.c_str() + c + 1, "%lf", v) == 1;
        };
        size_t pos = 0;
        const size_t open = text.find('{');
        if (open == std::string::npos) return;
        pos = open + 1;
        while (true) {
            const size_t q0 = text.find('"', pos);
            if (q0 == std::string::npos) break;
            const size_t q1 = text.find('"', q0 + 1);
            if (q1 == std::string::npos) break;
            const size_t b0 = text.find('{', q1);
            const size_t b1 = b0 == std::string::npos ? b0 : text.find('}', b0);
            if (b1 == std::string::npos) break;
            const std::string key = text.substr(q0 + 1, q1 - q0 - 1), obj = text.substr(b0, b1 - b0 + 1);
            double t = 0, c = 0, s = 0, pl = 1, us = 0;
            // range checks before any conversion: a value outside int's range would be undefined
            const bool has_planes = obj.find("\"planes\"") != std::string::npos;
            if (field(obj, "threads", &t) && field(obj, "cmax", &c) && field(obj, "sites", &s) && t >= 64 &&
                t <= MR_MAX_THREADS && (c == 4 || c == 16 || c == 32 || c == 64) && (s == 16 || s == 32) &&
                (!has_planes || (field(obj, "planes", &pl) && (pl == 1 || pl == 2 || pl == 4 || pl == 8)))) {
                field(obj, "us", &us);
                const MrShape sh{(int)t, (int)c, (int)s, (int)pl};
                if (sh.threads == t && sh.threads % 64 == 0) into[key] = {sh, us};
            }
            pos = b1 + 1;
        }
    }

    bool lookup(const std::string &key, MrShape *out)
    {
        std::lock_guard<std::mutex> lock(mu);
        if (!loaded) {
            loaded = true;
            const std::string p = path();
            if (!p.empty()) read_file(p, entries);
        }
        auto it = entries.find(key);
        if (it == entries.end()) return false;
        *out = it->second.first;
        return true;
    }

    // merge with what other processes wrote meanwhile, then replace the file atomically
    void store(const std::string &key, MrShape sh, double us)
    {
        std::lock_guard<std::mutex> lock(mu);
        entries[key] = {sh, us};
        const std::string p = path();
        if (p.empty()) return;
        const size_t slash = p.find_last_of('/');
        if (slash != std::string::npos && slash > 0) {
            const std::string dir = p.substr(0, slash);
            const std::string parent = dir.substr(0, dir.find_last_of('/'));
            if (!parent.empty()) mkdir(parent.c_str(), 0755);
            mkdir(dir.c_str(), 0755);
        }
        std::map<std::string, std::pair<MrShape, double>> merged;
        read_file(p, merged);
        for (auto &kv : entries) merged[kv.first] = kv.second;
        const std::string tmp = p + ".tmp" + std::to_string((long)getpid());
        FILE *f = fopen(tmp.c_str(), "w");
        if (!f) return;
        fprintf(f, "{\n");
        size_t n = 0;
        for (auto &kv : merged) {
            const MrShape &m = kv.second.first;
            fprintf(f, "  \"%s\": {\"threads\": %d, \"cmax\": %d, \"sites\": %d, \"planes\": %d, \"us\": %.1f}%s\n",
                    kv.first.c_str(), m.threads, m.cmax, m.sites, m.planes, kv.second.second,
                    ++n < merged.size() ? "," : "");
        }
        fprintf(f, "}\n");
        const bool ok = fclose(f) == 0;
        if (!ok || rename(tmp.c_str(), p.c_str()) != 0) remove(tmp.c_str());
    }
};

inline TuneCache &tune_cache()
{
    static TuneCache c;
    return c;
}

inline std::string device_arch()
{
    static std::string arch;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            arch = prop.gcnArchName;
            const size_t c = arch.find(':');
            if (c != std::string::npos) arch = arch.substr(0, c);
        }
        if (arch.empty()) arch = "unknown";
    });
    return arch;
}

template <int NR, int RS, class S>
struct MrTuner {
    typedef std::array<int, 5> Key;  // sources and the four extents
    std::mutex mu;
    std::map<Key, MrShape> best;

    static Key key(const HopArgs<S> &b) { return Key{b.n_rhs, b.g.d[0], b.g.d[1], b.g.d[2], b.g.d[3]}; }

    static std::string cache_key(const HopArgs<S> &b)
    {
        int vc = 0;
        while ((1LL << vc) < (long long)b.g.half) ++vc;
        static const char *names[] = {"f64", "f32", "bf16", "f16"};
        char buf[160];
        // "w2": shapes that carry the walk's planes (entries of earlier files are not reused)
        snprintf(buf, sizeof buf, "%s/nr%d/rs%d/%s/n%d/v%d/w2", device_arch().c_str(), NR, RS, names[dtype_id<S>()],
                 b.n_rhs, vc);
        return buf;
    }

    bool lookup(const HopArgs<S> &b, MrShape *out)
    {
        {
            std::lock_guard<std::mutex> lock(mu);
            auto it = best.find(key(b));
            if (it != best.end()) {
                *out = it->second;
                return true;
            }
        }
        MrShape sh;
        if (!tune_cache().lookup(cache_key(b), &sh)) return false;
        if (sh.sites == 32 && !mr_has32<NR, RS, S>()) return false;
        if (sh.threads % mr_unit(NR / RS, sh.sites)) return false;  // not a shape of this instance
        std::lock_guard<std::mutex> lock(mu);
        best[key(b)] = sh;
        *out = sh;
        return true;
    }

    // time every candidate with the plain epilogue (out = H in: re-running it is
    // harmless); returns the fastest, or false if timing was not possible
    template <bool D>
    bool tune(const HopArgs<S> &b0, hipStream_t st, MrShape *out)
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = best.find(key(b0));
        if (it != best.end()) {
            *out = it->second;
            return true;
        }
        constexpr int G = NR / RS;
        hipEvent_t ev[2];
        if (hipEventCreate(&ev[0]) != hipSuccess) return false;
        if (hipEventCreate(&ev[1]) != hipSuccess) {
            (void)hipEventDestroy(ev[0]);
            return false;
        }
        float best_ms = 0;
        MrShape pick{0, 0, 0, 1};
        bool ok = true;
        for (int sites : {16, 32}) {
            if (sites == 32 && !mr_has32<NR, RS, S>()) continue;
            const int unit = mr_unit(G, sites);
            const size_t lds = mr_lds<NR, S>(sites);
            HopArgs<S> b = b0;
            b.grid_half = (b0.ngroups + sites / PG_SITES - 1) / (sites / PG_SITES);
            const dim3 grid(b0.parity < 0 ? 2 * b.grid_half : b.grid_half, 1);
            // walks: (chunk limit, planes); a candidate whose chunk and planes repeat
            // an earlier one's on this lattice is skipped
            const int walks[4][2] = {{16, 1}, {16, MR_PLANES}, {32, MR_PLANES}, {64, MR_PLANES}};
            int seen[4][2];
            int nseen = 0;
            for (const auto &wk : walks) {
                const int cmax = wk[0];
                hop_tiling(b.g, sites, &b.tile_ts, &b.tile_c, cmax);
                hop_tiling_planes(b.g, sites, wk[1], b.tile_ts, b.tile_c, &b.tile_p, &b.tile_b);
                bool dup = false;
                for (int k = 0; k < nseen; ++k) dup = dup || (seen[k][0] == b.tile_c && seen[k][1] == b.tile_p);
                if (dup) continue;
                seen[nseen][0] = b.tile_c;
                seen[nseen][1] = b.tile_p;
                ++nseen;
                for (int t = MR_MAX_THREADS; t >= unit && ok; t -= 64) {
                    if (t % unit) continue;
                    float ms = 0;
                    for (int rep = 0; rep < 2 && ok; ++rep) {
                        ok = hipEventRecord(ev[0], st) == hipSuccess;
                        if (sites == 32) {
                            if constexpr (mr_has32<NR, RS, S>())
                                hop_mrhs_kernel<NR, RS, S, D, EPI_PLAIN, 32><<<grid, dim3(t), lds, st>>>(b);
                        } else {
                            hop_mrhs_kernel<NR, RS, S, D, EPI_PLAIN, 16><<<grid, dim3(t), lds, st>>>(b);
                        }
                        ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(ev[1], st) == hipSuccess &&
                             hipEventSynchronize(ev[1]) == hipSuccess;
                        float e = 0;
                        ok = ok && hipEventElapsedTime(&e, ev[0], ev[1]) == hipSuccess;
                        if (ok && (rep == 0 || e < ms)) ms = e;
                    }
                    if (ok && (pick.threads == 0 || ms < best_ms)) {
                        best_ms = ms;
                        pick = MrShape{t, cmax, sites, wk[1]};
                    }
                }
            }
        }
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        if (!ok || pick.threads == 0) return false;
        best[key(b0)] = pick;
        tune_cache().store(cache_key(b0), pick, best_ms * 1e3);
        *out = pick;
        return true;
    }
};

template <int NR, int RS, class S>
MrTuner<NR, RS, S> &mr_tuner()
{
    static MrTuner<NR, RS, S> t;
    return t;
}

// HRW_MRHS_SITES=16 or 32 pins the sites per workgroup (threads from the
// occupancy model, chunk 16; no tuning): for tests and experiments
inline int mr_forced_sites()
{
    const char *e = getenv("HRW_MRHS_SITES");
    if (!e) return 0;
    const int v = atoi(e);
    return v == 16 || v == 32 ? v : 0;
}

// shape for this launch (see MrTuner); tunes on a plain-epilogue launch
template <int NR, int RS, class S, bool D, int E>
MrShape mr_shape(const HopArgs<S> &b, hipStream_t st)
{
    MrShape sh;
    const int forced = mr_forced_sites();
    if (forced == 32 && mr_has32<NR, RS, S>())
        return MrShape{mr_block<NR, RS, S, D, E, 32>(b.n_rhs, mr_lds<NR, S>(32)), 16, 32, MR_PLANES};
    if (forced == 16)
        return MrShape{mr_block<NR, RS, S, D, E, 16>(b.n_rhs, mr_lds<NR, S>(16)), 16, 16, MR_PLANES};
    auto &tuner = mr_tuner<NR, RS, S>();
    if (tuner.lookup(b, &sh)) return sh;
    if (E == EPI_PLAIN && mr_tuning_enabled()) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone &&
            tuner.template tune<D>(b, st, &sh))
            return sh;
    }
    return MrShape{mr_block<NR, RS, S, D, E, 16>(b.n_rhs, mr_lds<NR, S>(16)), 16, 16, MR_PLANES};
}

template <int NR, int RS, class S, bool D, int E>
void launch_mrhs(const HopArgs<S> &b, hipStream_t st)
{
    const MrShape sh = mr_shape<NR, RS, S, D, E>(b, st);
    HopArgs<S> bt = b;
    bt.grid_half = (b.ngroups + sh.sites / PG_SITES - 1) / (sh.sites / PG_SITES);
    hop_tiling(bt.g, sh.sites, &bt.tile_ts, &bt.tile_c, sh.cmax);
    const int forced_planes = mr_planes_env();
    hop_tiling_planes(bt.g, sh.sites, forced_planes > 0 ? forced_planes : sh.planes, bt.tile_ts, bt.tile_c,
                      &bt.tile_p, &bt.tile_b);
    const dim3 grid(b.parity < 0 ? 2 * bt.grid_half : bt.grid_half, 1);
    if constexpr (mr_has32<NR, RS, S>()) {
        if (sh.sites == 32) {
            hop_mrhs_kernel<NR, RS, S, D, E, 32><<<grid, dim3(sh.threads), mr_lds<NR, S>(32), st>>>(bt);
            return;
        }
    }
    hop_mrhs_kernel<NR, RS, S, D, E, 16><<<grid, dim3(sh.threads), mr_lds<NR, S>(16), st>>>(bt);
}

// Input staging of the one-thread-per-site kernels (stage_input): opt-in
// (HRW_HOP_STAGE=1), built for 32-bit and 16-bit storage with N_R <= 4, and
// used only where the staged range fits the default 64 KB of LDS.  Measured
// on MI355X it does not pay: D_hat at 32^4 SU(3) fund FP32 204 us staged
// against 180 us unstaged, two-row 180 against 151 us, SU(2) adj 24^3x48
// 150 against 129 us (the neighbour reads it replaces mostly hit L2 already,
// and the copy into LDS, its barrier and the lower occupancy cost more); an
// FP64 variant (two workgroups per CU with 55 KB of staged spinors) was
// slower still, and compiling the range check into the unstaged FP64 hop
// alone cost it 7%, so the staged kernels are separate instances.  Returns
// the dynamic LDS bytes of the launch and sets b.stage.
inline bool hop_stage_enabled()
{
    const char *e = getenv("HRW_HOP_STAGE");
    return e && e[0] == '1';
}

// whether the staged instances of an (N_R, storage, threads per site) family are built
template <int NR, class S, int G>
constexpr bool stage_built() { return G == 1 && dtype_id<S>() != 0 && NR <= 4; }

template <int NR, class S, int G>
size_t plan_stage(HopArgs<S> &b)
{
    b.stage = 0;
    if (!stage_built<NR, S, G>() || !hop_stage_enabled()) return 0;
    const size_t bytes = (size_t)(WG + 2 * b.g.n3h) * 4 * NR * sizeof(cpx<S>);
    if (bytes > 65536) return 0;
    b.stage = 1;
    return bytes;
}

template <int NR, int RS, class S, bool MRK>
void launch_hop_rs(bool dagger, int epi, dim3 grid, size_t lds, const HopArgs<S> &b, hipStream_t st)
{
#define HRW_LAUNCH(D, E)                                                                           \
    do {                                                                                           \
        if (MRK) launch_mrhs<NR, RS, S, D, E>(b, st);                                              \
        else if (b.stage) hop_kernel<NR, RS, S, D, E, stage_built<NR, S, NR / RS>()><<<grid, WG, lds, st>>>(b); \
        else hop_kernel<NR, RS, S, D, E><<<grid, WG, 0, st>>>(b);                                  \
    } while (0)
    if (epi == EPI_PLAIN) {
        if (dagger) HRW_LAUNCH(true, EPI_PLAIN);
        else HRW_LAUNCH(false, EPI_PLAIN);
    } else if (epi == EPI_AXPY) {
        if (dagger) HRW_LAUNCH(true, EPI_AXPY);
        else HRW_LAUNCH(false, EPI_AXPY);
    } else {
        HRW_LAUNCH(true, EPI_CG);
    }
#undef HRW_LAUNCH
}

template <int NR, int RS, class S>
hipError_t allow_lds()
{
    // the multi-source instances may need more than the default 64 KB of LDS
    static bool done = false;
    if (done) return hipSuccess;
    hipError_t e = hipSuccess;
    auto set = [&](const void *f, size_t lds) {
        if (e == hipSuccess && lds > 65536)
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    };
#define HRW_ALLOW(M)                                                                                 \
    set((const void *)hop_mrhs_kernel<NR, RS, S, true, EPI_PLAIN, M>, mr_lds<NR, S>(M));               \
    set((const void *)hop_mrhs_kernel<NR, RS, S, false, EPI_PLAIN, M>, mr_lds<NR, S>(M));              \
    set((const void *)hop_mrhs_kernel<NR, RS, S, true, EPI_AXPY, M>, mr_lds<NR, S>(M));                \
    set((const void *)hop_mrhs_kernel<NR, RS, S, false, EPI_AXPY, M>, mr_lds<NR, S>(M));               \
    set((const void *)hop_mrhs_kernel<NR, RS, S, true, EPI_CG, M>, mr_lds<NR, S>(M));
    HRW_ALLOW(16)
    if constexpr (mr_has32<NR, RS, S>()) {
        HRW_ALLOW(32)
    }
#undef HRW_ALLOW
    done = e == hipSuccess;
    return e;
}

template <class S>
hipError_t launch_hop_impl(int nr, bool dagger, int epi, const HopArgs<S> &a, hipStream_t st)
{
    if (epi == EPI_CG && !dagger) return hipErrorInvalidValue;
    HopArgs<S> b = a;
    hipError_t err = hipSuccess;
    bool ok = dispatch_nr(nr, [&](auto nrc) {
        constexpr int NR = decltype(nrc)::value;
        constexpr int RS = hop_rows(NR, dtype_id<S>());
        constexpr int G = NR / RS;
        b.ngroups = hop_groups(a.g);
        if (hop_uses_mrhs(NR, dtype_id<S>(), a.n_rhs)) {
            // grid, tiling and LDS follow the launch shape (launch_mrhs)
            err = allow_lds<NR, RS, S>();
            if (err != hipSuccess) return;
            launch_hop_rs<NR, RS, S, true>(dagger, epi, dim3(1), 0, b, st);
        } else {
            const int gh = hop_grid(a.g, G);
            b.grid_half = gh;
            hop_tiling(a.g, WG / G, &b.tile_ts, &b.tile_c);
            dim3 grid(a.parity < 0 ? 2 * gh : gh, a.n_rhs);
            const size_t lds = plan_stage<NR, S, G>(b);
            launch_hop_rs<NR, RS, S, false>(dagger, epi, grid, lds, b, st);
        }
    });
    if (!ok) return hipErrorInvalidValue;
    if (err != hipSuccess) return err;
    return hipGetLastError();
}

// Fused representation map: one grid row per source (the multi-source kernel
// keeps its LDS copy of U_R), same tiling and partial-sum groups as hop_kernel.
template <class S>
hipError_t launch_hop_fused_impl(int nc, int rep, bool dagger, int epi, const HopArgs<S> &a, hipStream_t st)
{
    if (epi == EPI_CG && !dagger) return hipErrorInvalidValue;
    HopArgs<S> b = a;
    bool ok = false;
    auto go = [&](auto nv, auto rv) {
        constexpr int N = decltype(nv)::value;
        constexpr int REP = decltype(rv)::value;
        constexpr int NR = REP == 1 ? N * N - 1 : REP == 2 ? N * (N + 1) / 2 : N * (N - 1) / 2;
        constexpr int RS = hop_rows(NR, dtype_id<S>());
        constexpr int G = NR / RS;
        b.ngroups = hop_groups(a.g);
        const int gh = hop_grid(a.g, G);
        b.grid_half = gh;
        hop_tiling(a.g, WG / G, &b.tile_ts, &b.tile_c);
        dim3 grid(a.parity < 0 ? 2 * gh : gh, a.n_rhs);
        const size_t lds = plan_stage<NR, S, G>(b);
        constexpr bool SB = stage_built<NR, S, G>();
#define HRW_FUSED(D, E)                                                                            \
        do {                                                                                       \
            if (b.stage) hop_fused_kernel<N, REP, NR, RS, S, D, E, SB><<<grid, WG, lds, st>>>(b);  \
            else hop_fused_kernel<N, REP, NR, RS, S, D, E><<<grid, WG, 0, st>>>(b);                \
        } while (0)
        if (epi == EPI_PLAIN) {
            if (dagger) HRW_FUSED(true, EPI_PLAIN);
            else HRW_FUSED(false, EPI_PLAIN);
        } else if (epi == EPI_AXPY) {
            if (dagger) HRW_FUSED(true, EPI_AXPY);
            else HRW_FUSED(false, EPI_AXPY);
        } else {
            HRW_FUSED(true, EPI_CG);
        }
#undef HRW_FUSED
        ok = true;
    };
    if (nc == 2 && rep == 1) go(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{});
    else if (nc == 2 && rep == 2) go(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{});
    else if (nc == 3 && rep == 2) go(std::integral_constant<int, 3>{}, std::integral_constant<int, 2>{});
    else if (nc == 4 && rep == 3) go(std::integral_constant<int, 4>{}, std::integral_constant<int, 3>{});
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// SU(3) fundamental links read as two rows: same grid, tiling and partial-sum
// groups as hop_kernel at N_R = 3.
template <class S>
hipError_t launch_hop_su3_impl(bool dagger, int epi, const HopArgs<S> &a, hipStream_t st)
{
    static_assert(hop_rows(3, dtype_id<S>()) == 3, "one thread per site");
    if (epi == EPI_CG && !dagger) return hipErrorInvalidValue;
    HopArgs<S> b = a;
    b.ngroups = hop_groups(a.g);
    const int gh = hop_grid(a.g, 1);
    b.grid_half = gh;
    hop_tiling(a.g, WG, &b.tile_ts, &b.tile_c);
    dim3 grid(a.parity < 0 ? 2 * gh : gh, a.n_rhs);
    const size_t lds = plan_stage<3, S, 1>(b);
    constexpr bool SB = stage_built<3, S, 1>();
#define HRW_SU3(D, E)                                                                              \
    do {                                                                                           \
        if (b.stage) hop_su3_kernel<S, D, E, SB><<<grid, WG, lds, st>>>(b);                        \
        else hop_su3_kernel<S, D, E><<<grid, WG, 0, st>>>(b);                                      \
    } while (0)
    if (epi == EPI_PLAIN) {
        if (dagger) HRW_SU3(true, EPI_PLAIN);
        else HRW_SU3(false, EPI_PLAIN);
    } else if (epi == EPI_AXPY) {
        if (dagger) HRW_SU3(true, EPI_AXPY);
        else HRW_SU3(false, EPI_AXPY);
    } else {
        HRW_SU3(true, EPI_CG);
    }
#undef HRW_SU3
    return hipGetLastError();
}

}  // namespace hrw
