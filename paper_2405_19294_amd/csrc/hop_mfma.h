// Multi-source hopping kernel on the matrix cores (FP32 storage and
// arithmetic), for the even/odd hops of arXiv 2405.19294 Sec. 3.1 applied to
// several sources that share every link load.
//
// Per site and direction the link multiplies a block of half-spinors, one
// column per (source, half-spinor component):  G = U h  with U the N_R x N_R
// link and h the 2 x n_src half-spinors.  In real arithmetic this is the
// contraction  [Re G; Im G] = [[Ur, -Ui], [Ui, Ur]] [Re h; Im h], rows and
// inner index 2 N_R.  It runs on v_mfma_f32_4x4x1_16b_f32, whose 16
// independent 4x4 blocks are the 16 sites of the workgroup's site group (each
// site has its own link, the A operand):
//   lane l: site b = l / 4 of the group, column q = l % 4 of a 4-column tile;
//   A (4 x 1 per block): row i of block b from lane 4b + i;
//   B (1 x 4 per block): column j of block b from lane 4b + j;
//   result: lane 4b + j holds rows 0..3 of column j.
// A wave covers the 16 sites and 2 NT sources (NT tiles of 4 columns: two
// sources x the two half-spinor components); the waves of a workgroup cover
// further sources and share the group's links, staged in LDS once per launch.
// Each lane builds its own B column by projecting the neighbour spinor of its
// source (loads coalesce over the 16 sites, as in the vector kernel), so the
// operands never cross lanes; the reconstruction of the lower spin components
// exchanges the two half-spinor columns of a source between neighbouring
// lanes (DPP quad permute) where the projector swaps them.
//
// Lane (site b, source s, half h) accumulates the output spin components h
// and 2 + h of its source in real-embedded form (rows: Re of the N_R colours,
// then Im).  Projection and reconstruction, with sg = the projector sign of
// the hop direction and e_h = +1 for h = 0, -1 for h = 1, in the storage
// basis of the vector kernel (g_0 diagonal there):
//   mu = 0: sg = -1: h_h = 2 p_{h+2}; lower_h += g_h
//           sg = +1: h_h = 2 p_h;     upper_h += g_h
//   mu = 1: h_h = p_h - sg i p_{3-h};       lower_h +=  sg i g_{1-h}
//   mu = 2: h_h = p_h - e_h sg p_{3-h};     lower_h +=  e_h sg g_{1-h}
//   mu = 3: h_h = p_h - e_h sg i p_{2+h};   lower_h +=  e_h sg i g_h
// (for mu > 0 upper_h += g_h as well), the same table as the vector
// kernel's, split by half-spinor component.
#pragma once

#include <stdlib.h>

#include "hop_impl.h"

namespace hrw {

typedef float mf4 __attribute__((ext_vector_type(4)));

constexpr int MF_NT = 2;  // 4-column tiles (pairs of sources) per wave

__device__ __forceinline__ float lane_xor1(float v)
{
    // quad_perm [1, 0, 3, 2]: exchange with the neighbouring lane
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

template <int NR>
struct MfmaGeom {
    static constexpr int K = 2 * NR;            // real-embedded rows and inner index
    static constexpr int NM = (NR + 1) / 2;     // 4-row tiles: two Re and two Im rows each
    static constexpr int NC = 4 * NR;           // spinor components
    static constexpr int GC = 8 * NR * NR;      // link components per site
};

// One direction of the hop for the lane's site and all its columns.
template <int MU, int DIR, bool DAG, int NR, int NT>
__device__ __forceinline__ void mfma_dir(const HopArgs<float> &a, const cpx<float> *__restrict__ in_base,
                                         const cpx<float> *lk, int b, int q, int src0, const int (&x)[4],
                                         float (&up)[NT][2 * NR], float (&lo)[NT][2 * NR])
{
    typedef MfmaGeom<NR> M;
    constexpr int K = M::K, NM = M::NM;
    constexpr int SG = (DIR == 0) ? (DAG ? 1 : -1) : (DAG ? -1 : 1);
    constexpr int DD = MU + 4 * DIR;
    const int h = q & 1;
    const float eh = h ? -1.0f : 1.0f;
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
    // spin components entering the lane's half-spinor component (one along mu = 0)
    const int sa = MU == 0 ? t_half<SG>() + h : h;
    const int sb = MU == 3 ? h + 2 : 3 - h;
    // A operand.  The 2 N_R real-embedded rows are ordered so that lanes q = 0, 1
    // hold the Re rows and q = 2, 3 the Im rows: lane row i of tile m is
    // Re row 2m + i (i < 2) or Im row 2m + i - 2 (i >= 2), i.e. the lane reads
    // link row 2m + (q & 1) as [Ur | -Ui] (Re rows) or [Ui | Ur] (Im rows):
    // the part it reads first is selected by a per-lane offset into the
    // interleaved (re, im) pairs, the second half takes a per-lane sign.
    float av[NM][K];
    const int first = q < 2 ? 0 : 1;             // Re rows start with Ur, Im rows with Ui
    const float sgn2 = q < 2 ? -1.0f : 1.0f;      // -Ui for Re rows, +Ur for Im rows
    const float *lkf = (const float *)lk;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
        const int r = 2 * m + (q & 1);
        const bool valid = r < NR;
        const float *row = lkf + 2 * (((DD * NR + (valid ? r : 0)) * NR) * MR_SITES + b);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            const float v1 = row[2 * c * MR_SITES + first];
            const float v2 = row[2 * c * MR_SITES + 1 - first];
            av[m][c] = valid ? v1 : 0.0f;
            av[m][NR + c] = valid ? sgn2 * v2 : 0.0f;
        }
    }
    // B columns: the projected neighbour spinor of each of the lane's sources
    float bv[NT][K];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int s = src0 + 2 * t + (q >> 1);
        float pr[2][NR], pi[2][NR];
        if (s < a.n_rhs && (!a.run || a.run[s])) {
            // component k of site j sits at lay(j, k) = lay(j, 0) + 64 k
            const cpx<float> *pa = in_base + (size_t)s * a.rstride + lay(j, sa * NR, M::NC);
            const cpx<float> *pb = in_base + (size_t)s * a.rstride + lay(j, sb * NR, M::NC);
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                load_c(pa + c * BLK, pr[0][c], pi[0][c]);
                if (MU != 0) load_c(pb + c * BLK, pr[1][c], pi[1][c]);
            }
        } else {
#pragma unroll
            for (int c = 0; c < NR; ++c) pr[0][c] = pi[0][c] = pr[1][c] = pi[1][c] = 0.0f;
        }
        // h = p_a + w p_b, w in {+-1, +-i}
        const float wr = (MU == 0) ? -(float)SG : (MU == 2 ? -eh * (float)SG : 0.0f);
        const float wi = (MU == 1) ? -(float)SG : (MU == 3 ? -eh * (float)SG : 0.0f);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            float hr, hi;
            if (MU == 0) {
                hr = 2 * pr[0][c];
                hi = 2 * pi[0][c];
            } else if (MU == 2) {
                hr = fmac(wr, pr[1][c], pr[0][c]);
                hi = fmac(wr, pi[1][c], pi[0][c]);
            } else {  // i z = (-z_im, z_re)
                hr = fmac(-wi, pi[1][c], pr[0][c]);
                hi = fmac(wi, pr[1][c], pi[0][c]);
            }
            if (wrap && !(a.ph_re[MU] == 1.0 && a.ph_im[MU] == 0.0)) {
                const float cr = (float)a.ph_re[MU];
                const float ci = DIR == 0 ? (float)a.ph_im[MU] : -(float)a.ph_im[MU];
                const float tr = hr * cr - hi * ci;
                const float ti = hr * ci + hi * cr;
                hr = tr;
                hi = ti;
            }
            bv[t][c] = hr;
            bv[t][NR + c] = hi;
        }
    }
    // G = A B on the matrix cores: NM x NT independent chains over the inner index
    mf4 d[NM][NT];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) d[m][t] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int m = 0; m < NM; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) d[m][t] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[m][k], bv[t][k], d[m][t], 0, 0, 0);
    // reconstruction into the upper (spin h) and lower (spin 2 + h) accumulators
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        // register i of tile m is Re row 2m + i (i < 2) or Im row 2m + i - 2
        float g[K];
#pragma unroll
        for (int m = 0; m < NM; ++m)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 2 * m + (i & 1);
                if (row < NR) g[(i < 2 ? 0 : NR) + row] = d[m][t][i];
            }
        if (MU == 0) {
#pragma unroll
            for (int rho = 0; rho < K; ++rho) {
                if (t_half<SG>() == 0) up[t][rho] += g[rho];
                else lo[t][rho] += g[rho];
            }
            continue;
        }
#pragma unroll
        for (int rho = 0; rho < K; ++rho) up[t][rho] += g[rho];
        if (MU == 1 || MU == 2) {
#pragma unroll
            for (int rho = 0; rho < K; ++rho) g[rho] = lane_xor1(g[rho]);  // the other component's column
        }
        const float cf = (MU == 0) ? -(float)SG : (MU == 1 ? (float)SG : eh * (float)SG);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            if (MU == 0 || MU == 2) {
                lo[t][c] = fmac(cf, g[c], lo[t][c]);
                lo[t][NR + c] = fmac(cf, g[NR + c], lo[t][NR + c]);
            } else {  // cf i g
                lo[t][c] = fmac(-cf, g[NR + c], lo[t][c]);
                lo[t][NR + c] = fmac(cf, g[c], lo[t][NR + c]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int rho = 0; rho < K; ++rho) asm volatile("" : "+v"(up[t][rho]), "+v"(lo[t][rho]));
    // keep the next direction's loads from being hoisted over this one (registers)
    __builtin_amdgcn_sched_barrier(0);
}

// FP64 sum over the 32 lanes of one source (16 sites x 2 half-spinor
// components) in a fixed tree; valid in every lane of the group.
__device__ __forceinline__ double mfma_source_sum(double v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

template <int NR, bool DAG, int EPI>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(1))) hop_mfma_kernel(const HopArgs<float> a)
{
    typedef MfmaGeom<NR> M;
    constexpr int NT = MF_NT, K = M::K, NC = M::NC, GC = M::GC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<float> *lk = (cpx<float> *)smem_raw;
    __shared__ double sh[4];
    const int nt = blockDim.x;  // whole wavefronts
    int parity = a.parity, bx = blockIdx.x;
    if (parity < 0) {
        parity = bx >= a.grid_half;
        if (parity) bx -= a.grid_half;
    }
    bx = tile_remap(xcd_remap(bx, a.grid_half), a.grid_half, a.tile_ts, a.tile_c);
    if (EPI == EPI_PLAIN) hop_alpha_on_the_side(a, sh);
    const int i0 = bx * MR_SITES;
    const cpx<float> *__restrict__ gauge = a.gauge[parity];
    for (int e = threadIdx.x; e < GC * MR_SITES; e += nt) {
        const int comp = e / MR_SITES, s = e - comp * MR_SITES;
        const int i = i0 + s;
        cpx<float> v;
        v.re = v.im = 0.0f;
        if (i < a.g.half) load_c_nt(gauge + lay(i, comp, GC), v.re, v.im);
        lk[e] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = nt >> 6;
    const int b = lane >> 2, q = lane & 3, h = q & 1;
    const int i = i0 + b;
    const bool site_ok = i < a.g.half;
    int x[4];
    eo_coords(a.g, parity, site_ok ? i : 0, x);
    const cpx<float> *__restrict__ in_base = a.in[1 - parity];
    for (int src0 = wave * 2 * NT; src0 < a.n_rhs; src0 += waves * 2 * NT) {
        // an opaque copy of the LDS pointer per round keeps the compiler from
        // hoisting all eight directions' A operands out of the loop
        const cpx<float> *lkr = lk;
        asm volatile("" : "+v"(lkr));
        float up[NT][K], lo[NT][K];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int rho = 0; rho < K; ++rho) up[t][rho] = lo[t][rho] = 0.0f;
        mfma_dir<0, 0, DAG, NR, NT>(a, in_base, lkr, b, q, src0, x, up, lo);
        mfma_dir<0, 1, DAG, NR, NT>(a, in_base, lkr, b, q, src0, x, up, lo);
        mfma_dir<1, 0, DAG, NR, NT>(a, in_base, lkr, b, q, src0, x, up, lo);
        mfma_dir<1, 1, DAG, NR, NT>(a, in_base, lkr, b, q, src0, x, up, lo);
        mfma_dir<2, 0, DAG, NR, NT>(a, in_base, lkr, b, q, src0, x, up, lo);
        mfma_dir<2, 1, DAG, NR, NT>(a, in_base, lkr, b, q, src0, x, up, lo);
        mfma_dir<3, 0, DAG, NR, NT>(a, in_base, lkr, b, q, src0, x, up, lo);
        mfma_dir<3, 1, DAG, NR, NT>(a, in_base, lkr, b, q, src0, x, up, lo);
        // epilogue for each of the lane's sources: spin components h and 2 + h
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int s = src0 + 2 * t + (q >> 1);
            const bool live = s < a.n_rhs && (!a.run || a.run[s]);
            const bool ok = site_ok && live;
            double nrm = 0;
            if (ok) {
                const size_t roff = (size_t)s * a.rstride;
                if (EPI == EPI_PLAIN) {
                    cpx<float> *out = a.out[parity] + roff;
#pragma unroll
                    for (int c = 0; c < NR; ++c) {
                        store_c_nt(out + lay(i, h * NR + c, NC), up[t][c], up[t][NR + c]);
                        store_c_nt(out + lay(i, (2 + h) * NR + c, NC), lo[t][c], lo[t][NR + c]);
                    }
                } else {
                    const float cf = (float)a.coef[s];
                    const cpx<float> *self = a.self[parity] + roff;
#pragma unroll
                    for (int half = 0; half < 2; ++half)
#pragma unroll
                        for (int c = 0; c < NR; ++c) {
                            const float accr = half ? lo[t][c] : up[t][c];
                            const float acci = half ? lo[t][NR + c] : up[t][NR + c];
                            const size_t o = lay(i, (half ? 2 + h : h) * NR + c, NC);
                            float sr, si;
                            load_c_nt(self + o, sr, si);
                            const float vr = sr - cf * accr, vi = si - cf * acci;
                            if (EPI == EPI_AXPY) {
                                store_c_nt(a.out[parity] + roff + o, vr, vi);
                                nrm += (double)vr * (double)vr + (double)vi * (double)vi;
                            } else {  // EPI_CG
                                cpx<float> *r = a.r[parity] + roff;
                                float rr_, ri;
                                load_c_nt(r + o, rr_, ri);
                                if (a.active[s]) {
                                    const float al = (float)a.alpha[s];
                                    rr_ -= al * vr;
                                    ri -= al * vi;
                                    store_c_nt(r + o, rr_, ri);
                                }
                                nrm += (double)rr_ * (double)rr_ + (double)ri * (double)ri;
                            }
                        }
                }
            }
            if (EPI != EPI_PLAIN && a.partial) {
                const double tot = mfma_source_sum(nrm);
                if (b == 0 && h == 0 && live)
                    a.partial[(size_t)s * a.pstride + (a.parity < 0 ? parity * a.ngroups : 0) + bx] = tot;
            }
        }
    }
}

// Whether the matrix-core kernel serves a launch: FP32 N_R = 6 with at least
// 6 sources, and only when asked for (environment HRW_MRHS_MFMA=1).  It is
// not the default: at SU(3) sym 32^4 with 24 sources it takes 232 us per
// source against 112 us for the vector multi-source kernel (operand
// preparation and reconstruction are ~6000 VALU instructions per wave against
// 576 MFMAs, at ~250 VGPRs; measured at two waves per SIMD with 36-44 bytes of
// spill per lane; it is compiled for one wave per SIMD now, with no scratch).
inline bool hop_uses_mfma(int nr, int dt, int n_rhs)
{
    if (dt != 1 || nr != 6 || n_rhs < 6) return false;
    const char *e = getenv("HRW_MRHS_MFMA");
    return e && e[0] == '1';
}

// Workgroup of one wavefront per 2 MF_NT sources, at most four.
inline int mfma_threads(int n_rhs)
{
    int w = (n_rhs + 2 * MF_NT - 1) / (2 * MF_NT);
    if (w > 4) w = 4;
    if (w < 1) w = 1;
    return 64 * w;
}

template <int NR>
hipError_t launch_hop_mfma(bool dagger, int epi, const HopArgs<float> &a, hipStream_t st)
{
    HopArgs<float> b = a;
    b.ngroups = hop_groups(a.g);
    const int gh = b.ngroups;  // one workgroup per 16-site group
    b.grid_half = gh;
    hop_tiling(a.g, MR_SITES, &b.tile_ts, &b.tile_c);
    const size_t lds = sizeof(cpx<float>) * 8 * NR * NR * MR_SITES;
    dim3 grid(a.parity < 0 ? 2 * gh : gh, 1), block(mfma_threads(a.n_rhs));
    if (epi == EPI_PLAIN) {
        if (dagger) hop_mfma_kernel<NR, true, EPI_PLAIN><<<grid, block, lds, st>>>(b);
        else hop_mfma_kernel<NR, false, EPI_PLAIN><<<grid, block, lds, st>>>(b);
    } else if (epi == EPI_AXPY) {
        if (dagger) hop_mfma_kernel<NR, true, EPI_AXPY><<<grid, block, lds, st>>>(b);
        else hop_mfma_kernel<NR, false, EPI_AXPY><<<grid, block, lds, st>>>(b);
    } else {
        if (!dagger) return hipErrorInvalidValue;
        hop_mfma_kernel<NR, true, EPI_CG><<<grid, block, lds, st>>>(b);
    }
    return hipGetLastError();
}

}  // namespace hrw
