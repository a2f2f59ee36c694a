// Internal definitions of libhrw: storage types, device layout, geometry.
//
// Device layout ("site-blocked SoA").  A half-parity field of n_half sites is
// cut into blocks of BLK = 64 consecutive sites (one wavefront).  Inside a
// block the complex components are stored component-major, so that lane l
// of a wavefront reads component k of site 64*b + l from
//     base + (b * K + k) * BLK + l           (K components per site)
// and every load instruction of a wavefront touches one contiguous run of
// 64 complex numbers.  Spinors have K = 4*N_R components (spin-major,
// colour-minor); the hopping block of the gauge field for one output parity
// has K = 8*N_R*N_R: directions 0..3 hold U_mu(x) and directions 4..7 hold
// U_mu(x - mu)^+ (already conjugate-transposed), each N_R x N_R row-major.
// Every link is therefore stored twice (once per parity's block) and one
// hop streams exactly the links it needs, once, fully coalesced.  Padding
// lanes (site index >= n_half) are kept at zero.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace hrw {

constexpr int BLK = 64;       // sites per layout block = wavefront width
constexpr int WG = 256;       // threads per workgroup for streaming kernels
constexpr int MAX_RHS = 64;   // right-hand sides per call

// ------------------------------------------------------------------ storage types

struct bf16_t {
    uint16_t bits;
};
typedef _Float16 f16_t;

template <class S>
struct alignas(2 * sizeof(S)) cpx {
    S re, im;
};

// arithmetic type for a storage type: FP64 stays FP64, everything else is FP32
template <class S> struct acc_of { typedef float type; };
template <> struct acc_of<double> { typedef double type; };

__host__ __device__ inline float bf16_to_f32(bf16_t v)
{
    union { uint32_t u; float f; } c;
    c.u = (uint32_t)v.bits << 16;
    return c.f;
}

// float -> bfloat16, round to nearest even (NaN stays NaN)
__host__ __device__ inline bf16_t f32_to_bf16(float f)
{
    union { uint32_t u; float f; } c;
    c.f = f;
    bf16_t r;
    if ((c.u & 0x7f800000u) == 0x7f800000u && (c.u & 0x007fffffu)) {
        r.bits = (uint16_t)((c.u >> 16) | 0x40u);
        return r;
    }
    const uint32_t lsb = (c.u >> 16) & 1u;
    c.u += 0x7fffu + lsb;
    r.bits = (uint16_t)(c.u >> 16);
    return r;
}

// double -> float rounded to odd: truncate, then set the last bit when the
// truncation was inexact.  Rounding that result to a format with at least two
// fewer significand bits gives the correctly rounded (ties-to-even) value of
// the original double (Boldo & Melquiond, IEEE TC 57 (2008)).
__device__ inline float f64_to_f32_odd(double x)
{
    float t = __double2float_rz(x);
    if ((double)t != x && x == x) {
        union { uint32_t u; float f; } c;
        c.f = t;
        c.u |= 1u;
        t = c.f;
    }
    return t;
}

// conversions between storage and arithmetic types
template <class S> struct conv;
template <> struct conv<double> {
    __device__ static double to_acc(double v) { return v; }
    __device__ static double from_acc(double v) { return v; }
    __device__ static double from_f64(double v) { return v; }
};
template <> struct conv<float> {
    __device__ static float to_acc(float v) { return v; }
    __device__ static float from_acc(float v) { return v; }
    __device__ static float from_f64(double v) { return (float)v; }
};
template <> struct conv<bf16_t> {
    __device__ static float to_acc(bf16_t v) { return bf16_to_f32(v); }
    __device__ static bf16_t from_acc(float v) { return f32_to_bf16(v); }
    __device__ static bf16_t from_f64(double v) { return f32_to_bf16(f64_to_f32_odd(v)); }
};
template <> struct conv<f16_t> {
    __device__ static float to_acc(f16_t v) { return (float)v; }
    __device__ static f16_t from_acc(float v) { return (f16_t)v; }
    __device__ static f16_t from_f64(double v) { return (f16_t)f64_to_f32_odd(v); }
};

template <class S>
__device__ inline void load_c(const cpx<S> *p, typename acc_of<S>::type &re,
                              typename acc_of<S>::type &im)
{
    cpx<S> v = *p;
    re = conv<S>::to_acc(v.re);
    im = conv<S>::to_acc(v.im);
}

// Streaming (non-temporal) loads for data read exactly once per kernel, such as
// the links of a hop: they bypass the cache-retention policy so that they do
// not evict reusable lines (neighbour spinors) from L2.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));

template <class S>
__device__ inline void load_c_nt(const cpx<S> *p, typename acc_of<S>::type &re,
                                 typename acc_of<S>::type &im);
template <>
__device__ inline void load_c_nt<double>(const cpx<double> *p, double &re, double &im)
{
    const nt_d2 v = __builtin_nontemporal_load((const nt_d2 *)p);
    re = v.x;
    im = v.y;
}
template <>
__device__ inline void load_c_nt<float>(const cpx<float> *p, float &re, float &im)
{
    const nt_f2 v = __builtin_nontemporal_load((const nt_f2 *)p);
    re = v.x;
    im = v.y;
}
template <>
__device__ inline void load_c_nt<bf16_t>(const cpx<bf16_t> *p, float &re, float &im)
{
    const uint32_t w = __builtin_nontemporal_load((const uint32_t *)p);
    bf16_t a, b;
    a.bits = (uint16_t)(w & 0xffffu);
    b.bits = (uint16_t)(w >> 16);
    re = bf16_to_f32(a);
    im = bf16_to_f32(b);
}
template <>
__device__ inline void load_c_nt<f16_t>(const cpx<f16_t> *p, float &re, float &im)
{
    const uint32_t w = __builtin_nontemporal_load((const uint32_t *)p);
    union { uint16_t u; f16_t h; } a, b;
    a.u = (uint16_t)(w & 0xffffu);
    b.u = (uint16_t)(w >> 16);
    re = (float)a.h;
    im = (float)b.h;
}

template <class S>
__device__ inline void store_c(cpx<S> *p, typename acc_of<S>::type re, typename acc_of<S>::type im)
{
    cpx<S> v;
    v.re = conv<S>::from_acc(re);
    v.im = conv<S>::from_acc(im);
    *p = v;
}

// streaming store (written once, not re-read by this kernel)
template <class S>
__device__ inline void store_c_nt(cpx<S> *p, typename acc_of<S>::type re, typename acc_of<S>::type im);
template <>
__device__ inline void store_c_nt<double>(cpx<double> *p, double re, double im)
{
    nt_d2 v = {re, im};
    __builtin_nontemporal_store(v, (nt_d2 *)p);
}
template <>
__device__ inline void store_c_nt<float>(cpx<float> *p, float re, float im)
{
    nt_f2 v = {re, im};
    __builtin_nontemporal_store(v, (nt_f2 *)p);
}
template <>
__device__ inline void store_c_nt<bf16_t>(cpx<bf16_t> *p, float re, float im)
{
    const uint32_t w = (uint32_t)f32_to_bf16(re).bits | ((uint32_t)f32_to_bf16(im).bits << 16);
    __builtin_nontemporal_store(w, (uint32_t *)p);
}
template <>
__device__ inline void store_c_nt<f16_t>(cpx<f16_t> *p, float re, float im)
{
    union { uint16_t u; f16_t h; } a, b;
    a.h = (f16_t)re;
    b.h = (f16_t)im;
    const uint32_t w = (uint32_t)a.u | ((uint32_t)b.u << 16);
    __builtin_nontemporal_store(w, (uint32_t *)p);
}

// fused multiply-add in the accumulation type (one rounding per step)
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ------------------------------------------------------------------ reductions

// Sum of p[k] for k = first, first + step, ... below n, added in increasing k.
// Loads are issued eight at a time before the additions, so a thread keeps
// eight requests in flight; the order of the additions (and so the result) is
// that of the plain one-at-a-time loop.
__device__ inline double strided_sum(const double *p, int first, int n, int step)
{
    double s = 0;
    int k = first;
    for (; k + 7 * step < n; k += 8 * step) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p[k + j * step];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; k < n; k += step) s += p[k];
    return s;
}

// ------------------------------------------------------------------ geometry

struct Geom {
    int d[4];      // extents, d[0] = time
    int half;      // sites per parity = V/2
    int nblk;      // layout blocks per half field = ceil(half / BLK)
    int n3h;       // d[3] / 2
    int pad_;
};

inline Geom make_geom(const int dims[4])
{
    Geom g;
    for (int m = 0; m < 4; ++m) g.d[m] = dims[m];
    const long long v = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    g.half = (int)(v / 2);
    g.nblk = (g.half + BLK - 1) / BLK;
    g.n3h = dims[3] / 2;
    g.pad_ = 0;
    return g;
}

// complex elements of one packed half-parity spinor field with nr colours
inline size_t spinor_elems(const Geom &g, int nr) { return (size_t)g.nblk * BLK * 4 * nr; }
// complex elements of one packed hopping block of the gauge field
inline size_t gauge_block_elems(const Geom &g, int nr) { return (size_t)g.nblk * BLK * 8 * nr * nr; }

__device__ inline size_t lay(int site, int comp, int ncomp)
{
    return ((size_t)(site / BLK) * ncomp + comp) * BLK + (site % BLK);
}

// coordinates of the i-th site of parity p (requires every extent even)
__device__ inline void eo_coords(const Geom &g, int p, int i, int x[4])
{
    const int row = i / g.n3h;
    const int j = i - row * g.n3h;
    const int t = row / g.d[2];
    x[2] = row - t * g.d[2];
    x[0] = t / g.d[1];
    x[1] = t - x[0] * g.d[1];
    x[3] = 2 * j + ((x[0] + x[1] + x[2] + p) & 1);
}

__device__ inline int eo_index(const Geom &g, const int x[4])
{
    const long long lex = (((long long)x[0] * g.d[1] + x[1]) * g.d[2] + x[2]) * g.d[3] + x[3];
    return (int)(lex >> 1);
}

// ------------------------------------------------------------------ timing classes

// 0 = every hopping launch; 3/4/5 = hopping launches with the plain / axpy /
// fused-CG epilogue (each is one kernel instance per N_R and dtype)
enum KernelClass { KC_HOP = 0, KC_BLAS = 1, KC_REDUCE = 2, KC_HOP_PLAIN = 3, KC_HOP_AXPY = 4,
                   KC_HOP_CG = 5, KC_COUNT = 6 };

}  // namespace hrw
