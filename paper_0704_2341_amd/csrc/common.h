// Internal definitions shared by the kernels and the host engine.
//
// Internal field layout (private; the boundary is canonical): sites are
// grouped in tiles of 64 consecutive lexicographic sites (one wavefront), and
// inside a tile every component is a contiguous run of 64 values.
//   spinor field with nrhs right-hand sides, site s, RHS r, c = 3*spin + colour:
//     fidx = ((tile(s) * nrhs + r) * 12 + c) * 64 + lane(s)
//   gauge field, direction mu, entry e = 3*row + col:
//     lidx = ((tile(s) * 4 + mu) * 9 + e) * 64 + lane(s)
//   with the boundary sign bc[mu] folded into U_mu(x) on the last slice
//   x_mu = L_mu - 1.
// A wavefront's loads for one component are one coalesced 64-wide run, and all
// the data of a tile (every RHS) sits in one contiguous block, so the pages a
// wavefront touches are few (a component-major layout would put each of the
// 12 x 9 neighbour components and 72 link entries a field's length apart).
// One complex number per element: double2 (FP64), float2 (FP32) or a 32-bit
// word holding two bfloat16 (re in the low half, im in the high half).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grg.h"

namespace grg {

typedef uint32_t bf16x2;

// ------------------------------------------------------------------ geometry
struct Geom {
    int L[4];
    int V;   // number of sites
    int Vs;  // V rounded up to a whole number of 64-site tiles (a multiple of 256)
};

// Work decomposition of the site-parallel kernels: blocks of SB sites
// (a power of two), right-hand sides handled in groups of RG by one thread
// (looped), items ordered so that each of the 8 XCDs owns one contiguous
// eighth of the lattice.
struct Launch {
    int SB;       // sites per work item
    int RG;       // right-hand sides per work item (looped inside a thread)
    int grid;     // workgroups (multiple of 8)
};

__host__ __device__ __forceinline__ size_t fidx(int s, int r, int c, int nrhs)
{
    return ((((size_t)(s >> 6) * nrhs + r) * 12 + c) << 6) + (s & 63);
}
__host__ __device__ __forceinline__ size_t lidx(int s, int mu, int e)
{
    return ((((size_t)(s >> 6) * 4 + mu) * 9 + e) << 6) + (s & 63);
}

static inline size_t spinor_elems(const Geom &g, int nrhs) { return (size_t)nrhs * 12 * g.Vs; }
static inline size_t gauge_elems(const Geom &g) { return (size_t)4 * 9 * g.Vs; }
static inline size_t prec_bytes(int prec) { return prec == GRG_FP64 ? 16 : prec == GRG_FP32 ? 8 : 4; }

// ------------------------------------------------------------------ complex
template <class R>
struct cpx {
    R re, im;
};

template <class R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <class R>
__device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

// acc += m * h and acc += conj(m) * h as four fused multiply-adds
template <class R>
__device__ __forceinline__ void cmac(cpx<R> &acc, cpx<R> m, cpx<R> h)
{
    acc.re = fma(m.re, h.re, acc.re);
    acc.re = fma(-m.im, h.im, acc.re);
    acc.im = fma(m.re, h.im, acc.im);
    acc.im = fma(m.im, h.re, acc.im);
}
template <class R>
__device__ __forceinline__ void cmacc(cpx<R> &acc, cpx<R> m, cpx<R> h)
{
    acc.re = fma(m.re, h.re, acc.re);
    acc.re = fma(m.im, h.im, acc.re);
    acc.im = fma(m.re, h.im, acc.im);
    acc.im = fma(-m.im, h.re, acc.im);
}

// ------------------------------------------------------------------ storage
template <int P>
struct Store;
template <>
struct Store<GRG_FP64> {
    typedef double2 S;
    typedef double R;
};
template <>
struct Store<GRG_FP32> {
    typedef float2 S;
    typedef float R;
};
template <>
struct Store<GRG_BF16> {
    typedef bf16x2 S;
    typedef float R;
};

__device__ __forceinline__ cpx<double> ldc(const double2 *p, size_t i)
{
    double2 v = p[i];
    return {v.x, v.y};
}
__device__ __forceinline__ cpx<float> ldc(const float2 *p, size_t i)
{
    float2 v = p[i];
    return {v.x, v.y};
}
__device__ __forceinline__ cpx<float> ldc(const bf16x2 *p, size_t i)
{
    uint32_t u = p[i];
    return {__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u)};
}

// load converted to the compute type R
template <class R, class S>
__device__ __forceinline__ cpx<R> ldr(const S *p, size_t i)
{
    const auto v = ldc(p, i);
    return {(R)v.re, (R)v.im};
}

// float -> bfloat16 bits, round to nearest even; NaN stays NaN.
__device__ __forceinline__ uint32_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ void stc(double2 *p, size_t i, cpx<double> v) { p[i] = make_double2(v.re, v.im); }
__device__ __forceinline__ void stc(float2 *p, size_t i, cpx<float> v) { p[i] = make_float2(v.re, v.im); }
// Both halves at once with the gfx950 packed conversion (round to nearest
// even, the rounding of f2bf above).
typedef float f32x2_v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float re, float im)
{
    const f32x2_v v = {re, im};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_v));
}
__device__ __forceinline__ void stc(bf16x2 *p, size_t i, cpx<float> v) { p[i] = pack_bf16(v.re, v.im); }

// ------------------------------------------------------------------ work items
// Work item w in [0, nitems) of a grid-stride loop, XCD-aware: workgroup b
// runs on XCD b % 8 and walks the b-th eighth of the items.
struct ItemRange {
    int begin, end, step;
};
__device__ __forceinline__ ItemRange xcd_items(int nitems)
{
    const int xcd = blockIdx.x & 7;
    const int per_xcd_wg = gridDim.x >> 3;
    const int nper = (nitems + 7) >> 3;
    ItemRange r;
    r.begin = xcd * nper + (blockIdx.x >> 3);
    r.end = min((xcd + 1) * nper, nitems);
    r.step = per_xcd_wg;
    return r;
}

// Chunked XCD mapping: items are cut into chunks of C consecutive items and
// chunk k belongs to XCD k % 8.  Workgroups of one XCD share its L2 and walk
// its chunks in order, so neighbouring sites of a chunk meet in that L2,
// while the eight XCDs stay in the same region of the lattice, so that data
// evicted from one L2 is still in the shared last-level cache when a
// neighbouring chunk needs it.  C = ceil(nitems / 8) gives each XCD one
// contiguous eighth; C = 1 is plain round-robin.  Returns -1 past the end.
__device__ __forceinline__ int xcd_chunk_item(int j, int C, int nitems)
{
    const int ch = (int)(blockIdx.x & 7) + 8 * (j / C);
    const int item = ch * C + (j - (j / C) * C);
    return item < nitems ? item : -1;
}

// wave64 sum
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace grg
