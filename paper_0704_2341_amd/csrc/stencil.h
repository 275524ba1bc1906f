// Device building blocks of the Wilson stencil, shared by the single-lattice
// and the many-lattice kernels.
//
//   D psi(x) = (4 + m0) psi(x)
//              - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x + mu)
//                           + (1 + g_mu) U_mu(x - mu)^+ psi(x - mu) ]
//
// DeGrand-Rossi basis: g_mu = [[0, B_mu], [B_mu^+, 0]] on (spins 0,1 | 2,3),
//   B_x = [[0, i], [i, 0]], B_y = [[0, -1], [1, 0]], B_z = [[i, 0], [0, -i]],
//   B_t = 1, so (1 -/+ g_mu) psi = (h, -/+ B_mu^+ h), h = psi_up -/+ B_mu psi_lo.
#pragma once

#include "common.h"

namespace grg {

// ------------------------------------------------------------------ stencil
// One hop's arithmetic on loaded data: p = psi at the neighbour, u = link.
// Projection: h = psi_up -/+ B_mu psi_lo   (- for the forward hop, + for the
// backward), from the neighbour's four spin components l0..l3 (colour a).
template <int MU, bool FWD, class R>
__device__ __forceinline__ void project1(cpx<R> &h0, cpx<R> &h1, cpx<R> u0, cpx<R> u1, cpx<R> l0, cpx<R> l1)
{
    const R sg = FWD ? R(-1) : R(1);
    cpx<R> b0, b1;
    if (MU == 0) {        // (i l1, i l0)
        b0 = {-l1.im, l1.re};
        b1 = {-l0.im, l0.re};
    } else if (MU == 1) { // (-l1, l0)
        b0 = {-l1.re, -l1.im};
        b1 = l0;
    } else if (MU == 2) { // (i l0, -i l1)
        b0 = {-l0.im, l0.re};
        b1 = {l1.im, -l1.re};
    } else {              // (l0, l1)
        b0 = l0;
        b1 = l1;
    }
    h0 = {u0.re + sg * b0.re, u0.im + sg * b0.im};
    h1 = {u1.re + sg * b1.re, u1.im + sg * b1.im};
}

// w = U h (forward) or U^+ h (backward), one colour vector per spin, each
// complex multiply-add four fused multiply-adds; then the upper spins take
// -1/2 w and the lower spins -1/2 (-/+ B^+ w) = +/- 1/2 B^+ w.
template <int MU, bool FWD, class R>
__device__ __forceinline__ void hop_mult(cpx<R> (&acc)[12], const cpx<R> (&h0)[3], const cpx<R> (&h1)[3],
                                         const cpx<R> (&u)[9])
{
    const R hu = R(-0.5);
    const R hl = FWD ? R(0.5) : R(-0.5);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        cpx<R> w0 = {0, 0}, w1 = {0, 0};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (FWD) {
                cmac(w0, u[3 * r + c], h0[c]);
                cmac(w1, u[3 * r + c], h1[c]);
            } else {
                cmacc(w0, u[3 * c + r], h0[c]);
                cmacc(w1, u[3 * c + r], h1[c]);
            }
        }
        acc[r].re = fma(hu, w0.re, acc[r].re);
        acc[r].im = fma(hu, w0.im, acc[r].im);
        acc[3 + r].re = fma(hu, w1.re, acc[3 + r].re);
        acc[3 + r].im = fma(hu, w1.im, acc[3 + r].im);
        cpx<R> d0, d1;  // B^+ w
        if (MU == 0) {        // (-i w1, -i w0)
            d0 = {w1.im, -w1.re};
            d1 = {w0.im, -w0.re};
        } else if (MU == 1) { // (w1, -w0)
            d0 = w1;
            d1 = {-w0.re, -w0.im};
        } else if (MU == 2) { // (-i w0, i w1)
            d0 = {w0.im, -w0.re};
            d1 = {-w1.im, w1.re};
        } else {              // (w0, w1)
            d0 = w0;
            d1 = w1;
        }
        acc[6 + r].re = fma(hl, d0.re, acc[6 + r].re);
        acc[6 + r].im = fma(hl, d0.im, acc[6 + r].im);
        acc[9 + r].re = fma(hl, d1.re, acc[9 + r].re);
        acc[9 + r].im = fma(hl, d1.im, acc[9 + r].im);
    }
}

template <int MU, bool FWD, class R>
__device__ __forceinline__ void hop_math(cpx<R> (&acc)[12], const cpx<R> (&p)[12],
                                         const cpx<R> (&u)[9])
{
    cpx<R> h0[3], h1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) project1<MU, FWD>(h0[a], h1[a], p[a], p[3 + a], p[6 + a], p[9 + a]);
    hop_mult<MU, FWD>(acc, h0, h1, u);
}

// ------------------------------------------------------------------ BF16 hop
// The same hop with BF16 operands kept packed: one 32-bit word per complex
// (re in the low half, im in the high half), multiplied with the gfx950
// two-way BF16 dot product (products exact in FP32, sums in FP32).  By
// linearity U h = U psi_up +/- U (B psi_lo), so the projected h is never
// rounded: each complex multiply-add of a link entry m with a packed x is two
// dot products,
//     U x:      re = (m.re, -m.im).x    im = (m.im, m.re).x
//     U^+ x:    re = (m.re,  m.im).x    im = (-m.im, m.re).x
// The sign flips are the dot product's negation of the low or high half of a
// source, not instructions of their own; the B_mu phases of psi_lo are half
// swaps and sign flips too, and a half swap of x is moved onto the link
// (a.swap(x) = swap(a).x), so a hop spends one half swap per link entry
// beyond its 72 dot products.
__device__ __forceinline__ float dot2bf(uint32_t a, uint32_t b, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_v, a),
                                           __builtin_bit_cast(bf16x2_v, b), c, false);
}
__device__ __forceinline__ uint32_t swap_halves(uint32_t w) { return (w << 16) | (w >> 16); }
constexpr uint32_t kNegHi = 0x80000000u, kNegLo = 0x00008000u, kNegBoth = 0x80008000u;

// c + (-1)^NL a.lo b.lo + (-1)^NH a.hi b.hi (Z: c = 0), the VOP3P dot
// product with its source negations.  Written as assembly, so the compiler's
// hazard tracking does not see it as a dot product: a chain of these reads
// only its own results as the accumulator (forwarded between dot products of
// one opcode), and dot_fence closes a chain before any other instruction
// reads its result.
template <int NL, int NH, bool Z = false>
__device__ __forceinline__ float dot2n(uint32_t a, uint32_t b, float c = 0.f)
{
    float d;
    if constexpr (Z) {
        if constexpr (NL && NH)
            asm("v_dot2_f32_bf16 %0, %1, %2, 0 neg_lo:[1,0,0] neg_hi:[1,0,0]" : "=v"(d) : "v"(a), "v"(b));
        else if constexpr (NL)
            asm("v_dot2_f32_bf16 %0, %1, %2, 0 neg_lo:[1,0,0]" : "=v"(d) : "v"(a), "v"(b));
        else if constexpr (NH)
            asm("v_dot2_f32_bf16 %0, %1, %2, 0 neg_hi:[1,0,0]" : "=v"(d) : "v"(a), "v"(b));
        else
            asm("v_dot2_f32_bf16 %0, %1, %2, 0" : "=v"(d) : "v"(a), "v"(b));
    } else {
        if constexpr (NL && NH)
            asm("v_dot2_f32_bf16 %0, %1, %2, %3 neg_lo:[1,0,0] neg_hi:[1,0,0]" : "=v"(d) : "v"(a), "v"(b), "v"(c));
        else if constexpr (NL)
            asm("v_dot2_f32_bf16 %0, %1, %2, %3 neg_lo:[1,0,0]" : "=v"(d) : "v"(a), "v"(b), "v"(c));
        else if constexpr (NH)
            asm("v_dot2_f32_bf16 %0, %1, %2, %3 neg_hi:[1,0,0]" : "=v"(d) : "v"(a), "v"(b), "v"(c));
        else
            asm("v_dot2_f32_bf16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    }
    return d;
}
// Three wait states between the last dot products of the chains a0 .. b1
// and the first other VALU instruction that reads them (the results pass
// through this statement, so every reader comes after it).
__device__ __forceinline__ void dot_fence(float &a0, float &b0, float &a1, float &b1)
{
    asm("s_nop 2" : "+v"(a0), "+v"(b0), "+v"(a1), "+v"(b1));
}

// FIRST: the first hop of a site writes the accumulators instead of adding
// to them (the same values as adding to zero, without clearing them first).
template <int MU, bool FWD, bool FIRST = false>
__device__ __forceinline__ void hop_bf16(cpx<float> (&acc)[12], const uint32_t (&p)[12],
                                         const uint32_t (&u)[9])
{
    // y_s = sg (B_mu psi_lo)_s, sg = -1 forward, +1 backward, i (re, im) =
    // (-im, re): the lower spin YS feeding y_s, swapped halves (SW), and the
    // signs of y_s's low / high halves (Fs*)
    constexpr int Y0 = (MU == 0 || MU == 1) ? 1 : 0, Y1 = 1 - Y0;
    constexpr bool SW = MU == 0 || MU == 2;
    constexpr int F0L = MU == 0 ? !FWD : MU == 1 ? !FWD : MU == 2 ? !FWD : FWD;
    constexpr int F0H = MU == 0 ? FWD : MU == 1 ? !FWD : MU == 2 ? FWD : FWD;
    constexpr int F1L = MU == 0 ? !FWD : MU == 1 ? FWD : MU == 2 ? FWD : FWD;
    constexpr int F1H = MU == 0 ? FWD : MU == 1 ? FWD : MU == 2 ? !FWD : FWD;
    // the link forms: re on m with signs PR*, im on swap(m) with signs PI*
    constexpr int PRL = 0, PRH = FWD, PIL = !FWD, PIH = 0;
    cpx<float> w0[3], w1[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        float a0, b0, a1, b1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint32_t m = FWD ? u[3 * r + c] : u[3 * c + r];
            const uint32_t ms = swap_halves(m);
            const uint32_t l0 = p[6 + 3 * Y0 + c], l1 = p[6 + 3 * Y1 + c];
            if (c == 0) {
                a0 = dot2n<PRL, PRH, true>(m, p[c]);
                b0 = dot2n<PIL, PIH, true>(ms, p[c]);
                a1 = dot2n<PRL, PRH, true>(m, p[3 + c]);
                b1 = dot2n<PIL, PIH, true>(ms, p[3 + c]);
            } else {
                a0 = dot2n<PRL, PRH>(m, p[c], a0);
                b0 = dot2n<PIL, PIH>(ms, p[c], b0);
                a1 = dot2n<PRL, PRH>(m, p[3 + c], a1);
                b1 = dot2n<PIL, PIH>(ms, p[3 + c], b1);
            }
            if constexpr (SW) {
                a0 = dot2n<PRH ^ F0H, PRL ^ F0L>(ms, l0, a0);
                b0 = dot2n<PIH ^ F0H, PIL ^ F0L>(m, l0, b0);
                a1 = dot2n<PRH ^ F1H, PRL ^ F1L>(ms, l1, a1);
                b1 = dot2n<PIH ^ F1H, PIL ^ F1L>(m, l1, b1);
            } else {
                a0 = dot2n<PRL ^ F0L, PRH ^ F0H>(m, l0, a0);
                b0 = dot2n<PIL ^ F0L, PIH ^ F0H>(ms, l0, b0);
                a1 = dot2n<PRL ^ F1L, PRH ^ F1H>(m, l1, a1);
                b1 = dot2n<PIL ^ F1L, PIH ^ F1H>(ms, l1, b1);
            }
        }
        dot_fence(a0, b0, a1, b1);
        w0[r] = {a0, b0};
        w1[r] = {a1, b1};
    }
    const float hl = FWD ? 0.5f : -0.5f;
    // a + b f with a = 0 on the first hop (exact: f is a power of two)
    auto mad = [](float f, float b, float a) { return FIRST ? f * b : fmaf(f, b, a); };
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        acc[r].re = mad(-0.5f, w0[r].re, acc[r].re);
        acc[r].im = mad(-0.5f, w0[r].im, acc[r].im);
        acc[3 + r].re = mad(-0.5f, w1[r].re, acc[3 + r].re);
        acc[3 + r].im = mad(-0.5f, w1[r].im, acc[3 + r].im);
        cpx<float> d0, d1;  // B^+ w
        if (MU == 0) {
            d0 = {w1[r].im, -w1[r].re};
            d1 = {w0[r].im, -w0[r].re};
        } else if (MU == 1) {
            d0 = w1[r];
            d1 = {-w0[r].re, -w0[r].im};
        } else if (MU == 2) {
            d0 = {w0[r].im, -w0[r].re};
            d1 = {-w1[r].im, w1[r].re};
        } else {
            d0 = w0[r];
            d1 = w1[r];
        }
        acc[6 + r].re = mad(hl, d0.re, acc[6 + r].re);
        acc[6 + r].im = mad(hl, d0.im, acc[6 + r].im);
        acc[9 + r].re = mad(hl, d1.re, acc[9 + r].re);
        acc[9 + r].im = mad(hl, d1.im, acc[9 + r].im);
    }
}

// Operands of a hop as the kernels hold them: converted complex numbers, or
// for BF16 spinors with BF16 links and FP32 sums the packed words.
template <class S, class R>
struct Operand {
    typedef cpx<R> T;
    static constexpr bool kPacked = false;
    __device__ static T load(const S *p, size_t i) { return ldr<R>(p, i); }
};
template <>
struct Operand<bf16x2, float> {
    typedef uint32_t T;
    static constexpr bool kPacked = true;
    __device__ static T load(const bf16x2 *p, size_t i) { return p[i]; }
};
// BF16 spinors in an FP64 stencil (the defect correction of a BF16 inner
// solution): held packed, widened when used
template <>
struct Operand<bf16x2, double> {
    typedef uint32_t T;
    static constexpr bool kPacked = true;
    __device__ static T load(const bf16x2 *p, size_t i) { return p[i]; }
};

template <int MU, bool FWD, class R>
__device__ __forceinline__ void hop(cpx<R> (&acc)[12], const cpx<R> (&p)[12], const cpx<R> (&u)[9])
{
    hop_math<MU, FWD>(acc, p, u);
}
template <int MU, bool FWD>
__device__ __forceinline__ void hop(cpx<float> (&acc)[12], const uint32_t (&p)[12], const uint32_t (&u)[9])
{
    hop_bf16<MU, FWD>(acc, p, u);
}
template <int MU, bool FWD>
__device__ __forceinline__ void hop(cpx<double> (&acc)[12], const uint32_t (&p)[12],
                                    const cpx<double> (&u)[9])
{
    // the projection straight from the packed words (sums of two BF16
    // values, exact in FP64), without widening all twelve components first
    auto wd = [](uint32_t w) -> cpx<double> {
        return {(double)__uint_as_float(w << 16), (double)__uint_as_float(w & 0xffff0000u)};
    };
    cpx<double> h0[3], h1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        project1<MU, FWD>(h0[a], h1[a], wd(p[a]), wd(p[3 + a]), wd(p[6 + a]), wd(p[9 + a]));
    hop_mult<MU, FWD>(acc, h0, h1, u);
}
template <class R>
__device__ __forceinline__ cpx<R> as_cpx(const cpx<R> &v) { return v; }
__device__ __forceinline__ cpx<float> as_cpx(uint32_t w)
{
    return {__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u)};
}

// Site coordinates and the four lattice strides.
struct SiteGeo {
    int c[4];
};

__device__ __forceinline__ SiteGeo site_geo(int s, const Geom &g)
{
    SiteGeo q;
    const int t1 = s / g.L[0];
    q.c[0] = s - t1 * g.L[0];
    const int t2 = t1 / g.L[1];
    q.c[1] = t1 - t2 * g.L[1];
    const int t3 = t2 / g.L[2];
    q.c[2] = t2 - t3 * g.L[2];
    q.c[3] = t3;
    return q;
}

// Neighbours of s along mu (mu is wave-uniform; selects, not array indexing,
// so that nothing lands in scratch).
__device__ __forceinline__ void nbr(int s, int mu, const SiteGeo &q, const Geom &g, int &sp, int &sm)
{
    const int L = mu == 0 ? g.L[0] : mu == 1 ? g.L[1] : mu == 2 ? g.L[2] : g.L[3];
    const int x = mu == 0 ? q.c[0] : mu == 1 ? q.c[1] : mu == 2 ? q.c[2] : q.c[3];
    const int st = mu == 0 ? 1 : mu == 1 ? g.L[0] : mu == 2 ? g.L[0] * g.L[1]
                                                             : g.L[0] * g.L[1] * g.L[2];
    sp = x == L - 1 ? s - (L - 1) * st : s + st;
    sm = x == 0 ? s + (L - 1) * st : s - st;
}

// Operands of hop h (0..7 = +x, -x, +y, -y, +z, -z, +t, -t) of site s.
template <class OP, class OU, class S, class SU>
__device__ __forceinline__ void load_hop(int h, typename OP::T (&p)[12], typename OU::T (&u)[9],
                                         const S *__restrict__ in, const SU *__restrict__ U, int s,
                                         const SiteGeo &q, const Geom &g, int r, int nrhs)
{
    const int mu = h >> 1;
    int sp, sm;
    nbr(s, mu, q, g, sp, sm);
    const int n = (h & 1) ? sm : sp;
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = OP::load(in, fidx(n, r, c, nrhs));
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = OU::load(U, lidx((h & 1) ? sm : s, mu, e));
}

// acc = (D in)(s) for RHS r of a field with nrhs RHS.  HOPS selects how the
// eight hops are scheduled:
//   0: loop over directions, each iteration loading one direction's two
//      neighbours and links (24 + 18 complex) and consuming them;
//   1: loop over single hops (12 + 9 complex per iteration);
//   2: (packed BF16 operands: 21 registers per hop) single hops, double
//      buffered: the operands of hop h + 1 are requested before hop h is
//      computed, so every wavefront keeps a hop's loads in flight while it
//      computes.
// Loops 0 and 1 are not unrolled, which bounds the live registers and keeps
// several wavefronts per SIMD in flight.  HOPS = 2 with unpacked operands
// runs as 1.
template <class S, class R, int HOPS, class SU = S>
__device__ __forceinline__ void dslash_site(cpx<R> (&acc)[12], const S *__restrict__ in,
                                            const SU *__restrict__ U, int s, const SiteGeo &q,
                                            const Geom &g, int r, int nrhs, R diag)
{
    typedef Operand<S, R> OP;
    typedef Operand<SU, R> OU;
    typedef typename OP::T PT;
    typedef typename OU::T UT;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const cpx<R> v = ldr<R>(in, fidx(s, r, c, nrhs));
        acc[c] = {diag * v.re, diag * v.im};
    }
    if constexpr (HOPS == 2 && OP::kPacked && OU::kPacked) {
        // double buffer: A holds the forward hop of direction mu, B the
        // backward one; each buffer is refilled right after it is consumed
        PT pa[12], pb[12];
        UT ua[9], ub[9];
        load_hop<OP, OU>(0, pa, ua, in, U, s, q, g, r, nrhs);
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            load_hop<OP, OU>(2 * mu + 1, pb, ub, in, U, s, q, g, r, nrhs);
            switch (mu) {
            case 0: hop<0, true>(acc, pa, ua); break;
            case 1: hop<1, true>(acc, pa, ua); break;
            case 2: hop<2, true>(acc, pa, ua); break;
            default: hop<3, true>(acc, pa, ua); break;
            }
            if (mu < 3) load_hop<OP, OU>(2 * mu + 2, pa, ua, in, U, s, q, g, r, nrhs);
            switch (mu) {
            case 0: hop<0, false>(acc, pb, ub); break;
            case 1: hop<1, false>(acc, pb, ub); break;
            case 2: hop<2, false>(acc, pb, ub); break;
            default: hop<3, false>(acc, pb, ub); break;
            }
        }
        return;
    }
    if (HOPS >= 1) {
#pragma unroll 1
        for (int h = 0; h < 8; ++h) {
            const int mu = h >> 1;
            int sp, sm;
            nbr(s, mu, q, g, sp, sm);
            const int n = (h & 1) ? sm : sp;
            PT p[12];
            UT u[9];
#pragma unroll
            for (int c = 0; c < 12; ++c) p[c] = OP::load(in, fidx(n, r, c, nrhs));
#pragma unroll
            for (int e = 0; e < 9; ++e) u[e] = OU::load(U, lidx((h & 1) ? sm : s, mu, e));
            switch (h) {
            case 0: hop<0, true>(acc, p, u); break;
            case 1: hop<0, false>(acc, p, u); break;
            case 2: hop<1, true>(acc, p, u); break;
            case 3: hop<1, false>(acc, p, u); break;
            case 4: hop<2, true>(acc, p, u); break;
            case 5: hop<2, false>(acc, p, u); break;
            case 6: hop<3, true>(acc, p, u); break;
            default: hop<3, false>(acc, p, u); break;
            }
        }
        return;
    }
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        int sp, sm;
        nbr(s, mu, q, g, sp, sm);
        PT pf[12], pb[12];
        UT uf[9], ub[9];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            pf[c] = OP::load(in, fidx(sp, r, c, nrhs));
            pb[c] = OP::load(in, fidx(sm, r, c, nrhs));
        }
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            uf[e] = OU::load(U, lidx(s, mu, e));
            ub[e] = OU::load(U, lidx(sm, mu, e));
        }
        switch (mu) {
        case 0: hop<0, true>(acc, pf, uf); hop<0, false>(acc, pb, ub); break;
        case 1: hop<1, true>(acc, pf, uf); hop<1, false>(acc, pb, ub); break;
        case 2: hop<2, true>(acc, pf, uf); hop<2, false>(acc, pb, ub); break;
        default: hop<3, true>(acc, pf, uf); hop<3, false>(acc, pb, ub); break;
        }
    }
}

}  // namespace grg
