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
template <int MU, bool FWD, class R>
__device__ __forceinline__ void hop_math(cpx<R> (&acc)[12], const cpx<R> (&p)[12],
                                         const cpx<R> (&u)[9])
{
    // h = psi_up -/+ B_mu psi_lo   (- for the forward hop, + for the backward)
    const R sg = FWD ? R(-1) : R(1);
    cpx<R> h0[3], h1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cpx<R> l0 = p[6 + a], l1 = p[9 + a];
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
        h0[a] = {p[a].re + sg * b0.re, p[a].im + sg * b0.im};
        h1[a] = {p[3 + a].re + sg * b1.re, p[3 + a].im + sg * b1.im};
    }
    // w = U h (forward) or U^+ h (backward), one colour vector per spin;
    // each complex multiply-add is four fused multiply-adds
    cpx<R> w0[3], w1[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        cpx<R> s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (FWD) {
                cmac(s0, u[3 * r + c], h0[c]);
                cmac(s1, u[3 * r + c], h1[c]);
            } else {
                cmacc(s0, u[3 * c + r], h0[c]);
                cmacc(s1, u[3 * c + r], h1[c]);
            }
        }
        w0[r] = s0;
        w1[r] = s1;
    }
    // upper spins: -1/2 w ; lower spins: -1/2 (-/+ B^+ w) = +/- 1/2 B^+ w
    const R hu = R(-0.5);
    const R hl = FWD ? R(0.5) : R(-0.5);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        acc[r].re = fma(hu, w0[r].re, acc[r].re);
        acc[r].im = fma(hu, w0[r].im, acc[r].im);
        acc[3 + r].re = fma(hu, w1[r].re, acc[3 + r].re);
        acc[3 + r].im = fma(hu, w1[r].im, acc[3 + r].im);
        cpx<R> d0, d1;  // B^+ w
        if (MU == 0) {        // (-i w1, -i w0)
            d0 = {w1[r].im, -w1[r].re};
            d1 = {w0[r].im, -w0[r].re};
        } else if (MU == 1) { // (w1, -w0)
            d0 = w1[r];
            d1 = {-w0[r].re, -w0[r].im};
        } else if (MU == 2) { // (-i w0, i w1)
            d0 = {w0[r].im, -w0[r].re};
            d1 = {-w1[r].im, w1[r].re};
        } else {              // (w0, w1)
            d0 = w0[r];
            d1 = w1[r];
        }
        acc[6 + r].re = fma(hl, d0.re, acc[6 + r].re);
        acc[6 + r].im = fma(hl, d0.im, acc[6 + r].im);
        acc[9 + r].re = fma(hl, d1.re, acc[9 + r].re);
        acc[9 + r].im = fma(hl, d1.im, acc[9 + r].im);
    }
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

// acc = (D in)(s) for RHS r of a field with nrhs RHS.  The hop loop is not
// unrolled: each iteration loads one direction's two neighbours and links
// (24 + 18 complex; SPLIT: one hop, 12 + 9 complex) and consumes them, which
// bounds the live registers and keeps several wavefronts per SIMD in flight.
template <class S, class R, bool SPLIT, class SU = S>
__device__ __forceinline__ void dslash_site(cpx<R> (&acc)[12], const S *__restrict__ in,
                                            const SU *__restrict__ U, int s, const SiteGeo &q,
                                            const Geom &g, int r, int nrhs, R diag)
{
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const cpx<R> v = ldr<R>(in, fidx(s, r, c, nrhs));
        acc[c] = {diag * v.re, diag * v.im};
    }
    if (SPLIT) {
#pragma unroll 1
        for (int h = 0; h < 8; ++h) {
            const int mu = h >> 1;
            int sp, sm;
            nbr(s, mu, q, g, sp, sm);
            const int n = (h & 1) ? sm : sp;
            cpx<R> p[12], u[9];
#pragma unroll
            for (int c = 0; c < 12; ++c) p[c] = ldr<R>(in, fidx(n, r, c, nrhs));
#pragma unroll
            for (int e = 0; e < 9; ++e) u[e] = ldr<R>(U, lidx((h & 1) ? sm : s, mu, e));
            switch (h) {
            case 0: hop_math<0, true>(acc, p, u); break;
            case 1: hop_math<0, false>(acc, p, u); break;
            case 2: hop_math<1, true>(acc, p, u); break;
            case 3: hop_math<1, false>(acc, p, u); break;
            case 4: hop_math<2, true>(acc, p, u); break;
            case 5: hop_math<2, false>(acc, p, u); break;
            case 6: hop_math<3, true>(acc, p, u); break;
            default: hop_math<3, false>(acc, p, u); break;
            }
        }
        return;
    }
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
        int sp, sm;
        nbr(s, mu, q, g, sp, sm);
        cpx<R> pf[12], pb[12], uf[9], ub[9];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            pf[c] = ldr<R>(in, fidx(sp, r, c, nrhs));
            pb[c] = ldr<R>(in, fidx(sm, r, c, nrhs));
        }
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            uf[e] = ldr<R>(U, lidx(s, mu, e));
            ub[e] = ldr<R>(U, lidx(sm, mu, e));
        }
        switch (mu) {
        case 0: hop_math<0, true>(acc, pf, uf); hop_math<0, false>(acc, pb, ub); break;
        case 1: hop_math<1, true>(acc, pf, uf); hop_math<1, false>(acc, pb, ub); break;
        case 2: hop_math<2, true>(acc, pf, uf); hop_math<2, false>(acc, pb, ub); break;
        default: hop_math<3, true>(acc, pf, uf); hop_math<3, false>(acc, pb, ub); break;
        }
    }
}

}  // namespace grg
