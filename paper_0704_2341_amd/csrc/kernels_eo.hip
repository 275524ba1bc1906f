// Even-odd (red-black) reduction of the D_rr solve.
//
// The hopping term of the Wilson operator only couples sites of opposite
// parity (x + y + z + t mod 2), so on the rest sites R = R_e + R_o
//     D_rr = [[d, H_eo], [H_oe, d]],   d = 4 + m0,
// and D_rr z = b is solved through the Schur complement on one parity p
// (the reduction this library applies to D_rr is the same block elimination
// the coarse operator itself is built from):
//     b^_p = b_p - H_pq b_q / d,   (d - H_pq H_qp / d) z_p = b^_p,
//     z_q = (b_q - H_qp z_p) / d,               q = 1 - p.
// The residual of the reduced system is the residual of the full one on R_p
// and zero on R_q, so the inner tolerance carries over unchanged.
//
// Fields of one parity are compact: half-site index h = s / 2 (the x extent
// is even, so sites 2h and 2h + 1 have opposite parities), tiled like the
// full fields (fidx(h, ...)), so that a stencil over one parity reads and
// writes only lines of that parity.  The links are kept in the same compact
// form per parity (lidx(h, ...) in block p of a [2][...] array) and the
// coarse/rest mask per parity ([2][Vhs], padding marked coarse).
#include <algorithm>

#include "common.h"
#include "engine.h"
#include "stencil.h"

namespace grg {

// site of half index h with parity p, and its coordinates
__device__ __forceinline__ int eo_site(int h, int p, const Geom &g, SiteGeo &q)
{
    const int s0 = 2 * h;
    q = site_geo(s0, g);
    const int b = (p ^ q.c[1] ^ q.c[2] ^ q.c[3]) & 1;  // parity of s0 is y + z + t (x0 even)
    q.c[0] += b;
    return s0 + b;
}

__device__ __forceinline__ int site_parity(int s, const Geom &g)
{
    const SiteGeo q = site_geo(s, g);
    return (q.c[0] ^ q.c[1] ^ q.c[2] ^ q.c[3]) & 1;
}

// Operands of hop k (0..7 = +x, -x, ..., -t) of the site s = (h, parity po):
// the neighbour's compact input and the link, U_mu(s) from the output
// parity's links for a forward hop, U_mu(s - mu) from the input parity's
// links for a backward one.
template <class OP, class S>
__device__ __forceinline__ void eo_load_hop(int k, typename OP::T (&p)[12], typename OP::T (&u)[9],
                                            const S *__restrict__ in, const S *__restrict__ Uo,
                                            const S *__restrict__ Ui, int s, int h,
                                            const SiteGeo &q, const Geom &g, int r, int nrhs,
                                            bool in_full)
{
    const int mu = k >> 1;
    int sp, sm;
    nbr(s, mu, q, g, sp, sm);
    const int n = (k & 1) ? sm : sp;
    const int hn = n >> 1;
    const int ni = in_full ? n : hn;
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = OP::load(in, fidx(ni, r, c, nrhs));
    if (k & 1) {
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = OP::load(Ui, lidx(hn, mu, e));
    } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = OP::load(Uo, lidx(h, mu, e));
    }
}

template <class R, class PT>
__device__ __forceinline__ void eo_hop_k(int k, cpx<R> (&acc)[12], const PT (&p)[12], const PT (&u)[9])
{
    switch (k) {
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

// t-marching form of the compact half-stencil (packed BF16).  A workgroup
// takes 64 columns (x/2, y, z) of the half lattice and four RHS (one per
// wavefront) and walks `march` time slices.  The t-neighbours of an output
// site are the sites of the other parity in the same column one slice up
// and one down, so every input site of the column is loaded once: as the
// forward neighbour of one output and, two slices later, the backward
// neighbour of the next.  The two slices in between wait in LDS (a ring of
// two slots per wavefront, written by each lane for its own column, so no
// barrier is needed), which keeps the register count of the one-hop loop;
// the x hops read the slot of the current slice at the lanes of the same
// x-row instead of loading.
// Each XCD walks the columns of its own z-slab (an eighth of a slice), so
// that the x, y and z neighbours, loaded by the columns next to it at nearly
// the same time, are in its own L2.  Per-RHS sums go to red[r] (one
// wavefront per RHS of a workgroup, so no two wavefronts share a row).
template <int P, class OP, int IO>
__device__ __forceinline__ void eo_march(const EoArgs &a, double (*red)[3])
{
    // IO as for eo_hop_kernel: 0 compact fields, 1 in and in2 in the full
    // layout, 2 in2 and out in the full layout (with the partner copy), 3
    // out alone in the full layout
    constexpr bool in_full = IO == 1, in2_full = IO == 1 || IO == 2, out_full = IO >= 2;
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    typedef typename OP::T PT;
    static_assert(sizeof(PT) == 4, "the LDS ring holds packed BF16 complex words");
    __shared__ PT ring[4][2][12][64];
    const S *__restrict__ in = (const S *)a.in;
    const S *__restrict__ in2 = (const S *)a.in2;
    S *__restrict__ out = (S *)a.out;
    const S *__restrict__ Uo = (const S *)a.U + (size_t)a.po * 36 * a.Vhs;
    const S *__restrict__ Ui = (const S *)a.U + (size_t)(1 - a.po) * 36 * a.Vhs;
    const uint8_t *__restrict__ mk = a.mask + (size_t)a.po * a.Vhs;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool dots = a.partials != nullptr;
    const R al = (R)a.alpha, be = (R)a.beta;
    const int Lt = a.g.L[3];
    const int Vs3 = a.Vh / Lt;  // half-sites per time slice (a multiple of 64)
    const int nT = Vs3 >> 6;
    const int xcd = (int)(blockIdx.x & 7), slot = (int)(blockIdx.x >> 3), slots = (int)(gridDim.x >> 3);
    const int T0 = (xcd * nT) >> 3, ntx = (((xcd + 1) * nT) >> 3) - T0;
    const int nq = (a.nrhs + 3) >> 2;
    const int ML = a.march, nc = (Lt + ML - 1) / ML;
    const int nx = ntx * nq * nc;
    const int nr = a.nrhs;
    PT (*q)[12][64] = ring[wave];
    // element index of the input site with compact index hq (other parity)
    auto iidx = [&](int hq) -> int {
        if constexpr (in_full) {
            SiteGeo tq;
            return eo_site(hq, 1 - a.po, a.g, tq);
        } else {
            return hq;
        }
    };
    for (int j = slot; j < nx; j += slots) {
        const int quad = j % nq, rest = j / nq;
        const int T = T0 + rest % ntx, ch = rest / ntx;
        const int r = 4 * quad + wave;
        if (r >= nr) continue;
        const int col = T * 64 + lane;
        const int t0 = ch * ML, t1 = min(t0 + ML, Lt);
        // the column's input one slice below t0 and at t0: slot (t & 1)
        // holds slice t
        {
            const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                q[(t0 - 1) & 1][c][lane] = OP::load(in, fidx(iidx(tm * Vs3 + col), r, c, nr));
                q[t0 & 1][c][lane] = OP::load(in, fidx(iidx(t0 * Vs3 + col), r, c, nr));
            }
        }
        double dre = 0, dim = 0, dqq = 0;
#pragma unroll 1
        for (int t = t0; t < t1; ++t) {
            const int h = t * Vs3 + col;
            const int hf = (t + 1 == Lt ? 0 : (t + 1) * Vs3) + col;
            const int hbk = (t == 0 ? Lt - 1 : t - 1) * Vs3 + col;
            const bool on = mk[h] == 0;
            // the forward t-neighbour: used at the end of this slice, then
            // kept for the output two slices up
            PT qc[12];
            {
                const int fi = iidx(hf);
#pragma unroll
                for (int c = 0; c < 12; ++c) qc[c] = OP::load(in, fidx(fi, r, c, nr));
            }
            SiteGeo sq;
            const int s = eo_site(h, a.po, a.g, sq);
            cpx<R> acc[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
            if (on) {
                // x hops from the ring: the other parity's sites of slice t in
                // this wavefront's columns are in slot t & 1, and an x
                // neighbour is the site of this column or of the next or
                // previous column of the same x-row (which one: the parity of
                // x; x-rows of Lx / 2 columns tile the 64 lanes)
                {
                    const int Lh = a.g.L[0] >> 1;
                    const int xh = col % Lh, rs = lane - xh;
                    const bool b = (s & 1) != 0;
                    const int lp = b ? rs + (xh + 1 == Lh ? 0 : xh + 1) : lane;
                    const int lm = b ? lane : rs + (xh == 0 ? Lh - 1 : xh - 1);
                    PT p[12], u[9];
#pragma unroll
                    for (int e = 0; e < 9; ++e) u[e] = OP::load(Uo, lidx(h, 0, e));
#pragma unroll
                    for (int c = 0; c < 12; ++c) p[c] = q[t & 1][c][lp];
                    eo_hop_k(0, acc, p, u);
                    // U_x(s - x) at the x- neighbour's compact index
#pragma unroll
                    for (int e = 0; e < 9; ++e) u[e] = OP::load(Ui, lidx(h - lane + lm, 0, e));
#pragma unroll
                    for (int c = 0; c < 12; ++c) p[c] = q[t & 1][c][lm];
                    eo_hop_k(1, acc, p, u);
                }
#pragma unroll 1
                for (int k = 2; k < 6; ++k) {
                    PT p[12], u[9];
                    eo_load_hop<OP>(k, p, u, in, Uo, Ui, s, h, sq, a.g, r, nr, in_full);
                    eo_hop_k(k, acc, p, u);
                }
                {
                    PT u[9];
#pragma unroll
                    for (int e = 0; e < 9; ++e) u[e] = OP::load(Uo, lidx(h, 3, e));
                    eo_hop_k(6, acc, qc, u);
                }
                {
                    PT p[12], u[9];
#pragma unroll
                    for (int e = 0; e < 9; ++e) u[e] = OP::load(Ui, lidx(hbk, 3, e));
#pragma unroll
                    for (int c = 0; c < 12; ++c) p[c] = q[(t - 1) & 1][c][lane];
                    eo_hop_k(7, acc, p, u);
                }
            }
            // slice t + 1 replaces slice t - 1 (read above, by this lane only)
#pragma unroll
            for (int c = 0; c < 12; ++c) q[(t + 1) & 1][c][lane] = qc[c];
            R sre = 0, sim = 0, sqq = 0;
            const bool act = a.active == nullptr || a.active[r] != 0;
            // the sums against in2 itself reuse its loaded value
            const bool dot_in2 = !in2_full && a.dot_with == a.in2;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(h, r, c, nr);
                cpx<R> o = {0, 0}, v2 = {0, 0};
                if (in2 && on) v2 = ldr<R>(in2, in2_full ? fidx(s, r, c, nr) : i);
                if (on && act) {
                    o = {be * acc[c].re, be * acc[c].im};
                    if (in2) {
                        o.re = fma(al, v2.re, o.re);
                        o.im = fma(al, v2.im, o.im);
                    }
                }
                if constexpr (out_full) {
                    // this site, and the other parity's site of the same index
                    stc(out, fidx(s, r, c, nr), o);
                    out[fidx(s ^ 1, r, c, nr)] = ((const S *)a.partner)[i];
                } else {
                    stc(out, i, o);
                }
                if (dots && on) {
                    const cpx<R> v = dot_in2 ? v2 : a.dot_with ? ldr<R>((const S *)a.dot_with, i) : cpx<R>{0, 0};
                    sre = fma(o.re, v.re, fma(o.im, v.im, sre));
                    sim = fma(o.re, v.im, fma(-o.im, v.re, sim));
                    sqq = fma(o.re, o.re, fma(o.im, o.im, sqq));
                }
            }
            dre += (double)sre;
            dim += (double)sim;
            dqq += (double)sqq;
        }
        if (dots) {
            dre = wave_sum(dre);
            dim = wave_sum(dim);
            dqq = wave_sum(dqq);
            if (lane == 0) {
                red[r][0] += dre;
                red[r][1] += dim;
                red[r][2] += dqq;
            }
        }
    }
}

// RHS-simultaneous form of the compact half-stencil: the RS right-hand sides
// of a work item are carried through each hop together, so that the hop's
// link is loaded once for all of them and a wavefront has RS spinor loads
// plus one link load in flight per hop instead of one of each.
template <int P, class OP, int RS>
__device__ __forceinline__ void eo_multi(const EoArgs &a, double (*red)[kMaxRhs][3])
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    typedef typename OP::T PT;
    const S *__restrict__ in = (const S *)a.in;
    const S *__restrict__ in2 = (const S *)a.in2;
    S *__restrict__ out = (S *)a.out;
    const S *__restrict__ Uo = (const S *)a.U + (size_t)a.po * 36 * a.Vhs;
    const S *__restrict__ Ui = (const S *)a.U + (size_t)(1 - a.po) * 36 * a.Vhs;
    const uint8_t *__restrict__ mk = a.mask + (size_t)a.po * a.Vhs;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool dots = a.partials != nullptr;
    const R al = (R)a.alpha, be = (R)a.beta;
    const int nr = a.nrhs;
    const int ngroups = (nr + RS - 1) / RS;
    const int nsb = (a.Vh + a.SB - 1) / a.SB;
    const int nitems = nsb * ngroups;
    const int C = a.chunk > 0 ? a.chunk : (nitems + 7) / 8;
    for (int j = blockIdx.x >> 3;; j += gridDim.x >> 3) {
        const int w = xcd_chunk_item(j, C, nitems);
        if (w < 0) break;
        const int sb = w / ngroups, grp = w - sb * ngroups;
        const int h = sb * a.SB + (int)threadIdx.x;
        const bool valid = h < a.Vh;
        const bool on = valid && mk[h] == 0;
        SiteGeo q;
        int s = 0;
        if (on) s = eo_site(h, a.po, a.g, q);
        const int r0 = grp * RS;
        cpx<R> acc[RS][12];
#pragma unroll
        for (int k = 0; k < RS; ++k)
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[k][c] = {0, 0};
        if (on) {
#pragma unroll 1
            for (int k = 0; k < 8; ++k) {
                const int mu = k >> 1;
                int sp, sm;
                nbr(s, mu, q, a.g, sp, sm);
                const int hn = ((k & 1) ? sm : sp) >> 1;
                const S *__restrict__ Ul = (k & 1) ? Ui : Uo;
                const int hl = (k & 1) ? hn : h;
                PT u[9], p[RS][12];
#pragma unroll
                for (int e = 0; e < 9; ++e) u[e] = OP::load(Ul, lidx(hl, mu, e));
#pragma unroll
                for (int jr = 0; jr < RS; ++jr) {
                    const int r = min(r0 + jr, nr - 1);  // a ragged last group repeats the last RHS
#pragma unroll
                    for (int c = 0; c < 12; ++c) p[jr][c] = OP::load(in, fidx(hn, r, c, nr));
                }
#pragma unroll
                for (int jr = 0; jr < RS; ++jr) eo_hop_k(k, acc[jr], p[jr], u);
            }
        }
#pragma unroll
        for (int jr = 0; jr < RS; ++jr) {
            const int r = r0 + jr;
            if (r >= nr) break;
            R sre = 0, sim = 0, sqq = 0;
            const bool act = a.active == nullptr || a.active[r] != 0;
            if (valid) {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const size_t i = fidx(h, r, c, nr);
                    cpx<R> o = {0, 0};
                    if (on && act) {
                        o = {be * acc[jr][c].re, be * acc[jr][c].im};
                        if (in2) {
                            const cpx<R> v = ldr<R>(in2, i);
                            o.re = fma(al, v.re, o.re);
                            o.im = fma(al, v.im, o.im);
                        }
                    }
                    stc(out, i, o);
                    if (dots && on) {
                        const cpx<R> v = a.dot_with ? ldr<R>((const S *)a.dot_with, i) : cpx<R>{0, 0};
                        sre = fma(o.re, v.re, fma(o.im, v.im, sre));
                        sim = fma(o.re, v.im, fma(-o.im, v.re, sim));
                        sqq = fma(o.re, o.re, fma(o.im, o.im, sqq));
                    }
                }
            }
            if (dots) {
                const double dre = wave_sum((double)sre);
                const double dim = wave_sum((double)sim);
                const double dqq = wave_sum((double)sqq);
                if (lane == 0) {
                    red[wave][r][0] += dre;
                    red[wave][r][1] += dim;
                    red[wave][r][2] += dqq;
                }
            }
        }
    }
}

// out = alpha in2 + beta (H in) on the rest sites of parity po (zero on its
// coarse sites); in has parity 1 - po, in2 and out parity po.  With partials,
// also the per-workgroup sums conj(out).w (re, im) and |out|^2 per RHS,
// w = dot_with (parity po).  HOPS = 2 double-buffers the hop operands (packed
// BF16), otherwise one hop per loop iteration.
template <int P, int HOPS, int IO>
__global__ void __launch_bounds__(256) eo_hop_kernel(EoArgs a)
{
    // IO = 0: compact fields; 1: in and in2 in the full layout; 2: in2 and
    // out in the full layout; 3: out alone in the full layout (the
    // full-layout modes run once per reduced solve, the compact one every
    // iteration: separate instances keep the latter free of their indexing)
    constexpr bool in_full = IO == 1, in2_full = IO == 1 || IO == 2, out_full = IO >= 2;
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    typedef Operand<S, R> OP;
    typedef typename OP::T PT;
    __shared__ double red[4][kMaxRhs][3];
    const S *__restrict__ in = (const S *)a.in;
    const S *__restrict__ in2 = (const S *)a.in2;
    S *__restrict__ out = (S *)a.out;
    const S *__restrict__ Uo = (const S *)a.U + (size_t)a.po * 36 * a.Vhs;
    const S *__restrict__ Ui = (const S *)a.U + (size_t)(1 - a.po) * 36 * a.Vhs;
    const uint8_t *__restrict__ mk = a.mask + (size_t)a.po * a.Vhs;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool dots = a.partials != nullptr;
    if (dots) {
        for (int i = lane; i < a.nrhs * 3; i += 64) red[wave][i / 3][i % 3] = 0.0;
        __syncthreads();
    }
    if constexpr (HOPS == 3) {
        static_assert(OP::kPacked, "t-marching form: packed fields only");
        eo_march<P, OP, IO>(a, red[0]);
    } else if constexpr (HOPS == 4 || HOPS == 5) {
        static_assert(IO == 0, "RHS-simultaneous form: compact fields only");
        eo_multi<P, OP, HOPS - 2>(a, red);
    } else {
    const R al = (R)a.alpha, be = (R)a.beta;
    const bool inf = in_full;
    const int ngroups = (a.nrhs + a.RG - 1) / a.RG;
    const int nsb = (a.Vh + a.SB - 1) / a.SB;
    const int nitems = nsb * ngroups;
    const int C = a.chunk > 0 ? a.chunk : (nitems + 7) / 8;
    for (int j = blockIdx.x >> 3;; j += gridDim.x >> 3) {
        const int w = xcd_chunk_item(j, C, nitems);
        if (w < 0) break;
        const int sb = w / ngroups, grp = w - sb * ngroups;
        const int h = sb * a.SB + (int)threadIdx.x;
        const bool valid = h < a.Vh;
        const bool on = valid && mk[h] == 0;
        SiteGeo q;
        int s = 0;
        if (on || (valid && (out_full || HOPS == 6))) s = eo_site(h, a.po, a.g, q);
        const int r0 = grp * a.RG, r1 = min(r0 + a.RG, a.nrhs);
#pragma unroll 1
        for (int r = r0; r < r1; ++r) {
            cpx<R> acc[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
            // HOPS = 6: the x hops' spinors from lane shuffles.  The other
            // parity's site with this site's compact index is its x neighbour
            // on one side (which side: the parity of x); the x neighbour on the
            // other side is the next or previous half-site of the same x-row,
            // held by another lane of this wavefront (x-rows of Lx / 2
            // half-sites tile the 64 lanes).  Done with every lane active
            // (the result of a lane whose site is not computed is dropped).
            if constexpr (HOPS == 6) {
                const int Lh = a.g.L[0] >> 1;
                const int xh = h % Lh, rs = lane - xh;
                const int lp = rs + (xh + 1 == Lh ? 0 : xh + 1);
                const int lm = rs + (xh == 0 ? Lh - 1 : xh - 1);
                const bool b = (s & 1) != 0;
                const int hv = valid ? h : 0;
                PT self[12];
#pragma unroll
                for (int c = 0; c < 12; ++c) self[c] = OP::load(in, fidx(hv, r, c, a.nrhs));
                {
                    PT xs[12], u[9];
#pragma unroll
                    for (int e = 0; e < 9; ++e) u[e] = OP::load(Uo, lidx(hv, 0, e));
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const PT v = (PT)__shfl((int)self[c], lp, 64);
                        xs[c] = b ? v : self[c];
                    }
                    eo_hop_k(0, acc, xs, u);
                }
                {
                    // U_x(s - x) sits at the x- neighbour's compact index
                    const int hm = b ? hv : hv - xh + (xh == 0 ? Lh - 1 : xh - 1);
                    PT xs[12], u[9];
#pragma unroll
                    for (int e = 0; e < 9; ++e) u[e] = OP::load(Ui, lidx(hm, 0, e));
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const PT v = (PT)__shfl((int)self[c], lm, 64);
                        xs[c] = b ? self[c] : v;
                    }
                    eo_hop_k(1, acc, xs, u);
                }
            }
            if (on) {
                if constexpr (HOPS == 6) {
#pragma unroll 1
                    for (int k = 2; k < 8; ++k) {
                        PT p[12], u[9];
                        eo_load_hop<OP>(k, p, u, in, Uo, Ui, s, h, q, a.g, r, a.nrhs, inf);
                        eo_hop_k(k, acc, p, u);
                    }
                } else if constexpr (HOPS == 2 && OP::kPacked) {
                    PT pa[12], pb[12], ua[9], ub[9];
                    eo_load_hop<OP>(0, pa, ua, in, Uo, Ui, s, h, q, a.g, r, a.nrhs, inf);
#pragma unroll 1
                    for (int mu = 0; mu < 4; ++mu) {
                        eo_load_hop<OP>(2 * mu + 1, pb, ub, in, Uo, Ui, s, h, q, a.g, r, a.nrhs, inf);
                        eo_hop_k(2 * mu, acc, pa, ua);
                        if (mu < 3) eo_load_hop<OP>(2 * mu + 2, pa, ua, in, Uo, Ui, s, h, q, a.g, r, a.nrhs, inf);
                        eo_hop_k(2 * mu + 1, acc, pb, ub);
                    }
                } else {
#pragma unroll 1
                    for (int k = 0; k < 8; ++k) {
                        PT p[12], u[9];
                        eo_load_hop<OP>(k, p, u, in, Uo, Ui, s, h, q, a.g, r, a.nrhs, inf);
                        eo_hop_k(k, acc, p, u);
                    }
                }
            }
            R sre = 0, sim = 0, sqq = 0;
            const bool act = a.active == nullptr || a.active[r] != 0;
            if (valid) {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const size_t i = fidx(h, r, c, a.nrhs);
                    cpx<R> o = {0, 0};
                    if (on && act) {
                        o = {be * acc[c].re, be * acc[c].im};
                        if (in2) {
                            const cpx<R> v = ldr<R>(in2, in2_full ? fidx(s, r, c, a.nrhs) : i);
                            o.re = fma(al, v.re, o.re);
                            o.im = fma(al, v.im, o.im);
                        }
                    }
                    if (out_full) {
                        // this site, and the other parity's site of the same index
                        stc(out, fidx(s, r, c, a.nrhs), o);
                        out[fidx(s ^ 1, r, c, a.nrhs)] = ((const S *)a.partner)[i];
                    } else {
                        stc(out, i, o);
                    }
                    if (dots && on) {
                        const cpx<R> v = a.dot_with ? ldr<R>((const S *)a.dot_with, i) : cpx<R>{0, 0};
                        sre = fma(o.re, v.re, fma(o.im, v.im, sre));
                        sim = fma(o.re, v.im, fma(-o.im, v.re, sim));
                        sqq = fma(o.re, o.re, fma(o.im, o.im, sqq));
                    }
                }
            }
            if (dots) {
                const double dre = wave_sum((double)sre);
                const double dim = wave_sum((double)sim);
                const double dqq = wave_sum((double)sqq);
                if (lane == 0) {
                    red[wave][r][0] += dre;
                    red[wave][r][1] += dim;
                    red[wave][r][2] += dqq;
                }
            }
        }
    }
    }
    if (dots) {
        __syncthreads();
        const int nw = blockDim.x >> 6;
        for (int i = threadIdx.x; i < a.nrhs * 3; i += blockDim.x) {
            double t = 0;
            for (int k = 0; k < nw; ++k) t += red[k][i / 3][i % 3];
            a.partials[(size_t)blockIdx.x * a.nrhs * 3 + i] = t;
        }
    }
}

// Plane form of the t-marching half-stencil (packed BF16).  A workgroup holds
// one x-y plane of the half lattice (P = Lx / 2 * Ly columns, one lane each,
// P a multiple of 64 and at most kMaxPlane) for one RHS and walks `march` time
// slices.  The other parity's sites of the plane at slices t - 1, t and t + 1
// wait in an LDS ring of three slots (slice t in slot (t - t0 + 1) mod 3 for
// a chunk starting at t0), so the x and y hops (the y neighbours
// of a column are the columns one x-row up and down, the plane being periodic
// in y) and the backward t hop read LDS; only the z hops, the forward t
// neighbour (which then enters the ring) and the links are loaded.  One
// barrier per slice: the slot of slice t is written during slice t - 1 and
// read across lanes in slice t; the slot of slice t + 1, that of slice t - 2
// before, was last read across lanes in slice t - 2, which every wave has
// left once the barrier of slice t opens.  Workgroups of the same plane and
// time chunk (consecutive RHS) run side by side on one XCD and share its
// links through L2; each XCD walks its own z-slab.
constexpr int kMaxPlane = 512;

// The slice body is straight-line: the site's coordinates come from the
// lane (x / 2, y), the plane z and the slice t with no divisions; the z and t
// neighbours are the same column one plane or one slice away; the epilogue
// (EPI 0: out = H in; 3: out = beta H in; 1: out = alpha in2 + beta H in; 2:
// the same with the fused sums) is chosen at compile time, and the twelve
// in2 words (and the dot_with words) are loaded together before they are
// used.  The fused sums <out, v> and |out|^2 are formed from the stored BF16
// words of out, two-way dot products exact in FP32: the values the solver's
// update then reads.
template <int IO, int EPI, int NPL>
__global__ void __launch_bounds__(kMaxPlane * NPL, 4) eo_plane_kernel(EoArgs a)
{
    constexpr bool in_full = IO == 1, in2_full = IO == 1 || IO == 2, out_full = IO >= 2;
    constexpr bool has_in2 = EPI == 1 || EPI == 2, dots = EPI == 2, scaled = EPI != 0;
    typedef bf16x2 S;
    typedef float R;
    typedef uint32_t PT;
    __shared__ PT ring[3][12][kMaxPlane * NPL];
    __shared__ double red[kMaxPlane * NPL / 64][kMaxRhs][3];
    const PT *__restrict__ in = (const PT *)a.in;
    const PT *__restrict__ in2 = (const PT *)a.in2;
    PT *__restrict__ out = (PT *)a.out;
    const PT *__restrict__ Uo = (const PT *)a.U + (size_t)a.po * 36 * a.Vhs;
    const PT *__restrict__ Ui = (const PT *)a.U + (size_t)(1 - a.po) * 36 * a.Vhs;
    const uint8_t *__restrict__ mk = a.mask + (size_t)a.po * a.Vhs;
    // NPL planes per workgroup (z0, z0 + 1 with two): lane tid holds column
    // l of plane pl, in the ring at index tid
    const int P = blockDim.x / NPL, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int pl = NPL == 1 ? 0 : tid / P, l = tid - pl * P;  // pl: the same in a wavefront
    const int nw = blockDim.x >> 6, nr = a.nrhs;
    if (dots) {
        for (int i = tid; i < nw * nr * 3; i += blockDim.x) red[i / (nr * 3)][(i / 3) % nr][i % 3] = 0.0;
    }
    const R al = (R)a.alpha, be = (R)a.beta;
    const int Lt = a.g.L[3], Lz = a.g.L[2], Lh = a.g.L[0] >> 1;
    const int Vs3 = a.Vh / Lt;  // half-sites per time slice = P * Lz
    const int xcd = (int)(blockIdx.x & 7), slot = (int)(blockIdx.x >> 3), slots = (int)(gridDim.x >> 3);
    const int Z0 = (xcd * Lz) >> 3, nz = ((((xcd + 1) * Lz) >> 3) - Z0) / NPL;
    const int ML = a.march, nc = (Lt + ML - 1) / ML;
    const int nx = nz * nr * nc;
    // this lane's column: x / 2 and y; its neighbours in the plane along its
    // x-row (x hops) and one x-row up and down (y hops), as ring indices
    const int xh = l % Lh, yy = l / Lh, rs = tid - xh;
    const int xp = rs + (xh + 1 == Lh ? 0 : xh + 1), xm = rs + (xh == 0 ? Lh - 1 : xh - 1);
    const int yp = pl * P + (l + Lh >= P ? l + Lh - P : l + Lh), ym = pl * P + (l < Lh ? l - Lh + P : l - Lh);
    // with two planes, the ring index of the same column in the other plane
    const int other = NPL == 2 ? (pl == 0 ? tid + P : tid - P) : tid;
    // the sums' second vector: in2 itself (its loaded words), none (|out|^2
    // only), or a field of its own
    const int dmode = !dots || a.dot_with == nullptr ? 0 : (!in2_full && a.dot_with == a.in2) ? 1 : 2;
    // input element of the other parity's site at compact index hq in slice
    // tq (full layout: the site itself, 2 hq plus its x bit)
    auto iidx = [&](int hq, int tq, int zq) -> int {
        if constexpr (in_full) return 2 * hq + (((1 - a.po) ^ yy ^ zq ^ tq) & 1);
        else return hq;
    };
    for (int j = slot; j < nx; j += slots) {
        const int r = j % nr, rest = j / nr;
        const int z = Z0 + NPL * (rest % nz) + pl, ch = rest / nz;
        const int col = z * P + l;
        const int t0 = ch * ML, t1 = min(t0 + ML, Lt);
        const bool act = a.active == nullptr || a.active[r] != 0;
        const int zf = z + 1 == Lz ? 0 : z + 1, zb = z == 0 ? Lz - 1 : z - 1;
        const int dzf = (zf - z) * P, dzb = (zb - z) * P;
        {
            const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
            const int im = iidx(tm * Vs3 + col, tm, z), i0 = iidx(t0 * Vs3 + col, t0, z);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                ring[0][c][tid] = in[fidx(im, r, c, nr)];
                ring[1][c][tid] = in[fidx(i0, r, c, nr)];
            }
        }
        // the slots of slices t - 1, t and t + 1
        int prv = 0, cur = 1, nxt = 2;
        double dre = 0, dim = 0, dqq = 0;
#pragma unroll 1
        for (int t = t0; t < t1; ++t) {
            __syncthreads();
            const int base = t * Vs3 + z * P - pl * P;  // compact index of ring index 0
            const int h = base + tid;
            const int tf = t + 1 == Lt ? 0 : t + 1, tb = t == 0 ? Lt - 1 : t - 1;
            const bool on = mk[h] == 0;
            // the output site: x = 2 xh + b, with b from the parity
            const int b = (a.po ^ yy ^ z ^ t) & 1;
            const int s = 2 * h + b;
            // the forward t-neighbour: used at the end of this slice, then
            // kept in the ring for the two slices after it
            PT qc[12];
            {
                const int fi = iidx(tf * Vs3 + col, tf, z);
#pragma unroll
                for (int c = 0; c < 12; ++c) qc[c] = in[fidx(fi, r, c, nr)];
            }
            // the x and y hops from the ring: neighbour column n, and the
            // link U_mu(s) (forward) or U_mu(s - mu) at the neighbour's index;
            // loads in batches: the x and y hops' links, the z+ hop's
            // operands, then the z- hop's with the t hops' links.  The first
            // hop runs on every lane (its operands are valid for a coarse
            // site too) and writes the accumulators; a coarse site's output
            // is replaced by zero below.
            PT u4[4][9];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int n = k == 0 ? (b ? xp : tid) : k == 1 ? (b ? tid : xm) : k == 2 ? yp : ym;
                const int mu = k >> 1;
#pragma unroll
                for (int e = 0; e < 9; ++e)
                    u4[k][e] = (k & 1) ? Ui[lidx(base + n, mu, e)] : Uo[lidx(h, mu, e)];
            }
            cpx<R> acc[12];
            {
                PT p[12];
#pragma unroll
                for (int c = 0; c < 12; ++c) p[c] = ring[cur][c][b ? xp : tid];
                hop_bf16<0, true, true>(acc, p, u4[0]);
            }
            if (on) {
#pragma unroll
                for (int k = 1; k < 4; ++k) {
                    const int n = k == 1 ? (b ? tid : xm) : k == 2 ? yp : ym;
                    PT p[12];
#pragma unroll
                    for (int c = 0; c < 12; ++c) p[c] = ring[cur][c][n];
                    if (k == 1) hop_bf16<0, false>(acc, p, u4[1]);
                    else if (k == 2) hop_bf16<1, true>(acc, p, u4[2]);
                    else hop_bf16<1, false>(acc, p, u4[3]);
                }
                PT pz[12], uz[9];
                {
                    // z+: the same column one plane up, U_z(s); with two
                    // planes, the lower plane's from the upper plane's ring
                    if (NPL == 2 && pl == 0) {
#pragma unroll
                        for (int c = 0; c < 12; ++c) pz[c] = ring[cur][c][other];
                    } else {
                        const int ni = iidx(h + dzf, t, zf);
#pragma unroll
                        for (int c = 0; c < 12; ++c) pz[c] = in[fidx(ni, r, c, nr)];
                    }
#pragma unroll
                    for (int e = 0; e < 9; ++e) uz[e] = Uo[lidx(h, 2, e)];
                }
                hop_bf16<2, true>(acc, pz, uz);
                PT ut[2][9];
                {
                    // z-: one plane down, U_z(s - z) at the neighbour's index;
                    // with two planes, the upper plane's from the lower's ring
                    const int hn = h + dzb;
                    if (NPL == 2 && pl == 1) {
#pragma unroll
                        for (int c = 0; c < 12; ++c) pz[c] = ring[cur][c][other];
                    } else {
                        const int ni = iidx(hn, t, zb);
#pragma unroll
                        for (int c = 0; c < 12; ++c) pz[c] = in[fidx(ni, r, c, nr)];
                    }
#pragma unroll
                    for (int e = 0; e < 9; ++e) uz[e] = Ui[lidx(hn, 2, e)];
                }
#pragma unroll
                for (int e = 0; e < 9; ++e) {
                    ut[0][e] = Uo[lidx(h, 3, e)];
                    ut[1][e] = Ui[lidx(tb * Vs3 + col, 3, e)];
                }
                hop_bf16<2, false>(acc, pz, uz);
                hop_bf16<3, true>(acc, qc, ut[0]);
                {
                    PT p[12];
#pragma unroll
                    for (int c = 0; c < 12; ++c) p[c] = ring[prv][c][tid];
                    hop_bf16<3, false>(acc, p, ut[1]);
                }
            }
            // slice t + 1 into the slot of slice t - 2 (read across lanes in
            // slice t - 2 only, which every wave has left)
#pragma unroll
            for (int c = 0; c < 12; ++c) ring[nxt][c][tid] = qc[c];
            {
                const int o = prv;
                prv = cur;
                cur = nxt;
                nxt = o;
            }
            // epilogue: every word of in2 (and of the sums' vector) first
            PT w2[12], wd[12];
            if constexpr (has_in2) {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    if constexpr (!in2_full)
                        // read once, whole lines: streamed past L2
                        w2[c] = __builtin_nontemporal_load(in2 + fidx(h, r, c, nr));
                    else
                        // the full layout: half of each line, the other half
                        // read by the neighbouring lanes' hops
                        w2[c] = in2[fidx(s, r, c, nr)];
                }
            }
            if constexpr (dots) {
                if (dmode == 2) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) wd[c] = ((const PT *)a.dot_with)[fidx(h, r, c, nr)];
                } else if (dmode == 1) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) wd[c] = w2[c];
                } else {
#pragma unroll
                    for (int c = 0; c < 12; ++c) wd[c] = 0u;
                }
            }
            const bool keep = on && act;
            R sre = 0, sim = 0, sqq = 0;
            // the partner copy of the last step is the input itself at this
            // column and slice, which the ring holds (now in slot prv)
            const bool partner_in = out_full && a.partner == a.in;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                cpx<R> o = acc[c];
                if constexpr (scaled) o = {be * acc[c].re, be * acc[c].im};
                if constexpr (has_in2) {
                    const cpx<R> v2 = as_cpx(w2[c]);
                    o.re = fmaf(al, v2.re, o.re);
                    o.im = fmaf(al, v2.im, o.im);
                }
                if (!keep) o = {0, 0};
                const PT ow = pack_bf16(o.re, o.im);
                if constexpr (out_full) {
                    // this site, and the other parity's site of the same index
                    // (two halves of each line: ordinary stores, merged in L2)
                    out[fidx(s, r, c, nr)] = ow;
                    out[fidx(s ^ 1, r, c, nr)] =
                        partner_in ? ring[prv][c][tid] : ((const PT *)a.partner)[fidx(h, r, c, nr)];
                } else {
                    // written once, whole lines: streamed past L2, which keeps
                    // the links and the input planes the next workgroups read
                    __builtin_nontemporal_store(ow, out + fidx(h, r, c, nr));
                }
                if constexpr (dots) {
                    // re <o, v> = o.re v.re + o.im v.im, im = o.re v.im - o.im v.re
                    sre = dot2bf(ow, wd[c], sre);
                    sqq = dot2bf(ow, ow, sqq);
                    sim = dot2n<0, 1>(ow, swap_halves(wd[c]), sim);
                }
            }
            if constexpr (dots) {
                asm("s_nop 2" : "+v"(sim));  // closes the chain of sim (see dot_fence)
                dre += (double)sre;
                dim += (double)sim;
                dqq += (double)sqq;
            }
        }
        // the next item's first loads overwrite slots read across lanes
        __syncthreads();
        if constexpr (dots) {
            dre = wave_sum(dre);
            dim = wave_sum(dim);
            dqq = wave_sum(dqq);
            if (lane == 0) {
                red[wave][r][0] += dre;
                red[wave][r][1] += dim;
                red[wave][r][2] += dqq;
            }
        }
    }
    if constexpr (dots) {
        __syncthreads();
        for (int i = tid; i < nr * 3; i += blockDim.x) {
            double t = 0;
            for (int k = 0; k < nw; ++k) t += red[k][i / 3][i % 3];
            a.partials[(size_t)blockIdx.x * nr * 3 + i] = t;
        }
    }
}

// A compact field of parity par <-> the full field that holds it on the
// sites of that parity and zero on the others (every RHS).
template <int P>
__global__ void __launch_bounds__(256) eo_scatter_kernel(Geom g, int nrhs, int par, const void *src_,
                                                         void *dst_, int to_full)
{
    typedef typename Store<P>::S S;
    const S *src = (const S *)src_;
    S *dst = (S *)dst_;
    const int n = to_full ? g.V : g.V / 2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int r = 0; r < nrhs; ++r) {
            if (to_full) {
                const bool mine = site_parity(i, g) == par;
#pragma unroll
                for (int c = 0; c < 12; ++c)
                    dst[fidx(i, r, c, nrhs)] = mine ? src[fidx(i >> 1, r, c, nrhs)] : S{};
            } else {
                SiteGeo q;
                const int s = eo_site(i, par, g, q);
#pragma unroll
                for (int c = 0; c < 12; ++c) dst[fidx(i, r, c, nrhs)] = src[fidx(s, r, c, nrhs)];
            }
        }
    }
}

// links [tiles][4][9][64] -> [2][half tiles][4][9][64]; mask -> [2][Vhs]
template <class S>
__global__ void __launch_bounds__(256) eo_pack_links_kernel(Geom g, int Vhs, const S *U, S *Ueo)
{
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.V; s += gridDim.x * blockDim.x) {
        S *dst = Ueo + (size_t)site_parity(s, g) * 36 * Vhs;
        const int h = s >> 1;
        for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int e = 0; e < 9; ++e) dst[lidx(h, mu, e)] = U[lidx(s, mu, e)];
    }
}

__global__ void __launch_bounds__(256) eo_pack_mask_kernel(Geom g, int Vhs, const uint8_t *mask,
                                                           uint8_t *meo)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * Vhs) return;
    const int p = i / Vhs, h = i - p * Vhs;
    uint8_t v = 1;  // padding: never a rest site
    if (h < g.V / 2) {
        SiteGeo q;
        const int s = eo_site(h, p, g, q);
        v = mask[s];
    }
    meo[i] = v;
}

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

hipError_t launch_eo_hop(int prec, const EoArgs &a, int grid, hipStream_t st)
{
    if (a.nrhs < 1 || a.nrhs > kMaxRhs || a.RG < 1 || grid < 8 || grid % 8) return hipErrorInvalidValue;
    int io = 0;
    if (a.in_full && a.in2_full && !a.out_full) io = 1;
    else if (!a.in_full && a.in2_full && a.out_full) io = 2;
    else if (!a.in_full && !a.in2_full && a.out_full) io = 3;
    else if (a.in_full || a.in2_full || a.out_full) return hipErrorInvalidValue;
    if (a.hops == 7) {
        // plane form: packed BF16, one workgroup of P = Lx / 2 * Ly lanes
        // per x-y plane
        const int P = (a.g.L[0] / 2) * a.g.L[1];
        if (prec != GRG_BF16 || a.SB != P || P % 64 || P > kMaxPlane || a.march < 1 || a.g.L[3] < 2 ||
            a.g.L[0] < 2 || a.Vh != P * a.g.L[2] * a.g.L[3])
            return hipErrorInvalidValue;
        // RG = 2: two planes per workgroup, which needs an even number of
        // planes in every XCD's z-slab
        const int npl = a.RG == 2 ? 2 : 1;
        if (npl == 2 && (a.g.L[2] % 16 || a.g.L[2] < 16)) return hipErrorInvalidValue;
        dim3 pb(P * npl), pg(grid);
        const int epi = a.partials ? 2 : a.in2 ? 1 : a.beta == 1.0 ? 0 : 3;
        if (epi == 2 && !a.in2) return hipErrorInvalidValue;  // the sums come with the alpha term
#define PLANE(I, E)                                                                \
    do {                                                                           \
        if (npl == 2) hipLaunchKernelGGL((eo_plane_kernel<I, E, 2>), pg, pb, 0, st, a); \
        else hipLaunchKernelGGL((eo_plane_kernel<I, E, 1>), pg, pb, 0, st, a);    \
    } while (0)
        if (io == 1) {
            if (epi == 2) PLANE(1, 2); else if (epi == 1) PLANE(1, 1); else return hipErrorInvalidValue;
        } else if (io == 2) {
            if (epi == 1) PLANE(2, 1); else return hipErrorInvalidValue;
        } else if (io == 3) {
            if (epi == 1) PLANE(3, 1); else return hipErrorInvalidValue;
        } else {
            if (epi == 2) PLANE(0, 2); else if (epi == 1) PLANE(0, 1); else if (epi == 3) PLANE(0, 3);
            else PLANE(0, 0);
        }
#undef PLANE
        return hipGetLastError();
    }
    if (a.SB != 64 && a.SB != 128 && a.SB != 256) return hipErrorInvalidValue;
    dim3 blk(a.SB), grd(grid);
    const bool pipe = a.hops == 2 && prec == GRG_BF16 && io == 0;
    if (a.hops == 3) {
        // t-marching: packed BF16, 256 threads, whole 64-column tiles per slice
        if (prec != GRG_BF16 || a.SB != 256 || a.march < 1 || a.g.L[3] < 2 || a.Vh % a.g.L[3] ||
            (a.Vh / a.g.L[3]) % 64 || a.g.L[0] < 2 || 64 % (a.g.L[0] / 2))
            return hipErrorInvalidValue;
        if (io == 1) hipLaunchKernelGGL((eo_hop_kernel<GRG_BF16, 3, 1>), grd, blk, 0, st, a);
        else if (io == 2) hipLaunchKernelGGL((eo_hop_kernel<GRG_BF16, 3, 2>), grd, blk, 0, st, a);
        else if (io == 3) hipLaunchKernelGGL((eo_hop_kernel<GRG_BF16, 3, 3>), grd, blk, 0, st, a);
        else hipLaunchKernelGGL((eo_hop_kernel<GRG_BF16, 3, 0>), grd, blk, 0, st, a);
        return hipGetLastError();
    }
    if (a.hops == 6 && io == 0) {
        // x hops from lane shuffles: packed BF16, x-rows tiling the wavefront
        if (prec != GRG_BF16 || 64 % (a.g.L[0] / 2) != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((eo_hop_kernel<GRG_BF16, 6, 0>), grd, blk, 0, st, a);
        return hipGetLastError();
    }
    if ((a.hops == 4 || a.hops == 5) && io == 0) {
        // RHS-simultaneous: packed BF16, RG = 2 or 3 right-hand sides per hop
        if (prec != GRG_BF16 || a.RG != a.hops - 2) return hipErrorInvalidValue;
        if (a.hops == 4) hipLaunchKernelGGL((eo_hop_kernel<GRG_BF16, 4, 0>), grd, blk, 0, st, a);
        else hipLaunchKernelGGL((eo_hop_kernel<GRG_BF16, 5, 0>), grd, blk, 0, st, a);
        return hipGetLastError();
    }
#define EOH(PP, H, IO) hipLaunchKernelGGL((eo_hop_kernel<PP, H, IO>), grd, blk, 0, st, a)
#define EOIO(PP)                     \
    if (io == 1) EOH(PP, 1, 1);      \
    else if (io == 2) EOH(PP, 1, 2); \
    else if (io == 3) EOH(PP, 1, 3); \
    else EOH(PP, 1, 0);
    switch (prec) {
    case GRG_FP64: EOIO(GRG_FP64) break;
    case GRG_FP32: EOIO(GRG_FP32) break;
    case GRG_BF16:
        if (pipe) EOH(GRG_BF16, 2, 0);
        else {
            EOIO(GRG_BF16)
        }
        break;
    default: return hipErrorInvalidValue;
    }
#undef EOIO
#undef EOH
    return hipGetLastError();
}

hipError_t launch_eo_scatter(int prec, const Geom &g, int nrhs, int par, const void *src, void *dst,
                             bool to_full, hipStream_t st)
{
    const int grid = std::min(cdiv(g.V, 256), 8192);
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(eo_scatter_kernel<GRG_FP64>, dim3(grid), dim3(256), 0, st, g, nrhs, par, src, dst, (int)to_full); break;
    case GRG_FP32: hipLaunchKernelGGL(eo_scatter_kernel<GRG_FP32>, dim3(grid), dim3(256), 0, st, g, nrhs, par, src, dst, (int)to_full); break;
    case GRG_BF16: hipLaunchKernelGGL(eo_scatter_kernel<GRG_BF16>, dim3(grid), dim3(256), 0, st, g, nrhs, par, src, dst, (int)to_full); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_eo_pack_links(int prec, const Geom &g, int Vhs, const void *U, void *Ueo, hipStream_t st)
{
    const int grid = std::min(cdiv(g.V, 256), 8192);
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(eo_pack_links_kernel<double2>, dim3(grid), dim3(256), 0, st, g, Vhs, (const double2 *)U, (double2 *)Ueo); break;
    case GRG_FP32: hipLaunchKernelGGL(eo_pack_links_kernel<float2>, dim3(grid), dim3(256), 0, st, g, Vhs, (const float2 *)U, (float2 *)Ueo); break;
    case GRG_BF16: hipLaunchKernelGGL(eo_pack_links_kernel<bf16x2>, dim3(grid), dim3(256), 0, st, g, Vhs, (const bf16x2 *)U, (bf16x2 *)Ueo); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_eo_pack_mask(const Geom &g, int Vhs, const uint8_t *mask, uint8_t *meo, hipStream_t st)
{
    hipLaunchKernelGGL(eo_pack_mask_kernel, dim3(cdiv(2L * Vhs, 256)), dim3(256), 0, st, g, Vhs, mask, meo);
    return hipGetLastError();
}

}  // namespace grg
