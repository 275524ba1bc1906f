// Wilson-Dirac stencil (dslash) and layout kernels for gfx950.
//
//   D psi(x) = (4 + m0) psi(x)
//              - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x + mu)
//                           + (1 + g_mu) U_mu(x - mu)^+ psi(x - mu) ]
//
// DeGrand-Rossi basis: every g_mu is block off-diagonal,
// g_mu = [[0, B_mu], [B_mu^+, 0]] on (spins 0,1 | spins 2,3), with
//   B_x = [[0, i], [i, 0]],  B_y = [[0, -1], [1, 0]],
//   B_z = [[i, 0], [0, -i]], B_t = [[1, 0], [0, 1]].
// Hence (1 -/+ g_mu) psi = (h, -/+ B_mu^+ h) with h = psi_up -/+ B_mu psi_lo:
// each hop projects to a 2-spin vector h, multiplies 2 colour vectors by the
// link, and reconstructs the lower spins with B_mu^+ (swaps and phases only).
//
// The operator is memory-bound (1320 flop per site against 24 + 24 + 72
// reals of compulsory traffic), so the kernel is organised around traffic:
// site-parallel SoA loads (one complex per lane per component, coalesced),
// one thread per site looping over a group of right-hand sides so that the
// links of a site are fetched from HBM once per group, and an XCD-aware
// grid-stride walk so that each XCD's L2 sees one contiguous eighth of the
// lattice.  Sub-blocks D_rr, D_rb, D_bb, D_br are the same stencil with an
// output-site mask (inputs vanish off their block by construction).
#include "common.h"
#include "engine.h"

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
    // w = U h (forward) or U^+ h (backward), one colour vector per spin
    cpx<R> w0[3], w1[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        cpx<R> s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cpx<R> m = FWD ? u[3 * r + c] : u[3 * c + r];
            const cpx<R> t0 = FWD ? cmul(m, h0[c]) : cmulc(m, h0[c]);
            const cpx<R> t1 = FWD ? cmul(m, h1[c]) : cmulc(m, h1[c]);
            s0.re += t0.re; s0.im += t0.im;
            s1.re += t1.re; s1.im += t1.im;
        }
        w0[r] = s0;
        w1[r] = s1;
    }
    // upper spins: -1/2 w ; lower spins: -1/2 (-/+ B^+ w) = +/- 1/2 B^+ w
    const R hu = R(-0.5);
    const R hl = FWD ? R(0.5) : R(-0.5);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        acc[r].re += hu * w0[r].re;
        acc[r].im += hu * w0[r].im;
        acc[3 + r].re += hu * w1[r].re;
        acc[3 + r].im += hu * w1[r].im;
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
        acc[6 + r].re += hl * d0.re;
        acc[6 + r].im += hl * d0.im;
        acc[9 + r].re += hl * d1.re;
        acc[9 + r].im += hl * d1.im;
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
template <class S, class R, bool SPLIT>
__device__ __forceinline__ void dslash_site(cpx<R> (&acc)[12], const S *__restrict__ in,
                                            const S *__restrict__ U, int s, const SiteGeo &q,
                                            const Geom &g, int r, int nrhs, R diag)
{
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const cpx<R> v = ldc(in, fidx(s, r, c, nrhs));
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
            for (int c = 0; c < 12; ++c) p[c] = ldc(in, fidx(n, r, c, nrhs));
#pragma unroll
            for (int e = 0; e < 9; ++e) u[e] = ldc(U, lidx((h & 1) ? sm : s, mu, e));
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
            pf[c] = ldc(in, fidx(sp, r, c, nrhs));
            pb[c] = ldc(in, fidx(sm, r, c, nrhs));
        }
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            uf[e] = ldc(U, lidx(s, mu, e));
            ub[e] = ldc(U, lidx(sm, mu, e));
        }
        switch (mu) {
        case 0: hop_math<0, true>(acc, pf, uf); hop_math<0, false>(acc, pb, ub); break;
        case 1: hop_math<1, true>(acc, pf, uf); hop_math<1, false>(acc, pb, ub); break;
        case 2: hop_math<2, true>(acc, pf, uf); hop_math<2, false>(acc, pb, ub); break;
        default: hop_math<3, true>(acc, pf, uf); hop_math<3, false>(acc, pb, ub); break;
        }
    }
}

// out = mask_sel D in, for nrhs fields.  With a.partials set, also the
// per-workgroup partial sums of conj(out).in (re, im) and |out|^2 per RHS.
template <int P, bool SPLIT>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs a)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    __shared__ double red[4][kMaxRhs][3];
    const S *__restrict__ in = (const S *)a.in;
    S *__restrict__ out = (S *)a.out;
    const S *__restrict__ U = (const S *)a.U;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool dots = a.partials != nullptr;
    if (dots) {
        for (int i = lane; i < a.nrhs * 3; i += 64) red[wave][i / 3][i % 3] = 0.0;
        __syncthreads();
    }
    const int ngroups = (a.nrhs + a.RG - 1) / a.RG;
    const int nsb = (a.g.V + a.SB - 1) / a.SB;
    const ItemRange it = xcd_items(nsb * ngroups);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int sb = w / ngroups, grp = w - sb * ngroups;
        const int s = sb * a.SB + (int)threadIdx.x;
        const bool valid = s < a.g.V;
        const bool on = valid && (a.mask == nullptr || a.mask[s] == a.sel);
        SiteGeo q;
        if (on) q = site_geo(s, a.g);
        const int r0 = grp * a.RG, r1 = min(r0 + a.RG, a.nrhs);
        for (int r = r0; r < r1; ++r) {
            cpx<R> acc[12];
            if (on) {
                dslash_site<S, R, SPLIT>(acc, in, U, s, q, a.g, r, a.nrhs, (R)a.diag);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
            }
            if (valid) {
#pragma unroll
                for (int c = 0; c < 12; ++c) stc(out, fidx(s, r, c, a.nrhs), acc[c]);
            }
            if (dots) {
                double dre = 0, dim = 0, dqq = 0;
                if (on) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const cpx<R> v = ldc(in, fidx(s, r, c, a.nrhs));
                        dre += (double)acc[c].re * v.re + (double)acc[c].im * v.im;
                        dim += (double)acc[c].re * v.im - (double)acc[c].im * v.re;
                        dqq += (double)acc[c].re * acc[c].re + (double)acc[c].im * acc[c].im;
                    }
                }
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

// y_b[rhs][k] = (D in)(q[k]) in canonical coarse layout, FP64.
__global__ void __launch_bounds__(256) dslash_coarse_kernel(CoarseArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.nb) return;
    const int s = a.q[k];
    const SiteGeo q = site_geo(s, a.g);
    const double2 *in = (const double2 *)a.in;
    const double2 *U = (const double2 *)a.U;
    for (int r = 0; r < a.nrhs; ++r) {
        cpx<double> acc[12];
        dslash_site<double2, double, true>(acc, in, U, s, q, a.g, r, a.nrhs, a.diag);
        double2 *o = (double2 *)a.out + ((size_t)r * a.nb + k) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = make_double2(acc[c].re, acc[c].im);
    }
}

// ------------------------------------------------------------------ layouts
// canonical links [V][4][3][3] complex128 -> internal tiles in three
// precisions, boundary sign folded into the last slice of each direction.
__global__ void pack_gauge_kernel(const double2 *__restrict__ src, Geom g, int4 bc,
                                  double2 *u64, float2 *u32, bf16x2 *u16)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.V * 4) return;
    const int s = idx >> 2, mu = idx & 3;
    const SiteGeo q = site_geo(s, g);
    const int b = mu == 0 ? bc.x : mu == 1 ? bc.y : mu == 2 ? bc.z : bc.w;
    const int x = mu == 0 ? q.c[0] : mu == 1 ? q.c[1] : mu == 2 ? q.c[2] : q.c[3];
    const int L = mu == 0 ? g.L[0] : mu == 1 ? g.L[1] : mu == 2 ? g.L[2] : g.L[3];
    const double sign = (x == L - 1) ? (double)b : 1.0;
    for (int e = 0; e < 9; ++e) {
        const double2 v = src[(size_t)idx * 9 + e];
        const cpx<double> d = {sign * v.x, sign * v.y};
        const size_t o = lidx(s, mu, e);
        stc(u64, o, d);
        stc(u32, o, cpx<float>{(float)d.re, (float)d.im});
        stc(u16, o, cpx<float>{(float)d.re, (float)d.im});
    }
}

// canonical [nrhs][V][12] complex128  <->  internal tiles
template <int P>
__global__ void pack_spinor_kernel(const double2 *__restrict__ src, void *dst, Geom g, int nrhs)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V || r >= nrhs) return;
    const double2 *p = src + ((size_t)r * g.V + s) * 12;
    S *o = (S *)dst;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 v = p[c];
        stc(o, fidx(s, r, c, nrhs), cpx<R>{(R)v.x, (R)v.y});
    }
}

template <int P>
__global__ void unpack_spinor_kernel(const void *src, double2 *__restrict__ dst, Geom g, int nrhs)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V || r >= nrhs) return;
    const S *p = (const S *)src;
    double2 *o = dst + ((size_t)r * g.V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const cpx<R> v = ldc(p, fidx(s, r, c, nrhs));
        o[c] = make_double2((double)v.re, (double)v.im);
    }
}

// canonical lattice field -> internal FP64 with the coarse sites zeroed
// (rhs of the D_rr solve), or the coarse-only part (keep = 1).
__global__ void pack_masked_kernel(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                   const uint8_t *__restrict__ mask, int keep, Geom g, int nrhs)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V || r >= nrhs) return;
    const bool k = mask[s] == keep;
    const double2 *p = src + ((size_t)r * g.V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[fidx(s, r, c, nrhs)] = k ? p[c] : make_double2(0.0, 0.0);
}

// coarse canonical [nrhs][nb][12] -> internal FP64 lattice field, zero on
// the other sites.  bidx[s] = coarse index of site s, or -1.
__global__ void scatter_coarse_kernel(const double2 *__restrict__ xb, double2 *__restrict__ dst,
                                      const int32_t *__restrict__ bidx, int nb, Geom g, int nrhs)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V || r >= nrhs) return;
    const int k = bidx[s];
    const double2 *p = xb + ((size_t)r * nb + (k < 0 ? 0 : k)) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[fidx(s, r, c, nrhs)] = k >= 0 ? p[c] : make_double2(0.0, 0.0);
}

// ------------------------------------------------------------------ launchers
static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

hipError_t launch_dslash(int prec, const DslashArgs &a, int grid, hipStream_t st)
{
    if (a.SB != 256 && a.SB != 128 && a.SB != 64) return hipErrorInvalidValue;
    if (a.nrhs < 1 || a.nrhs > kMaxRhs || a.RG < 1) return hipErrorInvalidValue;
    if (grid < 8 || grid % 8) return hipErrorInvalidValue;
    dim3 blk(a.SB), grd(grid);
#define DSL(PP)                                                                                 \
    if (a.split) hipLaunchKernelGGL((dslash_kernel<PP, true>), grd, blk, 0, st, a);             \
    else hipLaunchKernelGGL((dslash_kernel<PP, false>), grd, blk, 0, st, a);
    switch (prec) {
    case GRG_FP64: DSL(GRG_FP64) break;
    case GRG_FP32: DSL(GRG_FP32) break;
    case GRG_BF16: DSL(GRG_BF16) break;
    default: return hipErrorInvalidValue;
    }
#undef DSL
    return hipGetLastError();
}

hipError_t launch_dslash_coarse(const CoarseArgs &a, hipStream_t st)
{
    if (a.nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(dslash_coarse_kernel, dim3(cdiv(a.nb, 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_pack_gauge(const double *src, const Geom &g, const int bc[4], void *u64,
                             void *u32, void *u16, hipStream_t st)
{
    int4 b = make_int4(bc[0], bc[1], bc[2], bc[3]);
    hipLaunchKernelGGL(pack_gauge_kernel, dim3(cdiv((long)g.V * 4, 256)), dim3(256), 0, st,
                       (const double2 *)src, g, b, (double2 *)u64, (float2 *)u32, (bf16x2 *)u16);
    return hipGetLastError();
}

hipError_t launch_pack_spinor(int prec, const double *src, void *dst, const Geom &g, int nrhs,
                              hipStream_t st)
{
    dim3 grd(cdiv(g.V, 256), nrhs), blk(256);
    const double2 *s = (const double2 *)src;
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(pack_spinor_kernel<GRG_FP64>, grd, blk, 0, st, s, dst, g, nrhs); break;
    case GRG_FP32: hipLaunchKernelGGL(pack_spinor_kernel<GRG_FP32>, grd, blk, 0, st, s, dst, g, nrhs); break;
    case GRG_BF16: hipLaunchKernelGGL(pack_spinor_kernel<GRG_BF16>, grd, blk, 0, st, s, dst, g, nrhs); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(int prec, const void *src, double *dst, const Geom &g, int nrhs,
                                hipStream_t st)
{
    dim3 grd(cdiv(g.V, 256), nrhs), blk(256);
    double2 *d = (double2 *)dst;
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(unpack_spinor_kernel<GRG_FP64>, grd, blk, 0, st, src, d, g, nrhs); break;
    case GRG_FP32: hipLaunchKernelGGL(unpack_spinor_kernel<GRG_FP32>, grd, blk, 0, st, src, d, g, nrhs); break;
    case GRG_BF16: hipLaunchKernelGGL(unpack_spinor_kernel<GRG_BF16>, grd, blk, 0, st, src, d, g, nrhs); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_masked(const double *src, void *dst, const uint8_t *mask, int keep,
                              const Geom &g, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(pack_masked_kernel, dim3(cdiv(g.V, 256), nrhs), dim3(256), 0, st,
                       (const double2 *)src, (double2 *)dst, mask, keep, g, nrhs);
    return hipGetLastError();
}

hipError_t launch_scatter_coarse(const double *xb, void *dst, const int32_t *bidx, int nb,
                                 const Geom &g, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(scatter_coarse_kernel, dim3(cdiv(g.V, 256), nrhs), dim3(256), 0, st,
                       (const double2 *)xb, (double2 *)dst, bidx, nb, g, nrhs);
    return hipGetLastError();
}

}  // namespace grg
