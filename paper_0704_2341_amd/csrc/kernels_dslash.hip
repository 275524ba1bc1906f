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
template <int MU, bool FWD, class S, class R>
__device__ __forceinline__ void hop(cpx<R> (&acc)[12], const S *__restrict__ in,
                                    const S *__restrict__ U, int Vs, int n, int ls)
{
    cpx<R> p[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = ldc(in, (size_t)c * Vs + n);
    cpx<R> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ldc(U, (size_t)(MU * 9 + e) * Vs + ls);

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

struct Nbr {
    int p[4], m[4];
};

__device__ __forceinline__ Nbr neighbours(int s, const Geom &g)
{
    const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
    const int x = s % L0, t1 = s / L0;
    const int y = t1 % L1, t2 = t1 / L1;
    const int z = t2 % L2, t = t2 / L2;
    const int s1 = L0, s2 = L0 * L1, s3 = L0 * L1 * L2;
    Nbr nb;
    nb.p[0] = x == L0 - 1 ? s - (L0 - 1) : s + 1;
    nb.m[0] = x == 0 ? s + (L0 - 1) : s - 1;
    nb.p[1] = y == L1 - 1 ? s - (L1 - 1) * s1 : s + s1;
    nb.m[1] = y == 0 ? s + (L1 - 1) * s1 : s - s1;
    nb.p[2] = z == L2 - 1 ? s - (L2 - 1) * s2 : s + s2;
    nb.m[2] = z == 0 ? s + (L2 - 1) * s2 : s - s2;
    nb.p[3] = t == L3 - 1 ? s - (L3 - 1) * s3 : s + s3;
    nb.m[3] = t == 0 ? s + (L3 - 1) * s3 : s - s3;
    return nb;
}

template <class S, class R>
__device__ __forceinline__ void dslash_site(cpx<R> (&acc)[12], const S *__restrict__ in,
                                            const S *__restrict__ U, int Vs, int s,
                                            const Nbr &nb, R diag)
{
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const cpx<R> v = ldc(in, (size_t)c * Vs + s);
        acc[c] = {diag * v.re, diag * v.im};
    }
    hop<0, true>(acc, in, U, Vs, nb.p[0], s);
    hop<0, false>(acc, in, U, Vs, nb.m[0], nb.m[0]);
    hop<1, true>(acc, in, U, Vs, nb.p[1], s);
    hop<1, false>(acc, in, U, Vs, nb.m[1], nb.m[1]);
    hop<2, true>(acc, in, U, Vs, nb.p[2], s);
    hop<2, false>(acc, in, U, Vs, nb.m[2], nb.m[2]);
    hop<3, true>(acc, in, U, Vs, nb.p[3], s);
    hop<3, false>(acc, in, U, Vs, nb.m[3], nb.m[3]);
}

// out = mask_sel D in, for nrhs fields.  With a.partials set, also the
// per-workgroup partial sums of conj(out).in (re, im) and |out|^2 per RHS.
template <int P>
__global__ void __launch_bounds__(256) dslash_kernel(DslashArgs a)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    __shared__ double red[4][kMaxRhs][3];
    const S *__restrict__ in = (const S *)a.in;
    S *__restrict__ out = (S *)a.out;
    const S *__restrict__ U = (const S *)a.U;
    const int Vs = a.g.Vs;
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
        Nbr nb;
        if (on) nb = neighbours(s, a.g);
        const int r0 = grp * a.RG, r1 = min(r0 + a.RG, a.nrhs);
        for (int r = r0; r < r1; ++r) {
            const S *inr = in + (size_t)r * 12 * Vs;
            S *outr = out + (size_t)r * 12 * Vs;
            cpx<R> acc[12];
            if (on) {
                dslash_site<S, R>(acc, inr, U, Vs, s, nb, (R)a.diag);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
            }
            if (valid) {
#pragma unroll
                for (int c = 0; c < 12; ++c) stc(outr, (size_t)c * Vs + s, acc[c]);
            }
            if (dots) {
                double dre = 0, dim = 0, dqq = 0;
                if (on) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const cpx<R> v = ldc(inr, (size_t)c * Vs + s);
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
    const Nbr nb = neighbours(s, a.g);
    const double2 *in = (const double2 *)a.in;
    const double2 *U = (const double2 *)a.U;
    for (int r = 0; r < a.nrhs; ++r) {
        cpx<double> acc[12];
        dslash_site<double2, double>(acc, in + (size_t)r * 12 * a.g.Vs, U, a.g.Vs, s, nb, a.diag);
        double2 *o = (double2 *)a.out + ((size_t)r * a.nb + k) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = make_double2(acc[c].re, acc[c].im);
    }
}

// ------------------------------------------------------------------ layouts
// canonical links [V][4][3][3] complex128 -> internal [mu][9][Vs] in three
// precisions, boundary sign folded into the last slice of each direction.
__global__ void pack_gauge_kernel(const double2 *__restrict__ src, Geom g, int4 bc,
                                  double2 *u64, float2 *u32, bf16x2 *u16)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.V * 4) return;
    const int s = idx >> 2, mu = idx & 3;
    int c[4];
    int r = s;
    for (int nu = 0; nu < 4; ++nu) {
        c[nu] = r % g.L[nu];
        r /= g.L[nu];
    }
    const int b = mu == 0 ? bc.x : mu == 1 ? bc.y : mu == 2 ? bc.z : bc.w;
    const double sign = (c[mu] == g.L[mu] - 1) ? (double)b : 1.0;
    for (int e = 0; e < 9; ++e) {
        const double2 v = src[(size_t)idx * 9 + e];
        const cpx<double> d = {sign * v.x, sign * v.y};
        const size_t o = (size_t)(mu * 9 + e) * g.Vs + s;
        stc(u64, o, d);
        stc(u32, o, cpx<float>{(float)d.re, (float)d.im});
        stc(u16, o, cpx<float>{(float)d.re, (float)d.im});
    }
}

// canonical [nrhs][V][12] complex128  <->  internal [nrhs][12][Vs]
template <int P>
__global__ void pack_spinor_kernel(const double2 *__restrict__ src, void *dst, Geom g, int nrhs)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V || r >= nrhs) return;
    const double2 *p = src + ((size_t)r * g.V + s) * 12;
    S *o = (S *)dst + (size_t)r * 12 * g.Vs;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 v = p[c];
        stc(o, (size_t)c * g.Vs + s, cpx<R>{(R)v.x, (R)v.y});
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
    const S *p = (const S *)src + (size_t)r * 12 * g.Vs;
    double2 *o = dst + ((size_t)r * g.V + s) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const cpx<R> v = ldc(p, (size_t)c * g.Vs + s);
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
    double2 *o = dst + (size_t)r * 12 * g.Vs;
#pragma unroll
    for (int c = 0; c < 12; ++c) o[(size_t)c * g.Vs + s] = k ? p[c] : make_double2(0.0, 0.0);
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
    double2 *o = dst + (size_t)r * 12 * g.Vs;
    const double2 *p = xb + ((size_t)r * nb + (k < 0 ? 0 : k)) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) o[(size_t)c * g.Vs + s] = k >= 0 ? p[c] : make_double2(0.0, 0.0);
}

// ------------------------------------------------------------------ launchers
static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

hipError_t launch_dslash(int prec, const DslashArgs &a, int grid, hipStream_t st)
{
    if (a.SB != 256 && a.SB != 128 && a.SB != 64) return hipErrorInvalidValue;
    if (a.nrhs < 1 || a.nrhs > kMaxRhs || a.RG < 1) return hipErrorInvalidValue;
    if (grid < 8 || grid % 8) return hipErrorInvalidValue;
    dim3 blk(a.SB), grd(grid);
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(dslash_kernel<GRG_FP64>, grd, blk, 0, st, a); break;
    case GRG_FP32: hipLaunchKernelGGL(dslash_kernel<GRG_FP32>, grd, blk, 0, st, a); break;
    case GRG_BF16: hipLaunchKernelGGL(dslash_kernel<GRG_BF16>, grd, blk, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
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
