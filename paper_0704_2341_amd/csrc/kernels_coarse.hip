// b = D_rb x_b: the hopping term from the coarse sites onto the rest sites
// (section 1, step 1's block D_rb) for a field that is nonzero on the coarse
// sites only.  A rest site takes the hops from those of its eight neighbours
// that are coarse (with the all-even coarse set, two neighbours for a site
// with one odd coordinate, none otherwise), read straight from the canonical
// coarse vector; the full stencil over a field that is zero on 15 of 16 sites
// would read every neighbour.  Output: the internal FP64 field, zero on the
// coarse sites.
#include <algorithm>

#include "common.h"
#include "engine.h"
#include "stencil.h"

namespace grg {

template <int MU>
__device__ __forceinline__ void rb_hops(cpx<double> (&acc)[12], int s, const SiteGeo &q, const Geom &g,
                                        const double2 *__restrict__ xb, const int32_t *__restrict__ bidx,
                                        int nb, int r, const double2 *__restrict__ U)
{
    int sp, sm;
    nbr(s, MU, q, g, sp, sm);
    const int kp = bidx[sp], km = bidx[sm];
    if (kp >= 0) {
        cpx<double> p[12], u[9];
        const double2 *v = xb + ((size_t)r * nb + kp) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = {v[c].x, v[c].y};
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const double2 w = U[lidx(s, MU, e)];
            u[e] = {w.x, w.y};
        }
        hop_math<MU, true>(acc, p, u);
    }
    if (km >= 0) {
        cpx<double> p[12], u[9];
        const double2 *v = xb + ((size_t)r * nb + km) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = {v[c].x, v[c].y};
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const double2 w = U[lidx(sm, MU, e)];
            u[e] = {w.x, w.y};
        }
        hop_math<MU, false>(acc, p, u);
    }
}

// Work items (block of 256 sites, RHS) with the RHS fastest, one contiguous
// range per XCD: the RHS of a site block run side by side in one L2 and share
// its links and neighbour lists.  partials[workgroup][r]: the workgroup's sum
// of |out|^2 for RHS r.  PP >= 0: b also written, in precision PP, into the
// compact even-odd pair `pair` (parity `first` at compact index s / 2, the
// other parity `half` elements on), the reduced solve's right-hand side.
template <int PP>
__global__ void __launch_bounds__(256) rb_apply_kernel(Geom g, const double2 *__restrict__ xb,
                                                       const int32_t *__restrict__ bidx, int nb,
                                                       const double2 *__restrict__ U, double2 *__restrict__ out,
                                                       int nrhs, double *partials, void *pair, size_t half,
                                                       int first)
{
    __shared__ double red[4][kMaxRhs];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = lane; i < nrhs; i += 64) red[wave][i] = 0.0;
    const int nsb = (g.V + 255) >> 8;
    const ItemRange it = xcd_items(nsb * nrhs);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int sb = w / nrhs, r = w - sb * nrhs;
        const int s = sb * 256 + (int)threadIdx.x;
        double n2 = 0;
        if (s < g.V) {
            cpx<double> acc[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
            if (bidx[s] < 0) {
                const SiteGeo q = site_geo(s, g);
                rb_hops<0>(acc, s, q, g, xb, bidx, nb, r, U);
                rb_hops<1>(acc, s, q, g, xb, bidx, nb, r, U);
                rb_hops<2>(acc, s, q, g, xb, bidx, nb, r, U);
                rb_hops<3>(acc, s, q, g, xb, bidx, nb, r, U);
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                out[fidx(s, r, c, nrhs)] = make_double2(acc[c].re, acc[c].im);
                n2 += acc[c].re * acc[c].re + acc[c].im * acc[c].im;
            }
            if constexpr (PP >= 0) {
                typedef typename Store<PP>::S SP;
                typedef typename Store<PP>::R RP;
                const SiteGeo q = site_geo(s, g);
                const size_t base =
                    (((q.c[0] + q.c[1] + q.c[2] + q.c[3]) & 1) == first ? 0 : half) + fidx(s >> 1, r, 0, nrhs);
#pragma unroll
                for (int c = 0; c < 12; ++c) stc((SP *)pair, base + 64 * c, cpx<RP>{(RP)acc[c].re, (RP)acc[c].im});
            }
        }
        n2 = wave_sum(n2);  // every lane of the wavefront takes part
        if (lane == 0) red[wave][r] += n2;
    }
    if (partials) {
        __syncthreads();
        for (int i = threadIdx.x; i < nrhs; i += blockDim.x)
            partials[(size_t)blockIdx.x * nrhs + i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    }
}

int rb_apply_grid(const Geom &g)
{
    // whole XCD shares: a multiple of 8 workgroups, at least 8
    const long n = std::min<long>(((long)g.V + 255) / 256 * 4, 2048);
    return (int)std::max<long>(8, (n + 7) / 8 * 8);
}

hipError_t launch_rb_apply(const Geom &g, const double *xb, const int32_t *bidx, int nb, const void *U64,
                           void *out, int nrhs, hipStream_t st, double *partials, int pair_prec, void *pair,
                           size_t half, int first)
{
    if (nrhs < 1 || nrhs > kMaxRhs || nb < 1) return hipErrorInvalidValue;
#define RBA(PP)                                                                                        \
    hipLaunchKernelGGL(rb_apply_kernel<PP>, dim3(rb_apply_grid(g)), dim3(256), 0, st, g, (const double2 *)xb, \
                       bidx, nb, (const double2 *)U64, (double2 *)out, nrhs, partials, pair, half, first)
    switch (pair ? pair_prec : -1) {
    case -1: RBA(-1); break;
    case GRG_FP64: RBA(GRG_FP64); break;
    case GRG_FP32: RBA(GRG_FP32); break;
    case GRG_BF16: RBA(GRG_BF16); break;
    default: return hipErrorInvalidValue;
    }
#undef RBA
    return hipGetLastError();
}

}  // namespace grg

namespace grg {

// y_b = [D w]_b with w = u + sigma sum_j f_j e_j, u = x_b on the coarse sites
// (zero elsewhere) and the kept corrections e_j of the D_rr solve (zero on the
// coarse sites): the S_bb apply's last step, [D (u - z)]_b, read from the
// corrections at the coarse sites' neighbours only, instead of summing the
// iterate over the whole lattice first.
// w at the neighbour n of a coarse site: x_b there if n is coarse, else
// sigma sum_j f_j e_j(n), with the loads of e_(j+1) issued before e_j is added
template <int P>
__device__ __forceinline__ void coarse_w(cpx<double> (&w)[12], int n, const double2 *__restrict__ xb,
                                         const int32_t *__restrict__ bidx, int nb, int r, int nrhs,
                                         const CombineArgs &a)
{
    typedef typename Store<P>::S S;
    const int kb = bidx[n];
    if (kb >= 0) {
        const double2 *v = xb + ((size_t)r * nb + kb) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) w[c] = {v[c].x, v[c].y};
        return;
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = {0, 0};
    if (a.n < 1) return;
    S cur[12], nxt[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) cur[c] = ((const S *)a.e[0])[fidx(n, r, c, nrhs)];
#pragma unroll 1
    for (int j = 0; j < a.n; ++j) {
        if (j + 1 < a.n) {
            const S *e = (const S *)a.e[j + 1];
#pragma unroll
            for (int c = 0; c < 12; ++c) nxt[c] = e[fidx(n, r, c, nrhs)];
        }
        const double f = a.sigma * a.f[j * kMaxRhs + r];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const cpx<double> ev = ldr<double>(cur, c);
            w[c].re = fma(f, ev.re, w[c].re);
            w[c].im = fma(f, ev.im, w[c].im);
            cur[c] = nxt[c];
        }
    }
}

template <int P>
__global__ void __launch_bounds__(256) coarse_combine_apply_kernel(Geom g, const double2 *__restrict__ xb,
                                                                   const int32_t *__restrict__ qsites,
                                                                   const int32_t *__restrict__ bidx, int nb,
                                                                   const double2 *__restrict__ U, double diag,
                                                                   CombineArgs a, double2 *__restrict__ yb,
                                                                   int nrhs)
{
    // work items (block of 256 coarse sites, RHS), RHS fastest, one
    // contiguous range per XCD: the RHS of a block share its links in L2
    const int nkb = (nb + 255) >> 8;
    const ItemRange it = xcd_items(nkb * nrhs);
    for (int wi = it.begin; wi < it.end; wi += it.step) {
        const int kb = wi / nrhs, r = wi - kb * nrhs;
        const int k = kb * 256 + (int)threadIdx.x;
        if (k >= nb) continue;
        const int s = qsites[k];
        const SiteGeo q = site_geo(s, g);
        cpx<double> acc[12];
        const double2 *v = xb + ((size_t)r * nb + k) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {diag * v[c].x, diag * v[c].y};
        // one hop per iteration (+x, -x, ..., -t): the FP64 operands of a hop
        // are 84 registers, so the hops are not unrolled
#pragma unroll 1
        for (int h = 0; h < 8; ++h) {
            const int mu = h >> 1;
            int sp, sm;
            nbr(s, mu, q, g, sp, sm);
            const int n = (h & 1) ? sm : sp;
            cpx<double> w[12], u[9];
            coarse_w<P>(w, n, xb, bidx, nb, r, nrhs, a);
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                const double2 x = U[lidx((h & 1) ? sm : s, mu, e)];
                u[e] = {x.x, x.y};
            }
            switch (h) {
            case 0: hop_math<0, true>(acc, w, u); break;
            case 1: hop_math<0, false>(acc, w, u); break;
            case 2: hop_math<1, true>(acc, w, u); break;
            case 3: hop_math<1, false>(acc, w, u); break;
            case 4: hop_math<2, true>(acc, w, u); break;
            case 5: hop_math<2, false>(acc, w, u); break;
            case 6: hop_math<3, true>(acc, w, u); break;
            default: hop_math<3, false>(acc, w, u); break;
            }
        }
        double2 *o = yb + ((size_t)r * nb + k) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = make_double2(acc[c].re, acc[c].im);
    }
}

hipError_t launch_coarse_combine_apply(int prec, const Geom &g, const double *xb, const int32_t *qsites,
                                       const int32_t *bidx, int nb, const void *U64, double diag,
                                       const CombineArgs &a, double *yb, int nrhs, hipStream_t st)
{
    if (nrhs < 1 || nrhs > kMaxRhs || nb < 1 || a.n < 0 || a.n > kCorrPool) return hipErrorInvalidValue;
    const long items = (long)(nb + 255) / 256 * nrhs;
    dim3 grd((unsigned)std::max<long>(8, (std::min<long>(items, 2048) + 7) / 8 * 8)), blk(256);
#define CCA(PP)                                                                                        \
    hipLaunchKernelGGL(coarse_combine_apply_kernel<PP>, grd, blk, 0, st, g, (const double2 *)xb, qsites, bidx, nb, \
                       (const double2 *)U64, diag, a, (double2 *)yb, nrhs)
    switch (prec) {
    case GRG_FP64: CCA(GRG_FP64); break;
    case GRG_FP32: CCA(GRG_FP32); break;
    case GRG_BF16: CCA(GRG_BF16); break;
    default: return hipErrorInvalidValue;
    }
#undef CCA
    return hipGetLastError();
}

}  // namespace grg
