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
#include "stencil.h"

namespace grg {

// out = mask_sel D in, for nrhs fields.  With a.partials set, also the
// per-workgroup partial sums of conj(out).in (re, im) and |out|^2 per RHS.
template <int P, int SPLIT>
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
    const int nitems = nsb * ngroups;
    const int C = a.chunk > 0 ? a.chunk : (nitems + 7) / 8;
    for (int j = blockIdx.x >> 3;; j += gridDim.x >> 3) {
        const int w = xcd_chunk_item(j, C, nitems);
        if (w < 0) break;
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
                // a site's 12 terms in the compute precision, the sums over
                // sites and workgroups in FP64
                R sre = 0, sim = 0, sqq = 0;
                if (on) {
                    const S *dw = a.dot_with ? (const S *)a.dot_with : in;
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const cpx<R> v = ldc(dw, fidx(s, r, c, a.nrhs));
                        sre = fma(acc[c].re, v.re, fma(acc[c].im, v.im, sre));
                        sim = fma(acc[c].re, v.im, fma(-acc[c].im, v.re, sim));
                        sqq = fma(acc[c].re, acc[c].re, fma(acc[c].im, acc[c].im, sqq));
                    }
                }
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

// t-marching stencil.  A workgroup owns 64 sites of one x-y-z plane (one
// wavefront of sites) for RG right-hand sides (one wavefront per RHS), over a
// chunk of T consecutive time slices, and walks t upwards.  psi(t) is loaded
// once and used three times from registers: as the diagonal term of site t,
// in the backward t-hop of site t+1 and in the forward t-hop of site t-1;
// U_t(t) serves the backward hop of t+1 now and the forward hop of t on the
// next step.  The t-neighbours, whose reuse distance (a whole 3-d slice) no L2
// can hold at this footprint, thus cost nothing beyond the slice itself, and
// the links of a site are read once for all RG right-hand sides (the RG
// wavefronts of a workgroup request the same lines together).
// Epilogues of the t-marching stencil: what happens to the finished sum acc of
// site s, RHS r.  K partial sums per RHS are accumulated per workgroup.
//
// StoreEpi: out = acc on the selected rows (zero elsewhere), with the solver's
// fused sums conj(out).w (re, im) and |out|^2, w = dot_with or in.
template <int P>
struct StoreEpi {
    typedef typename Store<P>::S SIN;
    typedef SIN SU;
    typedef typename Store<P>::R R;
    typedef DslashArgs Args;
    static constexpr int K = 3;
    static constexpr int kThreads = P == GRG_FP64 ? 512 : 768;
    __device__ static const SIN *input(const Args &a) { return (const SIN *)a.in; }
    __device__ static const SU *links(const Args &a) { return (const SU *)a.U; }
    __device__ static double *partials(const Args &a) { return a.partials; }
    __device__ static void store(const Args &a, cpx<R> (&acc)[12], int s, int r, bool valid,
                                 double (&dot)[K])
    {
        if (!valid) return;
        const bool on = a.mask == nullptr || a.mask[s] == a.sel;
        SIN *out = (SIN *)a.out;
        const SIN *w = (const SIN *)(a.dot_with ? a.dot_with : a.in);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const size_t i = fidx(s, r, c, a.nrhs);
            const cpx<R> o = on ? acc[c] : cpx<R>{0, 0};
            stc(out, i, o);
            if (a.partials && on) {
                const cpx<R> v = ldc(w, i);
                dot[0] += (double)o.re * v.re + (double)o.im * v.im;
                dot[1] += (double)o.re * v.im - (double)o.im * v.re;
                dot[2] += (double)o.re * o.re + (double)o.im * o.im;
            }
        }
    }
};

// DcEpi: one FP64 defect-correction step on the rest sites (see
// dc_update_kernel): r_out = r_in - f acc, x_out = x_in + f e (skipped when
// x_out is null: the caller sums the corrections itself), r_next =
// s_next r_out, and |r_out|^2.  The stencil of e runs in FP64 with FP64 links.
// The defect correction's residual element i, stored in FP64 or (late steps,
// DcArgs::r_in32 / r_out32) in FP32 at the same element index.
__device__ __forceinline__ double2 dc_load_r(const DcArgs &a, const double2 *r, size_t i)
{
    if (a.r_in32) {
        const float2 v = ((const float2 *)r)[i];
        return make_double2((double)v.x, (double)v.y);
    }
    return r[i];
}
__device__ __forceinline__ void dc_store_r(const DcArgs &a, double2 *r, size_t i, double2 v)
{
    if (a.r_out32) ((float2 *)r)[i] = make_float2((float)v.x, (float)v.y);
    else r[i] = v;
}

// Where r_next's element (r, c) of site s goes: the full layout (i), or the
// compact half of the site's parity at its compact index s / 2.
struct DcNext {
    size_t base = 0;
    int hs;
    bool compact;
    __device__ DcNext(const DcArgs &a, int s) : hs(s), compact(a.next_half != 0)
    {
        if (compact) {
            const SiteGeo q = site_geo(s, a.g);
            base = ((q.c[0] ^ q.c[1] ^ q.c[2] ^ q.c[3]) & 1) == a.next_par ? 0 : a.next_half;
            hs = s >> 1;
        }
    }
    __device__ size_t at(size_t i, int r, int c, int nrhs) const
    {
        return compact ? base + fidx(hs, r, c, nrhs) : i;
    }
};

template <int P>
struct DcEpi {
    typedef typename Store<P>::S SIN;
    typedef double2 SU;
    typedef double R;
    typedef DcArgs Args;
    static constexpr int K = 1;
    static constexpr int kThreads = 512;
    static constexpr bool kGroupOrder = true;  // Args carries grp_first
    __device__ static const SIN *input(const Args &a) { return (const SIN *)a.e; }
    __device__ static const SU *links(const Args &a) { return (const SU *)a.U; }
    __device__ static double *partials(const Args &a) { return a.partials; }
    __device__ static void store(const Args &a, cpx<double> (&acc)[12], int s, int r, bool valid,
                                 double (&nrm)[K])
    {
        if (!valid) return;
        typedef typename Store<P>::R RN;
        const bool on = a.mask[s] == 0;
        const double2 *r_in = (const double2 *)a.r_in;
        const double2 *x_in = (const double2 *)a.x_in;
        double2 *r_out = (double2 *)a.r_out;
        double2 *x_out = (double2 *)a.x_out;
        SIN *r_next = (SIN *)a.r_next;
        const SIN *e = (const SIN *)a.e;
        const double f = a.f[r];
        const double sn = r_next ? a.s_next[r] : 0.0;
        const DcNext nx(a, s);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            // three components at a time: a compiler barrier keeps the
            // streams' loads from being hoisted all at once (registers)
            if (c % 3 == 0) asm volatile("" ::: "memory");
            const size_t i = fidx(s, r, c, a.nrhs);
            if (on) {
                const double2 rv = dc_load_r(a, r_in, i);
                const double2 d = make_double2(rv.x - f * acc[c].re, rv.y - f * acc[c].im);
                dc_store_r(a, r_out, i, d);
                if (r_next) stc(r_next, nx.at(i, r, c, a.nrhs), cpx<RN>{(RN)(sn * d.x), (RN)(sn * d.y)});
                nrm[0] += d.x * d.x + d.y * d.y;
                if (x_out) {
                    const cpx<double> ev = ldr<double>(e, i);
                    const double2 xv = x_in ? x_in[i] : make_double2(0.0, 0.0);
                    x_out[i] = make_double2(xv.x + f * ev.re, xv.y + f * ev.im);
                }
            } else {
                dc_store_r(a, r_out, i, make_double2(0.0, 0.0));
                if (x_out) x_out[i] = make_double2(0.0, 0.0);
                if (r_next) stc(r_next, nx.at(i, r, c, a.nrhs), cpx<RN>{0, 0});
            }
        }
    }
};

// t-marching stencil.  A workgroup owns 64 sites of one x-y-z plane (one
// wavefront of sites) for RG right-hand sides (one wavefront per RHS), over a
// chunk of T consecutive time slices, and walks t upwards.  psi(t) is loaded
// once and used three times from registers: as the diagonal term of site t,
// in the backward t-hop of site t+1 and in the forward t-hop of site t-1;
// U_t(t) serves the backward hop of t+1 now and the forward hop of t on the
// next step.  The t-neighbours, whose reuse distance (a whole 3-d slice) no L2
// can hold at this footprint, thus cost nothing beyond the slice itself, and
// the links of a site are read once for all RG right-hand sides (the RG
// wavefronts of a workgroup request the same lines together).  Wavefront wv
// of an item with RHS group grp holds RHS grp * RG + wv, so it only ever sees
// RHS with r % RG == wv: the per-RHS sums of the workgroup's items go to LDS
// rows no other wavefront writes.
template <class E>
__global__ void __launch_bounds__(E::kThreads) march_kernel(typename E::Args a)
{
    typedef typename E::SIN S;
    typedef typename E::SU SU;
    typedef typename E::R R;
    typedef Operand<S, R> OP;
    typedef Operand<SU, R> OU;
    typedef typename OP::T PT;
    typedef typename OU::T UT;
    constexpr int K = E::K;
    __shared__ double red[kMaxRhs][K];
    const S *__restrict__ in = E::input(a);
    const SU *__restrict__ U = E::links(a);
    double *partials = E::partials(a);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (partials) {
        for (int i = threadIdx.x; i < kMaxRhs * K; i += blockDim.x) red[i / K][i % K] = 0.0;
        __syncthreads();
    }
    const int V3 = a.g.L[0] * a.g.L[1] * a.g.L[2], Lt = a.g.L[3];
    const int nb3 = (V3 + 63) >> 6;
    const int T = a.march;
    const int ntc = (Lt + T - 1) / T;
    const int ngroups = (a.nrhs + a.RG - 1) / a.RG;
    const int nitems = nb3 * ntc * ngroups;
    const R diag = (R)a.diag;
    double dot[K];
#pragma unroll
    for (int k = 0; k < K; ++k) dot[k] = 0.0;
    const int C = a.chunk > 0 ? a.chunk : (nitems + 7) / 8;
    for (int j = blockIdx.x >> 3;; j += gridDim.x >> 3) {
        const int w = xcd_chunk_item(j, C, nitems);
        if (w < 0) break;
        const int b3 = w % nb3, rest = w / nb3;
        const int grp = rest % ngroups, tc = rest / ngroups;
        const int s3 = b3 * 64 + lane;
        const int r = grp * a.RG + wv;
        if (r >= a.nrhs) continue;  // whole wavefront idles
        const bool valid = s3 < V3;
        const int s3c = valid ? s3 : 0;  // keep idle lanes' addresses in range
        const int t0 = tc * T, t1 = min(t0 + T, Lt);
        SiteGeo q = site_geo(s3c, a.g);
        // prologue: backward t-hop of site t0 from psi(t0 - 1)
        cpx<R> acc_cur[12], acc_prev[12];
        UT ut_prev[9];
        {
            const int sm = s3c + V3 * (t0 == 0 ? Lt - 1 : t0 - 1);
            PT p[12];
            UT u[9];
#pragma unroll
            for (int c = 0; c < 12; ++c) p[c] = OP::load(in, fidx(sm, r, c, a.nrhs));
#pragma unroll
            for (int e = 0; e < 9; ++e) u[e] = OU::load(U, lidx(sm, 3, e));
#pragma unroll
            for (int c = 0; c < 12; ++c) acc_cur[c] = {0, 0};
            hop<3, false>(acc_cur, p, u);
        }
#pragma unroll 1
        for (int t = t0; t < t1; ++t) {
            const int s = s3c + V3 * t;
            q.c[3] = t;
            PT psi[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) psi[c] = OP::load(in, fidx(s, r, c, a.nrhs));
            // wide (FP64) psi is not kept live across the x, y, z hops: it is
            // loaded again (from cache) for the backward t-hop below
            constexpr bool kKeep = sizeof(PT) <= 8;
            if (t > t0) {  // finish site t - 1 with its forward t-hop
                hop<3, true>(acc_prev, psi, ut_prev);
                E::store(a, acc_prev, s - V3, r, valid, dot);
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const auto v = as_cpx(psi[c]);
                acc_cur[c].re += diag * (R)v.re;
                acc_cur[c].im += diag * (R)v.im;
            }
#pragma unroll 1
            for (int h = 0; h < 6; ++h) {  // x, y, z hops, one at a time
                const int mu = h >> 1;
                int sp, sm;
                nbr(s, mu, q, a.g, sp, sm);
                const int n = (h & 1) ? sm : sp;
                PT p[12];
                UT u[9];
#pragma unroll
                for (int c = 0; c < 12; ++c) p[c] = OP::load(in, fidx(n, r, c, a.nrhs));
#pragma unroll
                for (int e = 0; e < 9; ++e) u[e] = OU::load(U, lidx((h & 1) ? sm : s, mu, e));
                switch (h) {
                case 0: hop<0, true>(acc_cur, p, u); break;
                case 1: hop<0, false>(acc_cur, p, u); break;
                case 2: hop<1, true>(acc_cur, p, u); break;
                case 3: hop<1, false>(acc_cur, p, u); break;
                case 4: hop<2, true>(acc_cur, p, u); break;
                default: hop<2, false>(acc_cur, p, u); break;
                }
            }
            // backward t-hop of site t + 1, from psi(t) and U_t(t)
#pragma unroll
            for (int e = 0; e < 9; ++e) ut_prev[e] = OU::load(U, lidx(s, 3, e));
            if (!kKeep) {
#pragma unroll
                for (int c = 0; c < 12; ++c) psi[c] = OP::load(in, fidx(s, r, c, a.nrhs));
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                acc_prev[c] = acc_cur[c];
                acc_cur[c] = {0, 0};
            }
            hop<3, false>(acc_cur, psi, ut_prev);
        }
        // epilogue: forward t-hop of site t1 - 1 from psi(t1)
        {
            const int sp = s3c + V3 * (t1 == Lt ? 0 : t1);
            PT p[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) p[c] = OP::load(in, fidx(sp, r, c, a.nrhs));
            hop<3, true>(acc_prev, p, ut_prev);
            E::store(a, acc_prev, s3c + V3 * (t1 - 1), r, valid, dot);
        }
        if (partials) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double t = wave_sum(dot[k]);
                if (lane == 0) red[r][k] += t;
                dot[k] = 0.0;
            }
        }
    }
    if (partials) {
        __syncthreads();
        for (int i = threadIdx.x; i < a.nrhs * K; i += blockDim.x)
            partials[(size_t)blockIdx.x * a.nrhs * K + i] = red[i / K][i % K];
    }
}

// LDS-ring form of the t-marching stencil for packed BF16 input (the fused
// defect-correction step of a BF16 inner solve).  As march_kernel, a
// workgroup holds 64 sites of a 3-d slice for RG RHS and walks t, but each
// site is finished within its own slice: the column's input at t - 1 and t
// waits in an LDS ring (two slots per wavefront, each lane writing its own
// column), so the backward t hop and the x hops (the sites of the same
// x-row, lanes of the same wavefront) read LDS, and no second FP64
// accumulator is carried from one slice to the next.  The hops of a site are
// summed in march_kernel's order (backward t, diagonal, x, y, z, forward t).
constexpr int kRingWaves = 4;  // wavefronts (RHS) per workgroup of the LDS-ring form
template <class E>
__global__ void __launch_bounds__(64 * kRingWaves) ring_march_kernel(typename E::Args a)
{
    typedef typename E::SIN S;
    typedef typename E::SU SU;
    typedef typename E::R R;
    typedef Operand<S, R> OP;
    typedef Operand<SU, R> OU;
    typedef typename OP::T PT;
    typedef typename OU::T UT;
    static_assert(sizeof(PT) == 4, "the LDS ring holds packed BF16 words");
    constexpr int K = E::K;
    __shared__ PT ring[kRingWaves][2][12][64];
    // per wavefront, U_t of its column at the previous slice: the backward t
    // link of this slice (the forward one of the last), kept from there
    __shared__ double2 utl[kRingWaves][9][64];
    __shared__ double red[kMaxRhs][K];
    const S *__restrict__ in = E::input(a);
    const SU *__restrict__ U = E::links(a);
    double *partials = E::partials(a);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (partials) {
        for (int i = threadIdx.x; i < kMaxRhs * K; i += blockDim.x) red[i / K][i % K] = 0.0;
        __syncthreads();
    }
    const int Lx = a.g.L[0];
    const int V3 = Lx * a.g.L[1] * a.g.L[2], Lt = a.g.L[3];
    const int nb3 = V3 >> 6;  // whole tiles (V3 a multiple of 64)
    const int T = a.march;
    const int ntc = (Lt + T - 1) / T;
    const int ngroups = (a.nrhs + a.RG - 1) / a.RG;
    const int nitems = nb3 * ntc * ngroups;
    const R diag = (R)a.diag;
    // the x neighbours' lanes: x-rows of Lx sites tile the 64 lanes
    const int xh = lane % Lx, rs = lane - xh;
    const int lp = rs + (xh + 1 == Lx ? 0 : xh + 1), lm = rs + (xh == 0 ? Lx - 1 : xh - 1);
    PT (*q)[12][64] = ring[wv];
    double2 (*ut)[64] = utl[wv];
    double dot[K];
#pragma unroll
    for (int k = 0; k < K; ++k) dot[k] = 0.0;
    const int C = a.chunk > 0 ? a.chunk : (nitems + 7) / 8;
    for (int j = blockIdx.x >> 3;; j += gridDim.x >> 3) {
        const int w = xcd_chunk_item(j, C, nitems);
        if (w < 0) break;
        int b3, grp, tc;
        if (E::kGroupOrder && a.grp_first) {
            // the RHS groups of a tile adjacent: they run together on one
            // XCD and share the tile's links through its L2; with one
            // contiguous eighth of the items per XCD, each XCD walks a slab
            // of z-planes
            grp = w % ngroups;
            const int rest = w / ngroups;
            b3 = rest % nb3;
            tc = rest / nb3;
        } else {
            b3 = w % nb3;
            const int rest = w / nb3;
            grp = rest % ngroups;
            tc = rest / ngroups;
        }
        const int s3 = b3 * 64 + lane;
        const int r = grp * a.RG + wv;
        if (r >= a.nrhs) continue;  // whole wavefront idles
        const int t0 = tc * T, t1 = min(t0 + T, Lt);
        SiteGeo g3 = site_geo(s3, a.g);
        // slot (t & 1) holds slice t (counted from t0, so an odd Lt wraps too)
        {
            const int tm = t0 == 0 ? Lt - 1 : t0 - 1;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                q[(t0 - 1) & 1][c][lane] = OP::load(in, fidx(s3 + V3 * tm, r, c, a.nrhs));
                q[t0 & 1][c][lane] = OP::load(in, fidx(s3 + V3 * t0, r, c, a.nrhs));
            }
            // U_t one slice below t0 (each lane reads back only its own entries)
#pragma unroll
            for (int e = 0; e < 9; ++e) ut[e][lane] = ((const double2 *)U)[lidx(s3 + V3 * tm, 3, e)];
        }
#pragma unroll 1
        for (int t = t0; t < t1; ++t) {
            const int s = s3 + V3 * t;
            g3.c[3] = t;
            const int tf = t + 1 == Lt ? 0 : t + 1, tb = t == 0 ? Lt - 1 : t - 1;
            // the forward t-neighbour: used at the end of this slice, then
            // kept in the ring for the next two
            PT qc[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) qc[c] = OP::load(in, fidx(s3 + V3 * tf, r, c, a.nrhs));
            cpx<R> acc[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
            {
                PT p[12];
                UT u[9];
#pragma unroll
                for (int e = 0; e < 9; ++e) {
                    const double2 w = ut[e][lane];
                    u[e] = {w.x, w.y};
                }
#pragma unroll
                for (int c = 0; c < 12; ++c) p[c] = q[(t - 1) & 1][c][lane];
                hop<3, false>(acc, p, u);
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const auto v = as_cpx(q[t & 1][c][lane]);
                acc[c].re += diag * (R)v.re;
                acc[c].im += diag * (R)v.im;
            }
#pragma unroll 1
            for (int h = 0; h < 6; ++h) {  // x hops from the ring, y and z hops loaded
                const int mu = h >> 1;
                int sp, sm;
                nbr(s, mu, g3, a.g, sp, sm);
                PT p[12];
                UT u[9];
                if (h < 2) {
                    const int l = h == 0 ? lp : lm;
#pragma unroll
                    for (int c = 0; c < 12; ++c) p[c] = q[t & 1][c][l];
                } else {
                    const int n = (h & 1) ? sm : sp;
#pragma unroll
                    for (int c = 0; c < 12; ++c) p[c] = OP::load(in, fidx(n, r, c, a.nrhs));
                }
#pragma unroll
                for (int e = 0; e < 9; ++e) u[e] = OU::load(U, lidx((h & 1) ? sm : s, mu, e));
                switch (h) {
                case 0: hop<0, true>(acc, p, u); break;
                case 1: hop<0, false>(acc, p, u); break;
                case 2: hop<1, true>(acc, p, u); break;
                case 3: hop<1, false>(acc, p, u); break;
                case 4: hop<2, true>(acc, p, u); break;
                default: hop<2, false>(acc, p, u); break;
                }
            }
            {
                UT u[9];
#pragma unroll
                for (int e = 0; e < 9; ++e) u[e] = OU::load(U, lidx(s, 3, e));
                hop<3, true>(acc, qc, u);
                // the backward t link of the next slice
#pragma unroll
                for (int e = 0; e < 9; ++e) ut[e][lane] = make_double2(u[e].re, u[e].im);
            }
            // slice t + 1 into the slot of slice t - 1 (read above by this
            // lane only)
#pragma unroll
            for (int c = 0; c < 12; ++c) q[(t + 1) & 1][c][lane] = qc[c];
            E::store(a, acc, s, r, true, dot);
        }
        if (partials) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double t = wave_sum(dot[k]);
                if (lane == 0) red[r][k] += t;
                dot[k] = 0.0;
            }
        }
    }
    if (partials) {
        __syncthreads();
        for (int i = threadIdx.x; i < a.nrhs * K; i += blockDim.x)
            partials[(size_t)blockIdx.x * a.nrhs * K + i] = red[i / K][i % K];
    }
}

// One FP64 defect-correction step, fused.  e is the inner solution (stored in
// precision P, zero on coarse sites) of A e = r_in / f_k:
//     r_out = r_in - f (D_rr e)        x_out = x_in + f e        (FP64;
// r_in / r_out stored in FP32 instead with DcArgs::r_in32 / r_out32)
// on the r-sites; coarse sites are written as zero.  x_out == nullptr skips
// the iterate (the caller keeps the corrections); x_in == nullptr reads as
// zero.  With r_next set, also r_next = s_next r_out in precision P (the next
// inner right-hand side), and always the per-workgroup partial sums of
// |r_out|^2 per RHS.  r_out may alias r_in and x_out may alias x_in (each
// thread touches only its own site).
template <int P>
__global__ void __launch_bounds__(256) dc_update_kernel(DcArgs a)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    __shared__ double red[4][kMaxRhs];
    const S *__restrict__ e = (const S *)a.e;
    const double2 *__restrict__ U = (const double2 *)a.U;
    const double2 *r_in = (const double2 *)a.r_in;
    const double2 *x_in = (const double2 *)a.x_in;
    double2 *r_out = (double2 *)a.r_out;
    double2 *x_out = (double2 *)a.x_out;
    S *r_next = (S *)a.r_next;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = lane; i < a.nrhs; i += 64) red[wave][i] = 0.0;
    __syncthreads();
    const int nsb = (a.g.V + blockDim.x - 1) / blockDim.x;
    const ItemRange it = xcd_items(nsb);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int s = w * blockDim.x + (int)threadIdx.x;
        const bool valid = s < a.g.V;
        const bool on = valid && a.mask[s] == 0;
        SiteGeo q;
        if (on) q = site_geo(s, a.g);
        for (int r = 0; r < a.nrhs; ++r) {
            double nrm = 0;
            if (on) {
                cpx<double> acc[12];
                dslash_site<S, double, true, double2>(acc, e, U, s, q, a.g, r, a.nrhs, a.diag);
                const double f = a.f[r];
                const double sn = r_next ? a.s_next[r] : 0.0;
                const DcNext nx(a, s);
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const size_t i = fidx(s, r, c, a.nrhs);
                    const double2 rv = dc_load_r(a, r_in, i);
                    const double2 d = make_double2(rv.x - f * acc[c].re, rv.y - f * acc[c].im);
                    dc_store_r(a, r_out, i, d);
                    if (r_next) stc(r_next, nx.at(i, r, c, a.nrhs), cpx<R>{(R)(sn * d.x), (R)(sn * d.y)});
                    nrm += d.x * d.x + d.y * d.y;
                    if (x_out) {
                        const cpx<double> ev = ldr<double>(e, i);
                        const double2 xv = x_in ? x_in[i] : make_double2(0.0, 0.0);
                        x_out[i] = make_double2(xv.x + f * ev.re, xv.y + f * ev.im);
                    }
                }
            } else if (valid) {
                const DcNext nx(a, s);
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const size_t i = fidx(s, r, c, a.nrhs);
                    dc_store_r(a, r_out, i, make_double2(0.0, 0.0));
                    if (x_out) x_out[i] = make_double2(0.0, 0.0);
                    if (r_next) stc(r_next, nx.at(i, r, c, a.nrhs), cpx<R>{0, 0});
                }
            }
            nrm = wave_sum(nrm);
            if (lane == 0) red[wave][r] += nrm;
        }
    }
    __syncthreads();
    const int nw = blockDim.x >> 6;
    for (int i = threadIdx.x; i < a.nrhs; i += blockDim.x) {
        double t = 0;
        for (int k = 0; k < nw; ++k) t += red[k][i];
        a.partials[(size_t)blockIdx.x * a.nrhs + i] = t;
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
// mask != nullptr: sites with mask[s] != keep are written as zero
template <int P>
__global__ void pack_spinor_kernel(const double2 *__restrict__ src, void *dst, Geom g, int nrhs,
                                   const uint8_t *__restrict__ mask, int keep)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V || r >= nrhs) return;
    const bool k = mask == nullptr || mask[s] == keep;
    const double2 *p = src + ((size_t)r * g.V + s) * 12;
    S *o = (S *)dst;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 v = k ? p[c] : make_double2(0.0, 0.0);
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
    if (a.nrhs < 1 || a.nrhs > kMaxRhs || a.RG < 1) return hipErrorInvalidValue;
    if (grid < 8 || grid % 8) return hipErrorInvalidValue;
    if (a.march > 0) {
        // one wavefront per RHS of a group
        if (64 * a.RG > (prec == GRG_FP64 ? 512 : 768)) return hipErrorInvalidValue;
        dim3 blk(64 * a.RG), grd(grid);
        switch (prec) {
        case GRG_FP64: hipLaunchKernelGGL(march_kernel<StoreEpi<GRG_FP64>>, grd, blk, 0, st, a); break;
        case GRG_FP32: hipLaunchKernelGGL(march_kernel<StoreEpi<GRG_FP32>>, grd, blk, 0, st, a); break;
        case GRG_BF16: hipLaunchKernelGGL(march_kernel<StoreEpi<GRG_BF16>>, grd, blk, 0, st, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (a.SB != 256 && a.SB != 128 && a.SB != 64) return hipErrorInvalidValue;
    dim3 blk(a.SB), grd(grid);
#define DSL(PP)                                                                                 \
    if (a.split == 2) hipLaunchKernelGGL((dslash_kernel<PP, 2>), grd, blk, 0, st, a);           \
    else if (a.split) hipLaunchKernelGGL((dslash_kernel<PP, 1>), grd, blk, 0, st, a);           \
    else hipLaunchKernelGGL((dslash_kernel<PP, 0>), grd, blk, 0, st, a);
    switch (prec) {
    case GRG_FP64: DSL(GRG_FP64) break;
    case GRG_FP32: DSL(GRG_FP32) break;
    case GRG_BF16: DSL(GRG_BF16) break;
    default: return hipErrorInvalidValue;
    }
#undef DSL
    return hipGetLastError();
}

hipError_t launch_dc_update(int prec, const DcArgs &a, int grid, int SB, hipStream_t st)
{
    if (a.nrhs < 1 || a.nrhs > kMaxRhs || grid < 8 || grid % 8) return hipErrorInvalidValue;
    if (a.march > 0 && a.ring) {
        const int V3 = a.g.L[0] * a.g.L[1] * a.g.L[2];
        if (prec != GRG_BF16 || a.RG < 1 || a.RG > kRingWaves || V3 % 64 || 64 % a.g.L[0])
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(ring_march_kernel<DcEpi<GRG_BF16>>, dim3(grid), dim3(64 * a.RG), 0, st, a);
        return hipGetLastError();
    }
    if (a.march > 0) {
        if (a.RG < 1 || 64 * a.RG > 512) return hipErrorInvalidValue;
        dim3 blk(64 * a.RG), grd(grid);
        switch (prec) {
        case GRG_FP64: hipLaunchKernelGGL(march_kernel<DcEpi<GRG_FP64>>, grd, blk, 0, st, a); break;
        case GRG_FP32: hipLaunchKernelGGL(march_kernel<DcEpi<GRG_FP32>>, grd, blk, 0, st, a); break;
        case GRG_BF16: hipLaunchKernelGGL(march_kernel<DcEpi<GRG_BF16>>, grd, blk, 0, st, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (SB != 64 && SB != 128 && SB != 256) return hipErrorInvalidValue;
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(dc_update_kernel<GRG_FP64>, dim3(grid), dim3(SB), 0, st, a); break;
    case GRG_FP32: hipLaunchKernelGGL(dc_update_kernel<GRG_FP32>, dim3(grid), dim3(SB), 0, st, a); break;
    case GRG_BF16: hipLaunchKernelGGL(dc_update_kernel<GRG_BF16>, dim3(grid), dim3(SB), 0, st, a); break;
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
                              hipStream_t st, const uint8_t *mask, int keep)
{
    dim3 grd(cdiv(g.V, 256), nrhs), blk(256);
    const double2 *s = (const double2 *)src;
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(pack_spinor_kernel<GRG_FP64>, grd, blk, 0, st, s, dst, g, nrhs, mask, keep); break;
    case GRG_FP32: hipLaunchKernelGGL(pack_spinor_kernel<GRG_FP32>, grd, blk, 0, st, s, dst, g, nrhs, mask, keep); break;
    case GRG_BF16: hipLaunchKernelGGL(pack_spinor_kernel<GRG_BF16>, grd, blk, 0, st, s, dst, g, nrhs, mask, keep); break;
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
