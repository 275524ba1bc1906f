// Many-lattice batch: every kernel covers all lattices of the batch in one
// launch.  The lattices are concatenated in the site index (each starts on a
// 256-site boundary, so no workgroup straddles two of them); a per-tile table
// names the lattice of every 64-site tile, and per-lattice tables hold the
// extents, the first site and the diagonal 4 + m0.  A "system" is one
// (lattice, right-hand side) pair, sys = lattice * nrhs + rhs; step lengths,
// norms and convergence flags are per system.
#include "batch.h"
#include "common.h"
#include "engine.h"
#include "reduce.h"
#include "stencil.h"

namespace grg {

struct BSite {
    int l;      // lattice
    Geom g;     // its geometry (V = its volume)
    int local;  // site index inside it
};

__device__ __forceinline__ BSite bsite(const BatchTable &bt, int s)
{
    BSite b;
    b.l = bt.tile_lat[s >> 6];
    const int4 d = bt.dims[b.l];
    b.g.L[0] = d.x;
    b.g.L[1] = d.y;
    b.g.L[2] = d.z;
    b.g.L[3] = d.w;
    b.g.V = d.x * d.y * d.z * d.w;
    b.g.Vs = b.g.V;
    b.local = s - bt.off[b.l];
    return b;
}

// per-wave LDS accumulators over the systems, written as one partial per
// workgroup and system at the end
template <int K>
struct SysPartial {
    double *red;  // [4 waves][nsys][K]
    int nsys;
    __device__ void init(double *smem, int n)
    {
        red = smem;
        nsys = n;
        for (int i = threadIdx.x; i < 4 * n * K; i += blockDim.x) red[i] = 0.0;
        __syncthreads();
    }
    __device__ void add(int sys, const double (&v)[K])
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double t = wave_sum(v[k]);
            if (lane == 0) red[(wave * nsys + sys) * K + k] += t;
        }
    }
    __device__ void flush(double *partials)
    {
        __syncthreads();
        const int nw = blockDim.x >> 6;
        for (int i = threadIdx.x; i < nsys * K; i += blockDim.x) {
            double t = 0;
            for (int w = 0; w < nw; ++w) t += red[w * nsys * K + i];
            partials[(size_t)blockIdx.x * nsys * K + i] = t;
        }
    }
};

// Whether any of the n flags is set: the same answer in every thread of the
// workgroup (a gate read at the start of a launch, before any barrier of the
// kernel, so a launch with nothing to do returns as a whole).
__device__ bool any_set(const int *flags, int n)
{
    __shared__ int s_any;
    if (threadIdx.x == 0) s_any = 0;
    __syncthreads();
    int mine = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) mine |= flags[i];
    if (mine) s_any = 1;
    __syncthreads();
    return s_any != 0;
}

// out = mask_sel D in over all lattices; fused dots per system when partials.
template <int P>
__global__ void __launch_bounds__(256) dslash_batch_kernel(BatchDslashArgs a)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    extern __shared__ double smem[];
    const S *__restrict__ in = (const S *)a.in;
    S *__restrict__ out = (S *)a.out;
    const S *__restrict__ U = (const S *)a.U;
    const int nsys = a.bt.nlat * a.nrhs;
    if (a.act && !any_set(a.act, nsys)) return;
    const bool dots = a.partials != nullptr;
    SysPartial<3> part;
    if (dots) part.init(smem, nsys);
    const int ngroups = (a.nrhs + a.RG - 1) / a.RG;
    const int nsb = a.Vtot / blockDim.x;  // every lattice is a whole number of blocks
    const ItemRange it = xcd_items(nsb * ngroups);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int sb = w / ngroups, grp = w - sb * ngroups;
        const int s = sb * blockDim.x + (int)threadIdx.x;
        const BSite b = bsite(a.bt, s);
        const bool on = a.mask[s] == a.sel;
        const SiteGeo q = site_geo(b.local, b.g);
        const R diag = (R)a.bt.diag[b.l];
        const int r0 = grp * a.RG, r1 = min(r0 + a.RG, a.nrhs);
        for (int r = r0; r < r1; ++r) {
            // (a workgroup lies inside one lattice: the skip is uniform)
            if (a.act && !a.act[b.l * a.nrhs + r]) continue;
            cpx<R> acc[12];
            if (on) {
                dslash_site<S, R, true>(acc, in, U, s, q, b.g, r, a.nrhs, diag);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) stc(out, fidx(s, r, c, a.nrhs), acc[c]);
            if (dots) {
                R sre = 0, sim = 0, sqq = 0;
                if (on) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const cpx<R> v = ldc(in, fidx(s, r, c, a.nrhs));
                        sre = fma(acc[c].re, v.re, fma(acc[c].im, v.im, sre));
                        sim = fma(acc[c].re, v.im, fma(-acc[c].im, v.re, sim));
                        sqq = fma(acc[c].re, acc[c].re, fma(acc[c].im, acc[c].im, sqq));
                    }
                }
                const double d[3] = {(double)sre, (double)sim, (double)sqq};
                part.add(b.l * a.nrhs + r, d);
            }
        }
    }
    if (dots) part.flush(a.partials);
}

// x += alpha r ; r -= alpha q ; partial |r|^2  (per system)
template <int P>
__global__ void __launch_bounds__(256) batch_mr_update_kernel(BatchBlasArgs a, void *x_, void *r_,
                                                              const void *q_)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    extern __shared__ double smem[];
    if (a.act && !any_set(a.act, a.bt.nlat * a.nrhs)) return;
    if (a.ctr && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.ctr, 1);
    SysPartial<1> part;
    part.init(smem, a.bt.nlat * a.nrhs);
    S *x = (S *)x_, *r = (S *)r_;
    const S *q = (const S *)q_;
    const ItemRange it = xcd_items(a.Vtot / 256);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int s = w * 256 + threadIdx.x;
        const int l = a.bt.tile_lat[s >> 6];
        for (int k = 0; k < a.nrhs; ++k) {
            const int sys = l * a.nrhs + k;
            if (a.act && !a.act[sys]) continue;  // converged: x and r stay
            const double2 a2 = a.alpha[sys];
            const cpx<R> al = {(R)a2.x, (R)a2.y}, na = {(R)-a2.x, (R)-a2.y};
            R rr = 0;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, a.nrhs);
                cpx<R> xv = ldc(x, i), rv = ldc(r, i);
                const cpx<R> qv = ldc(q, i);
                cmac(xv, al, rv);
                cmac(rv, na, qv);
                stc(x, i, xv);
                stc(r, i, rv);
                const cpx<R> rs = ldc(r, i);
                rr = fma(rs.re, rs.re, fma(rs.im, rs.im, rr));
            }
            const double v[1] = {(double)rr};
            part.add(sys, v);
        }
    }
    part.flush(a.partials);
}

template <int P>
__global__ void __launch_bounds__(256) batch_norm2_kernel(BatchBlasArgs a, const void *v_)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    extern __shared__ double smem[];
    SysPartial<1> part;
    part.init(smem, a.bt.nlat * a.nrhs);
    const S *v = (const S *)v_;
    const ItemRange it = xcd_items(a.Vtot / 256);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int s = w * 256 + threadIdx.x;
        const int l = a.bt.tile_lat[s >> 6];
        for (int k = 0; k < a.nrhs; ++k) {
            double t = 0;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const cpx<R> z = ldc(v, fidx(s, k, c, a.nrhs));
                t += (double)z.re * z.re + (double)z.im * z.im;
            }
            const double vv[1] = {t};
            part.add(l * a.nrhs + k, vv);
        }
    }
    part.flush(a.partials);
}

// y = beta*y + f(scale[sys]) * x, f = identity / 1/sqrt / sqrt
template <int PI, int PO>
__global__ void __launch_bounds__(256) batch_axpy_convert_kernel(BatchBlasArgs a, const void *x_, void *y_,
                                                                 const double *scale, int mode, int beta)
{
    typedef typename Store<PI>::S SI;
    typedef typename Store<PI>::R RI;
    typedef typename Store<PO>::S SO;
    typedef typename Store<PO>::R RO;
    const SI *x = (const SI *)x_;
    SO *y = (SO *)y_;
    const ItemRange it = xcd_items(a.Vtot / 256);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int s = w * 256 + threadIdx.x;
        const int l = a.bt.tile_lat[s >> 6];
        for (int k = 0; k < a.nrhs; ++k) {
            double f = scale ? scale[l * a.nrhs + k] : 1.0;
            if (mode == 1) f = f > 0 ? 1.0 / sqrt(f) : 0.0;
            if (mode == 2) f = sqrt(f);
            const RO fo = (RO)f;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, a.nrhs);
                const cpx<RI> v = ldc(x, i);
                cpx<RO> o = {fo * (RO)v.re, fo * (RO)v.im};
                if (beta) {
                    const cpx<RO> yo = ldc(y, i);
                    o.re += yo.re;
                    o.im += yo.im;
                }
                stc(y, i, o);
            }
        }
    }
}

__global__ void __launch_bounds__(256) batch_sub_norm_kernel(BatchBlasArgs a, const double2 *b,
                                                             const double2 *ax, double2 *r)
{
    extern __shared__ double smem[];
    SysPartial<1> part;
    part.init(smem, a.bt.nlat * a.nrhs);
    const ItemRange it = xcd_items(a.Vtot / 256);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int s = w * 256 + threadIdx.x;
        const int l = a.bt.tile_lat[s >> 6];
        for (int k = 0; k < a.nrhs; ++k) {
            double t = 0;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, a.nrhs);
                const double2 bv = b[i], av = ax[i];
                const double2 d = make_double2(bv.x - av.x, bv.y - av.y);
                r[i] = d;
                t += d.x * d.x + d.y * d.y;
            }
            const double vv[1] = {t};
            part.add(l * a.nrhs + k, vv);
        }
    }
    part.flush(a.partials);
}

// r_out = r_in - f (D_rr e), x_out = x_in + f e in FP64, f = sqrt(fr2[sys])
template <int P>
__global__ void __launch_bounds__(128) batch_dc_update_kernel(BatchDcArgs a)
{
    typedef typename Store<P>::S S;
    extern __shared__ double smem[];
    SysPartial<1> part;
    part.init(smem, a.bt.nlat * a.nrhs);
    const S *__restrict__ e = (const S *)a.e;
    const double2 *__restrict__ U = (const double2 *)a.U;
    const double2 *r_in = (const double2 *)a.r_in;
    const double2 *x_in = (const double2 *)a.x_in;
    double2 *r_out = (double2 *)a.r_out;
    double2 *x_out = (double2 *)a.x_out;
    const int nsys = a.bt.nlat * a.nrhs;
    const bool in_place = a.r_in == a.r_out && a.x_in == a.x_out;
    if (a.act) {
        const bool any = any_set(a.act, nsys);
        if (any && a.ctr && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.ctr, 1);
        if (a.gate && !any) return;
    }
    const ItemRange it = xcd_items(a.Vtot / blockDim.x);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int s = w * blockDim.x + threadIdx.x;
        const BSite b = bsite(a.bt, s);
        const bool on = a.mask[s] == 0;
        const SiteGeo q = site_geo(b.local, b.g);
        for (int r = 0; r < a.nrhs; ++r) {
            const int sys = b.l * a.nrhs + r;
            const bool sys_on = a.act == nullptr || a.act[sys] != 0;
            if (in_place && !sys_on) continue;  // converged: r and x stay
            double nrm = 0;
            if (on && !sys_on) {
                // converged before this step: r and x copied, e not read
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const size_t i = fidx(s, r, c, a.nrhs);
                    const double2 rv = r_in[i];
                    r_out[i] = rv;
                    nrm += rv.x * rv.x + rv.y * rv.y;
                    x_out[i] = x_in ? x_in[i] : make_double2(0.0, 0.0);
                }
            } else if (on) {
                cpx<double> acc[12];
                dslash_site<S, double, true, double2>(acc, e, U, s, q, b.g, r, a.nrhs, a.bt.diag[b.l]);
                const double f = sqrt(a.fr2[sys]);
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const size_t i = fidx(s, r, c, a.nrhs);
                    const double2 rv = r_in[i];
                    const double2 d = make_double2(rv.x - f * acc[c].re, rv.y - f * acc[c].im);
                    r_out[i] = d;
                    nrm += d.x * d.x + d.y * d.y;
                    const cpx<double> ev = ldr<double>(e, i);
                    const double2 xv = x_in ? x_in[i] : make_double2(0.0, 0.0);
                    x_out[i] = make_double2(xv.x + f * ev.re, xv.y + f * ev.im);
                }
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const size_t i = fidx(s, r, c, a.nrhs);
                    r_out[i] = make_double2(0.0, 0.0);
                    x_out[i] = make_double2(0.0, 0.0);
                }
            }
            const double v[1] = {nrm};
            part.add(sys, v);
        }
    }
    part.flush(a.partials);
}

// coarse canonical -> internal FP64 lattice field (zero elsewhere).  The
// coarse vectors of lattice l are one block [nrhs][nb_l][12] at complex
// offset coff[l]; bidx[s] is the coarse index of site s inside its lattice.
__global__ void batch_scatter_kernel(BatchTable bt, const double2 *xb, double2 *dst,
                                     const int32_t *bidx, const int *nb, const long long *coff,
                                     int Vtot, int nrhs)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= Vtot || r >= nrhs) return;
    const int l = bt.tile_lat[s >> 6];
    const int k = bidx[s];
    const double2 *p = xb + coff[l] + ((size_t)r * nb[l] + (k < 0 ? 0 : k)) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[fidx(s, r, c, nrhs)] = k >= 0 ? p[c] : make_double2(0.0, 0.0);
}

// y_b = (D in)(coarse sites), FP64, into the per-lattice coarse blocks
__global__ void __launch_bounds__(128) batch_coarse_kernel(BatchTable bt, const double2 *in,
                                                           const double2 *U, double2 *yb,
                                                           const int32_t *qg, const int *clat,
                                                           const int *nb, const int *nboff,
                                                           const long long *coff, int nbtot, int nrhs)
{
    const int kg = blockIdx.x * blockDim.x + threadIdx.x;
    if (kg >= nbtot) return;
    const int l = clat[kg];
    const int s = qg[kg];
    const BSite b = bsite(bt, s);
    const SiteGeo q = site_geo(b.local, b.g);
    const int k = kg - nboff[l];
    for (int r = 0; r < nrhs; ++r) {
        cpx<double> acc[12];
        dslash_site<double2, double, true>(acc, in, U, s, q, b.g, r, nrhs, bt.diag[l]);
        double2 *o = yb + coff[l] + ((size_t)r * nb[l] + k) * 12;
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = make_double2(acc[c].re, acc[c].im);
    }
}

// in_r = r_src / sqrt(fr2) in the inner precision, in_x = 0, partial |in_r|^2
// (of the stored values); systems whose flag is 0 get zeros
template <int PO>
__global__ void __launch_bounds__(256) batch_inner_init_kernel(BatchBlasArgs a, const double2 *r_src,
                                                               const double *fr2, void *in_r_, void *in_x_)
{
    typedef typename Store<PO>::S S;
    typedef typename Store<PO>::R R;
    extern __shared__ double smem[];
    const int nsys = a.bt.nlat * a.nrhs;
    if (a.act && !any_set(a.act, nsys)) return;
    SysPartial<1> part;
    part.init(smem, nsys);
    S *in_r = (S *)in_r_, *in_x = (S *)in_x_;
    const ItemRange it = xcd_items(a.Vtot / 256);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int s = w * 256 + threadIdx.x;
        const int l = a.bt.tile_lat[s >> 6];
        for (int k = 0; k < a.nrhs; ++k) {
            const int sys = l * a.nrhs + k;
            const bool on = a.act == nullptr || a.act[sys] != 0;
            const double f2 = fr2[sys];
            const double f = on && f2 > 0 ? 1.0 / sqrt(f2) : 0.0;
            double t = 0;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, a.nrhs);
                const double2 v = on ? r_src[i] : make_double2(0.0, 0.0);
                stc(in_r, i, cpx<R>{(R)(f * v.x), (R)(f * v.y)});
                stc(in_x, i, cpx<R>{(R)0, (R)0});
                const cpx<R> st = ldc(in_r, i);
                t += (double)st.re * st.re + (double)st.im * st.im;
            }
            const double vv[1] = {t};
            part.add(sys, vv);
        }
    }
    part.flush(a.partials);
}

// one workgroup per system: the fixed-order sum of its partials (as the
// single-lattice reduction), gated by act_in
__global__ void __launch_bounds__(256) batch_reduce_kernel(int mode, const double *partials, int nparts,
                                                           int nsys, double2 *alpha, double *out2,
                                                           const double *thr2, const int *act_in,
                                                           int *act_out)
{
    __shared__ double sm[3][256];
    if (act_in && !any_set(act_in, nsys)) return;
    const int r = blockIdx.x;
    if (act_in && !act_in[r]) {
        if (threadIdx.x == 0) {
            if (mode == kAlpha) alpha[r] = make_double2(0.0, 0.0);
            if (act_out && act_out != act_in) act_out[r] = 0;
        }
        return;
    }
    const int K = mode == kNorm ? 1 : 3;
    double acc[3] = {0, 0, 0};
    if (K == 1) strided_sum<1>(partials, nparts, nsys, r, acc);
    else strided_sum<3>(partials, nparts, nsys, r, acc);
    for (int k = 0; k < K; ++k) sm[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < K; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (mode == kAlpha) {
        const double qq = sm[2][0];
        alpha[r] = qq > 0 ? make_double2(sm[0][0] / qq, sm[1][0] / qq) : make_double2(0.0, 0.0);
    } else {
        const double n2 = sm[mode == kNorm3 ? 2 : 0][0];
        if (out2) out2[r] = n2;
        if (act_out) act_out[r] = n2 > thr2[r] ? 1 : 0;
    }
}

// the outer control of the defect correction, one thread per system: the
// relative FP64 residual against tol, the next inner threshold (the inner
// solve reduces the scaled residual by max(inner_tol, need / 2), or by need
// itself in FP64, need = tol |b| / |r|) and the scale |r|^2
__global__ void __launch_bounds__(256) batch_ctl_kernel(BatchCtlArgs c)
{
    if (c.init && blockIdx.x == 0 && threadIdx.x < 2) c.ctr[threadIdx.x] = 0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < c.nsys; k += gridDim.x * blockDim.x) {
        const double b2 = c.bn2[k];
        if (c.init) c.rn2[k] = b2;
        const double r2 = c.rn2[k];
        const double rel = b2 > 0 ? sqrt(r2 / b2) : 0.0;
        const bool on = b2 > 0 && rel > c.tol;  // a NaN residual is left to the host's check
        const double need = b2 > 0 && r2 > 0 ? c.tol * sqrt(b2 / r2) : 1.0;
        const double relt = c.fp64_inner ? need : fmax(c.inner_tol, 0.5 * need);
        c.thr2[k] = on ? relt * relt : 2.0;
        c.fr2[k] = r2;
        c.oact[k] = on ? 1 : 0;
    }
}

// y = x - y, FP64
__global__ void __launch_bounds__(256) batch_xmy_kernel(BatchBlasArgs a, const double2 *x, double2 *y)
{
    const ItemRange it = xcd_items(a.Vtot / 256);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int s = w * 256 + threadIdx.x;
        for (int k = 0; k < a.nrhs; ++k) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, a.nrhs);
                const double2 u = x[i], v = y[i];
                y[i] = make_double2(u.x - v.x, u.y - v.y);
            }
        }
    }
}

// ------------------------------------------------------------------ launchers
static size_t lds_sys(int nsys, int K) { return (size_t)4 * nsys * K * sizeof(double); }

// ------------------------------------------------------------------ even-odd reduced form
// The site of side po (0: the lattice's reduced parity, 1: the other) at
// half-site h: 2h and 2h + 1 differ in parity (Lx even), 2h having the
// parity of y + z + t.
__device__ __forceinline__ int half_site(int h, int4 d, int parity)
{
    const int t1 = (2 * h) / d.x;
    const int y = t1 % d.y, t2 = t1 / d.y;
    const int z = t2 % d.z, t = t2 / d.z;
    return 2 * h + ((parity ^ (y + z + t)) & 1);
}

template <int P>
__global__ void __launch_bounds__(256) batch_eo_kernel(BatchEoArgs a)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    typedef Operand<S, R> OP;
    typedef typename OP::T PT;
    extern __shared__ double smem[];
    const S *__restrict__ in = (const S *)a.in;
    const S *__restrict__ in2 = (const S *)a.in2;
    S *__restrict__ out = (S *)a.out;
    const S *__restrict__ U = (const S *)a.U;
    const int nsys = a.bt.nlat * a.nrhs;
    if (a.act && !any_set(a.act, nsys)) return;
    const bool dots = a.partials != nullptr;
    SysPartial<3> part;
    if (dots) part.init(smem, nsys);
    const uint8_t *mk = a.hf.mask + (size_t)a.po * a.hf.Vtot;
    // work items: a block of 256 half-sites with one RHS (the RHS of a block
    // adjacent, so that they share its links in L2)
    const ItemRange it = xcd_items(a.hf.Vtot / 256 * a.nrhs);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int blk = w / a.nrhs, r = w - blk * a.nrhs;
        const int H = blk * 256 + (int)threadIdx.x;
        const int l = a.hf.tile_lat[H >> 6];  // a block of 256 lies in one lattice
        const int4 d = a.bt.dims[l];
        Geom g;
        g.L[0] = d.x;
        g.L[1] = d.y;
        g.L[2] = d.z;
        g.L[3] = d.w;
        g.V = g.Vs = d.x * d.y * d.z * d.w;
        const bool on = mk[H] == 0;  // rest site (coarse sites and padding are masked)
        const int par = a.po ? 1 - a.hf.par[l] : a.hf.par[l];
        const int s = half_site(on ? H - a.hf.off[l] : 0, d, par);  // local full site
        const SiteGeo q = site_geo(s, g);
        const int fo = a.bt.off[l], co = a.hf.off[l];
        const R ca = (R)a.ca[l], cb = (R)a.cb[l];
        {
            if (a.act && !a.act[l * a.nrhs + r]) continue;  // uniform (one lattice, one RHS)
            cpx<R> acc[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
            if (on) {
#pragma unroll 1
                for (int hp = 0; hp < 8; ++hp) {
                    const int mu = hp >> 1;
                    int sp, sm;
                    nbr(s, mu, q, g, sp, sm);
                    // the neighbour (other side) at its half-site index
                    const int n = co + (((hp & 1) ? sm : sp) >> 1);
                    PT p[12], u[9];
#pragma unroll
                    for (int c = 0; c < 12; ++c) p[c] = OP::load(in, fidx(n, r, c, a.nrhs));
#pragma unroll
                    for (int e = 0; e < 9; ++e) u[e] = OP::load(U, lidx(fo + ((hp & 1) ? sm : s), mu, e));
                    switch (hp) {
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
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const cpx<R> v2 = in2 ? ldc(in2, fidx(H, r, c, a.nrhs)) : cpx<R>{0, 0};
                    acc[c] = {ca * v2.re + cb * acc[c].re, ca * v2.im + cb * acc[c].im};
                }
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) stc(out, fidx(H, r, c, a.nrhs), acc[c]);
            if (dots) {
                R sre = 0, sim = 0, sqq = 0;
                if (on) {
#pragma unroll
                    for (int c = 0; c < 12; ++c) {
                        const cpx<R> v = in2 ? ldc(in2, fidx(H, r, c, a.nrhs)) : cpx<R>{0, 0};
                        sre = fma(acc[c].re, v.re, fma(acc[c].im, v.im, sre));
                        sim = fma(acc[c].re, v.im, fma(-acc[c].im, v.re, sim));
                        sqq = fma(acc[c].re, acc[c].re, fma(acc[c].im, acc[c].im, sqq));
                    }
                }
                const double dd[3] = {(double)sre, (double)sim, (double)sqq};
                part.add(l * a.nrhs + r, dd);
            }
        }
    }
    if (dots) part.flush(a.partials);
}

template <int P>
__global__ void __launch_bounds__(256) batch_eo_split_kernel(BatchTable bt, BatchHalf hf, int nrhs, void *x_,
                                                             void *xp_, void *xq_, int to_full)
{
    typedef typename Store<P>::S S;
    S *x = (S *)x_, *xp = (S *)xp_, *xq = (S *)xq_;
    const size_t n = (size_t)hf.Vtot * nrhs * 12;
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x) {
        // j = fidx(H, r, c): compact tile, RHS, component, lane
        const size_t rest = j >> 6;
        const int tile = (int)(rest / ((size_t)nrhs * 12)), rc = (int)(rest - (size_t)tile * nrhs * 12);
        const int r = rc / 12, c = rc - r * 12;
        const int H = tile * 64 + (int)(j & 63);
        const int l = hf.tile_lat[tile];
        const int4 d = bt.dims[l];
        const int h = H - hf.off[l];
        const bool valid = 2 * h < d.x * d.y * d.z * d.w;
        const int sp = half_site(valid ? h : 0, d, hf.par[l]);
        const int sq = sp ^ 1;  // the other site of the pair
        const size_t gp = fidx(bt.off[l] + sp, r, c, nrhs), gq = fidx(bt.off[l] + sq, r, c, nrhs);
        if (!to_full) {
            const S zero = {};
            xp[j] = valid ? x[gp] : zero;
            xq[j] = valid ? x[gq] : zero;
        } else if (valid) {
            x[gp] = xp[j];
            x[gq] = xq[j];
        }
    }
}

hipError_t launch_batch_eo(int prec, const BatchEoArgs &a, int grid, hipStream_t st)
{
    const size_t lds = a.partials ? lds_sys(a.bt.nlat * a.nrhs, 3) : 0;
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(batch_eo_kernel<GRG_FP64>, dim3(grid), dim3(256), lds, st, a); break;
    case GRG_FP32: hipLaunchKernelGGL(batch_eo_kernel<GRG_FP32>, dim3(grid), dim3(256), lds, st, a); break;
    case GRG_BF16: hipLaunchKernelGGL(batch_eo_kernel<GRG_BF16>, dim3(grid), dim3(256), lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_eo_split(int prec, const BatchTable &bt, const BatchHalf &hf, int nrhs, void *x,
                                 void *xp, void *xq, int to_full, int grid, hipStream_t st)
{
    switch (prec) {
    case GRG_FP64:
        hipLaunchKernelGGL(batch_eo_split_kernel<GRG_FP64>, dim3(grid), dim3(256), 0, st, bt, hf, nrhs, x, xp, xq,
                           to_full);
        break;
    case GRG_FP32:
        hipLaunchKernelGGL(batch_eo_split_kernel<GRG_FP32>, dim3(grid), dim3(256), 0, st, bt, hf, nrhs, x, xp, xq,
                           to_full);
        break;
    case GRG_BF16:
        hipLaunchKernelGGL(batch_eo_split_kernel<GRG_BF16>, dim3(grid), dim3(256), 0, st, bt, hf, nrhs, x, xp, xq,
                           to_full);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dslash_batch(int prec, const BatchDslashArgs &a, int grid, int SB, hipStream_t st)
{
    if (SB != 64 && SB != 128 && SB != 256) return hipErrorInvalidValue;
    const size_t lds = a.partials ? lds_sys(a.bt.nlat * a.nrhs, 3) : 0;
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(dslash_batch_kernel<GRG_FP64>, dim3(grid), dim3(SB), lds, st, a); break;
    case GRG_FP32: hipLaunchKernelGGL(dslash_batch_kernel<GRG_FP32>, dim3(grid), dim3(SB), lds, st, a); break;
    case GRG_BF16: hipLaunchKernelGGL(dslash_batch_kernel<GRG_BF16>, dim3(grid), dim3(SB), lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define BDISP(prec, KERNEL, lds, ...)                                                                  \
    switch (prec) {                                                                                    \
    case GRG_FP64: hipLaunchKernelGGL(KERNEL<GRG_FP64>, dim3(a.grid), dim3(256), lds, st, __VA_ARGS__); break; \
    case GRG_FP32: hipLaunchKernelGGL(KERNEL<GRG_FP32>, dim3(a.grid), dim3(256), lds, st, __VA_ARGS__); break; \
    case GRG_BF16: hipLaunchKernelGGL(KERNEL<GRG_BF16>, dim3(a.grid), dim3(256), lds, st, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                                             \
    }

hipError_t launch_batch_mr_update(int prec, const BatchBlasArgs &a, void *x, void *r, const void *q,
                                  hipStream_t st)
{
    BDISP(prec, batch_mr_update_kernel, lds_sys(a.bt.nlat * a.nrhs, 1), a, x, r, q);
    return hipGetLastError();
}

hipError_t launch_batch_norm2(int prec, const BatchBlasArgs &a, const void *v, hipStream_t st)
{
    BDISP(prec, batch_norm2_kernel, lds_sys(a.bt.nlat * a.nrhs, 1), a, v);
    return hipGetLastError();
}

hipError_t launch_batch_axpy_convert(int pin, int pout, const BatchBlasArgs &a, const void *x, void *y,
                                     const double *scale, int mode, int beta, hipStream_t st)
{
    dim3 g(a.grid), b(256);
#define BAX(PI, PO)                                                                                  \
    if (pin == PI && pout == PO) {                                                                   \
        hipLaunchKernelGGL((batch_axpy_convert_kernel<PI, PO>), g, b, 0, st, a, x, y, scale, mode, beta); \
        return hipGetLastError();                                                                    \
    }
    BAX(GRG_FP64, GRG_FP64) BAX(GRG_FP64, GRG_FP32) BAX(GRG_FP64, GRG_BF16)
    BAX(GRG_FP32, GRG_FP64) BAX(GRG_FP32, GRG_FP32) BAX(GRG_FP32, GRG_BF16)
    BAX(GRG_BF16, GRG_FP64) BAX(GRG_BF16, GRG_FP32) BAX(GRG_BF16, GRG_BF16)
#undef BAX
    return hipErrorInvalidValue;
}

hipError_t launch_batch_sub_norm(const BatchBlasArgs &a, const void *b, const void *ax, void *r,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(batch_sub_norm_kernel, dim3(a.grid), dim3(256), lds_sys(a.bt.nlat * a.nrhs, 1), st,
                       a, (const double2 *)b, (const double2 *)ax, (double2 *)r);
    return hipGetLastError();
}

hipError_t launch_batch_dc_update(int prec, const BatchDcArgs &a, int grid, hipStream_t st)
{
    const size_t lds = lds_sys(a.bt.nlat * a.nrhs, 1);
    dim3 g(grid), b(128);
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(batch_dc_update_kernel<GRG_FP64>, g, b, lds, st, a); break;
    case GRG_FP32: hipLaunchKernelGGL(batch_dc_update_kernel<GRG_FP32>, g, b, lds, st, a); break;
    case GRG_BF16: hipLaunchKernelGGL(batch_dc_update_kernel<GRG_BF16>, g, b, lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_scatter(const BatchTable &bt, const double *xb, void *dst, const int32_t *bidx,
                                const int *nb, const long long *coff, int Vtot, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(batch_scatter_kernel, dim3((Vtot + 255) / 256, nrhs), dim3(256), 0, st, bt,
                       (const double2 *)xb, (double2 *)dst, bidx, nb, coff, Vtot, nrhs);
    return hipGetLastError();
}

hipError_t launch_batch_inner_init(int prec, const BatchBlasArgs &a, const void *r_src, const double *fr2,
                                   void *in_r, void *in_x, hipStream_t st)
{
    BDISP(prec, batch_inner_init_kernel, lds_sys(a.bt.nlat * a.nrhs, 1), a, (const double2 *)r_src, fr2, in_r,
          in_x);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(int mode, const double *partials, int nparts, int nsys, double2 *alpha,
                               double *out2, const double *thr2, const int *act_in, int *act_out,
                               hipStream_t st)
{
    if (nsys < 1 || nparts < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(nsys), dim3(256), 0, st, mode, partials, nparts, nsys, alpha,
                       out2, thr2, act_in, act_out);
    return hipGetLastError();
}

hipError_t launch_batch_ctl(const BatchCtlArgs &c, hipStream_t st)
{
    if (c.nsys < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_ctl_kernel, dim3((c.nsys + 255) / 256), dim3(256), 0, st, c);
    return hipGetLastError();
}

hipError_t launch_batch_xmy(const BatchBlasArgs &a, const void *x, void *y, hipStream_t st)
{
    hipLaunchKernelGGL(batch_xmy_kernel, dim3(a.grid), dim3(256), 0, st, a, (const double2 *)x, (double2 *)y);
    return hipGetLastError();
}

hipError_t launch_batch_coarse(const BatchTable &bt, const void *in, const void *U, double *yb,
                               const int32_t *qg, const int *clat, const int *nb, const int *nboff,
                               const long long *coff, int nbtot, int nrhs, hipStream_t st)
{
    hipLaunchKernelGGL(batch_coarse_kernel, dim3((nbtot + 127) / 128), dim3(128), 0, st, bt,
                       (const double2 *)in, (const double2 *)U, (double2 *)yb, qg, clat, nb, nboff,
                       coff, nbtot, nrhs);
    return hipGetLastError();
}

}  // namespace grg
