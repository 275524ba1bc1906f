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
    const ItemRange it = xcd_items(a.Vtot / blockDim.x);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int s = w * blockDim.x + threadIdx.x;
        const BSite b = bsite(a.bt, s);
        const bool on = a.mask[s] == 0;
        const SiteGeo q = site_geo(b.local, b.g);
        for (int r = 0; r < a.nrhs; ++r) {
            const int sys = b.l * a.nrhs + r;
            double nrm = 0;
            if (on) {
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

// ------------------------------------------------------------------ launchers
static size_t lds_sys(int nsys, int K) { return (size_t)4 * nsys * K * sizeof(double); }

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
