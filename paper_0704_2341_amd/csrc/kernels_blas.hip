// Krylov vector operations on internal fields, with deterministic reductions.
//
// Every kernel is a grid-stride walk over blocks of 256 sites (XCD-aware, as
// the stencil) with all right-hand sides looped inside the thread.  Sums are
// formed per thread in FP64, reduced over the wavefront by shuffles, over the
// workgroup through LDS, and written as one partial per workgroup and RHS;
// launch_reduce then adds the partials in a fixed tree order.  No floating
// point atomics anywhere, so every reduction is bitwise reproducible.
#include "common.h"
#include "engine.h"
#include "reduce.h"

namespace grg {

constexpr int kBlasSB = 256;

#define SITE_LOOP_BEGIN(sh)                                            \
    const int nsb_ = ((sh).g.V + kBlasSB - 1) / kBlasSB;               \
    const ItemRange it_ = xcd_items(nsb_);                             \
    for (int w_ = it_.begin; w_ < it_.end; w_ += it_.step) {           \
        const int s = w_ * kBlasSB + (int)threadIdx.x;                 \
        const bool valid = s < (sh).g.V;

#define SITE_LOOP_END }

// per-wave LDS accumulators, summed and written at the end of the kernel
template <int K>
struct Partial {
    double (*red)[K];  // [4 * nrhs] rows of K, row = wave * nrhs + rhs
    int nrhs;
    __device__ void init(double *smem, int nrhs_)
    {
        red = (double (*)[K])smem;
        nrhs = nrhs_;
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int i = lane; i < nrhs * K; i += 64) red[wave * nrhs + i / K][i % K] = 0.0;
        __syncthreads();
    }
    __device__ void add(int r, const double (&v)[K])
    {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double t = wave_sum(v[k]);
            if (lane == 0) red[wave * nrhs + r][k] += t;
        }
    }
    __device__ void flush(double *partials)
    {
        __syncthreads();
        const int nw = blockDim.x >> 6;
        for (int i = threadIdx.x; i < nrhs * K; i += blockDim.x) {
            double t = 0;
            for (int w = 0; w < nw; ++w) t += red[w * nrhs + i / K][i % K];
            partials[(size_t)blockIdx.x * nrhs * K + i] = t;
        }
    }
};

// ------------------------------------------------------------------ MR / GCR step
// 16-byte vectors of a field: 4 complex in BF16, 2 in FP32, 1 in FP64.
template <int P>
struct VecIO;
template <>
struct VecIO<GRG_BF16> {
    static constexpr int N = 4;
    typedef float R;
    __device__ static void get(const uint4 &v, cpx<float> (&c)[N])
    {
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < N; ++e) c[e] = {__uint_as_float(w[e] << 16), __uint_as_float(w[e] & 0xffff0000u)};
    }
    __device__ static uint4 put(const cpx<float> (&c)[N])
    {
        return make_uint4(pack_bf16(c[0].re, c[0].im), pack_bf16(c[1].re, c[1].im),
                          pack_bf16(c[2].re, c[2].im), pack_bf16(c[3].re, c[3].im));
    }
};
template <>
struct VecIO<GRG_FP32> {
    static constexpr int N = 2;
    typedef float R;
    __device__ static void get(const uint4 &v, cpx<float> (&c)[N])
    {
        c[0] = {__uint_as_float(v.x), __uint_as_float(v.y)};
        c[1] = {__uint_as_float(v.z), __uint_as_float(v.w)};
    }
    __device__ static uint4 put(const cpx<float> (&c)[N])
    {
        return make_uint4(__float_as_uint(c[0].re), __float_as_uint(c[0].im), __float_as_uint(c[1].re),
                          __float_as_uint(c[1].im));
    }
};
template <>
struct VecIO<GRG_FP64> {
    static constexpr int N = 1;
    typedef double R;
    __device__ static void get(const uint4 &v, cpx<double> (&c)[N])
    {
        c[0] = {__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z)};
    }
    __device__ static uint4 put(const cpx<double> (&c)[N])
    {
        const long long a = __double_as_longlong(c[0].re), b = __double_as_longlong(c[0].im);
        return make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
    }
};

// x += alpha_k p, r -= alpha_k q, and the partial sums of |r|^2 (of the values
// as stored) per RHS.  HAS_P = false: p is r itself (minimal residual).
//
// All RHS of a 64-site tile are one contiguous block, and one RHS of a tile
// (12 components x 64 sites) is a contiguous unit; a wavefront streams whole
// units with 16-byte accesses, so every load and store instruction of the
// wavefront moves 1 KB of consecutive memory, and alpha and the norm of a
// unit belong to one RHS.  Units are walked in tile order, XCD-aware.
// X0: x is taken as zero (not read): the first update of a solve started
// from x = 0.
template <int P, bool HAS_P, bool X0 = false>
__global__ void __launch_bounds__(256) mr_update_kernel(BlasShape sh, void *x_, void *r_,
                                                        const void *q_, const void *p_,
                                                        const double2 *alpha, double *partials)
{
    typedef VecIO<P> IO;
    typedef typename IO::R R;
    constexpr int N = IO::N;
    constexpr int UV = 12 * 64 / N;  // 16-byte vectors per unit
    constexpr int NV = UV / 64;      // per lane
    __shared__ double red[4][kMaxRhs];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = lane; i < sh.nrhs; i += 64) red[wave][i] = 0.0;
    uint4 *x = (uint4 *)x_, *r = (uint4 *)r_;
    const uint4 *q = (const uint4 *)q_, *p = (const uint4 *)p_;
    const int ntiles = (sh.g.V + 63) >> 6;
    const int nunits = ntiles * sh.nrhs;
    const ItemRange it = xcd_items((nunits + 3) >> 2);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int u = w * 4 + wave;
        if (u >= nunits) continue;  // the whole wavefront
        const int tile = u / sh.nrhs, k = u - tile * sh.nrhs;
        const double2 a2 = alpha[k];
        const cpx<R> a = {(R)a2.x, (R)a2.y}, na = {-a.re, -a.im};
        const size_t base = (size_t)u * UV;
        R rr = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int site = tile * 64 + (((v * 64 + lane) * N) & 63);
            if (site < sh.g.V) {
                const size_t i = base + v * 64 + lane;
                const uint4 xv = X0 ? make_uint4(0, 0, 0, 0) : x[i], rv = r[i], qv = q[i];
                cpx<R> xc[N], rc[N], qc[N], pc[N];
                IO::get(xv, xc);
                IO::get(rv, rc);
                IO::get(qv, qc);
                if (HAS_P) IO::get(p[i], pc);
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    cmac(xc[e], a, HAS_P ? pc[e] : rc[e]);
                    cmac(rc[e], na, qc[e]);
                }
                const uint4 ro = IO::put(rc);
                x[i] = IO::put(xc);
                r[i] = ro;
                IO::get(ro, rc);  // the norm of the values as stored
#pragma unroll
                for (int e = 0; e < N; ++e) rr = fma(rc[e].re, rc[e].re, fma(rc[e].im, rc[e].im, rr));
            }
        }
        const double t = wave_sum((double)rr);
        if (lane == 0) red[wave][k] += t;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < sh.nrhs; i += blockDim.x)
        partials[(size_t)blockIdx.x * sh.nrhs + i] = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
}

// BiCGstab vector steps (per-RHS scalars sc[0..3][kMaxRhs] = rho, alpha,
// omega, beta), in the unit walk of mr_update_kernel:
//   kBicgS:   s = r - alpha v                      (a = r, b = v, out = s)
//   kBicgUpd: x += alpha p + omega s, r = s - omega t, and the partial sums
//             of <r0, r> (re, im) and |r|^2 of the stored r
//             (x_ = x, r_ = r, a = p, b = s, c = t, d = r0)
//   kBicgP:   p = r + beta (p - omega v)          (r_ = p, a = r, b = v)
template <int P, int MODE>
__global__ void __launch_bounds__(256) bicg_kernel(BlasShape sh, void *x_, void *r_, const void *a_,
                                                   const void *b_, const void *c_, const void *d_,
                                                   const double2 *sc, double *partials)
{
    typedef VecIO<P> IO;
    typedef typename IO::R R;
    constexpr int N = IO::N;
    constexpr int UV = 12 * 64 / N;
    constexpr int NV = UV / 64;
    __shared__ double red[4][kMaxRhs][3];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (MODE == kBicgUpd)
        for (int i = lane; i < sh.nrhs * 3; i += 64) red[wave][i / 3][i % 3] = 0.0;
    uint4 *x = (uint4 *)x_, *r = (uint4 *)r_;
    const uint4 *a = (const uint4 *)a_, *b = (const uint4 *)b_, *c = (const uint4 *)c_,
                *d = (const uint4 *)d_;
    const int ntiles = (sh.g.V + 63) >> 6;
    const int nunits = ntiles * sh.nrhs;
    const ItemRange it = xcd_items((nunits + 3) >> 2);
    for (int w = it.begin; w < it.end; w += it.step) {
        const int u = w * 4 + wave;
        if (u >= nunits) continue;
        const int tile = u / sh.nrhs, k = u - tile * sh.nrhs;
        const double2 al2 = sc[kMaxRhs + k], om2 = sc[2 * kMaxRhs + k], be2 = sc[3 * kMaxRhs + k];
        const cpx<R> al = {(R)al2.x, (R)al2.y}, om = {(R)om2.x, (R)om2.y}, be = {(R)be2.x, (R)be2.y};
        const size_t base = (size_t)u * UV;
        R sre = 0, sim = 0, srr = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int site = tile * 64 + (((v * 64 + lane) * N) & 63);
            if (site >= sh.g.V) continue;
            const size_t i = base + v * 64 + lane;
            cpx<R> ac[N], bc[N];
            IO::get(a[i], ac);
            IO::get(b[i], bc);
            if (MODE == kBicgS) {
                cpx<R> o[N];
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    o[e] = ac[e];
                    cmac(o[e], cpx<R>{-al.re, -al.im}, bc[e]);
                }
                r[i] = IO::put(o);
            } else if (MODE == kBicgUpd) {
                cpx<R> xc[N], cc[N], dc[N], rc[N];
                IO::get(x[i], xc);
                IO::get(c[i], cc);
                IO::get(d[i], dc);
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    cmac(xc[e], al, ac[e]);
                    cmac(xc[e], om, bc[e]);
                    rc[e] = bc[e];
                    cmac(rc[e], cpx<R>{-om.re, -om.im}, cc[e]);
                }
                x[i] = IO::put(xc);
                const uint4 ro = IO::put(rc);
                r[i] = ro;
                IO::get(ro, rc);  // the sums of the values as stored
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    // conj(r0) r
                    sre = fma(dc[e].re, rc[e].re, fma(dc[e].im, rc[e].im, sre));
                    sim = fma(dc[e].re, rc[e].im, fma(-dc[e].im, rc[e].re, sim));
                    srr = fma(rc[e].re, rc[e].re, fma(rc[e].im, rc[e].im, srr));
                }
            } else {
                cpx<R> pc[N];
                IO::get(r[i], pc);
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    cpx<R> t = pc[e];
                    cmac(t, cpx<R>{-om.re, -om.im}, bc[e]);  // p - omega v
                    pc[e] = ac[e];
                    cmac(pc[e], be, t);                       // r + beta (p - omega v)
                }
                r[i] = IO::put(pc);
            }
        }
        if (MODE == kBicgUpd) {
            const double t0 = wave_sum((double)sre), t1 = wave_sum((double)sim), t2 = wave_sum((double)srr);
            if (lane == 0) {
                red[wave][k][0] += t0;
                red[wave][k][1] += t1;
                red[wave][k][2] += t2;
            }
        }
    }
    if (MODE == kBicgUpd) {
        __syncthreads();
        for (int i = threadIdx.x; i < sh.nrhs * 3; i += blockDim.x) {
            const int k = i / 3, j = i % 3;
            partials[(size_t)blockIdx.x * sh.nrhs * 3 + i] =
                ((red[0][k][j] + red[1][k][j]) + red[2][k][j]) + red[3][k][j];
        }
    }
}

// BiCGstab scalars from per-workgroup partials, one workgroup per RHS:
//   kBicgInit:  K = 1 (|r0|^2): rho = |r0|^2, out2 = |r0|^2, active = |r0|^2 > thr2
//   kBicgAlpha: K = 3 (sum conj(v) r0, |v|^2): alpha = rho / <r0, v>
//   kBicgBeta:  K = 3 (<r0, r>, |r|^2): beta = (rho' / rho) (alpha / omega),
//               rho = rho', out2 = |r|^2, active = |r|^2 > thr2
// An inactive RHS (or a zero denominator) gets alpha = beta = 0, which
// freezes its x and r in the vector steps (omega comes from the MR reduction
// with the same active flags).
__global__ void __launch_bounds__(256) bicg_reduce_kernel(int mode, const double *partials, int nparts,
                                                          int nrhs, double2 *sc, double *out2,
                                                          const double *thr2, int *active)
{
    __shared__ double sm[3][256];
    const int r = blockIdx.x;
    const int K = mode == kBicgInit ? 1 : 3;
    double acc[3] = {0, 0, 0};
    if (K == 1) strided_sum<1>(partials, nparts, nrhs, r, acc);
    else strided_sum<3>(partials, nparts, nrhs, r, acc);
    for (int k = 0; k < K; ++k) sm[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < K; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double2 *rho = sc, *alpha = sc + kMaxRhs, *omega = sc + 2 * kMaxRhs, *beta = sc + 3 * kMaxRhs;
    const bool on = active == nullptr || active[r];
    if (mode == kBicgInit) {
        rho[r] = make_double2(sm[0][0], 0.0);
        out2[r] = sm[0][0];
        if (active) active[r] = sm[0][0] > thr2[r] ? 1 : 0;
    } else if (mode == kBicgAlpha) {
        // <r0, v> = conj(sum conj(v) r0)
        const double sr = sm[0][0], si = -sm[1][0];
        const double den = sr * sr + si * si;
        const double2 rh = rho[r];
        alpha[r] = on && den > 0 ? make_double2((rh.x * sr + rh.y * si) / den, (rh.y * sr - rh.x * si) / den)
                                 : make_double2(0.0, 0.0);
    } else {
        const double2 rn = make_double2(sm[0][0], sm[1][0]), rh = rho[r], al = alpha[r], om = omega[r];
        const double d1 = rh.x * rh.x + rh.y * rh.y, d2 = om.x * om.x + om.y * om.y;
        double2 b = make_double2(0.0, 0.0);
        if (on && d1 > 0 && d2 > 0) {
            // (rn / rh) (al / om)
            const double2 q1 = make_double2((rn.x * rh.x + rn.y * rh.y) / d1, (rn.y * rh.x - rn.x * rh.y) / d1);
            const double2 q2 = make_double2((al.x * om.x + al.y * om.y) / d2, (al.y * om.x - al.x * om.y) / d2);
            b = make_double2(q1.x * q2.x - q1.y * q2.y, q1.x * q2.y + q1.y * q2.x);
        }
        beta[r] = b;
        rho[r] = rn;
        out2[r] = sm[2][0];
        if (active) active[r] = sm[2][0] > thr2[r] ? 1 : 0;
    }
}

template <int P>
__global__ void __launch_bounds__(256) norm2_kernel(BlasShape sh, const void *v_, double *partials)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    __shared__ double smem[4 * kMaxRhs];
    Partial<1> part;
    part.init(smem, sh.nrhs);
    const S *v = (const S *)v_;
    SITE_LOOP_BEGIN(sh)
    for (int k = 0; k < sh.nrhs; ++k) {
        double t = 0;
        if (valid) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const cpx<R> a = ldc(v, fidx(s, k, c, sh.nrhs));
                t += (double)a.re * a.re + (double)a.im * a.im;
            }
        }
        const double vv[1] = {t};
        part.add(k, vv);
    }
    SITE_LOOP_END
    part.flush(partials);
}

__global__ void __launch_bounds__(256) sub_norm_kernel(BlasShape sh, const double2 *b,
                                                       const double2 *ax, double2 *r,
                                                       double *partials)
{
    __shared__ double smem[4 * kMaxRhs];
    Partial<1> part;
    part.init(smem, sh.nrhs);
    SITE_LOOP_BEGIN(sh)
    for (int k = 0; k < sh.nrhs; ++k) {
        double t = 0;
        if (valid) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, sh.nrhs);
                const double2 bv = b[i], av = ax[i];
                const double2 d = make_double2(bv.x - av.x, bv.y - av.y);
                r[i] = d;
                t += d.x * d.x + d.y * d.y;
            }
        }
        const double vv[1] = {t};
        part.add(k, vv);
    }
    SITE_LOOP_END
    part.flush(partials);
}

// y = beta*y + f(scale[k]) * x, f = identity / 1/sqrt / sqrt
// With y_half > 0, y is written as a compact even-odd pair instead (a site
// of parity y_first at compact index s / 2, the other parity y_half
// elements on; beta must be 0).
template <int PI, int PO>
__global__ void __launch_bounds__(256) axpy_convert_kernel(BlasShape sh, const void *x_, void *y_,
                                                           const double *scale, int mode,
                                                           int beta, const int *active,
                                                           size_t y_half, int y_first)
{
    typedef typename Store<PI>::S SI;
    typedef typename Store<PI>::R RI;
    typedef typename Store<PO>::S SO;
    typedef typename Store<PO>::R RO;
    const SI *x = (const SI *)x_;
    SO *y = (SO *)y_;
    SITE_LOOP_BEGIN(sh)
    if (valid) {
        size_t ybase = 0;
        if (y_half) {
            const int x0 = s % sh.g.L[0], s1 = s / sh.g.L[0];
            const int x1 = s1 % sh.g.L[1], s2 = s1 / sh.g.L[1];
            const int par = (x0 + x1 + s2 % sh.g.L[2] + s2 / sh.g.L[2]) & 1;
            ybase = par == y_first ? 0 : y_half;
        }
        for (int k = 0; k < sh.nrhs; ++k) {
            double f = scale ? scale[k] : 1.0;
            if (mode == 1) f = f > 0 ? 1.0 / sqrt(f) : 0.0;
            if (mode == 2) f = sqrt(f);
            if (active && !active[k]) f = 0.0;
            const RO fo = (RO)f;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, sh.nrhs);
                const cpx<RI> a = ldc(x, i);
                cpx<RO> o = {fo * (RO)a.re, fo * (RO)a.im};
                if (beta) {
                    const cpx<RO> yo = ldc(y, i);
                    o.re += yo.re;
                    o.im += yo.im;
                }
                stc(y, y_half ? ybase + fidx(s >> 1, k, c, sh.nrhs) : i, o);
            }
        }
    }
    SITE_LOOP_END
}

__global__ void __launch_bounds__(256) xmy_kernel(BlasShape sh, const double2 *x, double2 *y)
{
    SITE_LOOP_BEGIN(sh)
    if (valid) {
        for (int k = 0; k < sh.nrhs; ++k) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, sh.nrhs);
                const double2 a = x[i], b = y[i];
                y[i] = make_double2(a.x - b.x, a.y - b.y);
            }
        }
    }
    SITE_LOOP_END
}

static bool shape_ok(const BlasShape &sh);

// ------------------------------------------------------------------ section 3 approximation
// The pieces of S~_bb x = [D (u - M y)]_b, M = d^{-1} + d~^{-1} - d^{-1} D_rr d~^{-1},
// y = D_rb u, d = 4 + m0 and d~ = D_rr 1 (row sums):
//   ones:     1 on every rest-site dof (one field), 0 on the coarse sites
//   divide:   t = y / d~ on the rest sites, 0 on the coarse sites
//   combine:  w = u - ((y - D_rr t) / d + t) on the rest sites, u on the coarse sites
__global__ void __launch_bounds__(256) rest_ones_kernel(BlasShape sh, const uint8_t *mask, double2 *o)
{
    SITE_LOOP_BEGIN(sh)
    if (valid) {
        const double v = mask[s] == 0 ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < 12; ++c) o[fidx(s, 0, c, 1)] = make_double2(v, 0.0);
    }
    SITE_LOOP_END
}

__global__ void __launch_bounds__(256) reusken_divide_kernel(BlasShape sh, const double2 *y,
                                                             const double2 *dt, const uint8_t *mask,
                                                             double2 *t)
{
    SITE_LOOP_BEGIN(sh)
    if (valid) {
        const bool rest = mask[s] == 0;
        for (int k = 0; k < sh.nrhs; ++k) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, sh.nrhs);
                double2 o = make_double2(0.0, 0.0);
                if (rest) {
                    const double2 a = y[i], b = dt[fidx(s, 0, c, 1)];
                    const double den = b.x * b.x + b.y * b.y;
                    o = make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
                }
                t[i] = o;
            }
        }
    }
    SITE_LOOP_END
}

__global__ void __launch_bounds__(256) reusken_combine_kernel(BlasShape sh, const double2 *u,
                                                              const double2 *y, const double2 *z,
                                                              const double2 *t, const uint8_t *mask,
                                                              double inv_d, double2 *w)
{
    SITE_LOOP_BEGIN(sh)
    if (valid) {
        const bool rest = mask[s] == 0;
        for (int k = 0; k < sh.nrhs; ++k) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, sh.nrhs);
                const double2 uv = u[i];
                double2 o = uv;
                if (rest) {
                    const double2 yv = y[i];
                    const double2 zv = z ? z[i] : make_double2(0.0, 0.0);
                    const double2 tv = t ? t[i] : make_double2(0.0, 0.0);
                    o = make_double2(uv.x - ((yv.x - zv.x) * inv_d + tv.x),
                                     uv.y - ((yv.y - zv.y) * inv_d + tv.y));
                }
                w[i] = o;
            }
        }
    }
    SITE_LOOP_END
}

template <int P>
__global__ void __launch_bounds__(256) combine_kernel(BlasShape sh, CombineArgs a)
{
    typedef typename Store<P>::S S;
    const double2 *u = (const double2 *)a.u, *x = (const double2 *)a.x;
    double2 *out = (double2 *)a.out;
    SITE_LOOP_BEGIN(sh)
    if (valid) {
        for (int k = 0; k < sh.nrhs; ++k) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, sh.nrhs);
                double2 v = x ? x[i] : make_double2(0.0, 0.0);
                for (int j = 0; j < a.n; ++j) {
                    const double f = a.f[j * kMaxRhs + k];
                    const cpx<double> e = ldr<double>((const S *)a.e[j], i);
                    v.x = fma(f, e.re, v.x);
                    v.y = fma(f, e.im, v.y);
                }
                const double2 b = u ? u[i] : make_double2(0.0, 0.0);
                out[i] = make_double2(fma(a.sigma, v.x, b.x), fma(a.sigma, v.y, b.y));
            }
        }
    }
    SITE_LOOP_END
}

hipError_t launch_combine(int prec, const BlasShape &sh, const CombineArgs &a, hipStream_t st)
{
    if (!shape_ok(sh) || a.n < 0 || a.n > kCorrPool) return hipErrorInvalidValue;
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(combine_kernel<GRG_FP64>, dim3(sh.grid), dim3(kBlasSB), 0, st, sh, a); break;
    case GRG_FP32: hipLaunchKernelGGL(combine_kernel<GRG_FP32>, dim3(sh.grid), dim3(kBlasSB), 0, st, sh, a); break;
    case GRG_BF16: hipLaunchKernelGGL(combine_kernel<GRG_BF16>, dim3(sh.grid), dim3(kBlasSB), 0, st, sh, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rest_ones(const Geom &g, const uint8_t *mask, void *o, hipStream_t st)
{
    BlasShape sh;
    sh.g = g;
    sh.nrhs = 1;
    const int blocks = (g.V + 255) / 256;
    sh.grid = blocks < 8 ? 8 : blocks > 2048 ? 2048 : (blocks + 7) / 8 * 8;
    hipLaunchKernelGGL(rest_ones_kernel, dim3(sh.grid), dim3(kBlasSB), 0, st, sh, mask, (double2 *)o);
    return hipGetLastError();
}

hipError_t launch_reusken_divide(const BlasShape &sh, const void *y, const void *dt,
                                 const uint8_t *mask, void *t, hipStream_t st)
{
    if (!shape_ok(sh)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reusken_divide_kernel, dim3(sh.grid), dim3(kBlasSB), 0, st, sh,
                       (const double2 *)y, (const double2 *)dt, mask, (double2 *)t);
    return hipGetLastError();
}

hipError_t launch_reusken_combine(const BlasShape &sh, const void *u, const void *y, const void *z,
                                  const void *t, const uint8_t *mask, double inv_d, void *w,
                                  hipStream_t st)
{
    if (!shape_ok(sh)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reusken_combine_kernel, dim3(sh.grid), dim3(kBlasSB), 0, st, sh,
                       (const double2 *)u, (const double2 *)y, (const double2 *)z, (const double2 *)t,
                       mask, inv_d, (double2 *)w);
    return hipGetLastError();
}

template <int P>
__global__ void __launch_bounds__(256) copy_kernel(BlasShape sh, const void *x_, void *y_)
{
    typedef typename Store<P>::S S;
    const S *x = (const S *)x_;
    S *y = (S *)y_;
    SITE_LOOP_BEGIN(sh)
    if (valid) {
        for (int k = 0; k < sh.nrhs; ++k) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, k, c, sh.nrhs);
                y[i] = x[i];
            }
        }
    }
    SITE_LOOP_END
}

__global__ void fill_zero_kernel(uint4 *p, size_t n16, uint8_t *tail, size_t ntail)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ GCR(m > 1)
template <int P>
__global__ void __launch_bounds__(256) multidot_kernel(BlasShape sh, const void *Q_, int k,
                                                       const void *q_, double *partials)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    extern __shared__ double dsm[];
    const S *Q = (const S *)Q_, *q = (const S *)q_;
    const size_t vstride = (size_t)sh.nrhs * 12 * sh.g.Vs;
    const int nr = sh.nrhs * k;  // rows (rhs, j)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double (*red)[2] = (double (*)[2])dsm;  // [4 waves][nr][2]
    for (int i = lane; i < nr * 2; i += 64) red[wave * nr + i / 2][i % 2] = 0.0;
    __syncthreads();
    SITE_LOOP_BEGIN(sh)
    for (int r = 0; r < sh.nrhs; ++r) {
        cpx<R> qv[12];
        if (valid) {
#pragma unroll
            for (int c = 0; c < 12; ++c) qv[c] = ldc(q, fidx(s, r, c, sh.nrhs));
        }
        for (int j = 0; j < k; ++j) {
            double re = 0, im = 0;
            if (valid) {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const cpx<R> a = ldc(Q, j * vstride + fidx(s, r, c, sh.nrhs));
                    re += (double)a.re * qv[c].re + (double)a.im * qv[c].im;
                    im += (double)a.re * qv[c].im - (double)a.im * qv[c].re;
                }
            }
            re = wave_sum(re);
            im = wave_sum(im);
            if (lane == 0) {
                red[wave * nr + r * k + j][0] += re;
                red[wave * nr + r * k + j][1] += im;
            }
        }
    }
    SITE_LOOP_END
    __syncthreads();
    const int nw = blockDim.x >> 6;
    for (int i = threadIdx.x; i < nr * 2; i += blockDim.x) {
        double t = 0;
        for (int w = 0; w < nw; ++w) t += red[w * nr + i / 2][i % 2];
        partials[(size_t)blockIdx.x * nr * 2 + i] = t;
    }
}

template <int P>
__global__ void __launch_bounds__(256) orthogonalise_kernel(BlasShape sh, const void *Q_,
                                                            const void *P_, int k,
                                                            const double2 *beta, void *q_,
                                                            void *p_, const void *r_,
                                                            double *partials)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    __shared__ double smem[4 * kMaxRhs * 3];
    Partial<3> part;
    part.init(smem, sh.nrhs);
    const S *Q = (const S *)Q_, *Pm = (const S *)P_, *rr = (const S *)r_;
    S *q = (S *)q_, *p = (S *)p_;
    const size_t vstride = (size_t)sh.nrhs * 12 * sh.g.Vs;
    SITE_LOOP_BEGIN(sh)
    for (int r = 0; r < sh.nrhs; ++r) {
        double d[3] = {0, 0, 0};
        if (valid) {
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const size_t i = fidx(s, r, c, sh.nrhs);
                cpx<R> qv = ldc(q, i), pv = ldc(p, i);
                for (int j = 0; j < k; ++j) {
                    const double2 b2 = beta[r * kMaxRhs + j];
                    const cpx<R> b = {(R)b2.x, (R)b2.y};
                    const cpx<R> tq = cmul(b, ldc(Q, j * vstride + i));
                    const cpx<R> tp = cmul(b, ldc(Pm, j * vstride + i));
                    qv.re -= tq.re; qv.im -= tq.im;
                    pv.re -= tp.re; pv.im -= tp.im;
                }
                stc(q, i, qv);
                stc(p, i, pv);
                const cpx<R> qs = ldc(q, i), rv = ldc(rr, i);
                d[0] += (double)qs.re * rv.re + (double)qs.im * rv.im;
                d[1] += (double)qs.re * rv.im - (double)qs.im * rv.re;
                d[2] += (double)qs.re * qs.re + (double)qs.im * qs.im;
            }
        }
        part.add(r, d);
    }
    SITE_LOOP_END
    part.flush(partials);
}

// ------------------------------------------------------------------ reductions
__global__ void __launch_bounds__(256) reduce_kernel(int mode, const double *partials, int nparts,
                                                     int nrhs, double2 *alpha, double *out2,
                                                     const double *thr2, int *active, int *part)
{
    __shared__ double sm[3][256];
    const int r = blockIdx.x;
    const int K = mode == kNorm ? 1 : 3;
    double acc[3] = {0, 0, 0};
    if (K == 1) strided_sum<1>(partials, nparts, nrhs, r, acc);
    else strided_sum<3>(partials, nparts, nrhs, r, acc);
    for (int k = 0; k < K; ++k) sm[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < K; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (mode == kAlpha) {
            const double qq = sm[2][0];
            const bool on = (active == nullptr || active[r]) && qq > 0;
            alpha[r] = on ? make_double2(sm[0][0] / qq, sm[1][0] / qq) : make_double2(0.0, 0.0);
            if (out2) out2[r] = qq;
        } else {
            const double n2 = sm[mode == kNorm3 ? 2 : 0][0];
            out2[r] = n2;
            if (active) active[r] = n2 > thr2[r] ? 1 : 0;
            if (part) part[r] = isinf(thr2[r]) ? 0 : 1;
        }
    }
}

// beta[r][j] = <q_j, q> / |q_j|^2 ; qnorm2 laid out [j][kMaxRhs]
__global__ void __launch_bounds__(256) reduce_multi_kernel(const double *partials, int nparts,
                                                           int nrhs, int k, const double *qnorm2,
                                                           const int *active, double2 *beta)
{
    __shared__ double sm[2][256];
    const int r = blockIdx.x / k, j = blockIdx.x % k;
    const int nr = nrhs * k;
    double a0 = 0, a1 = 0;
    for (int i = threadIdx.x; i < nparts; i += 256) {
        a0 += partials[((size_t)i * nr + r * k + j) * 2];
        a1 += partials[((size_t)i * nr + r * k + j) * 2 + 1];
    }
    sm[0][threadIdx.x] = a0;
    sm[1][threadIdx.x] = a1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sm[0][threadIdx.x] += sm[0][threadIdx.x + o];
            sm[1][threadIdx.x] += sm[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n2 = qnorm2[j * kMaxRhs + r];
        const bool on = (active == nullptr || active[r]) && n2 > 0;
        beta[r * kMaxRhs + j] = on ? make_double2(sm[0][0] / n2, sm[1][0] / n2) : make_double2(0.0, 0.0);
    }
}

// ------------------------------------------------------------------ launchers
#define DISPATCH_P(prec, KERNEL, ...)                                                           \
    switch (prec) {                                                                             \
    case GRG_FP64: hipLaunchKernelGGL(KERNEL<GRG_FP64>, __VA_ARGS__); break;                    \
    case GRG_FP32: hipLaunchKernelGGL(KERNEL<GRG_FP32>, __VA_ARGS__); break;                    \
    case GRG_BF16: hipLaunchKernelGGL(KERNEL<GRG_BF16>, __VA_ARGS__); break;                    \
    default: return hipErrorInvalidValue;                                                       \
    }

static bool shape_ok(const BlasShape &sh)
{
    return sh.nrhs >= 1 && sh.nrhs <= kMaxRhs && sh.grid >= 8 && sh.grid % 8 == 0;
}

hipError_t launch_reduce(int mode, const double *partials, int nparts, int nrhs, double2 *alpha,
                         double *out2, const double *thr2, int *active, hipStream_t st, int *part)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(nrhs), dim3(256), 0, st, mode, partials, nparts, nrhs,
                       alpha, out2, thr2, active, part);
    return hipGetLastError();
}

hipError_t launch_mr_update(int prec, const BlasShape &sh, void *x, void *r, const void *q,
                            const void *p, const double2 *alpha, double *partials,
                            hipStream_t st, bool x_zero)
{
    if (!shape_ok(sh)) return hipErrorInvalidValue;
    dim3 g(sh.grid), b(kBlasSB);
#define MRU(PP)                                                                                    \
    if (p) hipLaunchKernelGGL((mr_update_kernel<PP, true>), g, b, 0, st, sh, x, r, q, p, alpha, partials); \
    else if (x_zero)                                                                                      \
        hipLaunchKernelGGL((mr_update_kernel<PP, false, true>), g, b, 0, st, sh, x, r, q, p, alpha, partials); \
    else hipLaunchKernelGGL((mr_update_kernel<PP, false>), g, b, 0, st, sh, x, r, q, p, alpha, partials);
    switch (prec) {
    case GRG_FP64: MRU(GRG_FP64) break;
    case GRG_FP32: MRU(GRG_FP32) break;
    case GRG_BF16: MRU(GRG_BF16) break;
    default: return hipErrorInvalidValue;
    }
#undef MRU
    return hipGetLastError();
}

hipError_t launch_bicg(int prec, int mode, const BlasShape &sh, void *x, void *r, const void *a,
                       const void *b, const void *c, const void *d, const double2 *sc,
                       double *partials, hipStream_t st)
{
    if (!shape_ok(sh) || mode < kBicgS || mode > kBicgP) return hipErrorInvalidValue;
    dim3 g(sh.grid), bl(kBlasSB);
#define BIC(PP)                                                                                         \
    if (mode == kBicgS) hipLaunchKernelGGL((bicg_kernel<PP, kBicgS>), g, bl, 0, st, sh, x, r, a, b, c, d, sc, partials); \
    else if (mode == kBicgUpd) hipLaunchKernelGGL((bicg_kernel<PP, kBicgUpd>), g, bl, 0, st, sh, x, r, a, b, c, d, sc, partials); \
    else hipLaunchKernelGGL((bicg_kernel<PP, kBicgP>), g, bl, 0, st, sh, x, r, a, b, c, d, sc, partials);
    switch (prec) {
    case GRG_FP64: BIC(GRG_FP64) break;
    case GRG_FP32: BIC(GRG_FP32) break;
    case GRG_BF16: BIC(GRG_BF16) break;
    default: return hipErrorInvalidValue;
    }
#undef BIC
    return hipGetLastError();
}

hipError_t launch_bicg_reduce(int mode, const double *partials, int nparts, int nrhs, double2 *sc,
                              double *out2, const double *thr2, int *active, hipStream_t st)
{
    if (nrhs < 1 || nrhs > kMaxRhs || mode < kBicgInit || mode > kBicgBeta) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bicg_reduce_kernel, dim3(nrhs), dim3(256), 0, st, mode, partials, nparts, nrhs, sc,
                       out2, thr2, active);
    return hipGetLastError();
}

hipError_t launch_norm2(int prec, const BlasShape &sh, const void *v, double *partials,
                        hipStream_t st)
{
    if (!shape_ok(sh)) return hipErrorInvalidValue;
    DISPATCH_P(prec, norm2_kernel, dim3(sh.grid), dim3(kBlasSB), 0, st, sh, v, partials);
    return hipGetLastError();
}

hipError_t launch_sub_norm(const BlasShape &sh, const void *b, const void *ax, void *r,
                           double *partials, hipStream_t st)
{
    if (!shape_ok(sh)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sub_norm_kernel, dim3(sh.grid), dim3(kBlasSB), 0, st, sh,
                       (const double2 *)b, (const double2 *)ax, (double2 *)r, partials);
    return hipGetLastError();
}

hipError_t launch_axpy_convert(int prec_in, int prec_out, const BlasShape &sh, const void *x,
                               void *y, const double *scale, int mode, int beta,
                               const int *active, hipStream_t st, size_t y_half, int y_first)
{
    if (!shape_ok(sh) || (y_half && beta)) return hipErrorInvalidValue;
    dim3 g(sh.grid), b(kBlasSB);
#define AXC(PI, PO)                                                                                \
    if (prec_in == PI && prec_out == PO) {                                                         \
        hipLaunchKernelGGL((axpy_convert_kernel<PI, PO>), g, b, 0, st, sh, x, y, scale, mode, beta, \
                           active, y_half, y_first);                                               \
        return hipGetLastError();                                                                  \
    }
    AXC(GRG_FP64, GRG_FP64) AXC(GRG_FP64, GRG_FP32) AXC(GRG_FP64, GRG_BF16)
    AXC(GRG_FP32, GRG_FP64) AXC(GRG_FP32, GRG_FP32) AXC(GRG_FP32, GRG_BF16)
    AXC(GRG_BF16, GRG_FP64) AXC(GRG_BF16, GRG_FP32) AXC(GRG_BF16, GRG_BF16)
#undef AXC
    return hipErrorInvalidValue;
}

hipError_t launch_xmy(const BlasShape &sh, const void *x, void *y, hipStream_t st)
{
    if (!shape_ok(sh)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(xmy_kernel, dim3(sh.grid), dim3(kBlasSB), 0, st, sh, (const double2 *)x,
                       (double2 *)y);
    return hipGetLastError();
}

hipError_t launch_copy(int prec, const BlasShape &sh, const void *x, void *y, hipStream_t st)
{
    if (!shape_ok(sh)) return hipErrorInvalidValue;
    DISPATCH_P(prec, copy_kernel, dim3(sh.grid), dim3(kBlasSB), 0, st, sh, x, y);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return hipSuccess;
    const size_t n16 = bytes / 16, ntail = bytes % 16;
    int grid = (int)std::min<size_t>((n16 + 255) / 256 + 1, 8192);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, st, (uint4 *)p, n16,
                       (uint8_t *)p + n16 * 16, ntail);
    return hipGetLastError();
}

hipError_t launch_multidot(int prec, const BlasShape &sh, const void *Q, int k, const void *q,
                           double *partials, hipStream_t st)
{
    if (!shape_ok(sh) || k < 1 || k > kMaxRhs) return hipErrorInvalidValue;
    const size_t lds = (size_t)4 * sh.nrhs * k * 2 * sizeof(double);
    DISPATCH_P(prec, multidot_kernel, dim3(sh.grid), dim3(kBlasSB), lds, st, sh, Q, k, q, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_multi(const double *partials, int nparts, int nrhs, int k,
                               const double *qnorm2, const int *active, double2 *beta,
                               hipStream_t st)
{
    hipLaunchKernelGGL(reduce_multi_kernel, dim3(nrhs * k), dim3(256), 0, st, partials, nparts,
                       nrhs, k, qnorm2, active, beta);
    return hipGetLastError();
}

hipError_t launch_orthogonalise(int prec, const BlasShape &sh, const void *Q, const void *P,
                                int k, const double2 *beta, void *q, void *p, const void *r,
                                double *partials, hipStream_t st)
{
    if (!shape_ok(sh) || k < 1 || k > kMaxRhs) return hipErrorInvalidValue;
    DISPATCH_P(prec, orthogonalise_kernel, dim3(sh.grid), dim3(kBlasSB), 0, st, sh, Q, P, k, beta,
               q, p, r, partials);
    return hipGetLastError();
}

}  // namespace grg
