// Kernels of the cyclic-reduction V-cycle (section 4): the blocked links of
// the next level, the restriction of a field to the coarse sites and its
// prolongation, and the canonical-field vector algebra of the BiCGstab solves
// that the cycle runs on full levels.
//
// With the all-even coarse set (Type I) the Schur complement that ignores the
// couplings inside D_rr is again a Wilson operator on the coarse lattice:
//     D_bb - D_br D_rb / d = (1/d) D_W(V, d^2 - 4),   d = 4 + m0,
//     V_mu(c) = U_mu(2c) U_mu(2c + mu)
// (from a coarse site, D_rb reaches x +- mu only, the return paths vanish
// since (1 - g)(1 + g) = 0, and x -> x + mu -> x + 2 mu carries
// (1/2 (1 - g_mu))^2 = (1 - g_mu)/2 with the link product V).  On that set
// the second-order approximation of section 3 coincides with it, so each
// level of the cycle is a Wilson operator with blocked links.
#include <algorithm>

#include "common.h"
#include "engine.h"

namespace grg {

// V_mu(c) = U_mu(2c) U_mu(2c + mu) from the fine lattice's internal FP64
// links (boundary signs folded in, so the product carries the sign of the
// one fine hop that wraps) into canonical [Vc][4][3][3] complex128.
__global__ void __launch_bounds__(256) vc_block_links_kernel(Geom gf, const double2 *__restrict__ U,
                                                             Geom gc, double2 *__restrict__ out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= gc.V * 4) return;
    const int sc = idx >> 2, mu = idx & 3;
    int c[4], t = sc;
    for (int k = 0; k < 4; ++k) {
        c[k] = t % gc.L[k];
        t /= gc.L[k];
    }
    int x[4];
    for (int k = 0; k < 4; ++k) x[k] = 2 * c[k];
    const int s0 = x[0] + gf.L[0] * (x[1] + gf.L[1] * (x[2] + gf.L[2] * x[3]));
    x[mu] += 1;  // 2 c + mu stays inside the lattice (the fine extent is even)
    const int s1 = x[0] + gf.L[0] * (x[1] + gf.L[1] * (x[2] + gf.L[2] * x[3]));
    double2 a[9], b[9];
    for (int e = 0; e < 9; ++e) {
        a[e] = U[lidx(s0, mu, e)];
        b[e] = U[lidx(s1, mu, e)];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double re = 0, im = 0;
            for (int k = 0; k < 3; ++k) {
                const double2 p = a[3 * i + k], q = b[3 * k + j];
                re += p.x * q.x - p.y * q.y;
                im += p.x * q.y + p.y * q.x;
            }
            out[(size_t)idx * 9 + 3 * i + j] = make_double2(re, im);
        }
}

// canonical fields [nrhs][V][12]: coarse[r][k] = full[r][q[k]] (restriction
// to the coarse sites, which are the next level's sites in its own order),
// and full[r][q[k]] = coarse[r][k] with full zero elsewhere (prolongation)
__global__ void __launch_bounds__(256) vc_restrict_kernel(const double2 *__restrict__ full,
                                                          double2 *__restrict__ coarse,
                                                          const int32_t *__restrict__ q, int nb, int V,
                                                          int nrhs)
{
    const size_t n = (size_t)nrhs * nb * 12;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % 12);
        const size_t rk = i / 12;
        const int k = (int)(rk % nb), r = (int)(rk / nb);
        coarse[i] = full[((size_t)r * V + q[k]) * 12 + c];
    }
}

__global__ void __launch_bounds__(256) vc_prolong_kernel(const double2 *__restrict__ coarse,
                                                         double2 *__restrict__ full,
                                                         const int32_t *__restrict__ q, int nb, int V,
                                                         int nrhs)
{
    const size_t n = (size_t)nrhs * nb * 12;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % 12);
        const size_t rk = i / 12;
        const int k = (int)(rk % nb), r = (int)(rk / nb);
        full[((size_t)r * V + q[k]) * 12 + c] = coarse[i];
    }
}

// out[r][i] = sum_j c[j][r] in_j[r][i] over the first n inputs (n <= 3);
// out may alias an input (each element is read before it is written)
__global__ void __launch_bounds__(256) vc_lincomb_kernel(size_t len, int nrhs, VcCoef cf, double2 *out,
                                                         const double2 *in0, const double2 *in1,
                                                         const double2 *in2)
{
    const size_t n = len * nrhs;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / len);
        const double2 *in[3] = {in0, in1, in2};
        double re = 0, im = 0;
        for (int j = 0; j < cf.n; ++j) {
            const double2 a = cf.c[j][r], v = in[j][i];
            re += a.x * v.x - a.y * v.y;
            im += a.x * v.y + a.y * v.x;
        }
        out[i] = make_double2(re, im);
    }
}

// per-workgroup partial sums per RHS: re and im of sum conj(a) b, and sum |b|^2
__global__ void __launch_bounds__(256) vc_dot_kernel(size_t len, int nrhs, const double2 *__restrict__ a,
                                                     const double2 *__restrict__ b, double *partials)
{
    __shared__ double sm[3][256];
    for (int r = 0; r < nrhs; ++r) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
             i += (size_t)gridDim.x * blockDim.x) {
            const double2 x = a[(size_t)r * len + i], y = b[(size_t)r * len + i];
            s0 += x.x * y.x + x.y * y.y;
            s1 += x.x * y.y - x.y * y.x;
            s2 += y.x * y.x + y.y * y.y;
        }
        sm[0][threadIdx.x] = s0;
        sm[1][threadIdx.x] = s1;
        sm[2][threadIdx.x] = s2;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) {
                sm[0][threadIdx.x] += sm[0][threadIdx.x + o];
                sm[1][threadIdx.x] += sm[1][threadIdx.x + o];
                sm[2][threadIdx.x] += sm[2][threadIdx.x + o];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double *p = partials + ((size_t)blockIdx.x * nrhs + r) * 3;
            p[0] = sm[0][0];
            p[1] = sm[1][0];
            p[2] = sm[2][0];
        }
        __syncthreads();
    }
}

static inline int vc_grid(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 2048); }

hipError_t launch_vc_block_links(const Geom &gf, const void *U64, const Geom &gc, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(vc_block_links_kernel, dim3((gc.V * 4 + 255) / 256), dim3(256), 0, st, gf,
                       (const double2 *)U64, gc, (double2 *)out);
    return hipGetLastError();
}

hipError_t launch_vc_restrict(const double *full, double *coarse, const int32_t *q, int nb, int V, int nrhs,
                              hipStream_t st)
{
    hipLaunchKernelGGL(vc_restrict_kernel, dim3(vc_grid((size_t)nrhs * nb * 12)), dim3(256), 0, st,
                       (const double2 *)full, (double2 *)coarse, q, nb, V, nrhs);
    return hipGetLastError();
}

hipError_t launch_vc_prolong(const double *coarse, double *full, const int32_t *q, int nb, int V, int nrhs,
                             hipStream_t st)
{
    hipLaunchKernelGGL(vc_prolong_kernel, dim3(vc_grid((size_t)nrhs * nb * 12)), dim3(256), 0, st,
                       (const double2 *)coarse, (double2 *)full, q, nb, V, nrhs);
    return hipGetLastError();
}

hipError_t launch_vc_lincomb(size_t len, int nrhs, const VcCoef &cf, double *out, const double *in0,
                             const double *in1, const double *in2, hipStream_t st)
{
    if (cf.n < 1 || cf.n > 3 || nrhs < 1 || nrhs > kMaxRhs) return hipErrorInvalidValue;
    hipLaunchKernelGGL(vc_lincomb_kernel, dim3(vc_grid(len * nrhs)), dim3(256), 0, st, len, nrhs, cf,
                       (double2 *)out, (const double2 *)in0, (const double2 *)in1, (const double2 *)in2);
    return hipGetLastError();
}

int vc_dot_grid(size_t len) { return (int)std::min<size_t>((len + 255) / 256, 256); }

hipError_t launch_vc_dot(size_t len, int nrhs, const double *a, const double *b, double *partials,
                         hipStream_t st)
{
    hipLaunchKernelGGL(vc_dot_kernel, dim3(vc_dot_grid(len)), dim3(256), 0, st, len, nrhs,
                       (const double2 *)a, (const double2 *)b, partials);
    return hipGetLastError();
}

}  // namespace grg
