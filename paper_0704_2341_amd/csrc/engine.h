// Host-side engine: kernel launchers and handle structures.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "common.h"

namespace grg {

constexpr int kMaxRhs = 16;
constexpr int kMaxGridValue = 4096;  // largest stencil/BLAS grid (sizes partial sums)

void set_error(const char *fmt, ...);

#define GRG_TRY_HIP(expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            ::grg::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                      \
            return GRG_EHIP;                                                                 \
        }                                                                                    \
    } while (0)

#define GRG_TRY(expr)                        \
    do {                                     \
        grg_status s_ = (expr);              \
        if (s_ != GRG_OK) return s_;         \
    } while (0)

// ------------------------------------------------------------------ kernels
struct DslashArgs {
    const void *in;
    void *out;
    const void *U;
    const uint8_t *mask;  // output-site mask, nullptr = every site
    int sel;              // rows kept: mask[s] == sel
    double diag;          // 4 + m0
    Geom g;
    int nrhs;
    int SB;               // sites per work item == workgroup size
    int RG;               // right-hand sides per work item
    int split;            // 1: one hop per loop iteration, 0: one direction (two hops)
    int chunk;            // items per XCD chunk (0 = one contiguous eighth per XCD)
    int march;            // > 0: t-marching kernel with time chunks of this length
                          //      (64 sites x RG RHS wavefronts per workgroup)
    double *partials;     // [grid][nrhs][3] or nullptr
    const void *dot_with; // the fused dots use this field instead of `in` (or nullptr)
};

// Stencil between the compact parity halves of the even-odd reduction
// (kernels_eo.hip): out = alpha in2 + beta (H in) on the rest sites of parity
// po, H the hopping term (D minus its diagonal).
struct EoArgs {
    const void *in;       // compact field of parity 1 - po
    const void *in2;      // compact field of parity po, or nullptr (alpha term dropped)
    void *out;            // compact field of parity po
    const void *U;        // links, [2][compact tiles][4][9][64]
    const uint8_t *mask;  // [2][Vhs]: 1 on coarse sites and padding
    int po;               // output parity
    double alpha, beta;
    Geom g;               // the full lattice
    int Vh, Vhs;          // half volume, and padded to whole tiles (multiple of 256)
    int nrhs, SB, RG, hops, chunk;
    int march;            // hops == 3: time slices per workgroup item (t-marching form)
    double *partials;     // [grid][nrhs][3] or nullptr
    const void *dot_with; // parity po, or nullptr: the sums are |out|^2 only (re, im zero)
    const int *active;    // per RHS: 0 writes zero for that RHS (nullptr: all active)
    // full-layout variants (the first and last steps of a reduced solve read
    // and write the unreduced fields directly): in / in2 indexed by the full
    // site; out written to the full field, together with the same-index site
    // of the other parity, copied from `partner` (compact, parity 1 - po)
    int in_full, in2_full, out_full;
    const void *partner;
};

// out = u + sigma (x + sum_j f[j][rhs] e_j) in FP64 (u, x nullable): the
// defect correction's iterate from its kept corrections e_j (inner precision)
constexpr int kCorrPool = 16;
struct CombineArgs {
    const void *e[kCorrPool];
    const double *f;      // [kCorrPool][kMaxRhs]
    int n;                // corrections in use
    const void *u, *x;    // FP64 or nullptr
    void *out;            // FP64, may alias x or u
    double sigma;
};

// A tuned launch of the stencil for one precision and RHS count.
struct DslashTune {
    int valid = 0;
    int SB = 128, RG = 1, split = 0, grid = 0, chunk = 0, march = 0;
    float ms = 0;
};

struct CoarseArgs {
    const void *in;       // internal FP64 lattice field
    void *out;            // canonical coarse [nrhs][nb][12] complex128
    const void *U;        // internal FP64 links
    const int32_t *q;     // coarse index -> site
    int nb;
    double diag;
    Geom g;
    int nrhs;
};

// Fused FP64 defect-correction step (see dc_update_kernel).
struct DcArgs {
    const void *e;        // inner solution, internal tiles in the inner precision
    const void *U;        // FP64 links
    const void *r_in;     // FP64 residual before the step
    const void *x_in;     // FP64 iterate before the step, or nullptr for zero
    void *r_out, *x_out;  // FP64 results (may alias the inputs)
    const double *f;      // per-RHS factor of e (the inner right-hand side was r / f)
    void *r_next;         // r_out * s_next in the inner precision (next inner rhs), or nullptr
    const double *s_next; // per-RHS scale of r_next
    const uint8_t *mask;  // 1 on coarse sites
    double diag;          // 4 + m0
    Geom g;
    int nrhs;
    double *partials;     // [grid][nrhs]: |r_out|^2
    int RG, chunk, march; // t-marching launch (march > 0), as in DslashArgs
    int ring;             // with march > 0 and BF16 e: the LDS-ring form of the t-marching step
    int grp_first;        // ring form: work items ordered with the RHS group fastest, so the
                          // groups of one tile run together on one XCD and share its links
    int r_in32 = 0;       // r_in is stored in FP32 (float2 per complex), else FP64
    int r_out32 = 0;      // r_out is stored in FP32 (rounded from the FP64 result), else FP64
    // r_next in the compact even-odd halves (the reduced solve's right-hand
    // side) instead of the full layout: the half of parity next_par first, the
    // other next_half elements on (0: full layout)
    size_t next_half = 0;
    int next_par = 0;
};

hipError_t launch_dslash(int prec, const DslashArgs &a, int grid, hipStream_t st);
// SB: workgroup of the site-parallel kernel (a.march == 0); with a.march > 0
// the t-marching kernel runs with 64 * a.RG threads per workgroup (a.ring: its
// LDS-ring form, BF16 e only, 64 sites per x-y-z tile made of whole x-rows).
hipError_t launch_dc_update(int prec, const DcArgs &a, int grid, int SB, hipStream_t st);
hipError_t launch_dslash_coarse(const CoarseArgs &a, hipStream_t st);
// b = D_rb x_b from the canonical coarse vector (kernels_coarse.hip): internal
// FP64 field, zero on the coarse sites
// With partials set, also the per-workgroup |b|^2 per RHS ([rb_apply_grid(g)][nrhs]).
// With pair set, b also in precision pair_prec as a compact even-odd pair
// (parity `first` at compact index s / 2, the other parity `half` elements on).
hipError_t launch_rb_apply(const Geom &g, const double *xb, const int32_t *bidx, int nb, const void *U64,
                           void *out, int nrhs, hipStream_t st, double *partials = nullptr,
                           int pair_prec = -1, void *pair = nullptr, size_t half = 0, int first = 0);
int rb_apply_grid(const Geom &g);
// y_b = [D (u + sigma sum_j f_j e_j)]_b, u = x_b on the coarse sites, from the
// kept corrections (inner precision prec) at the coarse sites' neighbours
hipError_t launch_coarse_combine_apply(int prec, const Geom &g, const double *xb, const int32_t *qsites,
                                       const int32_t *bidx, int nb, const void *U64, double diag,
                                       const CombineArgs &a, double *yb, int nrhs, hipStream_t st);
hipError_t launch_eo_hop(int prec, const EoArgs &a, int grid, hipStream_t st);
// compact field of parity par <-> full field (zero off that parity)
hipError_t launch_eo_scatter(int prec, const Geom &g, int nrhs, int par, const void *src, void *dst,
                             bool to_full, hipStream_t st);
hipError_t launch_eo_pack_links(int prec, const Geom &g, int Vhs, const void *U, void *Ueo, hipStream_t st);
hipError_t launch_eo_pack_mask(const Geom &g, int Vhs, const uint8_t *mask, uint8_t *meo, hipStream_t st);
hipError_t launch_pack_gauge(const double *src, const Geom &g, const int bc[4], void *u64,
                             void *u32, void *u16, hipStream_t st);
hipError_t launch_pack_spinor(int prec, const double *src, void *dst, const Geom &g, int nrhs,
                              hipStream_t st, const uint8_t *mask = nullptr, int keep = 0);
hipError_t launch_unpack_spinor(int prec, const void *src, double *dst, const Geom &g, int nrhs,
                                hipStream_t st);
hipError_t launch_pack_masked(const double *src, void *dst, const uint8_t *mask, int keep,
                              const Geom &g, int nrhs, hipStream_t st);
hipError_t launch_scatter_coarse(const double *xb, void *dst, const int32_t *bidx, int nb,
                                 const Geom &g, int nrhs, hipStream_t st);

// BLAS-1 on internal fields.  Every kernel walks sites in work items of
// SB sites x all RHS (looped); partial sums go to [grid][nrhs][k] doubles.
struct BlasShape {
    Geom g;
    int nrhs;
    int grid;   // workgroups, multiple of 8
};

// partials -> per-RHS reductions (fixed-order tree, deterministic)
//  mode kAlpha: in k = 3 (re<q,r>, im<q,r>, |q|^2); alpha[r] = <q,r>/|q|^2 if
//               active[r], else 0.  Also stores |q|^2 in aux[r].
//  mode kNorm : in k = 1; out2[r] = sum; active[r] = sum > thr2[r].
//  mode kNorm3: as kNorm from the third of k = 3 sums (a stencil's fused |out|^2).
//  part (kNorm, kNorm3; optional): part[r] = thr2[r] finite (the RHS takes
//  part in the solve; an infinite threshold marks one that does not).
enum { kAlpha = 0, kNorm = 1, kNorm3 = 2 };
hipError_t launch_reduce(int mode, const double *partials, int nparts, int nrhs, double2 *alpha,
                         double *out2, const double *thr2, int *active, hipStream_t st,
                         int *part = nullptr);

// x += alpha r ; r -= alpha q ; partial |r|^2     (one MR/GCR step; x_zero:
// x is taken as zero and not read, the first step from x = 0)
hipError_t launch_mr_update(int prec, const BlasShape &sh, void *x, void *r, const void *q,
                            const void *p, const double2 *alpha, double *partials,
                            hipStream_t st, bool x_zero = false);
// partial |v|^2
hipError_t launch_norm2(int prec, const BlasShape &sh, const void *v, double *partials,
                        hipStream_t st);
// r = b - ax (FP64), partial |r|^2
hipError_t launch_sub_norm(const BlasShape &sh, const void *b, const void *ax, void *r,
                           double *partials, hipStream_t st);
// y (prec_out) = beta*y + scale[r] * x (prec_in); scale from a device array
// of per-RHS reals, multiplied by 1/sqrt(scale) when inv_sqrt != 0.  With
// y_half > 0, y is a compact even-odd pair (parity y_first's half first, the
// other y_half elements on; beta 0).
hipError_t launch_axpy_convert(int prec_in, int prec_out, const BlasShape &sh, const void *x,
                               void *y, const double *scale, int inv_sqrt, int beta,
                               const int *active, hipStream_t st, size_t y_half = 0, int y_first = 0);
// y = x - y (FP64), used for u - z
hipError_t launch_xmy(const BlasShape &sh, const void *x, void *y, hipStream_t st);
// Second-order Schur complement approximation (kernels_blas.hip): the
// rest-site ones field, t = y / d~ and w = u - ((y - z) / d + t) (z, t
// nullable: zero; w = u - y / d is the approximation that ignores D_rr).
hipError_t launch_rest_ones(const Geom &g, const uint8_t *mask, void *o, hipStream_t st);
hipError_t launch_combine(int prec, const BlasShape &sh, const CombineArgs &a, hipStream_t st);
hipError_t launch_reusken_divide(const BlasShape &sh, const void *y, const void *dt,
                                 const uint8_t *mask, void *t, hipStream_t st);
hipError_t launch_reusken_combine(const BlasShape &sh, const void *u, const void *y, const void *z,
                                  const void *t, const uint8_t *mask, double inv_d, void *w,
                                  hipStream_t st);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);
hipError_t launch_copy(int prec, const BlasShape &sh, const void *x, void *y, hipStream_t st);

// BiCGstab vector steps and scalar reductions (kernels_blas.hip); sc holds
// rho, alpha, omega, beta per RHS as double2[4][kMaxRhs]:
//   kBicgS   s = r - alpha v               (r := s, a := r, b := v)
//   kBicgUpd x += alpha p + omega s, r = s - omega t, partials <r0, r>, |r|^2
//            (x, r, a := p, b := s, c := t, d := r0)
//   kBicgP   p = r + beta (p - omega v)    (r := p, a := r, b := v)
// and reductions kBicgInit (rho = |r0|^2), kBicgAlpha (alpha = rho / <r0, v>
// from the stencil's fused sums against r0), kBicgBeta (beta, rho, |r|^2).
enum { kBicgS = 0, kBicgUpd = 1, kBicgP = 2 };
enum { kBicgInit = 0, kBicgAlpha = 1, kBicgBeta = 2 };
hipError_t launch_bicg(int prec, int mode, const BlasShape &sh, void *x, void *r, const void *a,
                       const void *b, const void *c, const void *d, const double2 *sc,
                       double *partials, hipStream_t st);
hipError_t launch_bicg_reduce(int mode, const double *partials, int nparts, int nrhs, double2 *sc,
                              double *out2, const double *thr2, int *active, hipStream_t st);

// V-cycle (kernels_vcycle.hip): blocked links of the next level, restriction
// to / prolongation from the coarse sites (canonical fields), and linear
// combinations and dot products of canonical FP64 fields.
struct VcCoef {
    int n;                     // inputs in use, 1..3
    double2 c[3][kMaxRhs];     // per input and RHS
};
hipError_t launch_vc_block_links(const Geom &gf, const void *U64, const Geom &gc, double *out, hipStream_t st);
hipError_t launch_vc_restrict(const double *full, double *coarse, const int32_t *q, int nb, int V, int nrhs,
                              hipStream_t st);
hipError_t launch_vc_prolong(const double *coarse, double *full, const int32_t *q, int nb, int V, int nrhs,
                             hipStream_t st);
hipError_t launch_vc_lincomb(size_t len, int nrhs, const VcCoef &cf, double *out, const double *in0,
                             const double *in1, const double *in2, hipStream_t st);
int vc_dot_grid(size_t len);
hipError_t launch_vc_dot(size_t len, int nrhs, const double *a, const double *b, double *partials,
                         hipStream_t st);

// GCR(m > 1): <q_j, q> for j < k, then q -= sum beta_j q_j, p -= sum beta_j p_j
// with beta_j = <q_j, q>/|q_j|^2, fused with the partials of
// (re<q,r>, im<q,r>, |q|^2) for the step length.
hipError_t launch_multidot(int prec, const BlasShape &sh, const void *Q, int k, const void *q,
                           double *partials, hipStream_t st);
hipError_t launch_reduce_multi(const double *partials, int nparts, int nrhs, int k,
                               const double *qnorm2, const int *active, double2 *beta,
                               hipStream_t st);
hipError_t launch_orthogonalise(int prec, const BlasShape &sh, const void *Q, const void *P,
                                int k, const double2 *beta, void *q, void *p, const void *r,
                                double *partials, hipStream_t st);

}  // namespace grg
