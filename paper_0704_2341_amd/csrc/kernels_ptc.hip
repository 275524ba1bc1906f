// Kernels of the learned preconditioner: a linear gauge-covariant convolution
// network (parallel-transported nearest-neighbour hops, channel mixing by
// complex weights, no bias, no activation function), its adjoint, its weight
// gradients, the loss and an Adam step.
//
// One layer:  Y_f(x) = sum_{h=0..8} sum_f' W_h[f, f'] (T_h X_f')(x), with
// T_0 = 1, T_{+mu} X(x) = U_mu(x) X(x+mu), T_{-mu} X(x) = U_mu(x-mu)^+ X(x-mu)
// (hop order 0, +x, -x, +y, -y, +z, -z, +t, -t; boundary signs folded in the
// links as for the stencil).
//
// Work split on gfx950: a workgroup takes 64 sites of one right-hand side.
// Phase 1 gathers the 9 transported neighbour fields (FP32 SU(3) products on
// the vector ALUs) into LDS as a bf16 matrix B[(site, colour)][(hop, f', re/im)].
// Phase 2 mixes channels on the matrix cores: with the complex weights embedded
// as a real matrix A[(f, re/im)][(hop, f', re/im)] (16 rows), Y = A B^T is a
// 16 x K by K x 192 product done with v_mfma_f32_16x16x32_bf16 (bf16 operands,
// FP32 accumulation), lane l holding A[l%16][8(l/16)+j], B[8(l/16)+j][l%16]
// and C[4(l/16)+i][l%16].
//
// Activations are bf16 complex in the tiled field layout with F*3 components
// per site (F colour vectors); a Dirac field is the F = 4 case.
#include "common.h"
#include "engine.h"
#include "ptc.h"
#include "stencil.h"

namespace grg {

typedef __bf16 bf16x8_v __attribute__((ext_vector_type(8)));
typedef float f32x4_v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ size_t aidx(int s, int r, int k, int nrhs, int F3)
{
    return ((((size_t)(s >> 6) * nrhs + r) * F3 + k) << 6) + (s & 63);
}

// A lane's site and its coordinates (computed once per tile).
struct LaneSite {
    int s, x[4];
};

__device__ __forceinline__ LaneSite lane_site(int s, const Geom &g)
{
    LaneSite c;
    c.s = s;
    const int t1 = s / g.L[0], t2 = t1 / g.L[1];
    c.x[0] = s - t1 * g.L[0];
    c.x[1] = t1 - t2 * g.L[1];
    c.x[3] = t2 / g.L[2];
    c.x[2] = t2 - c.x[3] * g.L[2];
    return c;
}

// An opaque copy: what is derived from the site (neighbour and link
// addresses) is recomputed where it is used instead of being hoisted out of
// the right-hand-side loop into registers for every task.
__device__ __forceinline__ void opaque_site(LaneSite &c)
{
    asm volatile("" : "+v"(c.s), "+v"(c.x[0]), "+v"(c.x[1]), "+v"(c.x[2]), "+v"(c.x[3]));
}

// neighbour of the lane's site for hop h (0 = the site itself) and the site
// whose link the hop uses
__device__ __forceinline__ void ptc_hop_site(const LaneSite &c, int h, const Geom &g, int &n, int &ls)
{
    if (h == 0) {
        n = ls = c.s;
        return;
    }
    const int mu = (h - 1) >> 1;
    const bool fwd = ((h - 1) & 1) == 0;
    const int L = mu == 0 ? g.L[0] : mu == 1 ? g.L[1] : mu == 2 ? g.L[2] : g.L[3];
    const int x = mu == 0 ? c.x[0] : mu == 1 ? c.x[1] : mu == 2 ? c.x[2] : c.x[3];
    const int st = mu == 0 ? 1 : mu == 1 ? g.L[0] : mu == 2 ? g.L[0] * g.L[1] : g.L[0] * g.L[1] * g.L[2];
    const int sp = x == L - 1 ? c.s - (L - 1) * st : c.s + st;
    const int sm = x == 0 ? c.s + (L - 1) * st : c.s - st;
    n = fwd ? sp : sm;
    ls = fwd ? c.s : sm;
}

// One gather task's operands: the raw link of the hop and the FH channels'
// colour vectors of the neighbour.
template <int FH>
struct GatherOps {
    uint32_t m[9];
    uint32_t v[FH][3];
};

template <int FIN, int FH>
__device__ __forceinline__ void ptc_task_load(int h, int f0, int n, int ls, const bf16x2 *__restrict__ x,
                                              const bf16x2 *__restrict__ U, int r, int nrhs,
                                              GatherOps<FH> &o)
{
    if (h > 0) {
        const int mu = (h - 1) >> 1;
#pragma unroll
        for (int e = 0; e < 9; ++e) o.m[e] = U[lidx(ls, mu, e)];
    }
#pragma unroll
    for (int i = 0; i < FH; ++i) {
        const int f = min(f0 + i, FIN - 1);
#pragma unroll
        for (int a = 0; a < 3; ++a) o.v[i][a] = x[aidx(n, r, 3 * f + a, nrhs, 3 * FIN)];
    }
}

template <int FIN, int FH, bool ROWK, int LD>
__device__ __forceinline__ void ptc_task_store(int h, int f0, const GatherOps<FH> &o, bool valid,
                                               int lane, __bf16 *lds, int kbase)
{
    const int f1 = min(f0 + FH, FIN);
    const bool fwd = h > 0 && ((h - 1) & 1) == 0;
    // link forms, fr[3a + b] and fi[3a + b] for output colour a
    uint32_t fr[9], fi[9];
    if (h > 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const uint32_t m = o.m[fwd ? 3 * a + b : 3 * b + a];
                fr[3 * a + b] = fwd ? m ^ kNegHi : m;
                fi[3 * a + b] = fwd ? swap_halves(m) : swap_halves(m) ^ kNegLo;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < FH; ++i) {
        const int f = f0 + i;
        if (f >= f1) break;
        uint32_t w[3];
        if (h == 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) w[a] = o.v[i][a];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float re = 0.f, im = 0.f;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    re = dot2bf(fr[3 * a + b], o.v[i][b], re);
                    im = dot2bf(fi[3 * a + b], o.v[i][b], im);
                }
                w[a] = pack_bf16(re, im);
            }
        }
        const int k0 = (h * FIN + f) * 2 - kbase;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int col = lane * 3 + a;
            const uint32_t word = valid ? w[a] : 0u;
            if (ROWK) {
                // (re, im) adjacent in a row: one 32-bit store (k0 even, LD even)
                *(uint32_t *)(lds + col * LD + k0) = word;
            } else {
                lds[k0 * LD + col] = __builtin_bit_cast(__bf16, (uint16_t)(word & 0xffffu));
                lds[(k0 + 1) * LD + col] = __builtin_bit_cast(__bf16, (uint16_t)(word >> 16));
            }
        }
    }
}

// Phase 1: T_h X_f' for hops [H0, H1), right-hand side r, the 64 sites of a
// tile into LDS.  Row-major layout B[row][col]: ROWK = true puts the (hop,
// f', re/im) index contiguous (rows = (site, colour)), ROWK = false puts the
// (site, colour) index contiguous; the (hop, f', re/im) index is stored
// relative to kbase.
//
// The transports run on packed BF16 operands: each complex product of a link
// entry m with a colour component x is two two-way BF16 dot products (exact
// products, FP32 sums) against the forms (m.re, -m.im), (m.im, m.re) for U x
// and (m.re, m.im), (-m.im, m.re) for U^+ x, made once per task and shared by
// its channels.  A wavefront loads its next slot's operands before it
// transports the current one, so that the memory latency of its tasks
// overlaps.
template <int FIN, bool ROWK, int LD>
__device__ __forceinline__ void ptc_gather(const bf16x2 *__restrict__ x, const bf16x2 *__restrict__ U,
                                           const Geom &g, const LaneSite &c, bool valid, int r, int nrhs,
                                           __bf16 *lds, int h0, int h1, int kbase)
{
    constexpr int FH = (FIN + 1) / 2;  // channels per task
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ntask = 2 * (h1 - h0);
    int task = wv;
    if (task >= ntask) return;
    auto load = [&](int t, GatherOps<FH> &o) {
        const int h = h0 + (t >> 1);
        int n, ls;
        ptc_hop_site(c, h, g, n, ls);
        ptc_task_load<FIN, FH>(h, (t & 1) * FH, n, ls, x, U, r, nrhs, o);
    };
    GatherOps<FH> A, B;
    load(task, A);
    for (;;) {
        const bool more = task + 4 < ntask;
        if (more) load(task + 4, B);
        ptc_task_store<FIN, FH, ROWK, LD>(h0 + (task >> 1), (task & 1) * FH, A, valid, lane, lds, kbase);
        if (!more) break;
        task += 4;
        const bool more2 = task + 4 < ntask;
        if (more2) load(task + 4, A);
        ptc_task_store<FIN, FH, ROWK, LD>(h0 + (task >> 1), (task & 1) * FH, B, valid, lane, lds, kbase);
        if (!more2) break;
        task += 4;
    }
}

// ------------------------------------------------------------------ layer
template <int FIN, int FOUT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) ptc_layer_kernel(PtcLayerArgs a)
{
    constexpr int KR = 9 * FIN * 2;
    constexpr int KP = (KR + 31) / 32 * 32;
    constexpr int NS = KP / 32;
    // The K dimension in two passes, hops 0..3 and 4..8 (K1 = 4 * FIN * 2 is a
    // whole number of 32-wide MFMA steps), so that LDS holds half the
    // transported fields at a time and four or five workgroups share a CU.
    constexpr int K1 = 4 * FIN * 2, NS1 = K1 / 32, K2 = KP - K1;
    constexpr int LD = (K1 > K2 ? K1 : K2) + 8;  // bf16 per LDS row (16-byte aligned rows)
    static_assert(K1 % 32 == 0, "first pass must be whole MFMA steps");
    __shared__ __attribute__((aligned(16))) __bf16 lds[192 * LD];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // zero the second pass's padding columns once; the gathers never write them
    for (int i = threadIdx.x; i < 192 * (KP - KR); i += blockDim.x)
        lds[(i / (KP - KR)) * LD + (KR - K1) + i % (KP - KR)] = (__bf16)0.f;
    // this lane's weight fragments: A[l%16][32 s + 8 (l/16) + j]
    // the embedded weights A[16][KP] in LDS (read per MFMA step rather than
    // held in registers: the gather's double-buffered operands need them)
    __shared__ __attribute__((aligned(16))) __bf16 wl[16 * KP];
    for (int i = threadIdx.x; i < 16 * KP / 8; i += blockDim.x)
        *(bf16x8_v *)(wl + 8 * i) = *(const bf16x8_v *)(a.A + 8 * i);
    const __bf16 *arow = wl + (lane & 15) * KP + 8 * (lane >> 4);
    const bf16x2 *x = (const bf16x2 *)a.x;
    bf16x2 *y = (bf16x2 *)a.y;
    const bf16x2 *U = (const bf16x2 *)a.U;
    // work items: (tile, group of rc right-hand sides); the sites a tile's
    // gather reads are found once per item
    const int ntiles = (a.g.V + 63) >> 6;
    const int ngrp = (a.nrhs + a.rc - 1) / a.rc;
    const int nitems = ntiles * ngrp;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int tile = w / ngrp, grp = w - tile * ngrp;
        const int r0 = grp * a.rc, r1 = min(r0 + a.rc, a.nrhs);
        const int s = tile * 64 + lane;
        const bool valid = s < a.g.V;
        const LaneSite ls = lane_site(valid ? s : 0, a.g);
        // this lane's output columns 16 t + l%16 = (site, colour), t = wv + 4 i
        bool on[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int site = tile * 64 + (16 * (wv + 4 * i) + (lane & 15)) / 3;
            on[i] = site < a.g.V && (a.mask == nullptr || a.mask[site] == a.sel);
        }
        for (int r = r0; r < r1; ++r) {
            // the links are re-read for every right-hand side (L1 hits): an
            // opaque copy of the pointer keeps the compiler from hoisting
            // the loads, and the link forms made from them, out of this loop
            // into registers the occupancy cannot spare
            const bf16x2 *Ur = U;
            asm volatile("" : "+s"(Ur));
            LaneSite lc = ls;
            opaque_site(lc);
            f32x4_v c[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) c[i] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int pass = 0; pass < 2; ++pass) {
                __syncthreads();  // the previous products are out of LDS
                if (pass == 0) ptc_gather<FIN, true, LD>(x, Ur, a.g, lc, valid, r, a.nrhs, lds, 0, 4, 0);
                else ptc_gather<FIN, true, LD>(x, Ur, a.g, lc, valid, r, a.nrhs, lds, 4, 9, K1);
                __syncthreads();
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int t = wv + 4 * i;
                    const __bf16 *brow = lds + (16 * t + (lane & 15)) * LD + 8 * (lane >> 4);
#pragma unroll
                    for (int k = (pass == 0 ? 0 : NS1); k < (pass == 0 ? NS1 : NS); ++k) {
                        const bf16x8_v bf = *(const bf16x8_v *)(brow + 32 * (k - (pass == 0 ? 0 : NS1)));
                        const bf16x8_v af = *(const bf16x8_v *)(arow + 32 * k);
                        c[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, c[i], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int t = wv + 4 * i;
                // rows 4 (l/16) + q = (f, re/im): two complex outputs per lane
                const int col = 16 * t + (lane & 15);
                const int site = tile * 64 + col / 3, colour = col % 3;
                if (site < a.g.V) {
                    const int f0 = 2 * (lane >> 4);
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int f = f0 + q;
                        if (f < FOUT) {
                            const float re = on[i] ? c[i][2 * q] : 0.f, im = on[i] ? c[i][2 * q + 1] : 0.f;
                            y[aidx(site, r, 3 * f + colour, a.nrhs, 3 * FOUT)] = pack_bf16(re, im);
                        }
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ weight gradient
// C[(g, re/im)][(h, f', re/im)] = sum over sites and colours of dY * (T_h X),
// accumulated per workgroup; partial[blockIdx][16][NP] in FP32.
template <int FIN, int FOUT>
__global__ void __launch_bounds__(256) ptc_wgrad_kernel(PtcGradArgs a)
{
    constexpr int KR = 9 * FIN * 2;
    constexpr int NP = (KR + 15) / 16 * 16;
    constexpr int LD = 192 + 8;
    constexpr int NT = NP / 16;
    __shared__ __attribute__((aligned(16))) __bf16 tx[NP * LD];
    __shared__ __attribute__((aligned(16))) __bf16 dy[16 * LD];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < (NP - KR) * LD; i += blockDim.x) tx[KR * LD + i] = (__bf16)0.f;
    for (int i = threadIdx.x; i < 16 * LD; i += blockDim.x) dy[i] = (__bf16)0.f;
    f32x4_v acc[(NT + 3) / 4];
#pragma unroll
    for (int k = 0; k < (NT + 3) / 4; ++k) acc[k] = {0.f, 0.f, 0.f, 0.f};
    const bf16x2 *x = (const bf16x2 *)a.x;
    const bf16x2 *dyg = (const bf16x2 *)a.dy;
    const bf16x2 *U = (const bf16x2 *)a.U;
    const int ntiles = (a.g.V + 63) >> 6;
    const int ngrp = (a.nrhs + a.rc - 1) / a.rc;
    const int nitems = ntiles * ngrp;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int tile = w / ngrp, grp = w - tile * ngrp;
        const int r0 = grp * a.rc, r1 = min(r0 + a.rc, a.nrhs);
        const int s = tile * 64 + lane;
        const bool valid = s < a.g.V;
        const LaneSite ls = lane_site(valid ? s : 0, a.g);
        for (int r = r0; r < r1; ++r) {
            const bf16x2 *Ur = U;  // not hoisted (as in the layer kernel)
            asm volatile("" : "+s"(Ur));
            LaneSite lc = ls;
            opaque_site(lc);
            __syncthreads();
            ptc_gather<FIN, false, LD>(x, Ur, a.g, lc, valid, r, a.nrhs, tx, 0, 9, 0);
            // dY rows (g, re/im), columns (site, colour)
            for (int gch = wv; gch < FOUT; gch += 4) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const cpx<float> v = valid ? ldc(dyg, aidx(s, r, 3 * gch + c, a.nrhs, 3 * FOUT))
                                               : cpx<float>{0.f, 0.f};
                    dy[(2 * gch) * LD + lane * 3 + c] = (__bf16)v.re;
                    dy[(2 * gch + 1) * LD + lane * 3 + c] = (__bf16)v.im;
                }
            }
            __syncthreads();
            int k = 0;
            for (int t = wv; t < NT; t += 4, ++k) {
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    const bf16x8_v af = *(const bf16x8_v *)(dy + (lane & 15) * LD + 32 * q + 8 * (lane >> 4));
                    const bf16x8_v bf =
                        *(const bf16x8_v *)(tx + (16 * t + (lane & 15)) * LD + 32 * q + 8 * (lane >> 4));
                    acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[k], 0, 0, 0);
                }
            }
        }
    }
    // partial[blockIdx][row][col]: lane holds rows 4 (l/16) + i of column 16 t + l%16
    int k = 0;
    for (int t = wv; t < NT; t += 4, ++k) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 4 * (lane >> 4) + i, col = 16 * t + (lane & 15);
            a.partials[((size_t)blockIdx.x * 16 + row) * NP + col] = acc[k][i];
        }
    }
}

// partials -> dL/dconj(W) (complex [9][FOUT][FIN], FP64), fixed-order sum;
// out += result when accumulate.
template <int FIN, int FOUT>
__global__ void ptc_wgrad_reduce_kernel(const float *partials, int nparts, double2 *out)
{
    constexpr int KR = 9 * FIN * 2;
    constexpr int NP = (KR + 15) / 16 * 16;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // (h, g, f')
    if (i >= 9 * FOUT * FIN) return;
    const int h = i / (FOUT * FIN), gch = (i / FIN) % FOUT, f = i % FIN;
    const int cre = (h * FIN + f) * 2, cim = cre + 1;
    const int rre = 2 * gch, rim = rre + 1;
    double rr = 0, ri = 0, ir = 0, ii = 0;
    for (int p = 0; p < nparts; ++p) {
        const float *P = partials + (size_t)p * 16 * NP;
        rr += P[rre * NP + cre];
        ri += P[rre * NP + cim];
        ir += P[rim * NP + cre];
        ii += P[rim * NP + cim];
    }
    // dY conj(TX) = (re re + im im) + i (im re - re im)
    out[i] = make_double2(rr + ii, ir - ri);
}

// ------------------------------------------------------------------ weights
// complex W[9][FOUT][FIN] (FP64) -> real-embedded bf16 A[16][KP]:
//   A[2f][2(h FIN + f')] = Re W, A[2f][2(h FIN + f') + 1] = -Im W,
//   A[2f+1][2(h FIN + f')] = Im W, A[2f+1][2(h FIN + f') + 1] = Re W;
// adjoint != 0 builds the weights of the adjoint layer instead:
//   W'_h[f'][f] = conj(W_{rev h}[f][f']), rev swapping +mu and -mu.
template <int FIN, int FOUT>
__global__ void ptc_embed_kernel(const double2 *w, __bf16 *A, int adjoint)
{
    constexpr int FI = FIN, FO = FOUT;
    // the layer whose A is built has FI' inputs and FO' outputs
    const int fin = adjoint ? FO : FI, fout = adjoint ? FI : FO;
    const int KP = (9 * fin * 2 + 31) / 32 * 32;
    for (int i = threadIdx.x; i < 16 * KP; i += blockDim.x) {
        const int row = i / KP, k = i % KP;
        float v = 0.f;
        const int f = row >> 1, ri = row & 1;
        if (f < fout && k < 9 * fin * 2) {
            const int h = k / (2 * fin), fp = (k / 2) % fin, ci = k & 1;
            double2 c;
            if (!adjoint) {
                c = w[(h * FO + f) * FI + fp];
            } else {
                const int hr = h == 0 ? 0 : (((h - 1) ^ 1) + 1);
                const double2 o = w[(hr * FO + fp) * FI + f];
                c = make_double2(o.x, -o.y);
            }
            const double re = c.x, im = c.y;
            v = (float)(ri == 0 ? (ci == 0 ? re : -im) : (ci == 0 ? im : re));
        }
        A[i] = (__bf16)v;
    }
}

// ------------------------------------------------------------------ loss
// Per pair: loss_i = |y - e|^2 / |e|^2 / B and dY = (y - e) / |e|^2 / B.
// Partials per workgroup and pair: (|y - e|^2, |e|^2); the second kernel
// turns them into dY once the norms are known.
__global__ void __launch_bounds__(256) ptc_loss_partials_kernel(const bf16x2 *y, const bf16x2 *e,
                                                                Geom g, int nrhs, double *partials)
{
    __shared__ double red[4][kMaxRhs][2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = lane; i < nrhs * 2; i += 64) red[wv][i / 2][i % 2] = 0.0;
    __syncthreads();
    const int nsb = (g.V + 255) / 256;
    for (int b = blockIdx.x; b < nsb; b += gridDim.x) {
        const int s = b * 256 + threadIdx.x;
        for (int r = 0; r < nrhs; ++r) {
            float d2 = 0.f, e2 = 0.f;
            if (s < g.V) {
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const size_t i = fidx(s, r, c, nrhs);
                    const cpx<float> yv = ldc(y, i), ev = ldc(e, i);
                    const float dre = yv.re - ev.re, dim = yv.im - ev.im;
                    d2 = fmaf(dre, dre, fmaf(dim, dim, d2));
                    e2 = fmaf(ev.re, ev.re, fmaf(ev.im, ev.im, e2));
                }
            }
            const double sd = wave_sum((double)d2), se = wave_sum((double)e2);
            if (lane == 0) {
                red[wv][r][0] += sd;
                red[wv][r][1] += se;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nrhs * 2; i += blockDim.x) {
        double t = 0;
        for (int k = 0; k < 4; ++k) t += red[k][i / 2][i % 2];
        partials[(size_t)blockIdx.x * nrhs * 2 + i] = t;
    }
}

// sums[r] = (|y - e|^2, |e|^2) from the partials; loss = sum_r d2/e2/B
__global__ void ptc_loss_reduce_kernel(const double *partials, int nparts, int nrhs, double *sums,
                                       double *loss)
{
    __shared__ double tot[kMaxRhs];
    const int r = threadIdx.x;
    if (r < nrhs) {
        double d2 = 0, e2 = 0;
        for (int p = 0; p < nparts; ++p) {
            d2 += partials[((size_t)p * nrhs + r) * 2];
            e2 += partials[((size_t)p * nrhs + r) * 2 + 1];
        }
        sums[2 * r] = d2;
        sums[2 * r + 1] = e2;
        tot[r] = e2 > 0 ? d2 / e2 / nrhs : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double l = 0;
        for (int k = 0; k < nrhs; ++k) l += tot[k];
        *loss = l;
    }
}

__global__ void __launch_bounds__(256) ptc_dy_kernel(const bf16x2 *y, const bf16x2 *e, Geom g,
                                                     int nrhs, const double *sums, bf16x2 *dy)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V || r >= nrhs) return;
    const double e2 = sums[2 * r + 1];
    const float f = e2 > 0 ? (float)(1.0 / (e2 * nrhs)) : 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const size_t i = fidx(s, r, c, nrhs);
        const cpx<float> yv = ldc(y, i), ev = ldc(e, i);
        dy[i] = pack_bf16(f * (yv.re - ev.re), f * (yv.im - ev.im));
    }
}

// ------------------------------------------------------------------ Adam
// Real parameters p (re and im of every weight), real gradient 2 dL/dconj(W).
__global__ void ptc_adam_kernel(double *w, const double *gconj, double *m, double *v, int n,
                                double lr, double b1, double b2, double eps, int step)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double g = 2.0 * gconj[i];
    m[i] = b1 * m[i] + (1 - b1) * g;
    v[i] = b2 * v[i] + (1 - b2) * g * g;
    const double mh = m[i] / (1 - pow(b1, (double)step));
    const double vh = v[i] / (1 - pow(b2, (double)step));
    w[i] -= lr * mh / (sqrt(vh) + eps);
}

// ------------------------------------------------------------------ random fields
// Gaussian complex field on the r-sites (mask[s] == 0), zero on coarse sites,
// stored bf16; counter-based: SplitMix64 (Steele, Lea and Flood 2014) of
// (seed, counter) gives two uniforms, Box-Muller gives the normal pair.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

template <int P>
__global__ void random_field_kernel(void *out, const uint8_t *mask, Geom g, int nrhs, uint64_t seed)
{
    typedef typename Store<P>::S S;
    typedef typename Store<P>::R R;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= g.V || r >= nrhs) return;
    const bool on = mask == nullptr || mask[s] == 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const uint64_t ctr = (((uint64_t)r * g.V + s) * 12 + c);
        const uint64_t h1 = splitmix64(seed ^ splitmix64(2 * ctr)), h2 = splitmix64(seed ^ splitmix64(2 * ctr + 1));
        const double u1 = ((h1 >> 11) + 1) * (1.0 / 9007199254740993.0);  // (0, 1]
        const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);        // [0, 1)
        const double rad = sqrt(-2.0 * log(u1)), th = 6.283185307179586 * u2;
        cpx<R> v = {on ? (R)(rad * cos(th)) : (R)0, on ? (R)(rad * sin(th)) : (R)0};
        stc((S *)out, fidx(s, r, c, nrhs), v);
    }
}

// ------------------------------------------------------------------ launchers
// Resident workgroups of a network kernel on the current device (cached per
// kernel: the occupancy depends on the kernel's registers and LDS only).
template <typename K>
static int ptc_resident(K kernel, int slot)
{
    static int cache[8] = {};
    if (cache[slot] > 0) return cache[slot];
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess || per < 1 ||
        cus < 1)
        return 1024;
    cache[slot] = per * cus;
    return cache[slot];
}

int ptc_launch_shape(int kind, int fin, int fout, const Geom &g, int nrhs, int *rc)
{
    int res = 1024;
    const int slot = kind * 3 + (fin == 4 ? 0 : fout == 8 ? 1 : 2);
    if (kind == 0) {
        if (fin == 4) res = ptc_resident(ptc_layer_kernel<4, 8>, slot);
        else if (fout == 8) res = ptc_resident(ptc_layer_kernel<8, 8>, slot);
        else res = ptc_resident(ptc_layer_kernel<8, 4>, slot);
    } else {
        if (fin == 4) res = ptc_resident(ptc_wgrad_kernel<4, 8>, slot);
        else if (fout == 8) res = ptc_resident(ptc_wgrad_kernel<8, 8>, slot);
        else res = ptc_resident(ptc_wgrad_kernel<8, 4>, slot);
    }
    res = std::max(1, std::min(res, kPtcMaxGrid));
    const long ntiles = (g.V + 63) / 64;
    // RHS groups: enough work items for about four per workgroup
    const long want = 4L * res;
    const int ngrp = (int)std::max(1L, std::min<long>(nrhs, (want + ntiles - 1) / ntiles));
    const int r = (nrhs + ngrp - 1) / ngrp;
    *rc = std::max(1, r);
    const long items = ntiles * ((nrhs + *rc - 1) / *rc);
    return (int)std::max(1L, std::min<long>(items, res));
}

hipError_t launch_ptc_layer(int fin, int fout, const PtcLayerArgs &a, int grid, hipStream_t st)
{
    dim3 g(grid), b(256);
    if (fin == 4 && fout == 8) hipLaunchKernelGGL((ptc_layer_kernel<4, 8>), g, b, 0, st, a);
    else if (fin == 8 && fout == 8) hipLaunchKernelGGL((ptc_layer_kernel<8, 8>), g, b, 0, st, a);
    else if (fin == 8 && fout == 4) hipLaunchKernelGGL((ptc_layer_kernel<8, 4>), g, b, 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ptc_wgrad(int fin, int fout, const PtcGradArgs &a, int grid, hipStream_t st)
{
    dim3 g(grid), b(256);
    if (fin == 4 && fout == 8) hipLaunchKernelGGL((ptc_wgrad_kernel<4, 8>), g, b, 0, st, a);
    else if (fin == 8 && fout == 8) hipLaunchKernelGGL((ptc_wgrad_kernel<8, 8>), g, b, 0, st, a);
    else if (fin == 8 && fout == 4) hipLaunchKernelGGL((ptc_wgrad_kernel<8, 4>), g, b, 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ptc_wgrad_reduce(int fin, int fout, const float *partials, int nparts,
                                   double2 *out, hipStream_t st)
{
    const int n = 9 * fin * fout;
    dim3 g((n + 127) / 128), b(128);
    if (fin == 4 && fout == 8) hipLaunchKernelGGL((ptc_wgrad_reduce_kernel<4, 8>), g, b, 0, st, partials, nparts, out);
    else if (fin == 8 && fout == 8) hipLaunchKernelGGL((ptc_wgrad_reduce_kernel<8, 8>), g, b, 0, st, partials, nparts, out);
    else if (fin == 8 && fout == 4) hipLaunchKernelGGL((ptc_wgrad_reduce_kernel<8, 4>), g, b, 0, st, partials, nparts, out);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ptc_embed(int fin, int fout, const double2 *w, __bf16 *A, int adjoint, hipStream_t st)
{
    if (fin == 4 && fout == 8) hipLaunchKernelGGL((ptc_embed_kernel<4, 8>), dim3(1), dim3(256), 0, st, w, A, adjoint);
    else if (fin == 8 && fout == 8) hipLaunchKernelGGL((ptc_embed_kernel<8, 8>), dim3(1), dim3(256), 0, st, w, A, adjoint);
    else if (fin == 8 && fout == 4) hipLaunchKernelGGL((ptc_embed_kernel<8, 4>), dim3(1), dim3(256), 0, st, w, A, adjoint);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ptc_loss(const void *y, const void *e, const Geom &g, int nrhs, double *partials,
                           int grid, double *sums, double *loss, void *dy, hipStream_t st)
{
    hipLaunchKernelGGL(ptc_loss_partials_kernel, dim3(grid), dim3(256), 0, st, (const bf16x2 *)y,
                       (const bf16x2 *)e, g, nrhs, partials);
    hipLaunchKernelGGL(ptc_loss_reduce_kernel, dim3(1), dim3(64), 0, st, partials, grid, nrhs, sums, loss);
    if (dy)
        hipLaunchKernelGGL(ptc_dy_kernel, dim3((g.V + 255) / 256, nrhs), dim3(256), 0, st,
                           (const bf16x2 *)y, (const bf16x2 *)e, g, nrhs, sums, (bf16x2 *)dy);
    return hipGetLastError();
}

hipError_t launch_ptc_adam(double *w, const double *gconj, double *m, double *v, int n, double lr,
                           double b1, double b2, double eps, int step, hipStream_t st)
{
    hipLaunchKernelGGL(ptc_adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, w, gconj, m, v, n,
                       lr, b1, b2, eps, step);
    return hipGetLastError();
}

hipError_t launch_random_field(int prec, void *out, const uint8_t *mask, const Geom &g, int nrhs,
                               uint64_t seed, hipStream_t st)
{
    dim3 grd((g.V + 255) / 256, nrhs), blk(256);
    switch (prec) {
    case GRG_FP64: hipLaunchKernelGGL(random_field_kernel<GRG_FP64>, grd, blk, 0, st, out, mask, g, nrhs, seed); break;
    case GRG_FP32: hipLaunchKernelGGL(random_field_kernel<GRG_FP32>, grd, blk, 0, st, out, mask, g, nrhs, seed); break;
    case GRG_BF16: hipLaunchKernelGGL(random_field_kernel<GRG_BF16>, grd, blk, 0, st, out, mask, g, nrhs, seed); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace grg
