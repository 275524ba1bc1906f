// Many-lattice batch: device tables and kernel arguments (kernels_batch.hip).
#pragma once

#include "engine.h"

namespace grg {

// Per-lattice geometry of a concatenated batch (device pointers).
struct BatchTable {
    int nlat;
    const int *tile_lat;  // lattice of every 64-site tile
    const int4 *dims;     // extents per lattice
    const int *off;       // first site of every lattice
    const double *diag;   // 4 + m0 per lattice
};

struct BatchDslashArgs {
    const void *in;
    void *out;
    const void *U;
    const uint8_t *mask;  // 1 on coarse sites
    int sel;              // rows kept: mask[s] == sel
    BatchTable bt;
    int Vtot;             // total sites (a multiple of 256)
    int nrhs;             // right-hand sides per lattice
    int RG;
    double *partials;     // [grid][nlat * nrhs][3] or nullptr
    const int *act;       // per-system flags, or nullptr: with flags, systems whose flag is 0
                          // are skipped and a launch with no flag set returns at once
};

struct BatchBlasArgs {
    BatchTable bt;
    int Vtot;
    int nrhs;
    int grid;
    const double2 *alpha;  // per system (mr update)
    double *partials;      // [grid][nlat * nrhs]
    const int *act;        // per-system flags as in BatchDslashArgs, or nullptr
    int *ctr;              // counter incremented once by a launch that ran (mr update), or nullptr
};

struct BatchDcArgs {
    const void *e;
    const void *U;
    const void *r_in, *x_in;
    void *r_out, *x_out;
    const double *fr2;  // per system
    const uint8_t *mask;
    BatchTable bt;
    int Vtot;
    int nrhs;
    double *partials;
    const int *act;  // per-system flags: systems with 0 are skipped when the update is in place
                     // (r_in == r_out, x_in == x_out); with gate, a launch with no flag set
                     // returns at once; nullptr: every system
    int gate;
    int *ctr;        // incremented once by a launch that ran with a flag set, or nullptr
};

// Device-side control of the batched defect correction (one thread per
// system): from |b|^2 and the FP64 |r|^2 of every system, the active flags
// (relative residual above tol), the inner thresholds on the scaled residual
// and the scales; with init, |r|^2 = |b|^2 first and the counters cleared.
struct BatchCtlArgs {
    int nsys;
    const double *bn2;
    double *rn2;
    double tol, inner_tol;
    int fp64_inner;
    double *thr2, *fr2;
    int *oact;
    int *ctr;  // [inner iterations, outer steps], cleared with init
    int init;
};

hipError_t launch_dslash_batch(int prec, const BatchDslashArgs &a, int grid, int SB, hipStream_t st);
hipError_t launch_batch_mr_update(int prec, const BatchBlasArgs &a, void *x, void *r, const void *q,
                                  hipStream_t st);
hipError_t launch_batch_norm2(int prec, const BatchBlasArgs &a, const void *v, hipStream_t st);
hipError_t launch_batch_axpy_convert(int pin, int pout, const BatchBlasArgs &a, const void *x, void *y,
                                     const double *scale, int mode, int beta, hipStream_t st);
hipError_t launch_batch_sub_norm(const BatchBlasArgs &a, const void *b, const void *ax, void *r,
                                 hipStream_t st);
hipError_t launch_batch_dc_update(int prec, const BatchDcArgs &a, int grid, hipStream_t st);
hipError_t launch_batch_scatter(const BatchTable &bt, const double *xb, void *dst, const int32_t *bidx,
                                const int *nb, const long long *coff, int Vtot, int nrhs, hipStream_t st);
// in_r = r_src / |r| (scale 1 / sqrt(fr2)) in the inner precision and in_x = 0, for the
// systems with a.act set (zero for the others), with the partial |in_r|^2
hipError_t launch_batch_inner_init(int prec, const BatchBlasArgs &a, const void *r_src, const double *fr2,
                                   void *in_r, void *in_x, hipStream_t st);
// The fixed-order reduction of per-workgroup partials per system (modes as
// launch_reduce), gated: with act_in, a launch with no flag set returns at
// once and systems whose flag is 0 keep out2 (kAlpha: alpha 0) and get
// act_out 0; act_out[sys] = |.|^2 > thr2[sys] otherwise (kNorm).
hipError_t launch_batch_reduce(int mode, const double *partials, int nparts, int nsys, double2 *alpha,
                               double *out2, const double *thr2, const int *act_in, int *act_out,
                               hipStream_t st);
hipError_t launch_batch_ctl(const BatchCtlArgs &c, hipStream_t st);
// y = x - y (FP64, every site and RHS)
hipError_t launch_batch_xmy(const BatchBlasArgs &a, const void *x, void *y, hipStream_t st);

// The even-odd reduced form of every lattice's D_rr on compact half-lattice
// fields.  Each lattice's half-sites h (the site pair 2h, 2h + 1 of opposite
// parities: Lx is even) form a block of its own, starting on a 256 boundary
// (padded: entries past V / 2 are zero and stay zero); within a block the
// field of one parity holds at h the site of that parity.  par[l] is the
// parity of lattice l's reduced system (its rest sites there are the fewer).
struct BatchHalf {
    const int *tile_lat;  // lattice of every 64-entry compact tile
    const int *off;       // first compact entry of every lattice
    const int *par;       // the reduced parity per lattice
    const uint8_t *mask;  // [2][Vtot]: 1 on coarse sites and padding, per output side (below)
    int Vtot;             // compact entries of the whole batch (a multiple of 256)
};

// out = ca[l] in2 + cb[l] H in on the output side po (0: each lattice's reduced
// parity, 1: the other), H the hopping term of D (no diagonal); in is a field
// of the other side, in2 one of side po (nullptr: zero).  Rows on coarse
// sites and padding are written as zero.  With partials, the fused sums
// <out, in2>, |out|^2 per system; act as in BatchDslashArgs.
struct BatchEoArgs {
    const void *in, *in2;
    void *out;
    const void *U;        // full-layout links of the batch, in the stencil's precision
    BatchTable bt;        // the full layout (extents, first sites, lattices of full tiles)
    BatchHalf hf;
    int po;
    int nrhs;
    const double *ca, *cb;  // per lattice
    double *partials;       // [grid][nsys][3] or nullptr
    const int *act;
};
hipError_t launch_batch_eo(int prec, const BatchEoArgs &a, int grid, hipStream_t st);
// full-layout field x -> its two halves (xp on each lattice's reduced parity,
// xq on the other), zero on padding; with to_full, the reverse (every site of
// the full field written from the halves)
hipError_t launch_batch_eo_split(int prec, const BatchTable &bt, const BatchHalf &hf, int nrhs, void *x,
                                 void *xp, void *xq, int to_full, int grid, hipStream_t st);
hipError_t launch_batch_coarse(const BatchTable &bt, const void *in, const void *U, double *yb,
                               const int32_t *qg, const int *clat, const int *nb, const int *nboff,
                               const long long *coff, int nbtot, int nrhs, hipStream_t st);

}  // namespace grg
