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
    const uint8_t *mask;  // 1 on coarse sites (the reduced mode: 0 / 2 on the rest sites of the
                          // reduced parity / the other parity)
    int sel;              // rows kept: mask[s] == sel
    BatchTable bt;
    int Vtot;             // total sites (a multiple of 256)
    int nrhs;             // right-hand sides per lattice
    int RG;
    double *partials;     // [grid][nlat * nrhs][3] or nullptr
    const int *act;       // per-system flags, or nullptr: with flags, systems whose flag is 0
                          // are skipped and a launch with no flag set returns at once
    // the even-odd reduced mode (ca != nullptr): out = ca[l] in2 + cb[l] H in on the
    // kept rows, H the hopping term of D (no diagonal), in2 == nullptr read as zero;
    // the fused sums are taken with in2; with keep, rows not kept are left as they are
    // (else written as zero)
    const void *in2 = nullptr;
    const double *ca = nullptr, *cb = nullptr;
    int keep = 0;
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
// y = x on the sites with mask[s] == sel, zero elsewhere (every RHS, precision prec)
hipError_t launch_batch_select(int prec, const BatchBlasArgs &a, const uint8_t *mask, int sel, const void *x,
                               void *y, hipStream_t st);
hipError_t launch_batch_coarse(const BatchTable &bt, const void *in, const void *U, double *yb,
                               const int32_t *qg, const int *clat, const int *nb, const int *nboff,
                               const long long *coff, int nbtot, int nrhs, hipStream_t st);

}  // namespace grg
