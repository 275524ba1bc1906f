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
};

struct BatchBlasArgs {
    BatchTable bt;
    int Vtot;
    int nrhs;
    int grid;
    const double2 *alpha;  // per system (mr update)
    double *partials;      // [grid][nlat * nrhs]
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
hipError_t launch_batch_coarse(const BatchTable &bt, const void *in, const void *U, double *yb,
                               const int32_t *qg, const int *clat, const int *nb, const int *nboff,
                               const long long *coff, int nbtot, int nrhs, hipStream_t st);

}  // namespace grg
