// Learned preconditioner: kernel arguments and launchers (kernels_ptc.hip).
#pragma once

#include "engine.h"

namespace grg {

constexpr int kPtcLayers = 3;
constexpr int kPtcChannels[kPtcLayers + 1] = {4, 8, 8, 4};
constexpr int kPtcWeights = 9 * (8 * 4 + 8 * 8 + 4 * 8);  // complex weights, all layers

// real-embedded weight matrix of a layer: 16 rows x KP columns, bf16
inline int ptc_kp(int fin) { return (9 * fin * 2 + 31) / 32 * 32; }
// columns of a layer's weight-gradient partials
inline int ptc_np(int fin) { return (9 * fin * 2 + 15) / 16 * 16; }

struct PtcLayerArgs {
    const void *x;        // input activations, bf16 tiles with 3 FIN components
    void *y;              // output activations, bf16 tiles with 3 FOUT components
    const void *U;        // bf16 links
    const __bf16 *A;      // [16][KP] real-embedded weights
    const uint8_t *mask;  // output-site mask or nullptr
    int sel;
    Geom g;
    int nrhs;
    int rc;  // right-hand sides per work item (ptc_launch_shape)
};

struct PtcGradArgs {
    const void *x;   // layer input
    const void *dy;  // dL/dconj(layer output)
    const void *U;
    Geom g;
    int nrhs;
    int rc;           // right-hand sides per work item (ptc_launch_shape)
    float *partials;  // [grid][16][NP]
};

// Largest grid of the layer and weight-gradient kernels (sizes the partials).
constexpr int kPtcMaxGrid = 1024;
// Grid of a layer (kind 0) or weight-gradient (kind 1) launch and, in *rc, the
// right-hand sides each work item takes: as many workgroups as the device
// holds at once (at most kPtcMaxGrid, at most one per work item) and all
// right-hand sides per tile unless the tiles alone give a workgroup fewer
// than about four items.
int ptc_launch_shape(int kind, int fin, int fout, const Geom &g, int nrhs, int *rc);
hipError_t launch_ptc_layer(int fin, int fout, const PtcLayerArgs &a, int grid, hipStream_t st);
hipError_t launch_ptc_wgrad(int fin, int fout, const PtcGradArgs &a, int grid, hipStream_t st);
hipError_t launch_ptc_wgrad_reduce(int fin, int fout, const float *partials, int nparts,
                                   double2 *out, hipStream_t st);
hipError_t launch_ptc_embed(int fin, int fout, const double2 *w, __bf16 *A, int adjoint,
                            hipStream_t st);
hipError_t launch_ptc_loss(const void *y, const void *e, const Geom &g, int nrhs, double *partials,
                           int grid, double *sums, double *loss, void *dy, hipStream_t st);
hipError_t launch_ptc_adam(double *w, const double *gconj, double *m, double *v, int n, double lr,
                           double b1, double b2, double eps, int step, hipStream_t st);
hipError_t launch_random_field(int prec, void *out, const uint8_t *mask, const Geom &g, int nrhs,
                               uint64_t seed, hipStream_t st);

}  // namespace grg
