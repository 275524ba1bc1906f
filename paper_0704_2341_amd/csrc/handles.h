// Handle structures behind the opaque grg_lattice / grg_schur pointers.
#pragma once

#include <vector>

#include "engine.h"

struct grg_lattice_s {
    grg::Geom g;
    int bc[4];
    int device;
    hipStream_t stream;
    void *U[3] = {nullptr, nullptr, nullptr};  // internal links per grg_precision
    // even-odd reduction (every extent even): links per parity, compact
    // half-lattice tiles ([2][Vhs / 64][4][9][64] per precision)
    bool eo_ok = false;
    int Vhs = 0;
    void *Ueo[3] = {nullptr, nullptr, nullptr};
    bool gauge_set = false;
    int gauge_version = 0;  // incremented by every grg_gauge_set (caches derived from the links)
    // grow-only scratch of grg_dirac_apply
    void *tmp_in = nullptr, *tmp_out = nullptr;
    size_t tmp_bytes = 0;
    double *tmp_links = nullptr;  // staging of host links
};

namespace grg {

// Slots of the event-timed profile: 0..2 full-lattice stencil per precision,
// 3..5 even-odd half-stencil, then the phases of a solve.
constexpr int kProfDc = 6, kProfBlas = 7, kProfPrec = 8, kProfSlots = 9;
constexpr int kProfStencilSlots = 6;

struct ProfilePool {
    bool on = false;
    // phases: the solve's phases are timed too; per_call: the event pairs are
    // read back at the end of every call (for the call's stats) rather than
    // when the totals are read
    bool phases = true, per_call = true;
    std::vector<hipEvent_t> start, stop;
    std::vector<int> prec;
    int used = 0;
    long long count[kProfSlots] = {};
    double total_ms[kProfSlots] = {};
};

// Times the enclosed region of a solve (the work it enqueues on the stream)
// into a profile slot when profiling is on.  Reserves its event pair at
// construction, so stencil launches timed inside it keep their own pairs.
struct PhaseTimer {
    ProfilePool *P = nullptr;
    hipStream_t st = nullptr;
    int idx = -1;
    PhaseTimer(ProfilePool &pool, hipStream_t stream, int slot) : P(&pool), st(stream)
    {
        if (!pool.on || !pool.phases || pool.used >= (int)pool.start.size()) return;
        idx = pool.used++;
        pool.prec[idx] = slot;
        (void)hipEventRecord(pool.start[idx], st);
    }
    ~PhaseTimer()
    {
        if (idx >= 0) (void)hipEventRecord(P->stop[idx], st);
    }
    PhaseTimer(const PhaseTimer &) = delete;
    PhaseTimer &operator=(const PhaseTimer &) = delete;
};

}  // namespace grg

// Learned preconditioner: three layer network, weights on the device.
struct grg_precond_s {
    grg_schur schur = nullptr;      // lattice, links and coarse mask it is bound to
    int max_rhs = 0;
    double2 *w = nullptr;           // master weights, kPtcWeights complex (FP64)
    double2 *grad = nullptr;        // dL/dconj(W)
    double *adam_m = nullptr, *adam_v = nullptr;
    int adam_step = 0;
    __bf16 *A[3] = {nullptr, nullptr, nullptr};     // forward layers, [16][KP]
    __bf16 *Aadj[3] = {nullptr, nullptr, nullptr};  // adjoint layers
    void *act[4] = {nullptr, nullptr, nullptr, nullptr};  // bf16 activations
    void *dact[4] = {nullptr, nullptr, nullptr, nullptr}; // their gradients
    void *ebuf = nullptr;           // training targets (bf16 Dirac field)
    void *gen[3] = {nullptr, nullptr, nullptr};  // pair generation: x, r, q (bf16)
    float *wpart = nullptr;         // weight-gradient partials
    double *lpart = nullptr, *lsums = nullptr, *loss = nullptr;
    double *neg_one = nullptr;      // -1 per RHS (e = e_0 - x)
    double *h_buf = nullptr;        // pinned host staging
    bool weights_finite = true;
};

struct grg_schur_s {
    grg_lattice lat;
    double m0;
    int nb;
    grg_solver_params prm;
    std::vector<int32_t> q_host;
    uint8_t *d_mask = nullptr;    // 1 on coarse sites
    int32_t *d_q = nullptr;       // coarse index -> site
    int32_t *d_bidx = nullptr;    // site -> coarse index or -1
    // FP64 outer fields, [max_rhs][12][Vs] each
    void *b64 = nullptr, *x64 = nullptr, *r64 = nullptr, *t64 = nullptr, *u64 = nullptr;
    // the defect correction's residual in FP32 once it is small ([max_rhs][12][Vs]
    // float2, allocated on first use)
    void *r32 = nullptr;
    // inner fields (one set per precision, allocated on first use)
    void *in_b[3] = {nullptr, nullptr, nullptr};
    void *in_x[3] = {nullptr, nullptr, nullptr};
    void *in_r[3] = {nullptr, nullptr, nullptr};
    void *in_q[3] = {nullptr, nullptr, nullptr};
    void *in_P[3] = {nullptr, nullptr, nullptr};  // GCR(m) search directions, m fields
    void *in_Q[3] = {nullptr, nullptr, nullptr};  // their images A p_j
    int in_m[3] = {0, 0, 0};
    // coarse-space staging for assembly
    double *cb_in = nullptr, *cb_out = nullptr;
    // row sums of D_rr (one FP64 field) for the section 3 approximation, and
    // the lattice's gauge_version they were computed from (-1: not yet)
    void *dt64 = nullptr;
    int dt_version = -1;
    // even-odd reduced inner solve: mask per parity ([2][Vhs]), the parity of
    // the reduced system, and compact fields per inner precision: r, x, q
    // (reduced parity), w (other parity) and the preconditioned direction p
    uint8_t *d_mask_eo = nullptr;
    // full-lattice mask of the reduced system: 0 on the rest sites of parity
    // eo_par, 1 elsewhere (training pairs of the reduced system)
    uint8_t *d_mask_par = nullptr;
    // the defect correction's corrections e_k (inner precision, full layout)
    // and their factors: the iterate is summed from them at the end
    std::vector<void *> epool[3];
    double *d_fk = nullptr, *h_fk = nullptr;  // [kCorrPool][kMaxRhs]
    int eo_par = 1;
    void *eo_f[3][5] = {};
    void *eo_b[3] = {};  // the reduced solve's right-hand side as written by the defect
                         // correction: both compact halves, parity eo_par's first
    // BiCGstab: p, v, s, t and the shadow residual (inner precision, full
    // size, also used as compact halves), and rho, alpha, omega, beta per RHS
    void *bicg_f[3][5] = {};
    double2 *bicg_sc = nullptr;
    grg::DslashTune eotune[3][grg::kMaxRhs + 1];
    // the launch of the full-layout half-stencils (first and last step of a
    // reduced solve) when eotune holds the t-marching form and the tuner found
    // this one-hop shape faster for them (not valid: they run eotune too)
    grg::DslashTune eotune_io[3][grg::kMaxRhs + 1];
    // reduction scratch
    double *partials = nullptr;
    size_t partials_elems = 0;
    double2 *alpha = nullptr, *beta = nullptr;
    // per-RHS scalars: residual norms, thresholds, GCR |q_j|^2, and bn2 =
    // [|b|^2 | 1/s | s | next s] of the defect correction (4 kMaxRhs)
    double *rn2 = nullptr, *thr2 = nullptr, *qn2 = nullptr, *bn2 = nullptr;
    int *active = nullptr;
    int *act0 = nullptr;      // RHS active when an inner solve started
    double *h_buf = nullptr;  // pinned host staging (12 * kMaxRhs doubles: reads, uploads, flags)
    grg::ProfilePool prof;
    int n_dslash = 0;
    grg::DslashTune tune[3][grg::kMaxRhs + 1];    // per precision and nrhs
    grg::DslashTune dctune[3][grg::kMaxRhs + 1];  // defect-correction step, per inner precision
    grg_precond precond = nullptr;  // right preconditioner of the inner GCR, or none
    int fallbacks = 0;              // inner solves redone without the preconditioner
};
