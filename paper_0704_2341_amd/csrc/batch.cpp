// Many independent lattices solved together: S_bb applies for every lattice
// of the batch in the same launches (kernels_batch.hip).
//
// The method is the single-lattice one (solver.cpp) applied to every
// (lattice, right-hand side) system at once: FP64 defect correction around an
// inner minimal-residual solve in the inner precision, with per-system step
// lengths.  Convergence is decided on the device: per-system flags (inner:
// residual above its threshold; outer: FP64 relative residual above tol) are
// set by the reductions and the control kernel, every kernel of a step skips
// the systems whose flag is clear, and a launch with no flag set returns at
// once.  So the whole apply -- set-up, every outer step with its inner
// iterations, the check of the final residual and the combine -- is one
// sequence of launches with no host decision inside, captured once as a HIP
// graph and replayed; its counts of outer steps and inner iterations per step
// come from an eager apply of the same batch, and an apply the graph did not
// finish is continued eagerly.  The eager mode launches the same kernels and
// reads the flags back every check_every inner iterations.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "batch.h"
#include "handles.h"

namespace grg {

int round8(long v);

struct BatchMember {
    int dims[4], bc[4];
    double m0;
    int V, off, nb, nboff;
    long long coff;
};

}  // namespace grg

struct grg_batch_s {
    int device = 0;
    hipStream_t st = nullptr;      // own stream (capturable), default priority
    hipStream_t caller = nullptr;  // the caller's stream, synchronised with at entry and exit
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int nlat = 0, nrhs = 0, nsys = 0, Vtot = 0, nbtot = 0;
    grg_solver_params prm;
    std::vector<grg::BatchMember> mem;
    grg::Geom gtot;
    void *U[3] = {nullptr, nullptr, nullptr};
    uint8_t *mask = nullptr;
    int32_t *bidx = nullptr, *qg = nullptr;
    int *clat = nullptr, *tile_lat = nullptr, *off = nullptr, *nb = nullptr, *nboff = nullptr;
    int4 *dims = nullptr;
    double *diag = nullptr;
    long long *coff = nullptr;
    void *b64 = nullptr, *x64 = nullptr, *r64 = nullptr, *t64 = nullptr, *u64 = nullptr;
    void *in_b = nullptr, *in_x = nullptr, *in_r = nullptr, *in_q = nullptr;
    // the even-odd reduced inner solve (every extent even, params.eo) on compact
    // half-lattice fields (BatchHalf): per lattice the parity with fewer rest
    // sites carries the reduced system; coef holds per lattice [1, 0, d, 1 / d,
    // -1 / d] (d = 4 + m0) as five arrays; the compact fields (inner precision):
    // the reduced iterate, residual, A r and the intermediate H_qp r, the inner
    // right-hand side's other parity b_q and the reconstructed e_q
    bool eo = false;
    int Vh = 0;  // compact entries (a multiple of 256)
    int *tile_lat_h = nullptr, *off_h = nullptr, *par_h = nullptr;
    uint8_t *mask_h = nullptr;
    double *coef = nullptr;
    void *hx = nullptr, *hr = nullptr, *hq = nullptr, *hw = nullptr, *hbq = nullptr, *heq = nullptr;
    double *partials = nullptr;
    double2 *alpha = nullptr;
    double *thr2 = nullptr, *fr2 = nullptr, *rn2i = nullptr;
    // one block read back at once: FP64 |r|^2, |b|^2 per system, then the
    // counters [inner iterations, outer steps] and the inner flags
    char *dsc = nullptr;
    double *rn2 = nullptr, *bn2 = nullptr;
    int *ctr = nullptr, *active = nullptr;
    size_t dsc_bytes = 0;
    int *oact = nullptr;           // outer flags: FP64 residual above tol
    double *h_buf = nullptr;       // pinned, mirrors dsc
    double *xb_in = nullptr, *yb_out = nullptr;  // coarse staging of the captured apply
    int SB[3] = {64, 64, 64}, RG[3] = {1, 1, 1}, grid[3] = {0, 0, 0};
    float tune_ms[3] = {-1, -1, -1};  // tuned stencil time per launch (every system), per precision
    float upd_ms = -1;                // the inner precision's MR update (every system)
    float eo_ms = -1;                 // with the reduced solve: one half-step (average of the two)
    hipGraphExec_t graph = nullptr;
    int g_outer = 0, g_inner = 0;  // counts the graph was captured with
    int e_outer = 0, e_inner = 0;  // counts the last eager apply needed
};

namespace grg {

static constexpr int kBatchMaxGrid = 2048;

static BatchTable table(grg_batch B)
{
    BatchTable t;
    t.nlat = B->nlat;
    t.tile_lat = B->tile_lat;
    t.dims = B->dims;
    t.off = B->off;
    t.diag = B->diag;
    return t;
}

static int dgrid(grg_batch B, int prec)
{
    const long items = (long)(B->Vtot / B->SB[prec]) * ((B->nrhs + B->RG[prec] - 1) / B->RG[prec]);
    return round8(std::min<long>(items, B->grid[prec] > 0 ? B->grid[prec] : kBatchMaxGrid));
}

static BatchBlasArgs blas(grg_batch B)
{
    BatchBlasArgs a;
    a.bt = table(B);
    a.Vtot = B->Vtot;
    a.nrhs = B->nrhs;
    a.grid = round8(std::min<long>(B->Vtot / 256, kBatchMaxGrid));
    a.alpha = B->alpha;
    a.partials = B->partials;
    a.act = nullptr;
    a.ctr = nullptr;
    return a;
}

enum { kC1 = 0, kC0 = 1, kCd = 2, kCinv = 3, kCminv = 4 };  // rows of B->coef

static grg_status dslash(grg_batch B, int prec, const void *in, void *out, int sel, bool dots,
                         const int *act = nullptr)
{
    BatchDslashArgs a;
    a.act = act;
    a.in = in;
    a.out = out;
    a.U = B->U[prec];
    a.mask = B->mask;
    a.sel = sel;
    a.bt = table(B);
    a.Vtot = B->Vtot;
    a.nrhs = B->nrhs;
    a.RG = B->RG[prec];
    a.partials = dots ? B->partials : nullptr;
    GRG_TRY_HIP(launch_dslash_batch(prec, a, dgrid(B, prec), B->SB[prec], B->st));
    return GRG_OK;
}

static BatchHalf half(grg_batch B)
{
    BatchHalf h;
    h.tile_lat = B->tile_lat_h;
    h.off = B->off_h;
    h.par = B->par_h;
    h.mask = B->mask_h;
    h.Vtot = B->Vh;
    return h;
}

static int hgrid(grg_batch B) { return round8(std::min<long>(B->Vh / 256, kBatchMaxGrid)); }
// the half-step's grid (its items: a block of 256 half-sites with one RHS)
static int egrid(grg_batch B) { return round8(std::min<long>((long)B->Vh / 256 * B->nrhs, kBatchMaxGrid)); }

// vector kernels over the compact fields
static BatchBlasArgs blas_h(grg_batch B)
{
    BatchBlasArgs a = blas(B);
    a.bt.tile_lat = B->tile_lat_h;
    a.bt.off = B->off_h;
    a.Vtot = B->Vh;
    a.grid = hgrid(B);
    return a;
}

// out = c[ka] in2 + c[kb] H in on side po of every lattice (BatchEoArgs)
static grg_status eo_half(grg_batch B, int prec, const void *in, const void *in2, void *out, int po, int ka,
                          int kb, bool dots, const int *act)
{
    BatchEoArgs a;
    a.in = in;
    a.in2 = in2;
    a.out = out;
    a.U = B->U[prec];
    a.bt = table(B);
    a.hf = half(B);
    a.po = po;
    a.nrhs = B->nrhs;
    a.ca = B->coef + (size_t)ka * B->nlat;
    a.cb = B->coef + (size_t)kb * B->nlat;
    a.partials = dots ? B->partials : nullptr;
    a.act = act;
    GRG_TRY_HIP(launch_batch_eo(prec, a, egrid(B), B->st));
    return GRG_OK;
}

// the read-back block (|r|^2, |b|^2, counters, inner flags) into h_buf
static grg_status read_back(grg_batch B)
{
    GRG_TRY_HIP(hipMemcpyAsync(B->h_buf, B->dsc, B->dsc_bytes, hipMemcpyDeviceToHost, B->st));
    GRG_TRY_HIP(hipStreamSynchronize(B->st));
    return GRG_OK;
}
static const double *h_rn2(grg_batch B) { return B->h_buf; }
static const double *h_bn2(grg_batch B) { return B->h_buf + B->nsys; }
static const int *h_ctr(grg_batch B) { return (const int *)(B->h_buf + 2 * B->nsys); }
static const int *h_active(grg_batch B) { return h_ctr(B) + 4; }

static grg_status ctl(grg_batch B, bool init)
{
    BatchCtlArgs c;
    c.nsys = B->nsys;
    c.bn2 = B->bn2;
    c.rn2 = B->rn2;
    c.tol = B->prm.tol;
    c.inner_tol = B->prm.inner_tol;
    c.fp64_inner = B->prm.inner == GRG_FP64;
    c.thr2 = B->thr2;
    c.fr2 = B->fr2;
    c.oact = B->oact;
    c.ctr = B->ctr;
    c.init = init ? 1 : 0;
    GRG_TRY_HIP(launch_batch_ctl(c, B->st));
    return GRG_OK;
}

// one inner minimal-residual iteration for the systems whose inner flag is
// set (a no-op launch sequence once none is)
static grg_status inner_step(grg_batch B, int prec)
{
    BatchBlasArgs a = B->eo ? blas_h(B) : blas(B);
    a.act = B->active;
    a.ctr = B->ctr;
    if (B->eo) {
        // q = (d - H_pq H_qp / d) r on the reduced parity, with <q, r>, |q|^2
        GRG_TRY(eo_half(B, prec, B->hr, nullptr, B->hw, 1, kC0, kC1, false, B->active));
        GRG_TRY(eo_half(B, prec, B->hw, B->hr, B->hq, 0, kCd, kCminv, true, B->active));
        GRG_TRY_HIP(launch_batch_reduce(kAlpha, B->partials, egrid(B), B->nsys, B->alpha, nullptr, nullptr,
                                        B->active, nullptr, B->st));
        GRG_TRY_HIP(launch_batch_mr_update(prec, a, B->hx, B->hr, B->hq, B->st));
        GRG_TRY_HIP(launch_batch_reduce(kNorm, B->partials, a.grid, B->nsys, nullptr, B->rn2i, B->thr2,
                                        B->active, B->active, B->st));
        return GRG_OK;
    }
    GRG_TRY(dslash(B, prec, B->in_r, B->in_q, 0, true, B->active));
    GRG_TRY_HIP(launch_batch_reduce(kAlpha, B->partials, dgrid(B, prec), B->nsys, B->alpha, nullptr, nullptr,
                                    B->active, nullptr, B->st));
    GRG_TRY_HIP(launch_batch_mr_update(prec, a, B->in_x, B->in_r, B->in_q, B->st));
    GRG_TRY_HIP(launch_batch_reduce(kNorm, B->partials, a.grid, B->nsys, nullptr, B->rn2i, B->thr2, B->active,
                                    B->active, B->st));
    return GRG_OK;
}

// One outer step of the defect correction for the systems whose outer flag
// is set: the scaled residual into the inner precision, the inner solve
// (eager: until no inner flag is set, read back every check_every
// iterations, at most maxit; captured: exactly n_inner iterations, the
// surplus ones no-ops), then r -= A e |r|, x += e |r| in FP64 and the control.
static grg_status outer_step(grg_batch B, int prec, const void *r_src, const void *x_src, bool eager,
                             int n_inner, int *taken)
{
    BatchBlasArgs a = blas(B);
    a.act = B->oact;
    GRG_TRY_HIP(launch_batch_inner_init(prec, a, r_src, B->fr2, B->in_r, B->in_x, B->st));
    GRG_TRY_HIP(launch_batch_reduce(kNorm, B->partials, a.grid, B->nsys, nullptr, B->rn2i, B->thr2, B->oact,
                                    B->active, B->st));
    if (B->eo) {
        // the halves b_p (into hq for the moment) and b_q of the inner right-hand
        // side, the reduced right-hand side b_p - H_pq b_q / d into hr with its
        // |.|^2 setting the inner flags, and the reduced iterate from zero
        GRG_TRY_HIP(launch_batch_eo_split(prec, table(B), half(B), B->nrhs, B->in_r, B->hq, B->hbq, 0, hgrid(B),
                                          B->st));
        GRG_TRY(eo_half(B, prec, B->hbq, B->hq, B->hr, 0, kC1, kCminv, true, B->oact));
        GRG_TRY_HIP(launch_batch_reduce(kNorm3, B->partials, egrid(B), B->nsys, nullptr, B->rn2i, B->thr2,
                                        B->oact, B->active, B->st));
        GRG_TRY_HIP(launch_fill_zero(B->hx, (size_t)B->Vh * B->nrhs * 12 * prec_bytes(prec), B->st));
    }
    int it = 0;
    if (eager) {
        const int chunk = std::max(1, B->prm.check_every);
        GRG_TRY(read_back(B));
        bool any = false;
        for (int k = 0; k < B->nsys; ++k) any = any || h_active(B)[k];
        const int c0 = h_ctr(B)[0];
        while (any && it < n_inner) {
            for (int k = 0; k < chunk && it < n_inner; ++k, ++it) GRG_TRY(inner_step(B, prec));
            GRG_TRY(read_back(B));
            any = false;
            for (int k = 0; k < B->nsys; ++k) any = any || h_active(B)[k];
        }
        if (taken) *taken = h_ctr(B)[0] - c0;
    } else {
        for (int k = 0; k < n_inner; ++k) GRG_TRY(inner_step(B, prec));
    }
    if (B->eo) {
        // the other parity of the correction, e_q = (b_q - H_qp e_p) / d, and
        // both halves into the full-layout correction in_x
        GRG_TRY(eo_half(B, prec, B->hx, B->hbq, B->heq, 1, kCinv, kCminv, false, B->oact));
        GRG_TRY_HIP(launch_batch_eo_split(prec, table(B), half(B), B->nrhs, B->in_x, B->hx, B->heq, 1, hgrid(B),
                                          B->st));
    }
    BatchDcArgs d;
    d.e = B->in_x;
    d.U = B->U[GRG_FP64];
    d.r_in = r_src;
    d.x_in = x_src;
    d.r_out = B->r64;
    d.x_out = B->x64;
    d.fr2 = B->fr2;
    d.mask = B->mask;
    d.bt = table(B);
    d.Vtot = B->Vtot;
    d.nrhs = B->nrhs;
    d.partials = B->partials;
    d.act = B->oact;
    d.gate = r_src == B->r64 ? 1 : 0;  // the first step writes r64 and x64 for every system
    d.ctr = B->ctr + 1;
    const int dcg = round8(std::min<long>(B->Vtot / 128, kBatchMaxGrid));
    GRG_TRY_HIP(launch_batch_dc_update(prec, d, dcg, B->st));
    GRG_TRY_HIP(launch_batch_reduce(kNorm, B->partials, dcg, B->nsys, nullptr, B->rn2, nullptr, B->oact, nullptr,
                                    B->st));
    GRG_TRY(ctl(B, false));
    return GRG_OK;
}

// b = D_rb x_b, |b|^2, control initialised (|r| = |b|, counters cleared)
static grg_status prologue(grg_batch B, const double *xb)
{
    const BatchBlasArgs a = blas(B);
    GRG_TRY_HIP(launch_batch_scatter(table(B), xb, B->u64, B->bidx, B->nb, B->coff, B->Vtot, B->nrhs, B->st));
    GRG_TRY(dslash(B, GRG_FP64, B->u64, B->b64, 0, false));
    GRG_TRY_HIP(launch_batch_norm2(GRG_FP64, a, B->b64, B->st));
    GRG_TRY_HIP(launch_batch_reduce(kNorm, B->partials, a.grid, B->nsys, nullptr, B->bn2, nullptr, nullptr, nullptr,
                                    B->st));
    GRG_TRY(ctl(B, true));
    return GRG_OK;
}

// r = b - D_rr x from the iterate (every system), control on it
static grg_status verify(grg_batch B)
{
    const BatchBlasArgs a = blas(B);
    GRG_TRY(dslash(B, GRG_FP64, B->x64, B->t64, 0, false));
    GRG_TRY_HIP(launch_batch_sub_norm(a, B->b64, B->t64, B->r64, B->st));
    GRG_TRY_HIP(launch_batch_reduce(kNorm, B->partials, a.grid, B->nsys, nullptr, B->rn2, nullptr, nullptr, nullptr,
                                    B->st));
    GRG_TRY(ctl(B, false));
    return GRG_OK;
}

// y_b = [D (u - z)]_b; leaves u - z in x64 (undone by applying it again:
// u and z have disjoint supports)
static grg_status epilogue(grg_batch B, double *yb)
{
    const BatchBlasArgs a = blas(B);
    GRG_TRY_HIP(launch_batch_xmy(a, B->u64, B->x64, B->st));
    GRG_TRY_HIP(launch_batch_coarse(table(B), B->x64, B->U[GRG_FP64], yb, B->qg, B->clat, B->nb, B->nboff,
                                    B->coff, B->nbtot, B->nrhs, B->st));
    return GRG_OK;
}

// convergence of every system from the read-back block
static int host_state(grg_batch B, double *worst)
{
    *worst = 0;
    int conv = 1;
    for (int k = 0; k < B->nsys; ++k) {
        const double b2 = h_bn2(B)[k], r2 = h_rn2(B)[k];
        if (!isfinite(r2) || !isfinite(b2)) return -1;
        const double rel = b2 > 0 ? sqrt(r2 / b2) : 0.0;
        *worst = std::max(*worst, rel);
        if (rel > B->prm.tol) conv = 0;
    }
    return conv;
}

// The whole apply, with the outer and inner counts fixed, as one captured
// graph reading x_b from xb_in and writing y_b to yb_out.
static grg_status build_graph(grg_batch B, int prec, int n_outer, int n_inner)
{
    if (B->graph) {
        (void)hipGraphExecDestroy(B->graph);
        B->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    GRG_TRY_HIP(hipStreamBeginCapture(B->st, hipStreamCaptureModeThreadLocal));
    grg_status s = prologue(B, B->xb_in);
    for (int o = 0; o < n_outer && s == GRG_OK; ++o)
        s = outer_step(B, prec, o == 0 ? B->b64 : B->r64, o == 0 ? nullptr : B->x64, false, n_inner, nullptr);
    if (s == GRG_OK) s = verify(B);
    if (s == GRG_OK) s = epilogue(B, B->yb_out);
    hipError_t e = hipStreamEndCapture(B->st, &g);
    if (s != GRG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    GRG_TRY_HIP(e);
    e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    GRG_TRY_HIP(e);
    B->g_outer = n_outer;
    B->g_inner = n_inner;
    return GRG_OK;
}

static grg_status batch_apply(grg_batch B, const double *xb, double *yb, bool use_graph,
                              grg_solver_stats *stats)
{
    const grg_solver_params &p = B->prm;
    const int prec = p.inner;
    hipStream_t st = B->st;
    const size_t cb = sizeof(double2) * 12 * (size_t)B->nrhs * B->nbtot;
    bool done_by_graph = false;
    if (use_graph && B->e_outer == 0 && !B->graph) {
        // counts unknown: this apply runs eagerly and records them
        use_graph = false;
    }
    const void *r_src = B->b64, *x_src = nullptr;
    int conv = 0;
    double worst = 0;
    if (use_graph) {
        if (!B->graph) GRG_TRY(build_graph(B, prec, B->e_outer, B->e_inner + 1));
        GRG_TRY_HIP(hipMemcpyAsync(B->xb_in, xb, cb, hipMemcpyDeviceToDevice, st));
        GRG_TRY_HIP(hipGraphLaunch(B->graph, st));
        GRG_TRY_HIP(hipMemcpyAsync(yb, B->yb_out, cb, hipMemcpyDeviceToDevice, st));
        GRG_TRY(read_back(B));
        conv = host_state(B, &worst);
        if (conv < 0) return set_error("non-finite FP64 residual"), GRG_ENONFINITE;
        done_by_graph = conv == 1;
        if (!done_by_graph) {
            // continue eagerly from the verified residual; the next graph
            // is captured with one more outer step
            GRG_TRY(epilogue(B, yb));  // restores the iterate in x64 (the combine's output is redone)
            (void)hipGraphExecDestroy(B->graph);
            B->graph = nullptr;
            r_src = B->r64;
            x_src = B->x64;
        }
    } else {
        GRG_TRY(prologue(B, xb));
        GRG_TRY(read_back(B));
        conv = host_state(B, &worst);
        if (conv < 0) return set_error("non-finite FP64 residual"), GRG_ENONFINITE;
    }
    grg_status status = GRG_OK;
    if (!done_by_graph) {
        bool verified = use_graph;  // the graph's last residual was recomputed from x
        int max_inner = 0;
        for (;;) {
            if (conv && (verified || x_src == nullptr)) break;
            if (conv) {
                GRG_TRY(verify(B));
                GRG_TRY(read_back(B));
                conv = host_state(B, &worst);
                if (conv < 0) return set_error("non-finite FP64 residual"), GRG_ENONFINITE;
                r_src = B->r64;
                verified = true;
                continue;
            }
            verified = false;
            const int outer = h_ctr(B)[1], total = h_ctr(B)[0];
            if (outer >= p.max_outer || total >= p.max_iter) {
                status = GRG_ENOCONV;
                set_error("batched D_rr solve: no convergence after %d outer / %d inner iterations "
                          "(residual %.3e > %.3e)", outer, total, worst, p.tol);
                break;
            }
            int taken = 0;
            GRG_TRY(outer_step(B, prec, r_src, x_src, true, p.max_iter - total, &taken));
            max_inner = std::max(max_inner, taken);
            GRG_TRY(read_back(B));
            conv = host_state(B, &worst);
            if (conv < 0) return set_error("non-finite FP64 residual"), GRG_ENONFINITE;
            r_src = B->r64;
            x_src = B->x64;
        }
        if (x_src == nullptr)
            GRG_TRY_HIP(launch_fill_zero(B->x64, spinor_elems(B->gtot, B->nrhs) * 16, st));
        GRG_TRY(epilogue(B, yb));
        if (status == GRG_OK) {
            // the counts the next captured apply of this batch is built with:
            // every outer step this apply took (the graph's and the eager
            // ones after it), and the most inner iterations one of them took
            B->e_outer = std::max(1, h_ctr(B)[1]);
            B->e_inner = std::max({B->e_inner, max_inner, use_graph ? B->g_inner : 0});
        }
    }
    if (stats) {
        stats->iters = h_ctr(B)[0];
        stats->outer = h_ctr(B)[1];
        stats->converged = status == GRG_OK;
        stats->true_rel_resid = worst;
    }
    return status;
}

static void batch_free(grg_batch B)
{
    auto f = [](void *q) {
        if (q) (void)hipFree(q);
    };
    for (int k = 0; k < 3; ++k) f(B->U[k]);
    f(B->mask);
    f(B->bidx);
    f(B->qg);
    f(B->clat);
    f(B->tile_lat);
    f(B->off);
    f(B->nb);
    f(B->nboff);
    f(B->dims);
    f(B->diag);
    f(B->coff);
    f(B->b64);
    f(B->x64);
    f(B->r64);
    f(B->t64);
    f(B->u64);
    f(B->in_b);
    f(B->in_x);
    f(B->in_r);
    f(B->in_q);
    f(B->tile_lat_h);
    f(B->off_h);
    f(B->par_h);
    f(B->mask_h);
    f(B->coef);
    for (void *p : {B->hx, B->hr, B->hq, B->hw, B->hbq, B->heq}) f(p);
    f(B->partials);
    f(B->alpha);
    f(B->dsc);  // rn2, bn2, the counters and the inner flags
    f(B->thr2);
    f(B->fr2);
    f(B->rn2i);
    f(B->oact);
    f(B->xb_in);
    f(B->yb_out);
    if (B->h_buf) (void)hipHostFree(B->h_buf);
    if (B->graph) (void)hipGraphExecDestroy(B->graph);
    if (B->ev_in) (void)hipEventDestroy(B->ev_in);
    if (B->ev_out) (void)hipEventDestroy(B->ev_out);
    if (B->st) (void)hipStreamDestroy(B->st);
}

}  // namespace grg

using namespace grg;

extern "C" {

grg_status grg_batch_create(const grg_batch_member *m, int count, int nrhs,
                            const grg_solver_params *params, void *stream, grg_batch *out)
{
    if (!m || !out) return set_error("null argument"), GRG_EINVAL;
    *out = nullptr;
    if (count < 1 || count > 4096) return set_error("count must be in 1..4096"), GRG_EINVAL;
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error("nrhs must be in 1..%d", kMaxRhs), GRG_EINVAL;
    grg_solver_params prm;
    if (params) prm = *params;
    else grg_solver_params_default(&prm);
    if (!(prm.tol > 0 && prm.tol < 1) || prm.max_iter < 1 || prm.max_outer < 1 || prm.check_every < 1 ||
        prm.inner < 0 || prm.inner > 2 || (prm.inner != GRG_FP64 && !(prm.inner_tol > 0 && prm.inner_tol < 1)))
        return set_error("bad solver parameters"), GRG_EINVAL;
    if (prm.method != 0)
        return set_error("the batch runs minimal residual only (params.method must be 0)"), GRG_EUNSUPPORTED;
    std::vector<BatchMember> mem(count);
    long long Vtot = 0, nbtot = 0, coff = 0;
    for (int i = 0; i < count; ++i) {
        BatchMember &b = mem[i];
        long long V = 1;
        for (int mu = 0; mu < 4; ++mu) {
            if (m[i].dims[mu] < 2) return set_error("member %d: extents must be >= 2", i), GRG_EINVAL;
            if (m[i].bc[mu] != 1 && m[i].bc[mu] != -1) return set_error("member %d: bad bc", i), GRG_EINVAL;
            b.dims[mu] = m[i].dims[mu];
            b.bc[mu] = m[i].bc[mu];
            V *= m[i].dims[mu];
        }
        if (V % 256) return set_error("member %d: volume %lld is not a multiple of 256", i, V), GRG_EUNSUPPORTED;
        if (!m[i].links || !m[i].q) return set_error("member %d: null links or q", i), GRG_EINVAL;
        if (m[i].n_coarse < 1 || m[i].n_coarse >= V) return set_error("member %d: bad n_coarse", i), GRG_EINVAL;
        if (!isfinite(m[i].m0)) return set_error("member %d: m0 not finite", i), GRG_EINVAL;
        b.m0 = m[i].m0;
        b.V = (int)V;
        b.off = (int)Vtot;
        b.nb = m[i].n_coarse;
        b.nboff = (int)nbtot;
        b.coff = coff;
        Vtot += V;
        nbtot += b.nb;
        coff += 12LL * nrhs * b.nb;
    }
    if (Vtot > (1LL << 27)) return set_error("batch too large"), GRG_ETOO_LARGE;
    grg_batch B = new (std::nothrow) grg_batch_s();
    if (!B) return set_error("out of host memory"), GRG_ENOMEM;
    B->prm = prm;
    B->prm.max_rhs = nrhs;
    B->nlat = count;
    B->nrhs = nrhs;
    B->nsys = count * nrhs;
    B->Vtot = (int)Vtot;
    B->nbtot = (int)nbtot;
    B->mem = mem;
    B->gtot.L[0] = B->gtot.L[1] = B->gtot.L[2] = B->gtot.L[3] = 1;
    B->gtot.V = B->Vtot;
    B->gtot.Vs = B->Vtot;
    B->caller = (hipStream_t)stream;
    (void)hipGetDevice(&B->device);
    // host tables
    std::vector<uint8_t> mask(Vtot, 0);
    std::vector<int32_t> bidx(Vtot, -1), qg(nbtot);
    std::vector<int> clat(nbtot), tile_lat(Vtot / 64), off(count), nb(count), nboff(count);
    std::vector<int4> dims(count);
    std::vector<double> diag(count);
    std::vector<long long> coffs(count);
    for (int i = 0; i < count; ++i) {
        const BatchMember &b = mem[i];
        std::vector<uint8_t> seen(b.V, 0);
        for (int k = 0; k < b.V; ++k) {
            const int s = m[i].q[k];
            if (s < 0 || s >= b.V || seen[s]) {
                delete B;
                return set_error("member %d: q is not a permutation", i), GRG_EINVAL;
            }
            seen[s] = 1;
        }
        for (int k = 0; k < b.nb; ++k) {
            const int s = b.off + m[i].q[k];
            mask[s] = 1;
            bidx[s] = k;
            qg[b.nboff + k] = s;
            clat[b.nboff + k] = i;
        }
        for (int t = 0; t < b.V / 64; ++t) tile_lat[b.off / 64 + t] = i;
        off[i] = b.off;
        nb[i] = b.nb;
        nboff[i] = b.nboff;
        dims[i] = make_int4(b.dims[0], b.dims[1], b.dims[2], b.dims[3]);
        diag[i] = 4.0 + b.m0;
        coffs[i] = b.coff;
    }
    // the even-odd reduced inner solve: every lattice with even extents and a
    // nonzero diagonal 4 + m0 (the reduced operator divides by it)
    bool eo = prm.eo != 0;
    for (int i = 0; i < count && eo; ++i) {
        if (4.0 + mem[i].m0 == 0.0) eo = false;
        for (int mu = 0; mu < 4; ++mu)
            if (mem[i].dims[mu] % 2) eo = false;
    }
    // compact halves: lattice i's block of V / 2 half-sites, padded to 256
    std::vector<int> off_h(count), par_h(count), tile_lat_h;
    std::vector<uint8_t> mask_h;
    std::vector<double> coef(eo ? 5 * (size_t)count : 0);
    long Vh = 0;
    if (eo) {
        for (int i = 0; i < count; ++i) {
            off_h[i] = (int)Vh;
            Vh += (mem[i].V / 2 + 255) / 256 * 256;
        }
        tile_lat_h.assign(Vh / 64, 0);
        mask_h.assign(2 * (size_t)Vh, 1);  // padding masked
        for (int i = 0; i < count; ++i) {
            const BatchMember &b = mem[i];
            long rest[2] = {0, 0};
            std::vector<uint8_t> par(b.V);
            for (int x = 0; x < b.V; ++x) {
                int c = x, sum = 0;
                for (int mu = 0; mu < 4; ++mu) {
                    sum += c % b.dims[mu];
                    c /= b.dims[mu];
                }
                par[x] = (uint8_t)(sum & 1);
                if (!mask[b.off + x]) ++rest[sum & 1];
            }
            // the reduced system on the parity with fewer rest sites (as one lattice)
            const int p = rest[0] < rest[1] ? 0 : 1;
            par_h[i] = p;
            const int nblk = (b.V / 2 + 255) / 256 * 256;
            for (int t = 0; t < nblk / 64; ++t) tile_lat_h[off_h[i] / 64 + t] = i;
            // side 0: the sites of parity p, side 1: the others (pair 2h, 2h + 1)
            for (int h = 0; h < b.V / 2; ++h)
                for (int k = 0; k < 2; ++k) {
                    const int x = 2 * h + k;
                    const int side = par[x] == p ? 0 : 1;
                    mask_h[(size_t)side * Vh + off_h[i] + h] = mask[b.off + x];
                }
            const double d = diag[i];
            coef[kC1 * (size_t)count + i] = 1.0;
            coef[kC0 * (size_t)count + i] = 0.0;
            coef[kCd * (size_t)count + i] = d;
            coef[kCinv * (size_t)count + i] = 1.0 / d;
            coef[kCminv * (size_t)count + i] = -1.0 / d;
        }
    }
    const size_t f64 = spinor_elems(B->gtot, nrhs) * 16;
    const size_t fin = spinor_elems(B->gtot, nrhs) * prec_bytes(prm.inner);
    bool ok = true;
    auto al = [&](void **p, size_t bytes) {
        if (ok && hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) {
            *p = nullptr;
            ok = false;
        }
    };
    for (int k = 0; k < 3; ++k) al(&B->U[k], gauge_elems(B->gtot) * prec_bytes(k));
    al((void **)&B->mask, Vtot);
    al((void **)&B->bidx, sizeof(int32_t) * Vtot);
    al((void **)&B->qg, sizeof(int32_t) * nbtot);
    al((void **)&B->clat, sizeof(int) * nbtot);
    al((void **)&B->tile_lat, sizeof(int) * (Vtot / 64));
    al((void **)&B->off, sizeof(int) * count);
    al((void **)&B->nb, sizeof(int) * count);
    al((void **)&B->nboff, sizeof(int) * count);
    al((void **)&B->dims, sizeof(int4) * count);
    al((void **)&B->diag, sizeof(double) * count);
    al((void **)&B->coff, sizeof(long long) * count);
    for (void **p : {&B->b64, &B->x64, &B->r64, &B->t64, &B->u64}) al(p, f64);
    for (void **p : {&B->in_b, &B->in_x, &B->in_r, &B->in_q}) al(p, fin);
    B->eo = eo;
    B->Vh = (int)Vh;
    const size_t fh = (size_t)Vh * nrhs * 12 * prec_bytes(prm.inner);
    if (eo) {
        al((void **)&B->tile_lat_h, sizeof(int) * (Vh / 64));
        al((void **)&B->off_h, sizeof(int) * count);
        al((void **)&B->par_h, sizeof(int) * count);
        al((void **)&B->mask_h, 2 * (size_t)Vh);
        al((void **)&B->coef, sizeof(double) * 5 * count);
        for (void **p : {&B->hx, &B->hr, &B->hq, &B->hw, &B->hbq, &B->heq}) al(p, fh);
    }
    al((void **)&B->partials, sizeof(double) * kBatchMaxGrid * B->nsys * 3);
    al((void **)&B->alpha, sizeof(double2) * B->nsys);
    for (double **p : {&B->thr2, &B->fr2, &B->rn2i}) al((void **)p, sizeof(double) * B->nsys);
    al((void **)&B->oact, sizeof(int) * B->nsys);
    B->dsc_bytes = sizeof(double) * 2 * B->nsys + sizeof(int) * (4 + B->nsys);
    al((void **)&B->dsc, B->dsc_bytes);
    if (ok) {
        B->rn2 = (double *)B->dsc;
        B->bn2 = B->rn2 + B->nsys;
        B->ctr = (int *)(B->bn2 + B->nsys);
        B->active = B->ctr + 4;
    }
    const size_t cbytes = sizeof(double2) * 12 * (size_t)nrhs * nbtot;
    al((void **)&B->xb_in, cbytes);
    al((void **)&B->yb_out, cbytes);
    if (ok && hipHostMalloc((void **)&B->h_buf, B->dsc_bytes) != hipSuccess) {
        B->h_buf = nullptr;
        ok = false;
    }
    if (ok && (hipStreamCreateWithFlags(&B->st, hipStreamNonBlocking) != hipSuccess ||
               hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess ||
               hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming) != hipSuccess))
        ok = false;
    if (!ok) {
        batch_free(B);
        delete B;
        return set_error("batch workspaces: allocation failed"), GRG_ENOMEM;
    }
    hipStream_t st = B->st;
#define UP(dst, src, n) GRG_TRY_HIP(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st))
    UP(B->mask, mask.data(), Vtot);
    UP(B->bidx, bidx.data(), sizeof(int32_t) * Vtot);
    UP(B->qg, qg.data(), sizeof(int32_t) * nbtot);
    UP(B->clat, clat.data(), sizeof(int) * nbtot);
    UP(B->tile_lat, tile_lat.data(), sizeof(int) * (Vtot / 64));
    UP(B->off, off.data(), sizeof(int) * count);
    UP(B->nb, nb.data(), sizeof(int) * count);
    UP(B->nboff, nboff.data(), sizeof(int) * count);
    UP(B->dims, dims.data(), sizeof(int4) * count);
    UP(B->diag, diag.data(), sizeof(double) * count);
    UP(B->coff, coffs.data(), sizeof(long long) * count);
    if (eo) {
        UP(B->tile_lat_h, tile_lat_h.data(), sizeof(int) * (Vh / 64));
        UP(B->off_h, off_h.data(), sizeof(int) * count);
        UP(B->par_h, par_h.data(), sizeof(int) * count);
        UP(B->mask_h, mask_h.data(), 2 * (size_t)Vh);
        UP(B->coef, coef.data(), sizeof(double) * 5 * count);
    }
    GRG_TRY_HIP(hipStreamSynchronize(st));
#undef UP
    for (void *p : {B->b64, B->x64, B->r64, B->t64, B->u64}) GRG_TRY_HIP(launch_fill_zero(p, f64, st));
    for (void *p : {B->in_b, B->in_x, B->in_r, B->in_q}) GRG_TRY_HIP(launch_fill_zero(p, fin, st));
    for (void *p : {B->hx, B->hr, B->hq, B->hw, B->hbq, B->heq})
        if (p) GRG_TRY_HIP(launch_fill_zero(p, fh, st));
    GRG_TRY_HIP(launch_fill_zero(B->dsc, B->dsc_bytes, st));
    GRG_TRY_HIP(launch_fill_zero(B->oact, sizeof(int) * B->nsys, st));
    // links, one member at a time through a staging buffer
    size_t maxlink = 0;
    for (const BatchMember &b : mem) maxlink = std::max(maxlink, (size_t)b.V * 4 * 9 * 16);
    void *stage = nullptr;
    GRG_TRY_HIP(hipMalloc(&stage, maxlink));
    grg_status s = GRG_OK;
    for (int i = 0; i < count && s == GRG_OK; ++i) {
        const BatchMember &b = mem[i];
        Geom g;
        for (int mu = 0; mu < 4; ++mu) g.L[mu] = b.dims[mu];
        g.V = b.V;
        g.Vs = b.V;
        const size_t toff = (size_t)(b.off / 64) * 36 * 64;  // link elements before this member
        if (hipMemcpy(stage, m[i].links, (size_t)b.V * 4 * 9 * 16, hipMemcpyHostToDevice) != hipSuccess ||
            launch_pack_gauge((const double *)stage, g, b.bc, (double2 *)B->U[GRG_FP64] + toff,
                              (float2 *)B->U[GRG_FP32] + toff, (bf16x2 *)B->U[GRG_BF16] + toff, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            s = GRG_EHIP;
    }
    (void)hipFree(stage);
    if (s != GRG_OK) {
        set_error("uploading the batch links failed");
        batch_free(B);
        delete B;
        return s;
    }
    for (int k = 0; k < 3; ++k) B->grid[k] = 0;
    *out = B;
    return GRG_OK;
}

grg_status grg_batch_destroy(grg_batch B)
{
    if (!B) return GRG_OK;
    (void)hipStreamSynchronize(B->st);
    batch_free(B);
    delete B;
    return GRG_OK;
}

grg_status grg_batch_layout(grg_batch B, int member, int64_t *offset, int32_t *n_coarse)
{
    if (!B || !offset || !n_coarse) return set_error("null argument"), GRG_EINVAL;
    if (member < 0 || member > B->nlat) return set_error("member out of range"), GRG_EINVAL;
    if (member == B->nlat) {
        *offset = 12LL * B->nrhs * B->nbtot;
        *n_coarse = B->nbtot;
    } else {
        *offset = B->mem[member].coff;
        *n_coarse = B->mem[member].nb;
    }
    return GRG_OK;
}

grg_status grg_batch_apply(grg_batch B, const double *x_b, double *y_b, int use_graph,
                           grg_solver_stats *stats)
{
    if (!B || !x_b || !y_b) return set_error("null argument"), GRG_EINVAL;
    if (stats) memset(stats, 0, sizeof *stats);
    const auto t0 = std::chrono::steady_clock::now();
    GRG_TRY_HIP(hipEventRecord(B->ev_in, B->caller));
    GRG_TRY_HIP(hipStreamWaitEvent(B->st, B->ev_in, 0));
    grg_status s = batch_apply(B, x_b, y_b, use_graph != 0, stats);
    hipError_t e = hipStreamSynchronize(B->st);
    if (s == GRG_OK && e != hipSuccess) {
        set_error("stream synchronise failed: %s", hipGetErrorString(e));
        s = GRG_EHIP;
    }
    if (stats)
        stats->t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return s;
}

grg_status grg_batch_tune_info(grg_batch B, int precision, int32_t info[3], float ms[2])
{
    if (!B || !info || !ms) return set_error("null argument"), GRG_EINVAL;
    if (precision < GRG_FP64 || precision > GRG_BF16) return set_error("bad precision"), GRG_EINVAL;
    info[0] = B->SB[precision];
    info[1] = B->RG[precision];
    info[2] = dgrid(B, precision);
    const bool inner = precision == B->prm.inner;
    ms[0] = inner && B->eo ? B->eo_ms : B->tune_ms[precision];
    ms[1] = inner ? B->upd_ms : -1.0f;
    return GRG_OK;
}

grg_status grg_batch_graph_info(grg_batch B, int32_t counts[2])
{
    if (!B || !counts) return set_error("null argument"), GRG_EINVAL;
    counts[0] = B->graph ? B->g_outer : 0;
    counts[1] = B->graph ? B->g_inner : 0;
    return GRG_OK;
}

grg_status grg_batch_tune(grg_batch B)
{
    if (!B) return set_error("null argument"), GRG_EINVAL;
    hipEvent_t e0, e1;
    GRG_TRY_HIP(hipEventCreate(&e0));
    GRG_TRY_HIP(hipEventCreate(&e1));
    const int precs[2] = {GRG_FP64, B->prm.inner};
    for (int pi = 0; pi < (B->prm.inner == GRG_FP64 ? 1 : 2); ++pi) {
        const int prec = precs[pi];
        void *in = prec == GRG_FP64 ? B->b64 : B->in_b, *out = prec == GRG_FP64 ? B->t64 : B->in_q;
        float best = 1e30f;
        int bsb = 64, brg = 1, bgrid = 0;
        for (int sb : {64, 128, 256}) {
            for (int rg = 1; rg <= B->nrhs; rg *= 2) {
                for (int cap : {1024, 2048}) {
                    B->SB[prec] = sb;
                    B->RG[prec] = rg;
                    B->grid[prec] = cap;
                    grg_status s = GRG_OK;
                    for (int k = 0; k < 4 && s == GRG_OK; ++k) {
                        if (k == 1) GRG_TRY_HIP(hipEventRecord(e0, B->st));
                        s = dslash(B, prec, in, out, 0, true);
                    }
                    GRG_TRY(s);
                    GRG_TRY_HIP(hipEventRecord(e1, B->st));
                    GRG_TRY_HIP(hipEventSynchronize(e1));
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ms /= 3;
                    if (ms < best) {
                        best = ms;
                        bsb = sb;
                        brg = rg;
                        bgrid = cap;
                    }
                }
            }
        }
        B->SB[prec] = bsb;
        B->RG[prec] = brg;
        B->grid[prec] = bgrid;
        B->tune_ms[prec] = best;
    }
    if (B->eo) {
        // the reduced operator's two half-steps as the inner solve runs them
        // (every system; overwrites workspaces)
        const int prec = B->prm.inner;
        for (int k = 0; k < 4; ++k) {
            if (k == 1) GRG_TRY_HIP(hipEventRecord(e0, B->st));
            GRG_TRY(eo_half(B, prec, B->hr, nullptr, B->hw, 1, kC0, kC1, false, nullptr));
            GRG_TRY(eo_half(B, prec, B->hw, B->hr, B->hq, 0, kCd, kCminv, true, nullptr));
        }
        GRG_TRY_HIP(hipEventRecord(e1, B->st));
        GRG_TRY_HIP(hipEventSynchronize(e1));
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        B->eo_ms = ms / 6;
    }
    {
        // the inner precision's MR update over every system (x += alpha r,
        // r -= alpha q with the step lengths in place; overwrites workspaces),
        // on the compact fields with the reduced solve
        const int prec = B->prm.inner;
        const BatchBlasArgs a = B->eo ? blas_h(B) : blas(B);
        void *ux = B->eo ? B->hx : B->in_x, *ur = B->eo ? B->hr : B->in_r, *uq = B->eo ? B->hq : B->in_q;
        for (int k = 0; k < 4; ++k) {
            if (k == 1) GRG_TRY_HIP(hipEventRecord(e0, B->st));
            GRG_TRY_HIP(launch_batch_mr_update(prec, a, ux, ur, uq, B->st));
        }
        GRG_TRY_HIP(hipEventRecord(e1, B->st));
        GRG_TRY_HIP(hipEventSynchronize(e1));
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        B->upd_ms = ms / 3;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (B->graph) {
        (void)hipGraphExecDestroy(B->graph);  // launch shapes are baked into the graph
        B->graph = nullptr;
    }
    return GRG_OK;
}

}  // extern "C"
