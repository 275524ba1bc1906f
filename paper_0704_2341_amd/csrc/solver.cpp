// D_rr solves and the Schur-complement apply.
//
// The coarse operator S_bb = D_bb - D_br D_rr^{-1} D_rb (section 1) is applied
// matrix-free:
//     u = x on the coarse sites, 0 elsewhere
//     y = (D u)_r                         (= D_rb x)
//     z = D_rr^{-1} y                     (the cost of the method: section 2)
//     S x = [ D (u - z) ]_b               (= D_bb x - D_br z)
//
// D_rr^{-1} is an FP64 defect correction (iterative refinement) around an
// inner restarted GCR(m) in FP64, FP32 or BF16 storage:
//     x = 0, r = b
//     repeat: e ~= A_low^{-1} (r / |r|) to a relative residual eps_in
//             x += |r| e ;  r = b - A x   (FP64)
//     until |r| <= tol |b| for every right-hand side.
// With FP64 inner iterations the loop is a plain FP64 GCR whose result is
// confirmed by the recomputed FP64 residual.  The inner GCR keeps its residual
// recursively across restarts (no extra matvec per restart); restart length 1
// is minimal residual.  Every right-hand side has its own step lengths and a
// device-side "active" flag that freezes it once it has converged, so the
// host only reads the residual norms every check_every iterations.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "handles.h"

namespace grg {

int round8(long v) { return (int)std::max<long>(8, ((v + 7) / 8) * 8); }

int dslash_grid(const Geom &g, int nrhs, int SB, int RG)
{
    const long items = (long)((g.V + SB - 1) / SB) * ((nrhs + RG - 1) / RG);
    return round8(std::min<long>(items, 2048));
}

BlasShape blas_shape(const Geom &g, int nrhs)
{
    BlasShape sh;
    sh.g = g;
    sh.nrhs = nrhs;
    sh.grid = round8(std::min<long>((g.V + 255) / 256, 2048));
    return sh;
}

static int dslash_sb(const Geom &g) { return g.V >= (1 << 16) ? 128 : 64; }

// Default stencil launch (before or without tuning).
DslashTune default_tune(const Geom &g, int prec, int nrhs)
{
    DslashTune t;
    t.SB = dslash_sb(g);
    t.RG = nrhs;
    t.split = prec == GRG_FP64 ? 1 : 0;
    t.grid = dslash_grid(g, nrhs, t.SB, t.RG);
    return t;
}

static grg_status launch_tuned(grg_lattice L, int prec, const DslashTune &t, const void *in,
                               void *out, const uint8_t *mask, int sel, double m0, int nrhs,
                               double *partials, const void *dot_with = nullptr)
{
    DslashArgs a;
    a.dot_with = dot_with;
    a.in = in;
    a.out = out;
    a.U = L->U[prec];
    a.mask = mask;
    a.sel = sel;
    a.diag = 4.0 + m0;
    a.g = L->g;
    a.nrhs = nrhs;
    a.SB = t.SB;
    a.RG = t.RG;
    a.split = t.split;
    a.chunk = t.chunk;
    a.march = t.march;
    a.partials = partials;
    GRG_TRY_HIP(launch_dslash(prec, a, t.grid, L->stream));
    return GRG_OK;
}

// Validity of a launch shape for (prec, nrhs).
bool launch_ok(const Geom &g, int prec, int nrhs, const DslashTune &t, bool)
{
    if (t.grid < 8 || t.grid % 8 || t.grid > kMaxGridValue || t.chunk < 0 || t.march < 0) return false;
    if (t.march > 0) {
        return t.march <= g.L[3] && t.RG >= 1 && t.RG <= nrhs &&
               64 * t.RG <= (prec == GRG_FP64 ? 512 : 768);
    }
    return (t.SB == 64 || t.SB == 128 || t.SB == 256) && t.RG >= 1 && t.RG <= nrhs &&
           (t.split == 0 || t.split == 1 || (t.split == 2 && prec == GRG_BF16));
}

// One stencil launch, bracketed by profiling events when enabled.
grg_status run_dslash(grg_schur S, int prec, const void *in, void *out, int sel, int nrhs,
                      double *partials, const void *dot_with = nullptr)
{
    grg_lattice L = S->lat;
    const DslashTune t = S->tune[prec][nrhs].valid ? S->tune[prec][nrhs] : default_tune(L->g, prec, nrhs);
    ProfilePool &P = S->prof;
    const bool ev = P.on && P.used < (int)P.start.size();
    if (ev) GRG_TRY_HIP(hipEventRecord(P.start[P.used], L->stream));
    GRG_TRY(launch_tuned(L, prec, t, in, out, sel < 0 ? nullptr : S->d_mask, sel < 0 ? 0 : sel,
                         S->m0, nrhs, partials, dot_with));
    if (ev) {
        GRG_TRY_HIP(hipEventRecord(P.stop[P.used], L->stream));
        P.prec[P.used] = prec;
        ++P.used;
    }
    ++S->n_dslash;
    return GRG_OK;
}

grg_status ensure_inner(grg_schur S, int prec);
grg_status precond_apply_inner(grg_schur S, int prec, const void *r, void *p, int nrhs);

// Largest grid any stencil or BLAS launch may use (sizes the partial sums).
constexpr int kMaxGrid = kMaxGridValue;
int partial_rows(const Geom &, int) { return kMaxGrid; }

// Autotuner: time every candidate launch of the D_rr stencil (with its fused
// dot products, as the solver runs it) on the handle's own workspaces and keep
// the fastest.  Every candidate computes each site in the same operation
// order, so the choice changes speed only, never the stencil's output.
grg_status tune_dslash(grg_schur S, int prec, int nrhs, int reps)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    GRG_TRY(ensure_inner(S, prec));
    const void *in = prec == GRG_FP64 ? S->b64 : S->in_b[prec];
    void *out = prec == GRG_FP64 ? S->t64 : S->in_q[prec];
    hipEvent_t e0, e1;
    GRG_TRY_HIP(hipEventCreate(&e0));
    GRG_TRY_HIP(hipEventCreate(&e1));
    grg_status status = GRG_OK;
    auto timeit = [&](DslashTune &t) {
        if (status != GRG_OK) return;
        status = launch_tuned(L, prec, t, in, out, S->d_mask, 0, S->m0, nrhs, S->partials);
        if (status != GRG_OK) return;
        if (hipEventRecord(e0, st) != hipSuccess) { status = GRG_EHIP; return; }
        for (int k = 0; k < reps && status == GRG_OK; ++k)
            status = launch_tuned(L, prec, t, in, out, S->d_mask, 0, S->m0, nrhs, S->partials);
        if (status != GRG_OK) return;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            status = GRG_EHIP;
            return;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        t.ms = ms / reps;
    };
    // stage 1: workgroup size, RHS per thread, hop grouping (default grid and mapping)
    std::vector<DslashTune> cands;
    const int sbs[3] = {64, 128, 256};
    for (int sb : sbs) {
        if (sb > 64 && g.V < 4 * sb) continue;
        for (int rg = 1; rg <= nrhs; ++rg) {
            if (nrhs % rg && rg != nrhs) continue;
            if (rg > 4 && rg != nrhs) continue;
            for (int split = 0; split < (prec == GRG_BF16 ? 3 : 2); ++split) {
                DslashTune t;
                t.SB = sb;
                t.RG = rg;
                t.split = split;
                t.grid = dslash_grid(g, nrhs, sb, rg);
                t.valid = 1;
                timeit(t);
                cands.push_back(t);
            }
        }
    }
    // t-marching kernel: one workgroup = 64 sites x RG RHS (one wavefront
    // each), time chunks of T; RG = nrhs or a divisor of it that fits a
    // workgroup
    const int V3 = g.L[0] * g.L[1] * g.L[2];
    const int nb3 = (V3 + 63) / 64;
    const int max_rg = (prec == GRG_FP64 ? 512 : 768) / 64;
    for (int rg = std::min(nrhs, max_rg); rg >= 1; --rg) {
        if (nrhs % rg) continue;
        for (int T = 2; T <= g.L[3]; T *= 2) {
            DslashTune t;
            t.march = T;
            t.SB = 64;
            t.RG = rg;
            t.split = 0;
            const long items = (long)nb3 * ((g.L[3] + T - 1) / T) * (nrhs / rg);
            t.grid = round8(std::min<long>(items, 2048));
            t.valid = 1;
            timeit(t);
            cands.push_back(t);
        }
    }
    std::sort(cands.begin(), cands.end(), [](const DslashTune &a, const DslashTune &b) { return a.ms < b.ms; });
    // stage 2: grid size and XCD chunking for the three best shapes
    DslashTune best = cands.empty() ? default_tune(g, prec, nrhs) : cands[0];
    for (size_t i = 0; i < std::min<size_t>(3, cands.size()); ++i) {
        const long items =
            cands[i].march > 0
                ? (long)((g.L[0] * g.L[1] * g.L[2] + 63) / 64) * ((g.L[3] + cands[i].march - 1) / cands[i].march)
                : (long)((g.V + cands[i].SB - 1) / cands[i].SB) * ((nrhs + cands[i].RG - 1) / cands[i].RG);
        const int caps[4] = {512, 1024, 2048, kMaxGrid};
        std::vector<int> chunks = {0, 1, 8, 64};
        if (cands[i].march == 0) {
            // one XCD per z-slab of a time slice, and multiples
            const long slab = (long)(g.L[0] * g.L[1] * g.L[2] / 8 / cands[i].SB) *
                              ((nrhs + cands[i].RG - 1) / cands[i].RG);
            for (long c : {slab, 2 * slab, 4 * slab})
                if (c >= 1 && std::find(chunks.begin(), chunks.end(), (int)c) == chunks.end())
                    chunks.push_back((int)c);
        }
        for (int cap : caps) {
            for (int ch : chunks) {
                DslashTune t = cands[i];
                t.grid = round8(std::min<long>(items, cap));
                t.chunk = ch;
                if (ch > 0 && ch * 8 >= items) continue;
                timeit(t);
                if (t.ms < best.ms) best = t;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != GRG_OK) return status;
    best.valid = 1;
    S->tune[prec][nrhs] = best;
    return GRG_OK;
}

// Launch of the fused defect-correction step: the site-parallel kernel
// (march == 0: SB threads, grid-stride over sites) or the t-marching kernel.
DslashTune default_dc_tune(const Geom &g)
{
    DslashTune t;
    t.SB = 128;
    t.RG = 1;
    t.grid = round8(std::min<long>((g.V + 127) / 128, 2048));
    return t;
}

// split 1: the LDS-ring form of the t-marching step (BF16 e, whole tiles of
// x-rows); otherwise split is 0
bool dc_launch_ok(const Geom &g, int prec, int nrhs, const DslashTune &t)
{
    if (t.grid < 8 || t.grid % 8 || t.grid > kMaxGridValue || t.chunk < 0 || t.march < 0) return false;
    // split: 0 the t-marching form, 1 its LDS-ring form, 3 the ring form with
    // the RHS groups of a tile adjacent in the item order
    if (t.split != 0 && t.split != 1 && t.split != 3) return false;
    const int V3 = g.L[0] * g.L[1] * g.L[2];
    if ((t.split & 1) && (t.march < 1 || prec != GRG_BF16 || V3 % 64 || 64 % g.L[0] || t.RG > 4)) return false;
    if (t.march > 0) return t.march <= g.L[3] && t.RG >= 1 && t.RG <= nrhs && 64 * t.RG <= 512;
    return t.SB == 64 || t.SB == 128 || t.SB == 256;
}

static void dc_fill_launch(DcArgs &d, const DslashTune &t)
{
    d.RG = t.RG;
    d.chunk = t.chunk;
    d.march = t.march;
    d.ring = (t.split & 1) != 0;
    d.grp_first = (t.split & 2) != 0;
}

// Autotuner of the defect-correction step (inner precision prec), timed on
// the handle's workspaces; every candidate computes the same sums in the
// same order per site.
grg_status tune_dc(grg_schur S, int prec, int nrhs, int reps)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    GRG_TRY(ensure_inner(S, prec));
    DcArgs d;
    d.e = S->in_b[prec];
    d.U = L->U[GRG_FP64];
    d.r_in = S->b64;
    d.x_in = nullptr;
    d.r_out = S->t64;
    d.x_out = nullptr;  // as the solver runs it: the iterate is summed at the end
    d.f = S->bn2 + kMaxRhs;
    d.r_next = S->in_q[prec];
    d.s_next = S->bn2 + 3 * kMaxRhs;
    d.mask = S->d_mask;
    d.diag = 4.0 + S->m0;
    d.g = g;
    d.nrhs = nrhs;
    d.partials = S->partials;
    hipEvent_t e0, e1;
    GRG_TRY_HIP(hipEventCreate(&e0));
    GRG_TRY_HIP(hipEventCreate(&e1));
    grg_status status = GRG_OK;
    DslashTune best = default_dc_tune(g);
    best.ms = 1e30f;
    auto timeit = [&](DslashTune t) {
        if (status != GRG_OK || !dc_launch_ok(g, prec, nrhs, t)) return;
        dc_fill_launch(d, t);
        hipError_t e = launch_dc_update(prec, d, t.grid, t.SB, st);
        for (int k = 0; k < reps && e == hipSuccess; ++k) {
            if (k == 0) e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = launch_dc_update(prec, d, t.grid, t.SB, st);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e != hipSuccess) {
            set_error("defect-correction tuning: %s", hipGetErrorString(e));
            status = GRG_EHIP;
            return;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        t.ms = ms / reps;
        if (t.ms < best.ms) best = t;
    };
    for (int sb : {64, 128, 256}) {
        DslashTune t = default_dc_tune(g);
        t.SB = sb;
        t.grid = round8(std::min<long>((g.V + sb - 1) / sb, 2048));
        timeit(t);
    }
    const int nb3 = (g.L[0] * g.L[1] * g.L[2] + 63) / 64;
    for (int rg = std::min(nrhs, 8); rg >= 1; --rg) {
        if (nrhs % rg) continue;
        for (int T = 2; T <= g.L[3]; T *= 2) {
            for (int ch : {0, 8, nb3 / 8, nb3 / 4, nb3 / 2}) {
                DslashTune t;
                t.march = T;
                t.SB = 64;
                t.RG = rg;
                t.chunk = ch;
                const long items = (long)nb3 * ((g.L[3] + T - 1) / T) * (nrhs / rg);
                if (ch > 0 && ch * 8 >= items) continue;
                t.grid = round8(std::min<long>(items, 2048));
                timeit(t);
                t.split = 1;  // the LDS-ring form (where valid)
                if (ch <= 8) timeit(t);
                // the ring form with the RHS groups of a tile together
                // (chunks: an eighth per XCD, or whole z-planes of tiles)
                t.split = 3;
                if (ch == 0 || ch == 8) timeit(t);
            }
            if (nrhs / rg > 1) {
                const int plane = (g.L[0] * g.L[1] + 63) / 64 * (nrhs / rg);
                for (int ch : {plane, 2 * plane}) {
                    DslashTune t;
                    t.march = T;
                    t.SB = 64;
                    t.RG = rg;
                    t.chunk = ch;
                    t.split = 3;
                    const long items = (long)nb3 * ((g.L[3] + T - 1) / T) * (nrhs / rg);
                    if (ch * 8 >= items) continue;
                    t.grid = round8(std::min<long>(items, 2048));
                    timeit(t);
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != GRG_OK) return status;
    best.valid = 1;
    S->dctune[prec][nrhs] = best;
    return GRG_OK;
}

static grg_status read_norms(grg_schur S, int nrhs, double *host)
{
    GRG_TRY_HIP(hipMemcpyAsync(S->h_buf, S->rn2, sizeof(double) * nrhs, hipMemcpyDeviceToHost,
                               S->lat->stream));
    GRG_TRY_HIP(hipStreamSynchronize(S->lat->stream));
    memcpy(host, S->h_buf, sizeof(double) * nrhs);
    return GRG_OK;
}

grg_status ensure_inner(grg_schur S, int prec)
{
    const Geom &g = S->lat->g;
    const int m = std::max(1, S->prm.restart);
    const size_t bytes = spinor_elems(g, S->prm.max_rhs) * prec_bytes(prec);
    void **bufs[4] = {&S->in_b[prec], &S->in_x[prec], &S->in_r[prec], &S->in_q[prec]};
    for (void **b : bufs) {
        if (*b) continue;
        if (hipMalloc(b, bytes) != hipSuccess) {
            *b = nullptr;
            set_error("inner workspace: hipMalloc of %zu bytes failed", bytes);
            return GRG_ENOMEM;
        }
        GRG_TRY_HIP(launch_fill_zero(*b, bytes, S->lat->stream));
    }
    const int need_m = (m > 1 || S->precond) ? m : 0;  // search directions kept
    if (need_m > 0 && S->in_m[prec] < need_m) {
        if (S->in_P[prec]) (void)hipFree(S->in_P[prec]);
        if (S->in_Q[prec]) (void)hipFree(S->in_Q[prec]);
        S->in_P[prec] = S->in_Q[prec] = nullptr;
        if (hipMalloc(&S->in_P[prec], bytes * need_m) != hipSuccess ||
            hipMalloc(&S->in_Q[prec], bytes * need_m) != hipSuccess) {
            set_error("GCR(%d) basis: hipMalloc of 2 x %zu bytes failed", m, bytes * need_m);
            return GRG_ENOMEM;
        }
        GRG_TRY_HIP(launch_fill_zero(S->in_P[prec], bytes * need_m, S->lat->stream));
        GRG_TRY_HIP(launch_fill_zero(S->in_Q[prec], bytes * need_m, S->lat->stream));
        S->in_m[prec] = need_m;
    }
    return GRG_OK;
}

// Inner GCR(m) on D_rr in precision prec: solves A x = b, with b already in
// in_r (it becomes the residual) and x in xdst, until |r|^2 <= thr[k] per RHS
// (thr: host copy of the device array thr2; HUGE_VAL for a RHS that takes no
// part, whose correction stays zero) or maxit iterations.
// Returns the iterations taken in *iters and the last |r|^2 read in rn2_out.
static grg_status inner_gcr(grg_schur S, int prec, int nrhs, const double *thr, int maxit,
                            int *iters, double *rn2_out, void *xdst)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    const BlasShape sh = blas_shape(g, nrhs);
    const size_t vbytes = spinor_elems(g, nrhs) * prec_bytes(prec);
    const size_t vstride = spinor_elems(g, nrhs) * prec_bytes(prec);
    const int m = std::max(1, S->prm.restart);
    const int check = std::max(1, S->prm.check_every);
    const DslashTune &tt = S->tune[prec][nrhs];
    const int dgrid = tt.valid ? tt.grid : default_tune(g, prec, nrhs).grid;
    void *x = xdst, *r = S->in_r[prec], *q = S->in_q[prec];
    char *Pm = (char *)S->in_P[prec], *Qm = (char *)S->in_Q[prec];

    GRG_TRY_HIP(launch_fill_zero(x, vbytes, st));
    GRG_TRY_HIP(launch_norm2(prec, sh, r, S->partials, st));
    GRG_TRY_HIP(launch_reduce(kNorm, S->partials, sh.grid, nrhs, nullptr, S->rn2, S->thr2,
                              S->active, st));
    double h[kMaxRhs];
    GRG_TRY(read_norms(S, nrhs, h));
    auto all_done = [&](const double *n2) {
        for (int k = 0; k < nrhs; ++k) {
            if (!isfinite(n2[k])) return -1;
            if (n2[k] > thr[k]) return 0;
        }
        return 1;
    };
    int it = 0;
    int done = all_done(h);
    while (done == 0 && it < maxit) {
        const int k = it % m;
        if (m == 1 && !S->precond) {
            GRG_TRY(run_dslash(S, prec, r, q, 0, nrhs, S->partials));
            PhaseTimer pt(S->prof, st, kProfBlas);
            GRG_TRY_HIP(launch_reduce(kAlpha, S->partials, dgrid, nrhs, S->alpha, nullptr, nullptr,
                                      S->active, st));
            GRG_TRY_HIP(launch_mr_update(prec, sh, x, r, q, nullptr, S->alpha, S->partials, st));
        } else {
            void *pk = Pm + (size_t)k * vstride, *qk = Qm + (size_t)k * vstride;
            if (S->precond) {
                PhaseTimer pt(S->prof, st, kProfPrec);
                GRG_TRY(precond_apply_inner(S, prec, r, pk, nrhs));  // p = M r
            } else {
                PhaseTimer pt(S->prof, st, kProfBlas);
                GRG_TRY_HIP(launch_copy(prec, sh, r, pk, st));
            }
            if (k == 0) {
                GRG_TRY(run_dslash(S, prec, pk, qk, 0, nrhs, S->partials, r));
                PhaseTimer pt(S->prof, st, kProfBlas);
                GRG_TRY_HIP(launch_reduce(kAlpha, S->partials, dgrid, nrhs, S->alpha, S->qn2,
                                          nullptr, S->active, st));
            } else {
                GRG_TRY(run_dslash(S, prec, pk, qk, 0, nrhs, nullptr));
                PhaseTimer pt(S->prof, st, kProfBlas);
                GRG_TRY_HIP(launch_multidot(prec, sh, Qm, k, qk, S->partials, st));
                GRG_TRY_HIP(launch_reduce_multi(S->partials, sh.grid, nrhs, k, S->qn2, S->active,
                                                S->beta, st));
                GRG_TRY_HIP(launch_orthogonalise(prec, sh, Qm, Pm, k, S->beta, qk, pk, r,
                                                 S->partials, st));
                GRG_TRY_HIP(launch_reduce(kAlpha, S->partials, sh.grid, nrhs, S->alpha,
                                          S->qn2 + (size_t)k * kMaxRhs, nullptr, S->active, st));
            }
            PhaseTimer pt(S->prof, st, kProfBlas);
            GRG_TRY_HIP(launch_mr_update(prec, sh, x, r, qk, pk, S->alpha, S->partials, st));
        }
        {
            PhaseTimer pt(S->prof, st, kProfBlas);
            GRG_TRY_HIP(launch_reduce(kNorm, S->partials, sh.grid, nrhs, nullptr, S->rn2, S->thr2,
                                      S->active, st));
        }
        ++it;
        if (it % check == 0 || it == maxit) {
            GRG_TRY(read_norms(S, nrhs, h));
            done = all_done(h);
        }
    }
    *iters = it;
    memcpy(rn2_out, h, sizeof(double) * nrhs);
    if (done < 0) {
        set_error("non-finite residual in the inner solve");
        return GRG_ENONFINITE;
    }
    return done ? GRG_OK : GRG_ENOCONV;
}

// ------------------------------------------------------------------ even-odd inner solve
// Geometry of the compact parity halves, for the vector kernels.
static Geom half_geom(grg_lattice L)
{
    Geom gh = L->g;
    gh.V = L->g.V / 2;
    gh.Vs = L->Vhs;
    return gh;
}

DslashTune default_eo_tune(const Geom &gh, int prec, int nrhs)
{
    DslashTune t;
    t.SB = 256;
    t.RG = std::min(nrhs, 3);
    t.split = prec == GRG_BF16 ? 2 : 1;  // hop schedule
    const long items = (long)((gh.V + t.SB - 1) / t.SB) * ((nrhs + t.RG - 1) / t.RG);
    t.grid = round8(std::min<long>(items, 2048));
    return t;
}

// Bytes of one compact half-lattice field at the handle's largest RHS count
// (the offset of the second half of a compact pair).
static size_t eo_half_bytes(grg_schur S, int prec)
{
    return spinor_elems(half_geom(S->lat), S->prm.max_rhs) * prec_bytes(prec);
}

// The compact pair the defect correction writes the next reduced solve's
// right-hand side into (parity eo_par's half first).
static grg_status ensure_eo_rhs(grg_schur S, int prec)
{
    if (S->eo_b[prec]) return GRG_OK;
    const size_t bytes = 2 * eo_half_bytes(S, prec);
    if (hipMalloc(&S->eo_b[prec], bytes) != hipSuccess) {
        S->eo_b[prec] = nullptr;
        set_error("even-odd workspace: hipMalloc of %zu bytes failed", bytes);
        return GRG_ENOMEM;
    }
    GRG_TRY_HIP(launch_fill_zero(S->eo_b[prec], bytes, S->lat->stream));
    return GRG_OK;
}

static grg_status ensure_eo(grg_schur S, int prec)
{
    grg_lattice L = S->lat;
    const size_t bytes = spinor_elems(half_geom(L), S->prm.max_rhs) * prec_bytes(prec);
    for (int k = 0; k < 5; ++k) {  // r, x, q, the other parity's w, and p
        void *&b = S->eo_f[prec][k];
        if (b) continue;
        if (hipMalloc(&b, bytes) != hipSuccess) {
            b = nullptr;
            set_error("even-odd workspace: hipMalloc of %zu bytes failed", bytes);
            return GRG_ENOMEM;
        }
        GRG_TRY_HIP(launch_fill_zero(b, bytes, L->stream));
    }
    return GRG_OK;
}

// out = alpha in2 + beta H in on the rest sites of parity po (compact fields)
// partials: per-workgroup sums, grid_out (if set) the number of workgroups
// that wrote them
static grg_status eo_hop(grg_schur S, int prec, const DslashTune &t, const void *in, const void *in2,
                         void *out, int po, double alpha, double beta, int nrhs, double *partials,
                         const void *dot_with, const int *active = nullptr, int in_full = 0,
                         int in2_full = 0, const void *partner = nullptr, int *grid_out = nullptr,
                         bool timed = true)
{
    grg_lattice L = S->lat;
    // the full-layout steps: with the t-marching form tuned, in the one-hop
    // shape the tuner recorded for them if it found that one faster
    const bool io = in_full || in2_full || partner;
    const DslashTune &tu =
        io && (t.split == 3 || t.split == 7) && S->eotune_io[prec][nrhs].valid ? S->eotune_io[prec][nrhs] : t;
    EoArgs a;
    a.in = in;
    a.in2 = in2;
    a.out = out;
    a.U = L->Ueo[prec];
    a.mask = S->d_mask_eo;
    a.po = po;
    a.alpha = alpha;
    a.beta = beta;
    a.g = L->g;
    a.Vh = L->g.V / 2;
    a.Vhs = L->Vhs;
    a.nrhs = nrhs;
    a.SB = tu.SB;
    a.RG = tu.RG;
    a.hops = tu.split;
    a.chunk = tu.chunk;
    a.march = tu.march;
    a.partials = partials;
    a.dot_with = dot_with;
    a.active = active;
    a.in_full = in_full;
    a.in2_full = in2_full;
    a.out_full = partner != nullptr;
    a.partner = partner;
    // profiled: the compact half-stencils of the reduced operator (the
    // per-iteration launches), not the full-layout first and last steps
    ProfilePool &P = S->prof;
    const bool ev = timed && !io && P.on && P.used < (int)P.start.size();
    if (ev) GRG_TRY_HIP(hipEventRecord(P.start[P.used], L->stream));
    GRG_TRY_HIP(launch_eo_hop(prec, a, tu.grid, L->stream));
    if (grid_out) *grid_out = tu.grid;
    if (ev) {
        GRG_TRY_HIP(hipEventRecord(P.stop[P.used], L->stream));
        P.prec[P.used] = prec + 3;
        ++P.used;
    }
    ++S->n_dslash;
    return GRG_OK;
}

bool eo_launch_ok(const Geom &gh, int prec, int nrhs, const DslashTune &t)
{
    // split 3: the t-marching form
    const int Lt = gh.L[3];
    const bool march_ok = t.split == 3 && prec == GRG_BF16 && t.SB == 256 && t.march >= 1 &&
                          t.march <= Lt && Lt >= 2 && gh.V % Lt == 0 && (gh.V / Lt) % 64 == 0 &&
                          gh.L[0] >= 2 && 64 % (gh.L[0] / 2) == 0;
    // split 4, 5: RG = 2, 3 right-hand sides carried through each hop together;
    // split 6: one hop per iteration with the x hops' spinors from lane
    // shuffles (x-rows of half-sites must tile a wavefront)
    const bool multi_ok = ((t.split == 4 || t.split == 5) && prec == GRG_BF16 && t.RG == t.split - 2) ||
                          (t.split == 6 && prec == GRG_BF16 && gh.L[0] >= 2 && 64 % (gh.L[0] / 2) == 0);
    // split 7: the plane form, one workgroup of Lx / 2 * Ly lanes per x-y plane
    // (RG = 1 one plane per workgroup, RG = 2 two planes z, z + 1, which
    // needs an even number of planes in every XCD's z-slab: Lz a multiple of 16)
    const int plane = (gh.L[0] / 2) * gh.L[1];
    const bool plane_ok = t.split == 7 && prec == GRG_BF16 && t.SB == plane && plane % 64 == 0 &&
                          plane <= 512 && t.march >= 1 && t.march <= Lt && Lt >= 2 &&
                          (t.RG == 1 || (t.RG == 2 && gh.L[2] % 16 == 0));
    if (t.split == 7)
        return plane_ok && t.grid >= 8 && t.grid % 8 == 0 && t.grid <= kMaxGridValue && t.chunk >= 0;
    return (t.SB == 64 || t.SB == 128 || t.SB == 256) && t.RG >= 1 && t.RG <= nrhs &&
           (t.split == 1 || (t.split == 2 && prec == GRG_BF16) || march_ok || multi_ok) && t.grid >= 8 &&
           t.grid % 8 == 0 && t.grid <= kMaxGridValue && t.chunk >= 0 && t.march >= 0 && gh.V > 0;
}

// Autotuner of the reduced operator's half-stencil (timed as the solver runs
// its second half: with the alpha term and the fused dot products).
grg_status tune_eo(grg_schur S, int prec, int nrhs, int reps)
{
    grg_lattice L = S->lat;
    if (!L->eo_ok) return GRG_OK;
    GRG_TRY(ensure_eo(S, prec));
    hipStream_t st = L->stream;
    const Geom gh = half_geom(L);
    void **f = S->eo_f[prec];
    hipEvent_t e0, e1;
    GRG_TRY_HIP(hipEventCreate(&e0));
    GRG_TRY_HIP(hipEventCreate(&e1));
    grg_status status = GRG_OK;
    auto timeit = [&](DslashTune &t) {
        if (status != GRG_OK) return;
        t.ms = 1e30f;
        if (!eo_launch_ok(gh, prec, nrhs, t)) return;
        status = eo_hop(S, prec, t, f[3], f[0], f[2], S->eo_par, 4.0, -0.25, nrhs, S->partials, f[0]);
        if (status == GRG_OK && hipEventRecord(e0, st) != hipSuccess) status = GRG_EHIP;
        for (int k = 0; k < reps && status == GRG_OK; ++k)
            status = eo_hop(S, prec, t, f[3], f[0], f[2], S->eo_par, 4.0, -0.25, nrhs, S->partials, f[0]);
        if (status == GRG_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            status = GRG_EHIP;
        if (status != GRG_OK) return;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        t.ms = ms / reps;
    };
    std::vector<DslashTune> cands;
    for (int sb : {64, 128, 256}) {
        for (int rg = 1; rg <= nrhs; ++rg) {
            if ((nrhs % rg && rg != nrhs) || (rg > 4 && rg != nrhs)) continue;
            for (int hops = 1; hops <= (prec == GRG_BF16 ? 6 : 1); ++hops) {
                if (hops == 3 || ((hops == 4 || hops == 5) && rg != hops - 2)) continue;
                DslashTune t = default_eo_tune(gh, prec, nrhs);
                t.SB = sb;
                t.RG = rg;
                t.split = hops;
                const long items = (long)((gh.V + sb - 1) / sb) * ((nrhs + rg - 1) / rg);
                t.grid = round8(std::min<long>(items, 2048));
                timeit(t);
                cands.push_back(t);
            }
        }
    }
    std::sort(cands.begin(), cands.end(), [](const DslashTune &a, const DslashTune &b) { return a.ms < b.ms; });
    DslashTune best = cands.empty() ? default_eo_tune(gh, prec, nrhs) : cands[0];
    DslashTune best_io;  // the best one-hop shape, for the full-layout steps
    best_io.ms = 1e30f;
    for (const DslashTune &c : cands)
        if (c.split == 1 && c.ms < best_io.ms) best_io = c;
    for (size_t i = 0; i < std::min<size_t>(2, cands.size()); ++i) {
        const long items = (long)((gh.V + cands[i].SB - 1) / cands[i].SB) *
                           ((nrhs + cands[i].RG - 1) / cands[i].RG);
        // chunks: one XCD per z-slab of a time slice (an eighth of its
        // half-sites) and multiples, besides the fixed sizes
        const long slab = (long)(gh.L[0] * gh.L[1] * gh.L[2] / 16 / cands[i].SB) *
                          ((nrhs + cands[i].RG - 1) / cands[i].RG);
        std::vector<int> chunks = {0, 8, 64};
        for (long c : {slab / 2, slab, 2 * slab, 4 * slab})
            if (c >= 1 && std::find(chunks.begin(), chunks.end(), (int)c) == chunks.end())
                chunks.push_back((int)c);
        for (int cap : {512, 1024, 2048, kMaxGridValue}) {
            for (int ch : chunks) {
                DslashTune t = cands[i];
                t.grid = round8(std::min<long>(items, cap));
                t.chunk = ch;
                if (ch > 0 && ch * 8 >= items) continue;
                timeit(t);
                if (t.ms < best.ms) best = t;
                if (t.split == 1 && t.ms < best_io.ms) best_io = t;
            }
        }
    }
    // the t-marching form: time slices per item, and grids of one, a half
    // and a quarter workgroup per item of the largest XCD share
    if (prec == GRG_BF16 && !cands.empty()) {
        const int Lt = gh.L[3];
        std::vector<int> mls;
        for (int ml : {Lt, Lt / 2, Lt / 4})
            if (ml >= 1 && std::find(mls.begin(), mls.end(), ml) == mls.end()) mls.push_back(ml);
        for (int ml : mls) {
            DslashTune t = cands[0];
            t.SB = 256;
            t.split = 3;
            t.march = ml;
            t.chunk = 0;
            const long nT = gh.V / Lt / 64;
            const long nx = (nT + 7) / 8 * ((nrhs + 3) / 4) * ((Lt + ml - 1) / ml);
            for (long div : {1, 2, 4}) {
                t.grid = round8(std::min<long>(8 * nx / div, kMaxGridValue));
                if (!eo_launch_ok(gh, prec, nrhs, t)) continue;
                timeit(t);
                if (t.ms < best.ms) best = t;
            }
        }
    }
    // the plane form: time slices per item, and grids of one, a half and a
    // quarter workgroup per item of the largest XCD share
    if (prec == GRG_BF16 && !cands.empty()) {
        const int Lt = gh.L[3];
        std::vector<int> mls;
        for (int ml : {Lt, Lt / 2, Lt / 4, Lt / 8})
            if (ml >= 1 && std::find(mls.begin(), mls.end(), ml) == mls.end()) mls.push_back(ml);
        for (int ml : mls) {
            for (int npl : {1, 2}) {
                DslashTune t = cands[0];
                t.SB = (gh.L[0] / 2) * gh.L[1];
                t.RG = npl;
                t.split = 7;
                t.march = ml;
                t.chunk = 0;
                const long nx = (long)((gh.L[2] + 7) / 8 / npl) * nrhs * ((Lt + ml - 1) / ml);
                for (long div : {1, 2, 4}) {
                    t.grid = round8(std::min<long>(8 * nx / div, kMaxGridValue));
                    if (!eo_launch_ok(gh, prec, nrhs, t)) continue;
                    timeit(t);
                    if (t.ms < best.ms) best = t;
                }
            }
        }
    }
    best_io.valid = best_io.ms < 1e29f ? 1 : 0;
    // the full-layout first and last steps with a t-marching form tuned:
    // that form or the best one-hop shape, whichever runs the pair faster
    if (status == GRG_OK && (best.split == 3 || best.split == 7) && best_io.valid) {
        status = ensure_inner(S, prec);
        const int P = S->eo_par, Q = 1 - P;
        const double d = 4.0 + S->m0;
        void *fb = S->in_r[prec], *fo = S->in_q[prec];
        auto time_io = [&](const DslashTune &t) -> float {
            float ms = 1e30f;
            for (int k = 0; k <= reps && status == GRG_OK; ++k) {
                if (k == 1 && hipEventRecord(e0, st) != hipSuccess) status = GRG_EHIP;
                if (status == GRG_OK)
                    status = eo_hop(S, prec, t, fb, fb, f[0], P, 1.0, -1.0 / d, nrhs, nullptr, nullptr,
                                    nullptr, 1, 1);
                if (status == GRG_OK)
                    status = eo_hop(S, prec, t, f[1], fb, fo, Q, 1.0 / d, -1.0 / d, nrhs, nullptr,
                                    nullptr, nullptr, 0, 1, f[1]);
            }
            if (status == GRG_OK &&
                (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                status = GRG_EHIP;
            if (status == GRG_OK) {
                (void)hipEventElapsedTime(&ms, e0, e1);
                ms /= reps;
            }
            return ms;
        };
        // with no one-hop shape recorded the full-layout steps run best itself
        S->eotune_io[prec][nrhs].valid = 0;
        const float ms_march = time_io(best);
        const float ms_one = time_io(best_io);
        if (ms_march <= ms_one) best_io.valid = 0;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != GRG_OK) return status;
    best.valid = 1;
    S->eotune[prec][nrhs] = best;
    S->eotune_io[prec][nrhs] = best_io;
    return GRG_OK;
}

// Minimal residual on the even-odd reduced system.  The inner right-hand
// side b is in in_r (full layout), or with bc in the compact pair the defect
// correction wrote (b_P at bc, b_Q one half on); the solution is written to
// xdst (full layout, zero on the coarse sites and for RHS that were already
// converged), as inner_gcr does.
static grg_status inner_mr_eo(grg_schur S, int prec, int nrhs, const double *thr, int maxit,
                              int *iters, double *rn2_out, void *xdst, const void *bc = nullptr)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    GRG_TRY(ensure_eo(S, prec));
    const Geom gh = half_geom(L);
    const BlasShape sh = blas_shape(gh, nrhs);
    const size_t vbytes = spinor_elems(gh, nrhs) * prec_bytes(prec);
    const DslashTune t = S->eotune[prec][nrhs].valid ? S->eotune[prec][nrhs]
                                                     : default_eo_tune(gh, prec, nrhs);
    const int P = S->eo_par, Q = 1 - P;
    void **f = S->eo_f[prec];
    void *r = f[0], *x = f[1], *q = f[2], *w = f[3];
    const void *b = S->in_r[prec];  // the unreduced right-hand side (full layout)
    const void *bQ = bc ? (const char *)bc + eo_half_bytes(S, prec) : nullptr;
    const double d = 4.0 + S->m0;
    const int check = std::max(1, S->prm.check_every);
    // the reduced right-hand side b_P - H_PQ b_Q / d, read from the full field
    // or the compact pair (with |r|^2 summed by the same launch)
    int pgrid = 0;
    if (bc)
        GRG_TRY(eo_hop(S, prec, t, bQ, bc, r, P, 1.0, -1.0 / d, nrhs, S->partials, nullptr, nullptr, 0, 0,
                       nullptr, &pgrid, false));
    else
        GRG_TRY(eo_hop(S, prec, t, b, b, r, P, 1.0, -1.0 / d, nrhs, S->partials, nullptr, nullptr, 1, 1,
                       nullptr, &pgrid));
    // |r|^2, the device's active flags, and act0: the RHS that take part
    // (finite threshold; the others keep a zero correction).  One whose
    // reduced right-hand side already meets its threshold takes no step,
    // x_P = 0, but its correction z_Q = b_Q / d is not zero.
    GRG_TRY_HIP(launch_reduce(kNorm3, S->partials, pgrid, nrhs, nullptr, S->rn2, S->thr2, S->active, st,
                              S->act0));
    double h[kMaxRhs];
    auto all_done = [&](const double *n2) {
        for (int k = 0; k < nrhs; ++k) {
            if (!isfinite(n2[k])) return -1;
            if (n2[k] > thr[k]) return 0;
        }
        return 1;
    };
    int it = 0;
    // the norms are first read after `check` iterations (inactive RHS leave
    // them unchanged), not before the first: one wait for the host fewer
    int done = 0;
    if (maxit <= 0) {
        GRG_TRY(read_norms(S, nrhs, h));
        done = all_done(h);
    }
    while (done == 0 && it < maxit) {
        // q = (d - H_PQ H_QP / d) r, with the sums for alpha
        GRG_TRY(eo_hop(S, prec, t, r, nullptr, w, Q, 0.0, 1.0, nrhs, nullptr, nullptr));
        GRG_TRY(eo_hop(S, prec, t, w, r, q, P, d, -1.0 / d, nrhs, S->partials, r));
        {
            PhaseTimer pt(S->prof, st, kProfBlas);
            GRG_TRY_HIP(launch_reduce(kAlpha, S->partials, t.grid, nrhs, S->alpha, nullptr, nullptr,
                                      S->active, st));
            // x starts at zero: the first step writes x = alpha r without reading it
            GRG_TRY_HIP(launch_mr_update(prec, sh, x, r, q, nullptr, S->alpha, S->partials, st, it == 0));
            GRG_TRY_HIP(launch_reduce(kNorm, S->partials, sh.grid, nrhs, nullptr, S->rn2, S->thr2,
                                      S->active, st));
        }
        ++it;
        if (it % check == 0 || it == maxit) {
            GRG_TRY(read_norms(S, nrhs, h));
            done = all_done(h);
        }
    }
    if (it == 0) GRG_TRY_HIP(launch_fill_zero(x, vbytes, st));
    *iters = it;
    memcpy(rn2_out, h, sizeof(double) * nrhs);
    // z_Q = (b_Q - H_QP z_P) / d (zero for the RHS that take no part),
    // written with z_P into the full layout
    GRG_TRY(eo_hop(S, prec, t, x, bc ? bQ : b, xdst, Q, 1.0 / d, -1.0 / d, nrhs, nullptr, nullptr, S->act0,
                   0, bc ? 0 : 1, x));
    if (done < 0) {
        set_error("non-finite residual in the inner solve");
        return GRG_ENONFINITE;
    }
    return done ? GRG_OK : GRG_ENOCONV;
}

// Minimal residual on the even-odd reduced system with a right
// preconditioner (flexible GCR(1)): p = M^ r, q = A^ p, x += alpha p,
// r -= alpha q, alpha = <q, r> / <q, q>.  M^ restricts the learned network
// to the reduced parity: r extended by zero to the other parity, the network,
// and its output on the reduced parity again.  Since the inverse of the
// reduced operator is the reduced-parity block of D_rr^{-1}, a network that
// approximates D_rr^{-1} approximates it too.  Same conventions as
// inner_mr_eo.
static grg_status inner_fgcr_eo(grg_schur S, int prec, int nrhs, const double *thr, int maxit,
                                int *iters, double *rn2_out, void *xdst)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    GRG_TRY(ensure_eo(S, prec));
    const Geom gh = half_geom(L);
    const BlasShape sh = blas_shape(gh, nrhs);
    const size_t vbytes = spinor_elems(gh, nrhs) * prec_bytes(prec);
    const DslashTune t = S->eotune[prec][nrhs].valid ? S->eotune[prec][nrhs]
                                                     : default_eo_tune(gh, prec, nrhs);
    const int P = S->eo_par, Q = 1 - P;
    void **f = S->eo_f[prec];
    void *r = f[0], *x = f[1], *q = f[2], *w = f[3], *pv = f[4];
    void *full_in = S->in_b[prec], *full_out = S->in_q[prec];
    const void *b = S->in_r[prec];
    const double d = 4.0 + S->m0;
    const int check = std::max(1, S->prm.check_every);
    // (with |r|^2 summed by the same launch)
    int pgrid = 0;
    GRG_TRY(eo_hop(S, prec, t, b, b, r, P, 1.0, -1.0 / d, nrhs, S->partials, nullptr, nullptr, 1, 1, nullptr,
                   &pgrid));
    GRG_TRY_HIP(launch_fill_zero(x, vbytes, st));
    GRG_TRY_HIP(launch_reduce(kNorm3, S->partials, pgrid, nrhs, nullptr, S->rn2, S->thr2, S->active, st));
    double h[kMaxRhs];
    GRG_TRY(read_norms(S, nrhs, h));
    {
        int *flags = (int *)(S->h_buf + 8 * kMaxRhs);
        for (int k = 0; k < nrhs; ++k) flags[k] = thr[k] < HUGE_VAL ? 1 : 0;  // taking part
        GRG_TRY_HIP(hipMemcpyAsync(S->act0, flags, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    }
    auto all_done = [&](const double *n2) {
        for (int k = 0; k < nrhs; ++k) {
            if (!isfinite(n2[k])) return -1;
            if (n2[k] > thr[k]) return 0;
        }
        return 1;
    };
    int it = 0;
    int done = all_done(h);
    while (done == 0 && it < maxit) {
        // p = M^ r
        {
            PhaseTimer pt(S->prof, st, kProfPrec);
            GRG_TRY_HIP(launch_eo_scatter(prec, g, nrhs, P, r, full_in, true, st));
            GRG_TRY(precond_apply_inner(S, prec, full_in, full_out, nrhs));
            GRG_TRY_HIP(launch_eo_scatter(prec, g, nrhs, P, full_out, pv, false, st));
        }
        // q = A^ p with the sums <q, r>, |q|^2
        GRG_TRY(eo_hop(S, prec, t, pv, nullptr, w, Q, 0.0, 1.0, nrhs, nullptr, nullptr));
        GRG_TRY(eo_hop(S, prec, t, w, pv, q, P, d, -1.0 / d, nrhs, S->partials, r));
        {
            PhaseTimer pt(S->prof, st, kProfBlas);
            GRG_TRY_HIP(launch_reduce(kAlpha, S->partials, t.grid, nrhs, S->alpha, nullptr, nullptr,
                                      S->active, st));
            GRG_TRY_HIP(launch_mr_update(prec, sh, x, r, q, pv, S->alpha, S->partials, st));
            GRG_TRY_HIP(launch_reduce(kNorm, S->partials, sh.grid, nrhs, nullptr, S->rn2, S->thr2,
                                      S->active, st));
        }
        ++it;
        if (it % check == 0 || it == maxit) {
            GRG_TRY(read_norms(S, nrhs, h));
            done = all_done(h);
        }
    }
    *iters = it;
    memcpy(rn2_out, h, sizeof(double) * nrhs);
    GRG_TRY(eo_hop(S, prec, t, x, b, xdst, Q, 1.0 / d, -1.0 / d, nrhs, nullptr, nullptr, S->act0,
                   0, 1, x));
    if (done < 0) {
        set_error("non-finite residual in the inner solve");
        return GRG_ENONFINITE;
    }
    return done ? GRG_OK : GRG_ENOCONV;
}

// BiCGstab (van der Vorst) for the inner solve, on D_rr or, with reduce, on
// its even-odd reduced system; same conventions as inner_gcr (right-hand
// side in in_r, correction to xdst, zero for RHS that took no step) and
// inner_mr_eo.  The shadow residual is the initial residual.  Per iteration:
// v = A p with the sums against r0 fused into the stencil, alpha =
// rho / <r0, v>, s = r - alpha v, t = A s with <t, s> and |t|^2 fused,
// omega = <t, s> / |t|^2, x += alpha p + omega s, r = s - omega t (with
// <r0, r> and |r|^2), beta = (rho' / rho)(alpha / omega), p = r + beta (p -
// omega v).  All scalars stay on the device.
static grg_status inner_bicgstab(grg_schur S, int prec, int nrhs, const double *thr, int maxit,
                                 int *iters, double *rn2_out, void *xdst, bool reduce)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    const size_t full_bytes = spinor_elems(g, S->prm.max_rhs) * prec_bytes(prec);
    for (int k = 0; k < 5; ++k) {
        void *&b = S->bicg_f[prec][k];
        if (b) continue;
        if (hipMalloc(&b, full_bytes) != hipSuccess) {
            b = nullptr;
            set_error("BiCGstab workspace: hipMalloc of %zu bytes failed", full_bytes);
            return GRG_ENOMEM;
        }
        GRG_TRY_HIP(launch_fill_zero(b, full_bytes, st));
    }
    void **bf = S->bicg_f[prec];
    void *pv = bf[0], *v = bf[1], *sv = bf[2], *tv = bf[3], *r0 = bf[4];
    const double d = 4.0 + S->m0;
    const int P = S->eo_par, Q = 1 - P;
    const void *b = S->in_r[prec];
    void *r, *x, *w = nullptr;
    Geom gv = g;
    DslashTune te;
    int nparts;
    if (reduce) {
        GRG_TRY(ensure_eo(S, prec));
        gv = half_geom(L);
        te = S->eotune[prec][nrhs].valid ? S->eotune[prec][nrhs] : default_eo_tune(gv, prec, nrhs);
        nparts = te.grid;
        r = S->eo_f[prec][0];
        x = S->eo_f[prec][1];
        w = S->eo_f[prec][3];
    } else {
        const DslashTune &tt = S->tune[prec][nrhs];
        nparts = tt.valid ? tt.grid : default_tune(g, prec, nrhs).grid;
        r = S->in_r[prec];
        x = xdst;
    }
    const BlasShape sh = blas_shape(gv, nrhs);
    const size_t vbytes = spinor_elems(gv, nrhs) * prec_bytes(prec);
    const int check = std::max(1, S->prm.check_every);
    double2 *sc = S->bicg_sc;
    auto apply = [&](const void *in, void *out, const void *dot_with) -> grg_status {
        if (reduce) {
            GRG_TRY(eo_hop(S, prec, te, in, nullptr, w, Q, 0.0, 1.0, nrhs, nullptr, nullptr));
            return eo_hop(S, prec, te, w, in, out, P, d, -1.0 / d, nrhs, S->partials, dot_with);
        }
        return run_dslash(S, prec, in, out, 0, nrhs, S->partials, dot_with);
    };
    // r: the (reduced) right-hand side; x = 0; r0 = p = r
    if (reduce)
        GRG_TRY(eo_hop(S, prec, te, b, b, r, P, 1.0, -1.0 / d, nrhs, nullptr, nullptr, nullptr, 1, 1));
    GRG_TRY_HIP(launch_fill_zero(x, vbytes, st));
    GRG_TRY_HIP(launch_norm2(prec, sh, r, S->partials, st));
    GRG_TRY_HIP(launch_bicg_reduce(kBicgInit, S->partials, sh.grid, nrhs, sc, S->rn2, S->thr2, S->active,
                                   st));
    GRG_TRY_HIP(launch_copy(prec, sh, r, r0, st));
    GRG_TRY_HIP(launch_copy(prec, sh, r, pv, st));
    double h[kMaxRhs];
    GRG_TRY(read_norms(S, nrhs, h));
    if (reduce) {
        int *flags = (int *)(S->h_buf + 8 * kMaxRhs);
        for (int k = 0; k < nrhs; ++k) flags[k] = thr[k] < HUGE_VAL ? 1 : 0;  // taking part
        GRG_TRY_HIP(hipMemcpyAsync(S->act0, flags, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    }
    auto all_done = [&](const double *n2) {
        for (int k = 0; k < nrhs; ++k) {
            if (!isfinite(n2[k])) return -1;
            if (n2[k] > thr[k]) return 0;
        }
        return 1;
    };
    int it = 0;
    int done = all_done(h);
    while (done == 0 && it < maxit) {
        GRG_TRY(apply(pv, v, r0));
        {
            PhaseTimer pt(S->prof, st, kProfBlas);
            GRG_TRY_HIP(launch_bicg_reduce(kBicgAlpha, S->partials, nparts, nrhs, sc, nullptr, nullptr,
                                           S->active, st));
            GRG_TRY_HIP(launch_bicg(prec, kBicgS, sh, nullptr, sv, r, v, nullptr, nullptr, sc, nullptr, st));
        }
        GRG_TRY(apply(sv, tv, sv));
        {
            PhaseTimer pt(S->prof, st, kProfBlas);
            GRG_TRY_HIP(launch_reduce(kAlpha, S->partials, nparts, nrhs, sc + 2 * kMaxRhs, nullptr, nullptr,
                                      S->active, st));
            GRG_TRY_HIP(launch_bicg(prec, kBicgUpd, sh, x, r, pv, sv, tv, r0, sc, S->partials, st));
            GRG_TRY_HIP(launch_bicg_reduce(kBicgBeta, S->partials, sh.grid, nrhs, sc, S->rn2, S->thr2,
                                           S->active, st));
            GRG_TRY_HIP(launch_bicg(prec, kBicgP, sh, nullptr, pv, r, v, nullptr, nullptr, sc, nullptr, st));
        }
        ++it;
        if (it % check == 0 || it == maxit) {
            GRG_TRY(read_norms(S, nrhs, h));
            done = all_done(h);
        }
    }
    *iters = it;
    memcpy(rn2_out, h, sizeof(double) * nrhs);
    if (reduce)
        GRG_TRY(eo_hop(S, prec, te, x, b, xdst, Q, 1.0 / d, -1.0 / d, nrhs, nullptr, nullptr, S->act0,
                       0, 1, x));
    if (done < 0) {
        set_error("non-finite residual in the inner solve");
        return GRG_ENONFINITE;
    }
    return done ? GRG_OK : GRG_ENOCONV;
}

// A training pair of the reduced system for the learned preconditioner.
// e (BF16, full layout) holds the error e_0 on the reduced parity's rest
// sites.  k minimal-residual steps on A^ x = A^ e_0 from x = 0 (the reduced
// inner solve without the network) leave e_k = e_0 - x_k in e and
// r_k = A^ e_k in r, both in the full layout and zero on the other parity:
// the residuals that the reduced inner solve hands the network, with the
// errors it should map them to.
grg_status eo_training_pair(grg_schur S, void *e, void *r_full, int nrhs, int k, const double *neg_one)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const int prec = GRG_BF16;
    GRG_TRY(ensure_eo(S, prec));
    const Geom gh = half_geom(L);
    const BlasShape sh = blas_shape(gh, nrhs);
    const DslashTune t = S->eotune[prec][nrhs].valid ? S->eotune[prec][nrhs]
                                                     : default_eo_tune(gh, prec, nrhs);
    const int P = S->eo_par, Q = 1 - P;
    const double d = 4.0 + S->m0;
    void **f = S->eo_f[prec];
    void *r = f[0], *x = f[1], *q = f[2], *w = f[3], *e0 = f[4];
    GRG_TRY_HIP(launch_eo_scatter(prec, L->g, nrhs, P, e, e0, false, st));
    GRG_TRY(eo_hop(S, prec, t, e0, nullptr, w, Q, 0.0, 1.0, nrhs, nullptr, nullptr));
    GRG_TRY(eo_hop(S, prec, t, w, e0, r, P, d, -1.0 / d, nrhs, nullptr, nullptr));
    GRG_TRY_HIP(launch_fill_zero(x, spinor_elems(gh, nrhs) * prec_bytes(prec), st));
    for (int j = 0; j < k; ++j) {
        GRG_TRY(eo_hop(S, prec, t, r, nullptr, w, Q, 0.0, 1.0, nrhs, nullptr, nullptr));
        GRG_TRY(eo_hop(S, prec, t, w, r, q, P, d, -1.0 / d, nrhs, S->partials, r));
        GRG_TRY_HIP(launch_reduce(kAlpha, S->partials, t.grid, nrhs, S->alpha, nullptr, nullptr,
                                  nullptr, st));
        GRG_TRY_HIP(launch_mr_update(prec, sh, x, r, q, nullptr, S->alpha, S->partials, st));
    }
    // e_k = e_0 - x_k and r_k = A^ e_k (recomputed, so that the pair is
    // consistent to rounding)
    GRG_TRY_HIP(launch_axpy_convert(prec, prec, sh, x, e0, neg_one, 0, 1, nullptr, st));
    GRG_TRY(eo_hop(S, prec, t, e0, nullptr, w, Q, 0.0, 1.0, nrhs, nullptr, nullptr));
    GRG_TRY(eo_hop(S, prec, t, w, e0, r, P, d, -1.0 / d, nrhs, nullptr, nullptr));
    GRG_TRY_HIP(launch_eo_scatter(prec, L->g, nrhs, P, e0, e, true, st));
    GRG_TRY_HIP(launch_eo_scatter(prec, L->g, nrhs, P, r, r_full, true, st));
    return GRG_OK;
}

// Inner iterations allowed to a preconditioned inner solve before the plain
// GCR fallback takes over.
constexpr int kPrecondInnerCap = 100;

// The inner right-hand side s_k r_k in the inner precision, from the FP64
// residual r (scale: device array of s_k).
static grg_status convert_rhs(grg_schur S, int prec, const BlasShape &sh, const void *r_src,
                              const double *scale, int r_prec = GRG_FP64, bool pair = false)
{
    PhaseTimer pt(S->prof, S->lat->stream, kProfBlas);
    if (pair) {
        // into the compact pair the reduced solve reads (parity eo_par first)
        GRG_TRY(ensure_eo_rhs(S, prec));
        GRG_TRY_HIP(launch_axpy_convert(r_prec, prec, sh, r_src, S->eo_b[prec], scale, 0, 0, nullptr,
                                        S->lat->stream, eo_half_bytes(S, prec) / prec_bytes(prec),
                                        S->eo_par));
        return GRG_OK;
    }
    GRG_TRY_HIP(launch_axpy_convert(r_prec, prec, sh, r_src, S->in_r[prec], scale, 0, 0, nullptr,
                                    S->lat->stream));
    return GRG_OK;
}

// The defect correction keeps its residual in FP64 until it is small: once
// |r_k| <= theta |b| for every RHS, the next steps store it in FP32.  Each
// later store rounds by at most 2^-24 |r_j| (relative), so the recursively
// updated residual drifts from b - A x by at most 2^-24 sum_j |r_j| <= 2^-24
// theta |b| (1 + inner_tol + ...) ~ 6e-8 theta |b|: theta = 1e5 tol keeps
// that below 1 % of the tolerance.
static double dc_fp32_threshold(double tol) { return std::min(1e-3, 1e5 * tol); }

// A slot of the correction pool (inner precision, full layout, max_rhs).
static grg_status pool_slot(grg_schur S, int prec, int k, void **out)
{
    auto &pool = S->epool[prec];
    while ((int)pool.size() <= k) {
        void *b = nullptr;
        const size_t bytes = spinor_elems(S->lat->g, S->prm.max_rhs) * prec_bytes(prec);
        if (hipMalloc(&b, bytes) != hipSuccess) {
            set_error("correction pool: hipMalloc of %zu bytes failed", bytes);
            return GRG_ENOMEM;
        }
        pool.push_back(b);
    }
    *out = pool[k];
    return GRG_OK;
}

// b64 (internal FP64, zero on coarse sites) -> x64 = D_rr^{-1} b64, or with
// u_minus set, x64 = u_minus - D_rr^{-1} b64 (what S_bb needs next).
//
// Outer loop, FP64 (r_0 = b, x_0 = 0), with a per-RHS scale s_k:
//     e_k ~= A^{-1} (s r)                          inner solve, inner precision
//     r   <- r - A e_k / s                         one fused FP64 kernel, which
//                                                  also writes s' r for the next
//                                                  inner solve
// until |r| <= tol |b|; the iterate x = sum_k e_k / s_k is formed once at the
// end from the kept corrections (in FP64, the same sum the steps would have
// accumulated), so the steps do not stream x.  s_0 = 1 / |b|; s' = 1 / (the
// new |r| the inner solve predicts), so the inner fields stay of order one (a
// scale off by a few orders of magnitude is harmless: BF16 and FP32 share an
// exponent range far wider than that); the inner thresholds are taken
// relative to the actual |s r|.  The FP64 residual r is updated with the
// exact FP64 operator at every step, so it is the residual of x up to FP64
// rounding; with params.verify it is also recomputed from x as b - A x at the
// end, and the loop resumes from that residual if it is above tol.
// With xb and yb (the S_bb apply): u_minus = x_b on the coarse sites is
// scattered into S->u64 only if the iterate is summed over the lattice, and
// when it is not (no pool overflow, no verification) the final step writes
// y_b = [D (u - z)]_b from the corrections directly and sets *fused.
grg_status drr_solve_internal(grg_schur S, int nrhs, grg_solver_stats *stats, const void *u_minus,
                              const double *xb, double *yb, bool *fused, int bn2_parts, bool rhs_pair)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    const grg_solver_params &p = S->prm;
    const int prec = p.inner;
    const BlasShape sh = blas_shape(g, nrhs);
    GRG_TRY(ensure_inner(S, prec));
    // device per-RHS scalars: |b|^2, then f = 1/s, s, and the next s
    double *d_f = S->bn2 + kMaxRhs, *d_s = S->bn2 + 2 * kMaxRhs, *d_sn = S->bn2 + 3 * kMaxRhs;

    // |b|^2: from the partial sums the producer of b left (bn2_parts > 0), or a pass over b
    if (bn2_parts <= 0) GRG_TRY_HIP(launch_norm2(GRG_FP64, sh, S->b64, S->partials, st));
    GRG_TRY_HIP(launch_reduce(kNorm, S->partials, bn2_parts > 0 ? bn2_parts : sh.grid, nrhs, nullptr, S->bn2,
                              nullptr, nullptr, st));
    double bn2[kMaxRhs], rn2[kMaxRhs], sc[kMaxRhs], scn[kMaxRhs], ih[kMaxRhs];
    GRG_TRY_HIP(hipMemcpyAsync(S->h_buf, S->bn2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    GRG_TRY_HIP(hipStreamSynchronize(st));
    memcpy(bn2, S->h_buf, sizeof(double) * nrhs);
    memcpy(rn2, bn2, sizeof(double) * nrhs);
    for (int k = 0; k < nrhs; ++k) sc[k] = bn2[k] > 0 && isfinite(bn2[k]) ? 1.0 / sqrt(bn2[k]) : 1.0;
    // rhs_pair: the producer of b also wrote it unscaled (s = 1) into the
    // compact pair of the reduced solve; used when that is the first inner
    // solve and every |b| is within [1e-10, 1e10] (the inner precision's
    // sums then stay far inside FP32's range), else converted as usual
    const bool pair_inner = p.eo && L->eo_ok && 4.0 + S->m0 != 0.0 && std::max(1, p.restart) == 1 &&
                            !S->precond && p.method == 0;
    bool pair_ok = rhs_pair && pair_inner;
    for (int k = 0; k < nrhs && pair_ok; ++k)
        if (!(bn2[k] == 0.0 || (bn2[k] >= 1e-20 && bn2[k] <= 1e20))) pair_ok = false;
    if (pair_ok)
        for (int k = 0; k < nrhs; ++k) sc[k] = 1.0;
    // the per-RHS scalar block bn2: row 0 |b|^2, rows 1..4 f = 1/s, s, the
    // next s and the inner thresholds (thr2), staged on the host at hb (row k
    // at hb + (k - 1) kMaxRhs; reads use the front of h_buf), rows k0..k1
    // uploaded by one copy
    double *hb = S->h_buf + 4 * kMaxRhs;
    auto stage = [&](int row, const double *src) { memcpy(hb + (row - 1) * kMaxRhs, src, sizeof(double) * nrhs); };
    auto upload_rows = [&](int k0, int k1) -> grg_status {
        GRG_TRY_HIP(hipMemcpyAsync(S->bn2 + k0 * kMaxRhs, hb + (k0 - 1) * kMaxRhs,
                                   sizeof(double) * kMaxRhs * (k1 - k0 + 1), hipMemcpyHostToDevice, st));
        return GRG_OK;
    };
    // the kept corrections and the part of x already summed into x64
    int npool = 0;
    int ncorr = 0, nsummed = 0;  // corrections made, and summed into x64
    bool have_x = false;
    bool u_ready = xb == nullptr;
    if (fused) *fused = false;
    auto combine = [&](const void *u, double sigma) -> grg_status {
        if (u && !u_ready) {
            GRG_TRY_HIP(launch_scatter_coarse(xb, (void *)u, S->d_bidx, S->nb, g, nrhs, st));
            u_ready = true;
        }
        CombineArgs c;
        for (int j = 0; j < kCorrPool; ++j) c.e[j] = j < npool ? S->epool[prec][j] : nullptr;
        c.f = S->d_fk;
        c.n = npool;
        c.u = u;
        c.x = have_x ? S->x64 : nullptr;
        c.out = S->x64;
        c.sigma = sigma;
        if (npool > 0)
            GRG_TRY_HIP(hipMemcpyAsync(S->d_fk, S->h_fk, sizeof(double) * kCorrPool * kMaxRhs,
                                       hipMemcpyHostToDevice, st));
        {
            PhaseTimer pt(S->prof, st, kProfBlas);
            GRG_TRY_HIP(launch_combine(prec, sh, c, st));
        }
        if (npool > 0) GRG_TRY_HIP(hipStreamSynchronize(st));  // h_fk is reused next
        npool = 0;
        nsummed = ncorr;
        have_x = true;
        return GRG_OK;
    };
    // per RHS the iterate of smallest FP64 residual so far (returned with
    // GRG_ENOCONV): that residual and the corrections it sums (0: x = 0)
    double best[kMaxRhs];
    int best_n[kMaxRhs];
    for (int k = 0; k < nrhs; ++k) {
        best[k] = bn2[k];
        best_n[k] = 0;
    }

    const void *r_src = S->b64;  // the residual of the current iterate
    int r_prec = GRG_FP64;       // its storage (FP32 in the late steps, see dc_fp32_threshold)
    bool rhs_ready = pair_ok;    // in_r holds s r_src in the inner precision
    bool rhs_compact = pair_ok;  // ... in the compact pair eo_b instead (the reduced solve's)
    int total = 0, outer = 0;
    bool verified = false;
    grg_status status = GRG_OK;
    double worst = 0;
    const DslashTune dct = S->dctune[prec][nrhs].valid ? S->dctune[prec][nrhs] : default_dc_tune(g);
    for (;;) {
        bool conv = true;
        worst = 0;
        for (int k = 0; k < nrhs; ++k) {
            if (!isfinite(rn2[k])) {
                set_error("non-finite FP64 residual");
                return GRG_ENONFINITE;
            }
            const double rel = bn2[k] > 0 ? sqrt(rn2[k] / bn2[k]) : 0.0;
            worst = std::max(worst, rel);
            if (rel > p.tol) conv = false;
        }
        if (conv && (verified || outer == 0 || !p.verify)) break;
        if (conv) {
            // confirm with the residual recomputed from the iterate
            GRG_TRY(combine(nullptr, 1.0));
            GRG_TRY(run_dslash(S, GRG_FP64, S->x64, S->t64, 0, nrhs, nullptr));
            GRG_TRY_HIP(launch_sub_norm(sh, S->b64, S->t64, S->r64, S->partials, st));
            GRG_TRY_HIP(launch_reduce(kNorm, S->partials, sh.grid, nrhs, nullptr, S->rn2, nullptr,
                                      nullptr, st));
            GRG_TRY(read_norms(S, nrhs, rn2));
            for (int k = 0; k < nrhs; ++k)
                if (best_n[k] == ncorr) best[k] = rn2[k];
            r_src = S->r64;
            r_prec = GRG_FP64;
            rhs_ready = false;
            verified = true;
            continue;
        }
        verified = false;
        if (outer >= p.max_outer || total >= p.max_iter) {
            status = GRG_ENOCONV;
            break;
        }
        if (npool == kCorrPool) GRG_TRY(combine(nullptr, 1.0));  // pool full: sum it into x64
        void *e = nullptr;
        GRG_TRY(pool_slot(S, prec, npool, &e));
        // inner thresholds on the scaled residual s r, |s r|^2 = s^2 |r|^2
        double thr[kMaxRhs], f[kMaxRhs];
        for (int k = 0; k < nrhs; ++k) {
            const double need = bn2[k] > 0 && rn2[k] > 0 ? p.tol * sqrt(bn2[k] / rn2[k]) : 1.0;
            const double rel = prec == GRG_FP64 ? need : std::max(p.inner_tol, 0.5 * need);
            const bool on = bn2[k] > 0 && sqrt(rn2[k] / bn2[k]) > p.tol;
            ih[k] = sc[k] * sc[k] * rn2[k];
            thr[k] = on ? rel * rel * ih[k] : HUGE_VAL;  // converged: takes no part
            f[k] = 1.0 / sc[k];
        }
        stage(4, thr);
        stage(1, f);
        if (!rhs_ready) stage(2, sc);
        GRG_TRY(upload_rows(1, 4));  // f, s (when it changes), thresholds
        // the reduced system divides by the diagonal d = 4 + m0: none at d = 0
        const bool eo_form = p.eo && L->eo_ok && 4.0 + S->m0 != 0.0;
        const bool reduce = eo_form && std::max(1, p.restart) == 1;
        // the inner right-hand side as the compact pair of the reduced solve
        // when that is the inner solve (converted here, or written so by the
        // previous defect-correction step)
        const bool pair_rhs = reduce && !S->precond && p.method == 0;
        if (!rhs_ready) {
            GRG_TRY(convert_rhs(S, prec, sh, r_src, d_s, r_prec, pair_rhs));
            rhs_compact = pair_rhs;
        }
        int it = 0;
        grg_status is;
        double h[kMaxRhs];
        if (p.method == 1) {
            is = inner_bicgstab(S, prec, nrhs, thr, p.max_iter - total, &it, h, e, eo_form);
            total += it;
        } else if (S->precond) {
            // preconditioned inner solve, with the plain solve as the fallback
            const int cap = std::min(p.max_iter - total, kPrecondInnerCap);
            is = reduce ? inner_fgcr_eo(S, prec, nrhs, thr, cap, &it, h, e)
                        : inner_gcr(S, prec, nrhs, thr, cap, &it, h, e);
            total += it;
            if (is != GRG_OK) {
                grg_precond keep = S->precond;
                S->precond = nullptr;
                ++S->fallbacks;
                stage(2, sc);
                GRG_TRY(upload_rows(2, 2));
                GRG_TRY(convert_rhs(S, prec, sh, r_src, d_s, r_prec));
                is = reduce ? inner_mr_eo(S, prec, nrhs, thr, p.max_iter - total, &it, h, e)
                            : inner_gcr(S, prec, nrhs, thr, p.max_iter - total, &it, h, e);
                S->precond = keep;
                total += it;
            }
        } else if (reduce) {
            is = inner_mr_eo(S, prec, nrhs, thr, p.max_iter - total, &it, h, e,
                             rhs_compact ? S->eo_b[prec] : nullptr);
            total += it;
        } else {
            is = inner_gcr(S, prec, nrhs, thr, p.max_iter - total, &it, h, e);
            total += it;
        }
        if (is != GRG_OK && is != GRG_ENOCONV) return is;
        ++outer;
        // scale of the next inner right-hand side: the new |r| is about
        // |s r_inner| / s
        for (int k = 0; k < nrhs; ++k) {
            const double est = sqrt(h[k] > 0 ? h[k] : 0.0) / sc[k];
            scn[k] = est > 0 && isfinite(est) && isfinite(1.0 / est) ? 1.0 / est : sc[k];
        }
        stage(3, scn);
        GRG_TRY(upload_rows(3, 3));
        // r -= A e / s ; next inner rhs s' r   (FP64, fused; x is summed at the end)
        // the residual's storage from here on: FP32 once it is small for
        // every RHS (r_src is that of the step's input)
        bool small = r_prec == GRG_FP32;
        if (!small && prec != GRG_FP64) {
            small = true;
            const double theta = dc_fp32_threshold(p.tol);
            for (int k = 0; k < nrhs; ++k)
                if (bn2[k] > 0 && !(rn2[k] <= theta * theta * bn2[k])) small = false;
        }
        if (small && !S->r32) {
            const size_t bytes = spinor_elems(g, S->prm.max_rhs) * prec_bytes(GRG_FP32);
            if (hipMalloc(&S->r32, bytes) != hipSuccess) {
                S->r32 = nullptr;
                small = false;  // keep FP64
            }
        }
        DcArgs d;
        d.e = e;
        d.U = L->U[GRG_FP64];
        d.r_in = r_src;
        d.r_in32 = r_prec == GRG_FP32;
        d.x_in = nullptr;
        d.r_out = small ? S->r32 : S->r64;
        d.r_out32 = small;
        d.x_out = nullptr;
        d.f = d_f;
        // the next inner right-hand side: straight into the compact pair of
        // the reduced solve when the next inner solve is that one
        const bool next_compact = pair_rhs;
        if (next_compact) GRG_TRY(ensure_eo_rhs(S, prec));
        d.r_next = next_compact ? S->eo_b[prec] : S->in_r[prec];
        d.next_half = next_compact ? eo_half_bytes(S, prec) / prec_bytes(prec) : 0;
        d.next_par = S->eo_par;
        d.s_next = d_sn;
        d.mask = S->d_mask;
        d.diag = 4.0 + S->m0;
        d.g = g;
        d.nrhs = nrhs;
        d.partials = S->partials;
        dc_fill_launch(d, dct);
        {
            PhaseTimer pt(S->prof, st, kProfDc);
            GRG_TRY_HIP(launch_dc_update(prec, d, dct.grid, dct.SB, st));
            GRG_TRY_HIP(launch_reduce(kNorm, S->partials, dct.grid, nrhs, nullptr, S->rn2, nullptr,
                                      nullptr, st));
        }
        for (int k = 0; k < kMaxRhs; ++k) S->h_fk[npool * kMaxRhs + k] = k < nrhs ? f[k] : 0.0;
        ++npool;
        ++ncorr;
        GRG_TRY(read_norms(S, nrhs, rn2));
        for (int k = 0; k < nrhs; ++k)
            if (rn2[k] < best[k]) {
                best[k] = rn2[k];
                best_n[k] = ncorr;
            }
        memcpy(sc, scn, sizeof(double) * nrhs);
        r_src = small ? S->r32 : S->r64;
        r_prec = small ? GRG_FP32 : GRG_FP64;
        rhs_ready = true;
        rhs_compact = next_compact;
    }
    if (status == GRG_ENOCONV) {
        // return each RHS's best iterate: drop the corrections after it that
        // are still kept (those summed into x64 already stay)
        worst = 0;
        for (int k = 0; k < nrhs; ++k) {
            if (best_n[k] < ncorr && best_n[k] >= nsummed) {
                for (int j = best_n[k] - nsummed; j < npool; ++j) S->h_fk[j * kMaxRhs + k] = 0.0;
                rn2[k] = best[k];
            }
            worst = std::max(worst, bn2[k] > 0 ? sqrt(rn2[k] / bn2[k]) : 0.0);
        }
        set_error("D_rr solve: no convergence after %d outer / %d inner iterations "
                  "(residual of the returned iterate %.3e > %.3e)", outer, total, worst, p.tol);
    }
    if (xb && yb && fused && u_minus && !have_x) {
        // y_b = [D (u - sum_j f_j e_j)]_b straight from the corrections
        CombineArgs c;
        for (int j = 0; j < kCorrPool; ++j) c.e[j] = j < npool ? S->epool[prec][j] : nullptr;
        c.f = S->d_fk;
        c.n = npool;
        c.u = nullptr;
        c.x = nullptr;
        c.out = nullptr;
        c.sigma = -1.0;
        if (npool > 0)
            GRG_TRY_HIP(hipMemcpyAsync(S->d_fk, S->h_fk, sizeof(double) * kCorrPool * kMaxRhs,
                                       hipMemcpyHostToDevice, st));
        GRG_TRY_HIP(launch_coarse_combine_apply(prec, g, xb, S->d_q, S->d_bidx, S->nb, L->U[GRG_FP64],
                                                4.0 + S->m0, c, yb, nrhs, st));
        if (npool > 0) GRG_TRY_HIP(hipStreamSynchronize(st));  // h_fk is reused next
        *fused = true;
    } else {
        // x64 = sum of the corrections, or u_minus minus it
        GRG_TRY(combine(u_minus, u_minus ? -1.0 : 1.0));
    }
    if (stats) {
        stats->fallbacks = S->fallbacks;
        stats->iters = total;
        stats->outer = outer;
        stats->converged = status == GRG_OK;
        stats->true_rel_resid = worst;
    }
    return status;
}

// out = D_{rows, cols} in on canonical lattice fields, in precision prec, with
// the handle's launch for (prec, nrhs).  rows / cols: 1 coarse sites, 0 the
// rest, -1 every site.
grg_status block_apply_internal(grg_schur S, int prec, int rows, int cols, const double *in,
                                double *out, int nrhs)
{
    grg_lattice L = S->lat;
    GRG_TRY(ensure_inner(S, prec));
    void *a = S->in_b[prec], *b = S->in_q[prec];
    GRG_TRY_HIP(launch_pack_spinor(prec, in, a, L->g, nrhs, L->stream, cols < 0 ? nullptr : S->d_mask,
                                   cols));
    GRG_TRY(run_dslash(S, prec, a, b, rows, nrhs, nullptr));
    GRG_TRY_HIP(launch_unpack_spinor(prec, b, out, L->g, nrhs, L->stream));
    return GRG_OK;
}

// out = (d - H_pq H_qp / d) in on the rest sites of parity p (canonical
// fields, device)
grg_status reduced_apply_internal(grg_schur S, int prec, int parity, const double *in, double *out,
                                  int nrhs)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    GRG_TRY(ensure_inner(S, prec));
    GRG_TRY(ensure_eo(S, prec));
    const Geom gh = half_geom(L);
    const DslashTune t = S->eotune[prec][nrhs].valid ? S->eotune[prec][nrhs]
                                                     : default_eo_tune(gh, prec, nrhs);
    const double d = 4.0 + S->m0;
    void **f = S->eo_f[prec];
    void *a = S->in_b[prec], *b = S->in_q[prec];
    GRG_TRY_HIP(launch_pack_spinor(prec, in, a, L->g, nrhs, st, S->d_mask, 0));
    GRG_TRY_HIP(launch_eo_scatter(prec, L->g, nrhs, parity, a, f[0], false, st));
    GRG_TRY(eo_hop(S, prec, t, f[0], nullptr, f[3], 1 - parity, 0.0, 1.0, nrhs, nullptr, nullptr));
    GRG_TRY(eo_hop(S, prec, t, f[3], f[0], f[2], parity, d, -1.0 / d, nrhs, nullptr, nullptr));
    GRG_TRY_HIP(launch_eo_scatter(prec, L->g, nrhs, parity, f[2], b, true, st));
    GRG_TRY_HIP(launch_unpack_spinor(prec, b, out, L->g, nrhs, st));
    return GRG_OK;
}

// x_b (canonical coarse, device) -> y_b
grg_status schur_apply_internal(grg_schur S, const double *xb, double *yb, int nrhs,
                                grg_solver_stats *stats)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    // b = (D u)_r = D_rb x_b (u = x_b on the coarse sites), from the coarse
    // vector's hops only; for a mixed-precision reduced solve also straight
    // into its compact right-hand side
    const grg_solver_params &p = S->prm;
    const bool pair = p.inner != GRG_FP64 && p.eo && L->eo_ok && 4.0 + S->m0 != 0.0 &&
                      std::max(1, p.restart) == 1 && !S->precond && p.method == 0;
    if (pair) {
        GRG_TRY(ensure_inner(S, p.inner));
        GRG_TRY(ensure_eo_rhs(S, p.inner));
    }
    GRG_TRY_HIP(launch_rb_apply(g, xb, S->d_bidx, S->nb, L->U[GRG_FP64], S->b64, nrhs, st, S->partials,
                                pair ? p.inner : -1, pair ? S->eo_b[p.inner] : nullptr,
                                pair ? eo_half_bytes(S, p.inner) / prec_bytes(p.inner) : 0, S->eo_par));
    // z = D_rr^{-1} b (|b|^2 from rb_apply's sums), and y_b = [D (u - z)]_b
    // fused into its last step, or x64 = u - z (u scattered into u64 when needed)
    bool fused = false;
    grg_status s = drr_solve_internal(S, nrhs, stats, S->u64, xb, yb, &fused, rb_apply_grid(g), pair);
    if (s != GRG_OK && s != GRG_ENOCONV) return s;
    if (fused) return s;
    // y_b = [D (u - z)]_b
    CoarseArgs c;
    c.in = S->x64;
    c.out = yb;
    c.U = L->U[GRG_FP64];
    c.q = S->d_q;
    c.nb = S->nb;
    c.diag = 4.0 + S->m0;
    c.g = g;
    c.nrhs = nrhs;
    GRG_TRY_HIP(launch_dslash_coarse(c, st));
    return s;
}

}  // namespace grg

namespace grg {

// y_b = S~_bb x_b, the second-order Schur complement approximation of
// section 3, in FP64 without any solve:
//     u = x_b on the coarse sites;  y = D_rb u;  d~ = D_rr 1 (row sums);
//     t = y / d~;  z = D_rr t;  w = u - ((y - z) / d + t);  y_b = (D w)_b,
// with d = 4 + m0 the diagonal of D_rr.  Three stencil launches on nrhs
// fields and one on a single field (d~, recomputed per call since the links
// may have been reset).
// D_bb x_b - D_br (D_rb x_b) / d: the Schur complement with the couplings
// inside D_rr ignored (D_rr^{-1} -> 1 / d, d = 4 + m0 its diagonal), which
// keeps the coarse operator's sparsity; two stencil launches, no solve.
grg_status diag_schur_apply_internal(grg_schur S, const double *xb, double *yb, int nrhs)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    const BlasShape sh = blas_shape(g, nrhs);
    GRG_TRY_HIP(launch_scatter_coarse(xb, S->u64, S->d_bidx, S->nb, g, nrhs, st));
    GRG_TRY_HIP(launch_rb_apply(g, xb, S->d_bidx, S->nb, L->U[GRG_FP64], S->b64, nrhs, st));
    GRG_TRY_HIP(launch_reusken_combine(sh, S->u64, S->b64, nullptr, nullptr, S->d_mask,
                                       1.0 / (4.0 + S->m0), S->x64, st));
    CoarseArgs c;
    c.in = S->x64;
    c.out = yb;
    c.U = L->U[GRG_FP64];
    c.q = S->d_q;
    c.nb = S->nb;
    c.diag = 4.0 + S->m0;
    c.g = g;
    c.nrhs = nrhs;
    GRG_TRY_HIP(launch_dslash_coarse(c, st));
    return GRG_OK;
}

grg_status reusken_apply_internal(grg_schur S, const double *xb, double *yb, int nrhs)
{
    grg_lattice L = S->lat;
    hipStream_t st = L->stream;
    const Geom &g = L->g;
    const BlasShape sh = blas_shape(g, nrhs);
    if (!S->dt64 && hipMalloc(&S->dt64, spinor_elems(g, 1) * 16) != hipSuccess) {
        S->dt64 = nullptr;
        set_error("row-sum field: hipMalloc failed");
        return GRG_ENOMEM;
    }
    if (S->dt_version != L->gauge_version) {
        // d~ = D_rr 1 (the row sums), once per gauge field
        GRG_TRY_HIP(launch_rest_ones(g, S->d_mask, S->t64, st));
        GRG_TRY(run_dslash(S, GRG_FP64, S->t64, S->dt64, 0, 1, nullptr));
        S->dt_version = L->gauge_version;
    }
    GRG_TRY_HIP(launch_scatter_coarse(xb, S->u64, S->d_bidx, S->nb, g, nrhs, st));
    GRG_TRY_HIP(launch_rb_apply(g, xb, S->d_bidx, S->nb, L->U[GRG_FP64], S->b64, nrhs, st));
    GRG_TRY_HIP(launch_reusken_divide(sh, S->b64, S->dt64, S->d_mask, S->t64, st));
    GRG_TRY(run_dslash(S, GRG_FP64, S->t64, S->r64, 0, nrhs, nullptr));
    GRG_TRY_HIP(launch_reusken_combine(sh, S->u64, S->b64, S->r64, S->t64, S->d_mask,
                                       1.0 / (4.0 + S->m0), S->x64, st));
    CoarseArgs c;
    c.in = S->x64;
    c.out = yb;
    c.U = L->U[GRG_FP64];
    c.q = S->d_q;
    c.nb = S->nb;
    c.diag = 4.0 + S->m0;
    c.g = g;
    c.nrhs = nrhs;
    GRG_TRY_HIP(launch_dslash_coarse(c, st));
    return GRG_OK;
}

}  // namespace grg
