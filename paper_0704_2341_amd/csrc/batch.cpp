// Many independent lattices solved together: S_bb applies for every lattice
// of the batch in the same launches (kernels_batch.hip), the inner iterations
// replayed from a HIP graph.
//
// The method is the single-lattice one (solver.cpp) applied to every
// (lattice, right-hand side) system at once: FP64 defect correction around an
// inner minimal-residual solve in the inner precision, per-system step
// lengths and per-system convergence flags that freeze converged systems
// inside the captured iterations, so the host reads the norms only between
// graph replays.
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
    double *partials = nullptr;
    double2 *alpha = nullptr;
    double *rn2 = nullptr, *thr2 = nullptr, *bn2 = nullptr, *fr2 = nullptr;
    int *active = nullptr;
    double *h_buf = nullptr;       // pinned, 4 * nsys
    int SB[3] = {64, 64, 64}, RG[3] = {1, 1, 1}, grid[3] = {0, 0, 0};
    hipGraphExec_t graph = nullptr;
    int graph_iters = 0;
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
    return a;
}

static grg_status dslash(grg_batch B, int prec, const void *in, void *out, int sel, bool dots)
{
    BatchDslashArgs a;
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

static grg_status read_rn2(grg_batch B, double *host)
{
    GRG_TRY_HIP(hipMemcpyAsync(B->h_buf, B->rn2, sizeof(double) * B->nsys, hipMemcpyDeviceToHost, B->st));
    GRG_TRY_HIP(hipStreamSynchronize(B->st));
    memcpy(host, B->h_buf, sizeof(double) * B->nsys);
    return GRG_OK;
}

// one inner minimal-residual iteration for every system (graph body)
static grg_status inner_step(grg_batch B, int prec)
{
    const BatchBlasArgs a = blas(B);
    GRG_TRY(dslash(B, prec, B->in_r, B->in_q, 0, true));
    GRG_TRY_HIP(launch_reduce(kAlpha, B->partials, dgrid(B, prec), B->nsys, B->alpha, nullptr, nullptr,
                              B->active, B->st));
    GRG_TRY_HIP(launch_batch_mr_update(prec, a, B->in_x, B->in_r, B->in_q, B->st));
    GRG_TRY_HIP(launch_reduce(kNorm, B->partials, a.grid, B->nsys, nullptr, B->rn2, B->thr2, B->active,
                              B->st));
    return GRG_OK;
}

static grg_status build_graph(grg_batch B, int prec, int iters)
{
    if (B->graph && B->graph_iters == iters) return GRG_OK;
    if (B->graph) {
        (void)hipGraphExecDestroy(B->graph);
        B->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    GRG_TRY_HIP(hipStreamBeginCapture(B->st, hipStreamCaptureModeThreadLocal));
    grg_status s = GRG_OK;
    for (int k = 0; k < iters && s == GRG_OK; ++k) s = inner_step(B, prec);
    hipError_t e = hipStreamEndCapture(B->st, &g);
    if (s != GRG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    GRG_TRY_HIP(e);
    e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    GRG_TRY_HIP(e);
    B->graph_iters = iters;
    return GRG_OK;
}

// inner solve of in_b -> in_x to |r|^2 <= thr (host copy) per system
static grg_status inner_solve(grg_batch B, int prec, const double *thr, int maxit, bool use_graph,
                              int *iters)
{
    const BatchBlasArgs a = blas(B);
    const size_t bytes = spinor_elems(B->gtot, B->nrhs) * prec_bytes(prec);
    BlasShape sh;
    sh.g = B->gtot;
    sh.nrhs = B->nrhs;
    sh.grid = a.grid;
    GRG_TRY_HIP(launch_fill_zero(B->in_x, bytes, B->st));
    GRG_TRY_HIP(launch_copy(prec, sh, B->in_b, B->in_r, B->st));
    GRG_TRY_HIP(launch_batch_norm2(prec, a, B->in_r, B->st));
    GRG_TRY_HIP(launch_reduce(kNorm, B->partials, a.grid, B->nsys, nullptr, B->rn2, B->thr2, B->active,
                              B->st));
    std::vector<double> h(B->nsys);
    GRG_TRY(read_rn2(B, h.data()));
    auto done = [&]() {
        for (int k = 0; k < B->nsys; ++k) {
            if (!isfinite(h[k])) return -1;
            if (h[k] > thr[k]) return 0;
        }
        return 1;
    };
    const int chunk = std::max(1, B->prm.check_every);
    int it = 0, d = done();
    if (use_graph) GRG_TRY(build_graph(B, prec, chunk));
    while (d == 0 && it < maxit) {
        if (use_graph) {
            GRG_TRY_HIP(hipGraphLaunch(B->graph, B->st));
        } else {
            for (int k = 0; k < chunk; ++k) GRG_TRY(inner_step(B, prec));
        }
        it += chunk;
        GRG_TRY(read_rn2(B, h.data()));
        d = done();
    }
    *iters = it;
    if (d < 0) return set_error("non-finite residual in the batched inner solve"), GRG_ENONFINITE;
    return GRG_OK;
}

static grg_status batch_apply(grg_batch B, const double *xb, double *yb, bool use_graph,
                              grg_solver_stats *stats)
{
    const grg_solver_params &p = B->prm;
    const int prec = p.inner;
    const int n = B->nsys;
    const BatchBlasArgs a = blas(B);
    hipStream_t st = B->st;
    GRG_TRY_HIP(launch_batch_scatter(table(B), xb, B->u64, B->bidx, B->nb, B->coff, B->Vtot, B->nrhs, st));
    GRG_TRY(dslash(B, GRG_FP64, B->u64, B->b64, 0, false));  // b = D_rb x
    GRG_TRY_HIP(launch_batch_norm2(GRG_FP64, a, B->b64, st));
    GRG_TRY_HIP(launch_reduce(kNorm, B->partials, a.grid, n, nullptr, B->bn2, nullptr, nullptr, st));
    std::vector<double> bn2(n), rn2(n), thr(n);
    GRG_TRY_HIP(hipMemcpyAsync(B->h_buf, B->bn2, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    GRG_TRY_HIP(hipStreamSynchronize(st));
    memcpy(bn2.data(), B->h_buf, sizeof(double) * n);
    rn2 = bn2;
    const void *r_src = B->b64, *x_src = nullptr;
    int total = 0, outer = 0;
    bool verified = false;
    double worst = 0;
    grg_status status = GRG_OK;
    const int dcg = round8(std::min<long>(B->Vtot / 128, kBatchMaxGrid));
    for (;;) {
        bool conv = true;
        worst = 0;
        for (int k = 0; k < n; ++k) {
            if (!isfinite(rn2[k])) return set_error("non-finite FP64 residual"), GRG_ENONFINITE;
            const double rel = bn2[k] > 0 ? sqrt(rn2[k] / bn2[k]) : 0.0;
            worst = std::max(worst, rel);
            if (rel > p.tol) conv = false;
        }
        if (conv && (verified || x_src == nullptr)) break;
        if (conv) {
            GRG_TRY(dslash(B, GRG_FP64, B->x64, B->t64, 0, false));
            GRG_TRY_HIP(launch_batch_sub_norm(a, B->b64, B->t64, B->r64, st));
            GRG_TRY_HIP(launch_reduce(kNorm, B->partials, a.grid, n, nullptr, B->rn2, nullptr, nullptr, st));
            GRG_TRY(read_rn2(B, rn2.data()));
            r_src = B->r64;
            verified = true;
            continue;
        }
        verified = false;
        if (outer >= p.max_outer || total >= p.max_iter) {
            status = GRG_ENOCONV;
            set_error("batched D_rr solve: no convergence after %d outer / %d inner iterations "
                      "(residual %.3e > %.3e)", outer, total, worst, p.tol);
            break;
        }
        for (int k = 0; k < n; ++k) {
            const double need = bn2[k] > 0 && rn2[k] > 0 ? p.tol * sqrt(bn2[k] / rn2[k]) : 1.0;
            const double rel = prec == GRG_FP64 ? need : std::max(p.inner_tol, 0.5 * need);
            const bool on = bn2[k] > 0 && sqrt(rn2[k] / bn2[k]) > p.tol;
            thr[k] = on ? rel * rel : 2.0;
        }
        memcpy(B->h_buf + n, thr.data(), sizeof(double) * n);
        GRG_TRY_HIP(hipMemcpyAsync(B->thr2, B->h_buf + n, sizeof(double) * n, hipMemcpyHostToDevice, st));
        memcpy(B->h_buf + 2 * n, rn2.data(), sizeof(double) * n);
        GRG_TRY_HIP(hipMemcpyAsync(B->fr2, B->h_buf + 2 * n, sizeof(double) * n, hipMemcpyHostToDevice, st));
        GRG_TRY_HIP(launch_batch_axpy_convert(GRG_FP64, prec, a, r_src, B->in_b, B->fr2, 1, 0, st));
        int it = 0;
        GRG_TRY(inner_solve(B, prec, thr.data(), p.max_iter - total, use_graph, &it));
        total += it;
        ++outer;
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
        GRG_TRY_HIP(launch_batch_dc_update(prec, d, dcg, st));
        GRG_TRY_HIP(launch_reduce(kNorm, B->partials, dcg, n, nullptr, B->rn2, nullptr, nullptr, st));
        GRG_TRY(read_rn2(B, rn2.data()));
        r_src = B->r64;
        x_src = B->x64;
    }
    if (x_src == nullptr)
        GRG_TRY_HIP(launch_fill_zero(B->x64, spinor_elems(B->gtot, B->nrhs) * 16, st));
    // S x = [D (u - z)]_b
    BlasShape sh;
    sh.g = B->gtot;
    sh.nrhs = B->nrhs;
    sh.grid = a.grid;
    GRG_TRY_HIP(launch_xmy(sh, B->u64, B->x64, st));
    GRG_TRY_HIP(launch_batch_coarse(table(B), B->x64, B->U[GRG_FP64], yb, B->qg, B->clat, B->nb,
                                    B->nboff, B->coff, B->nbtot, B->nrhs, st));
    if (stats) {
        stats->iters = total;
        stats->outer = outer;
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
    f(B->partials);
    f(B->alpha);
    f(B->rn2);
    f(B->thr2);
    f(B->bn2);
    f(B->fr2);
    f(B->active);
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
    al((void **)&B->partials, sizeof(double) * kBatchMaxGrid * B->nsys * 3);
    al((void **)&B->alpha, sizeof(double2) * B->nsys);
    for (double **p : {&B->rn2, &B->thr2, &B->fr2}) al((void **)p, sizeof(double) * B->nsys);
    al((void **)&B->bn2, sizeof(double) * B->nsys);
    al((void **)&B->active, sizeof(int) * B->nsys);
    if (ok && hipHostMalloc((void **)&B->h_buf, sizeof(double) * 4 * B->nsys) != hipSuccess) {
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
    GRG_TRY_HIP(hipStreamSynchronize(st));
#undef UP
    for (void *p : {B->b64, B->x64, B->r64, B->t64, B->u64}) GRG_TRY_HIP(launch_fill_zero(p, f64, st));
    for (void *p : {B->in_b, B->in_x, B->in_r, B->in_q}) GRG_TRY_HIP(launch_fill_zero(p, fin, st));
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
