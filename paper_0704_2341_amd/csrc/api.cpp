// C ABI of the library: argument validation, handles, workspaces and the
// host-side permutation builder.  All compute is enqueued on the lattice
// stream by the engine (solver.cpp) and the kernels (kernels_*.hip).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <numeric>
#include <vector>

#include "handles.h"

namespace grg {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

grg_status drr_solve_internal(grg_schur S, int nrhs, grg_solver_stats *stats,
                              const void *u_minus = nullptr, const double *xb = nullptr, double *yb = nullptr,
                              bool *fused = nullptr, int bn2_parts = 0, bool rhs_pair = false);
grg_status schur_apply_internal(grg_schur S, const double *xb, double *yb, int nrhs,
                                grg_solver_stats *stats);
grg_status run_dslash(grg_schur S, int prec, const void *in, void *out, int sel, int nrhs,
                      double *partials, const void *dot_with = nullptr);
int partial_rows(const Geom &g, int nrhs);
int dslash_grid(const Geom &g, int nrhs, int SB, int RG);
DslashTune default_tune(const Geom &g, int prec, int nrhs);
bool launch_ok(const Geom &g, int prec, int nrhs, const DslashTune &t, bool dots);
grg_status block_apply_internal(grg_schur S, int prec, int rows, int cols, const double *in,
                                double *out, int nrhs);
grg_status reduced_apply_internal(grg_schur S, int prec, int parity, const double *in, double *out,
                                  int nrhs);
grg_status tune_dslash(grg_schur S, int prec, int nrhs, int reps);
grg_status reusken_apply_internal(grg_schur S, const double *xb, double *yb, int nrhs);
grg_status diag_schur_apply_internal(grg_schur S, const double *xb, double *yb, int nrhs);
grg_status tune_dc(grg_schur S, int prec, int nrhs, int reps);
grg_status tune_eo(grg_schur S, int prec, int nrhs, int reps);
DslashTune default_eo_tune(const Geom &gh, int prec, int nrhs);
DslashTune default_dc_tune(const Geom &g);
bool dc_launch_ok(const Geom &g, int prec, int nrhs, const DslashTune &t);
bool eo_launch_ok(const Geom &gh, int prec, int nrhs, const DslashTune &t);

static grg_status dmalloc(void **p, size_t bytes, const char *what)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        set_error("%s: hipMalloc of %zu bytes failed: %s", what, bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? GRG_ENOMEM : GRG_EHIP;
    }
    return GRG_OK;
}

static void dfree(void *&p)
{
    if (p) hipFree(p);
    p = nullptr;
}

static grg_status validate_params(const grg_solver_params &p)
{
    if (!(p.tol > 0) || !(p.tol < 1)) return set_error("tol must be in (0, 1)"), GRG_EINVAL;
    if (p.max_iter < 1) return set_error("max_iter must be >= 1"), GRG_EINVAL;
    if (p.restart < 1 || p.restart > kMaxRhs)
        return set_error("restart must be in 1..%d", kMaxRhs), GRG_EINVAL;
    if (p.inner < GRG_FP64 || p.inner > GRG_BF16) return set_error("bad inner precision"), GRG_EINVAL;
    if (p.inner != GRG_FP64 && !(p.inner_tol > 0 && p.inner_tol < 1))
        return set_error("inner_tol must be in (0, 1)"), GRG_EINVAL;
    if (p.max_outer < 1) return set_error("max_outer must be >= 1"), GRG_EINVAL;
    if (p.max_rhs < 1 || p.max_rhs > kMaxRhs)
        return set_error("max_rhs must be in 1..%d", kMaxRhs), GRG_EINVAL;
    if (p.check_every < 1) return set_error("check_every must be >= 1"), GRG_EINVAL;
    if (p.verify != 0 && p.verify != 1) return set_error("verify must be 0 or 1"), GRG_EINVAL;
    if (p.eo != 0 && p.eo != 1) return set_error("eo must be 0 or 1"), GRG_EINVAL;
    if (p.method != 0 && p.method != 1) return set_error("method must be 0 (GCR) or 1 (BiCGstab)"), GRG_EINVAL;
    return GRG_OK;
}

// Scoped switch to the handle's device.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

// ------------------------------------------------------------------ permutation
// Ordering vector of section 2: coarse sites first.  Type I: all-even sites
// (blocking in every direction at once).  Type II: nested red-black blocking
// one direction at a time, x first -- a site's group is the first direction
// with an odd coordinate; the all-even group leads and the x-odd group is last.
// Inside a group the order is lexicographic.  The inverse ordering is q^{-1}.
static void build_permutation(const int32_t dims[4], int type, int inverse, int32_t *q)
{
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    std::vector<int> key(V);
    for (int64_t s = 0; s < V; ++s) {
        int64_t r = s;
        int c[4];
        for (int mu = 0; mu < 4; ++mu) {
            c[mu] = (int)(r % dims[mu]);
            r /= dims[mu];
        }
        if (type == GRG_PERM_I) {
            key[s] = (c[0] | c[1] | c[2] | c[3]) & 1;  // 0 = all even
        } else {
            int first_odd = 4;
            for (int mu = 3; mu >= 0; --mu)
                if (c[mu] & 1) first_odd = mu;
            key[s] = 4 - first_odd;  // all-even -> 0, x-odd -> 4
        }
    }
    std::vector<int32_t> order(V);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    if (!inverse) {
        std::copy(order.begin(), order.end(), q);
    } else {
        for (int64_t k = 0; k < V; ++k) q[order[k]] = (int32_t)k;
    }
}

}  // namespace grg

using namespace grg;

extern "C" {

const char *grg_last_error(void) { return g_err; }

const char *grg_version(void) { return "grg 0.1 (gfx950)"; }

grg_status grg_solver_params_default(grg_solver_params *p)
{
    if (!p) return set_error("null params"), GRG_EINVAL;
    p->tol = 1e-10;
    p->max_iter = 2000;
    p->restart = 1;
    p->inner = GRG_FP64;
    p->inner_tol = 1e-5;
    p->max_outer = 30;
    p->max_rhs = 12;
    p->check_every = 1;
    p->verify = 0;
    p->eo = 1;
    p->method = 0;
    return GRG_OK;
}

grg_status grg_lattice_create(const int32_t dims[4], const int32_t bc[4], void *stream,
                              grg_lattice *out)
{
    if (!dims || !bc || !out) return set_error("null argument"), GRG_EINVAL;
    *out = nullptr;
    int64_t V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 1) return set_error("dims[%d] = %d must be positive", mu, dims[mu]), GRG_EINVAL;
        if (bc[mu] != 1 && bc[mu] != -1) return set_error("bc[%d] must be +1 or -1", mu), GRG_EINVAL;
        V *= dims[mu];
    }
    if (V > (int64_t)1 << 28) return set_error("volume %lld too large", (long long)V), GRG_ETOO_LARGE;
    grg_lattice L = new (std::nothrow) grg_lattice_s();
    if (!L) return set_error("out of host memory"), GRG_ENOMEM;
    for (int mu = 0; mu < 4; ++mu) {
        L->g.L[mu] = dims[mu];
        L->bc[mu] = bc[mu];
    }
    L->g.V = (int)V;
    L->g.Vs = (int)((V + 255) / 256 * 256);
    L->stream = (hipStream_t)stream;
    if (hipGetDevice(&L->device) != hipSuccess) {
        delete L;
        return set_error("no HIP device available"), GRG_EHIP;
    }
    const size_t ge = gauge_elems(L->g);
    grg_status s = GRG_OK;
    for (int p = 0; p < 3 && s == GRG_OK; ++p) s = dmalloc(&L->U[p], ge * prec_bytes(p), "links");
    L->eo_ok = dims[0] % 2 == 0 && dims[1] % 2 == 0 && dims[2] % 2 == 0 && dims[3] % 2 == 0;
    if (L->eo_ok) {
        L->Vhs = (int)((V / 2 + 255) / 256 * 256);
        for (int p = 0; p < 3 && s == GRG_OK; ++p)
            s = dmalloc(&L->Ueo[p], (size_t)2 * 36 * L->Vhs * prec_bytes(p), "even-odd links");
    }
    if (s != GRG_OK) {
        grg_lattice_destroy(L);
        return s;
    }
    *out = L;
    return GRG_OK;
}

grg_status grg_lattice_destroy(grg_lattice L)
{
    if (!L) return GRG_OK;
    DeviceGuard dg(L->device);
    hipStreamSynchronize(L->stream);
    for (int p = 0; p < 3; ++p) dfree(L->U[p]);
    for (int p = 0; p < 3; ++p) dfree(L->Ueo[p]);
    dfree(L->tmp_in);
    dfree(L->tmp_out);
    void *tl = L->tmp_links;
    dfree(tl);
    delete L;
    return GRG_OK;
}

grg_status grg_lattice_volume(grg_lattice L, int64_t *v)
{
    if (!L || !v) return set_error("null argument"), GRG_EINVAL;
    *v = L->g.V;
    return GRG_OK;
}

grg_status grg_gauge_set(grg_lattice L, const double *links, int on_device)
{
    if (!L || !links) return set_error("null argument"), GRG_EINVAL;
    DeviceGuard dg(L->device);
    const size_t bytes = (size_t)L->g.V * 4 * 9 * 16;
    const double *src = links;
    if (!on_device) {
        if (!L->tmp_links) {
            void *p;
            GRG_TRY(dmalloc(&p, bytes, "link staging"));
            L->tmp_links = (double *)p;
        }
        GRG_TRY_HIP(hipMemcpyAsync(L->tmp_links, links, bytes, hipMemcpyHostToDevice, L->stream));
        src = L->tmp_links;
    }
    GRG_TRY_HIP(launch_pack_gauge(src, L->g, L->bc, L->U[GRG_FP64], L->U[GRG_FP32],
                                  L->U[GRG_BF16], L->stream));
    if (L->eo_ok)
        for (int p = 0; p < 3; ++p)
            GRG_TRY_HIP(launch_eo_pack_links(p, L->g, L->Vhs, L->U[p], L->Ueo[p], L->stream));
    GRG_TRY_HIP(hipStreamSynchronize(L->stream));
    if (L->tmp_links) {
        void *tl = L->tmp_links;
        dfree(tl);
        L->tmp_links = nullptr;
    }
    L->gauge_set = true;
    ++L->gauge_version;
    return GRG_OK;
}

grg_status grg_permutation_block(const int32_t dims[4], int type, int inverse, int32_t *q,
                                 int32_t *n_coarse)
{
    if (!dims || !q || !n_coarse) return set_error("null argument"), GRG_EINVAL;
    if (type != GRG_PERM_I && type != GRG_PERM_II) return set_error("type must be 1 or 2"), GRG_EINVAL;
    int64_t V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 2) return set_error("dims must be >= 2"), GRG_EINVAL;
        if (dims[mu] % 2) return set_error("dims[%d] = %d is odd", mu, dims[mu]), GRG_EODD_EXTENT;
        V *= dims[mu];
    }
    if (V > (int64_t)1 << 28) return set_error("volume too large"), GRG_ETOO_LARGE;
    build_permutation(dims, type, inverse, q);
    *n_coarse = (int32_t)(V / 16);
    return GRG_OK;
}

grg_status grg_dirac_apply(grg_lattice L, double m0, int precision, const double *in, double *out,
                           int nrhs)
{
    if (!L || !in || !out) return set_error("null argument"), GRG_EINVAL;
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error("nrhs must be in 1..%d", kMaxRhs), GRG_EINVAL;
    if (precision < GRG_FP64 || precision > GRG_BF16) return set_error("bad precision"), GRG_EINVAL;
    if (!L->gauge_set) return set_error("gauge field not set"), GRG_EINVAL;
    if (!isfinite(m0)) return set_error("m0 not finite"), GRG_EINVAL;
    DeviceGuard dg(L->device);
    const size_t bytes = spinor_elems(L->g, nrhs) * prec_bytes(precision);
    if (bytes > L->tmp_bytes) {
        dfree(L->tmp_in);
        dfree(L->tmp_out);
        L->tmp_bytes = 0;
        GRG_TRY(dmalloc(&L->tmp_in, bytes, "dirac_apply scratch"));
        GRG_TRY(dmalloc(&L->tmp_out, bytes, "dirac_apply scratch"));
        L->tmp_bytes = bytes;
    }
    GRG_TRY_HIP(launch_pack_spinor(precision, in, L->tmp_in, L->g, nrhs, L->stream));
    DslashArgs a;
    a.in = L->tmp_in;
    a.out = L->tmp_out;
    a.U = L->U[precision];
    a.mask = nullptr;
    a.sel = 0;
    a.diag = 4.0 + m0;
    a.g = L->g;
    a.nrhs = nrhs;
    const DslashTune t = default_tune(L->g, precision, nrhs);
    a.SB = t.SB;
    a.RG = t.RG;
    a.split = t.split;
    a.chunk = t.chunk;
    a.march = t.march;
    a.partials = nullptr;
    a.dot_with = nullptr;
    GRG_TRY_HIP(launch_dslash(precision, a, t.grid, L->stream));
    GRG_TRY_HIP(launch_unpack_spinor(precision, L->tmp_out, out, L->g, nrhs, L->stream));
    GRG_TRY_HIP(hipStreamSynchronize(L->stream));
    return GRG_OK;
}

// ------------------------------------------------------------------ no-alloc D apply
// The staging fields of grg_dirac_apply_noalloc live in this fixed array, one
// copy per GPU, held until the process ends.  In host code `scratch` is only
// the shadow of the device symbol; its device address is taken once per
// device with hipGetSymbolAddress and only that address is passed on.
static __device__ __align__(256) unsigned char scratch[GRG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// the device address of this device's scratch (the device current)
grg_status scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return set_error("device %d out of range", dev), GRG_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e)), GRG_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GRG_OK;
}
}  // namespace

grg_status grg_dirac_apply_noalloc(grg_lattice L, double m0, int precision, const double *in, double *out,
                                   int nrhs)
{
    if (!L || !in || !out) return set_error("null argument"), GRG_EINVAL;
    if (nrhs < 1 || nrhs > kMaxRhs) return set_error("nrhs must be in 1..%d", kMaxRhs), GRG_EINVAL;
    if (precision < GRG_FP64 || precision > GRG_BF16) return set_error("bad precision"), GRG_EINVAL;
    if (!L->gauge_set) return set_error("gauge field not set"), GRG_EINVAL;
    if (!isfinite(m0)) return set_error("m0 not finite"), GRG_EINVAL;
    // two fields, each starting on a 256-byte boundary
    const size_t bytes = (spinor_elems(L->g, nrhs) * prec_bytes(precision) + 255) & ~(size_t)255;
    if (2 * bytes > (size_t)GRG_NOALLOC_SCRATCH_BYTES)
        return set_error("dirac_apply_noalloc: %zu bytes of staging for %d RHS exceed the %u-byte scratch",
                         2 * bytes, nrhs, (unsigned)GRG_NOALLOC_SCRATCH_BYTES),
               GRG_ETOO_LARGE;
    DeviceGuard dg(L->device);
    void *base = nullptr;
    GRG_TRY(scratch_address(L->device, &base));
    void *sin = base, *sout = (char *)base + bytes;
    // every entry the stencil reads (sites < V of every RHS) is written by the
    // pack first, so nothing left by an earlier call is read
    GRG_TRY_HIP(launch_pack_spinor(precision, in, sin, L->g, nrhs, L->stream));
    DslashArgs a;
    a.in = sin;
    a.out = sout;
    a.U = L->U[precision];
    a.mask = nullptr;
    a.sel = 0;
    a.diag = 4.0 + m0;
    a.g = L->g;
    a.nrhs = nrhs;
    const DslashTune t = default_tune(L->g, precision, nrhs);
    a.SB = t.SB;
    a.RG = t.RG;
    a.split = t.split;
    a.chunk = t.chunk;
    a.march = t.march;
    a.partials = nullptr;
    a.dot_with = nullptr;
    GRG_TRY_HIP(launch_dslash(precision, a, t.grid, L->stream));
    GRG_TRY_HIP(launch_unpack_spinor(precision, sout, out, L->g, nrhs, L->stream));
    GRG_TRY_HIP(hipStreamSynchronize(L->stream));
    return GRG_OK;
}

static void schur_free(grg_schur S)
{
    dfree((void *&)S->d_mask);
    dfree((void *&)S->d_q);
    dfree((void *&)S->d_bidx);
    void **f64[5] = {&S->b64, &S->x64, &S->r64, &S->t64, &S->u64};
    for (void **p : f64) dfree(*p);
    dfree(S->r32);
    for (int p = 0; p < 3; ++p) {
        dfree(S->in_b[p]);
        dfree(S->in_x[p]);
        dfree(S->in_r[p]);
        dfree(S->in_q[p]);
        dfree(S->in_P[p]);
        dfree(S->in_Q[p]);
    }
    dfree((void *&)S->cb_in);
    dfree((void *&)S->cb_out);
    dfree(S->dt64);
    dfree((void *&)S->d_mask_eo);
    dfree((void *&)S->d_mask_par);
    for (int p = 0; p < 3; ++p) {
        for (void *&b : S->epool[p]) dfree(b);
        S->epool[p].clear();
    }
    dfree((void *&)S->d_fk);
    if (S->h_fk) hipHostFree(S->h_fk);
    S->h_fk = nullptr;
    for (int p = 0; p < 3; ++p) {
        for (int k = 0; k < 5; ++k) dfree(S->eo_f[p][k]);
        dfree(S->eo_b[p]);
        for (int k = 0; k < 5; ++k) dfree(S->bicg_f[p][k]);
    }
    dfree((void *&)S->partials);
    dfree((void *&)S->alpha);
    dfree((void *&)S->bicg_sc);
    dfree((void *&)S->beta);
    dfree((void *&)S->rn2);
    S->thr2 = nullptr;  // inside bn2
    dfree((void *&)S->qn2);
    dfree((void *&)S->bn2);
    dfree((void *&)S->active);
    dfree((void *&)S->act0);
    if (S->h_buf) hipHostFree(S->h_buf);
    S->h_buf = nullptr;
    for (auto e : S->prof.start) hipEventDestroy(e);
    for (auto e : S->prof.stop) hipEventDestroy(e);
    S->prof.start.clear();
    S->prof.stop.clear();
}

grg_status grg_schur_create(grg_lattice L, double m0, const int32_t *q, int32_t n_coarse,
                            const grg_solver_params *params, grg_schur *out)
{
    if (!L || !q || !out) return set_error("null argument"), GRG_EINVAL;
    *out = nullptr;
    if (!L->gauge_set) return set_error("gauge field not set"), GRG_EINVAL;
    if (!isfinite(m0)) return set_error("m0 not finite"), GRG_EINVAL;
    const int V = L->g.V;
    if (n_coarse < 1 || n_coarse >= V) return set_error("n_coarse must be in 1..V-1"), GRG_EINVAL;
    grg_solver_params prm;
    if (params) prm = *params;
    else grg_solver_params_default(&prm);
    GRG_TRY(validate_params(prm));
    // q must be a permutation of the sites
    std::vector<int32_t> bidx(V, -1);
    std::vector<uint8_t> seen(V, 0), mask(V, 0);
    for (int k = 0; k < V; ++k) {
        if (q[k] < 0 || q[k] >= V || seen[q[k]])
            return set_error("q is not a permutation of 0..V-1 (entry %d)", k), GRG_EINVAL;
        seen[q[k]] = 1;
    }
    for (int k = 0; k < n_coarse; ++k) {
        bidx[q[k]] = k;
        mask[q[k]] = 1;
    }
    DeviceGuard dg(L->device);
    grg_schur S = new (std::nothrow) grg_schur_s();
    if (!S) return set_error("out of host memory"), GRG_ENOMEM;
    S->lat = L;
    S->m0 = m0;
    S->nb = n_coarse;
    S->prm = prm;
    S->q_host.assign(q, q + V);
    const Geom &g = L->g;
    const size_t f64 = spinor_elems(g, prm.max_rhs) * 16;
    grg_status s = GRG_OK;
#define ALLOC(ptr, bytes) \
    if (s == GRG_OK) s = dmalloc((void **)&(ptr), (bytes), #ptr)
    ALLOC(S->d_mask, V);
    ALLOC(S->d_q, sizeof(int32_t) * n_coarse);
    ALLOC(S->d_bidx, sizeof(int32_t) * V);
    ALLOC(S->b64, f64);
    ALLOC(S->x64, f64);
    ALLOC(S->r64, f64);
    ALLOC(S->t64, f64);
    ALLOC(S->u64, f64);
    S->partials_elems = (size_t)partial_rows(g, prm.max_rhs) * prm.max_rhs * std::max(3, 2 * kMaxRhs);
    ALLOC(S->partials, S->partials_elems * sizeof(double));
    ALLOC(S->alpha, sizeof(double2) * kMaxRhs);
    ALLOC(S->bicg_sc, sizeof(double2) * 4 * kMaxRhs);
    ALLOC(S->beta, sizeof(double2) * kMaxRhs * kMaxRhs);
    ALLOC(S->rn2, sizeof(double) * kMaxRhs);
    ALLOC(S->qn2, sizeof(double) * kMaxRhs * kMaxRhs);
    // |b|^2, then the per-RHS scales f = 1/s, s and the next s, then the
    // inner thresholds (thr2): one block, so the host uploads a step's
    // scalars with one copy
    ALLOC(S->bn2, sizeof(double) * 5 * kMaxRhs);
    if (S->bn2) S->thr2 = S->bn2 + 4 * kMaxRhs;
    ALLOC(S->active, sizeof(int) * kMaxRhs);
    ALLOC(S->act0, sizeof(int) * kMaxRhs);
    if (L->eo_ok) ALLOC(S->d_mask_eo, (size_t)2 * L->Vhs);
    if (L->eo_ok) ALLOC(S->d_mask_par, (size_t)V);
    ALLOC(S->d_fk, sizeof(double) * kCorrPool * kMaxRhs);
#undef ALLOC
    if (s == GRG_OK && hipHostMalloc((void **)&S->h_fk, sizeof(double) * kCorrPool * kMaxRhs) != hipSuccess) {
        S->h_fk = nullptr;
        set_error("hipHostMalloc failed");
        s = GRG_ENOMEM;
    }
    if (s == GRG_OK && hipHostMalloc((void **)&S->h_buf, sizeof(double) * 12 * kMaxRhs) != hipSuccess) {
        S->h_buf = nullptr;
        set_error("hipHostMalloc failed");
        s = GRG_ENOMEM;
    }
    if (s != GRG_OK) {
        schur_free(S);
        delete S;
        return s;
    }
    hipStream_t st = L->stream;
    std::vector<uint8_t> mask_par(L->eo_ok ? (size_t)V : 0);
    GRG_TRY_HIP(hipMemcpyAsync(S->d_mask, mask.data(), V, hipMemcpyHostToDevice, st));
    GRG_TRY_HIP(hipMemcpyAsync(S->d_q, q, sizeof(int32_t) * n_coarse, hipMemcpyHostToDevice, st));
    GRG_TRY_HIP(hipMemcpyAsync(S->d_bidx, bidx.data(), sizeof(int32_t) * V, hipMemcpyHostToDevice, st));
    void *f64s[5] = {S->b64, S->x64, S->r64, S->t64, S->u64};
    for (void *p : f64s) GRG_TRY_HIP(launch_fill_zero(p, f64, st));
    if (L->eo_ok) {
        GRG_TRY_HIP(launch_eo_pack_mask(g, L->Vhs, S->d_mask, S->d_mask_eo, st));
        // the reduced system lives on the parity with fewer rest sites
        long rest[2] = {0, 0};
        for (int x = 0; x < V; ++x) {
            int c = x, par = 0;
            for (int mu = 0; mu < 4; ++mu) {
                par += c % g.L[mu];
                c /= g.L[mu];
            }
            mask_par[x] = (uint8_t)(par & 1);
            if (!mask[x]) ++rest[par & 1];
        }
        S->eo_par = rest[0] < rest[1] ? 0 : 1;
        for (int x = 0; x < V; ++x) mask_par[x] = !mask[x] && mask_par[x] == S->eo_par ? 0 : 1;
        GRG_TRY_HIP(hipMemcpyAsync(S->d_mask_par, mask_par.data(), V, hipMemcpyHostToDevice, st));
    }
    GRG_TRY_HIP(hipStreamSynchronize(st));
    *out = S;
    return GRG_OK;
}

grg_status grg_schur_destroy(grg_schur S)
{
    if (!S) return GRG_OK;
    DeviceGuard dg(S->lat->device);
    hipStreamSynchronize(S->lat->stream);
    if (S->precond) S->precond->schur = nullptr;
    schur_free(S);
    delete S;
    return GRG_OK;
}

grg_status grg_schur_set_params(grg_schur S, const grg_solver_params *params)
{
    if (!S || !params) return set_error("null argument"), GRG_EINVAL;
    GRG_TRY(validate_params(*params));
    if (params->max_rhs > S->prm.max_rhs)
        return set_error("max_rhs cannot grow after creation (%d > %d)", params->max_rhs,
                         S->prm.max_rhs), GRG_EINVAL;
    const int keep = S->prm.max_rhs;
    S->prm = *params;
    S->prm.max_rhs = keep;
    return GRG_OK;
}

static void collect_profile(grg_schur S)
{
    ProfilePool &P = S->prof;
    for (int i = 0; i < P.used; ++i) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, P.start[i], P.stop[i]) == hipSuccess) {
            P.count[P.prec[i]] += 1;
            P.total_ms[P.prec[i]] += ms;
        }
    }
    P.used = 0;
}

typedef std::chrono::steady_clock clk;

// Summed milliseconds per profile slot when a call starts.
struct ProfSnap {
    double ms[kProfSlots];
};
static ProfSnap prof_snap(grg_schur S)
{
    ProfSnap p;
    for (int k = 0; k < kProfSlots; ++k) p.ms[k] = S->prof.total_ms[k];
    return p;
}

static grg_status finish_call(grg_schur S, grg_status st, clk::time_point t0, grg_solver_stats *stats,
                              const ProfSnap &before)
{
    hipError_t e = hipStreamSynchronize(S->lat->stream);
    if (e != hipSuccess && st == GRG_OK) {
        set_error("stream synchronise failed: %s", hipGetErrorString(e));
        st = GRG_EHIP;
    }
    if (S->prof.per_call || 2 * S->prof.used > (int)S->prof.start.size()) collect_profile(S);
    if (stats) {
        stats->t_total_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        stats->n_dslash = S->n_dslash;
        double tot = 0, tot0 = 0;
        for (int p = 0; p < kProfStencilSlots; ++p) {
            tot += S->prof.total_ms[p];
            tot0 += before.ms[p];
        }
        stats->t_dslash_ms = tot - tot0;
        stats->t_dc_ms = S->prof.total_ms[kProfDc] - before.ms[kProfDc];
        stats->t_blas_ms = S->prof.total_ms[kProfBlas] - before.ms[kProfBlas];
        stats->t_prec_ms = S->prof.total_ms[kProfPrec] - before.ms[kProfPrec];
        if (S->prof.on && !S->prof.per_call)
            stats->t_dslash_ms = stats->t_dc_ms = stats->t_blas_ms = stats->t_prec_ms = -1.0;
    }
    return st;
}

static grg_status check_call(grg_schur S, const void *a, const void *b, int nrhs)
{
    if (!S || !a || !b) return set_error("null argument"), GRG_EINVAL;
    if (nrhs < 1 || nrhs > S->prm.max_rhs)
        return set_error("nrhs = %d outside 1..max_rhs = %d", nrhs, S->prm.max_rhs), GRG_EINVAL;
    return GRG_OK;
}

grg_status grg_drr_solve(grg_schur S, const double *rhs, double *x, int nrhs, grg_solver_stats *stats)
{
    GRG_TRY(check_call(S, rhs, x, nrhs));
    DeviceGuard dg(S->lat->device);
    if (stats) memset(stats, 0, sizeof *stats);
    const auto t0 = clk::now();
    const ProfSnap before = prof_snap(S);
    S->n_dslash = 0;
    S->fallbacks = 0;
    grg_lattice L = S->lat;
    GRG_TRY_HIP(launch_pack_masked(rhs, S->b64, S->d_mask, 0, L->g, nrhs, L->stream));
    grg_status st = drr_solve_internal(S, nrhs, stats);
    if (st == GRG_OK || st == GRG_ENOCONV)
        GRG_TRY_HIP(launch_unpack_spinor(GRG_FP64, S->x64, x, L->g, nrhs, L->stream));
    return finish_call(S, st, t0, stats, before);
}

grg_status grg_schur_apply(grg_schur S, const double *x_b, double *y_b, int nrhs,
                           grg_solver_stats *stats)
{
    GRG_TRY(check_call(S, x_b, y_b, nrhs));
    DeviceGuard dg(S->lat->device);
    if (stats) memset(stats, 0, sizeof *stats);
    const auto t0 = clk::now();
    const ProfSnap before = prof_snap(S);
    S->n_dslash = 0;
    S->fallbacks = 0;
    grg_status st = schur_apply_internal(S, x_b, y_b, nrhs, stats);
    return finish_call(S, st, t0, stats, before);
}

grg_status grg_reusken_apply(grg_schur S, const double *x_b, double *y_b, int nrhs)
{
    GRG_TRY(check_call(S, x_b, y_b, nrhs));
    if (4.0 + S->m0 == 0.0) return set_error("4 + m0 = 0: D_rr has a zero diagonal"), GRG_EINVAL;
    DeviceGuard dg(S->lat->device);
    const auto t0 = clk::now();
    const ProfSnap before = prof_snap(S);
    S->n_dslash = 0;
    grg_status st = reusken_apply_internal(S, x_b, y_b, nrhs);
    return finish_call(S, st, t0, nullptr, before);
}

grg_status grg_diag_schur_apply(grg_schur S, const double *x_b, double *y_b, int nrhs)
{
    GRG_TRY(check_call(S, x_b, y_b, nrhs));
    if (4.0 + S->m0 == 0.0) return set_error("4 + m0 = 0: D_rr has a zero diagonal"), GRG_EINVAL;
    DeviceGuard dg(S->lat->device);
    const auto t0 = clk::now();
    const ProfSnap before = prof_snap(S);
    S->n_dslash = 0;
    grg_status st = diag_schur_apply_internal(S, x_b, y_b, nrhs);
    return finish_call(S, st, t0, nullptr, before);
}

enum AssembleKind { kExact, kSecondOrder, kDiagonal };

// Dense coarse operator from its applies to unit vectors, max_rhs columns at
// a time: S_bb (solves), the section 3 approximation, or the one that
// ignores the couplings inside D_rr.
static grg_status assemble(grg_schur S, double *out, size_t cap_bytes, AssembleKind kind)
{
    if (!S || !out) return set_error("null argument"), GRG_EINVAL;
    const size_t n = (size_t)12 * S->nb;
    const size_t need = n * n * 16;
    if (need > cap_bytes)
        return set_error("dense S_bb needs %zu bytes > capacity %zu", need, cap_bytes), GRG_ETOO_LARGE;
    DeviceGuard dg(S->lat->device);
    const int R = S->prm.max_rhs;
    hipStream_t st = S->lat->stream;
    if (!S->cb_in) {
        GRG_TRY(dmalloc((void **)&S->cb_in, n * 16 * R, "assembly staging"));
        GRG_TRY(dmalloc((void **)&S->cb_out, n * 16 * R, "assembly staging"));
    }
    std::vector<double> unit(n * 2 * R);
    grg_status worst = GRG_OK;
    for (size_t j0 = 0; j0 < n; j0 += R) {
        const int cnt = (int)std::min<size_t>(R, n - j0);
        std::fill(unit.begin(), unit.end(), 0.0);
        for (int k = 0; k < cnt; ++k) unit[((size_t)k * n + j0 + k) * 2] = 1.0;
        GRG_TRY_HIP(hipMemcpyAsync(S->cb_in, unit.data(), n * 16 * cnt, hipMemcpyHostToDevice, st));
        grg_solver_stats sst;
        grg_status s = kind == kExact        ? grg_schur_apply(S, S->cb_in, S->cb_out, cnt, &sst)
                       : kind == kSecondOrder ? grg_reusken_apply(S, S->cb_in, S->cb_out, cnt)
                                              : grg_diag_schur_apply(S, S->cb_in, S->cb_out, cnt);
        if (s != GRG_OK && s != GRG_ENOCONV) return s;
        if (s == GRG_ENOCONV) worst = s;
        // column j0 + k of the column-major matrix is output vector k
        GRG_TRY_HIP(hipMemcpy(out + j0 * n * 2, S->cb_out, n * 16 * cnt, hipMemcpyDeviceToHost));
    }
    return worst;
}

grg_status grg_schur_assemble(grg_schur S, double *out, size_t cap_bytes)
{
    return assemble(S, out, cap_bytes, kExact);
}

grg_status grg_reusken_assemble(grg_schur S, double *out, size_t cap_bytes)
{
    return assemble(S, out, cap_bytes, kSecondOrder);
}

grg_status grg_diag_schur_assemble(grg_schur S, double *out, size_t cap_bytes)
{
    return assemble(S, out, cap_bytes, kDiagonal);
}

grg_status grg_schur_tune(grg_schur S, int nrhs)
{
    if (!S) return set_error("null argument"), GRG_EINVAL;
    if (nrhs < 1 || nrhs > S->prm.max_rhs)
        return set_error("nrhs = %d outside 1..max_rhs = %d", nrhs, S->prm.max_rhs), GRG_EINVAL;
    DeviceGuard dg(S->lat->device);
    GRG_TRY(tune_dslash(S, GRG_FP64, nrhs, 3));
    if (S->prm.inner != GRG_FP64) GRG_TRY(tune_dslash(S, S->prm.inner, nrhs, 3));
    GRG_TRY(tune_dc(S, S->prm.inner, nrhs, 3));
    if (S->prm.eo) GRG_TRY(tune_eo(S, S->prm.inner, nrhs, 3));
    GRG_TRY_HIP(hipStreamSynchronize(S->lat->stream));
    return GRG_OK;
}

grg_status grg_schur_dc_launch_info(grg_schur S, int precision, int nrhs, int32_t info[6], float *ms)
{
    if (!S || !info || !ms) return set_error("null argument"), GRG_EINVAL;
    if (precision < 0 || precision > 2 || nrhs < 1 || nrhs > kMaxRhs)
        return set_error("bad precision or nrhs"), GRG_EINVAL;
    const DslashTune &t = S->dctune[precision][nrhs];
    const DslashTune d = t.valid ? t : default_dc_tune(S->lat->g);
    const int32_t v[6] = {d.SB, d.RG, d.split, d.grid, d.chunk, d.march};
    memcpy(info, v, sizeof(v));
    *ms = t.valid ? t.ms : -1.0f;
    return GRG_OK;
}

grg_status grg_schur_set_dc_launch(grg_schur S, int precision, int nrhs, const int32_t info[6])
{
    if (!S || !info) return set_error("null argument"), GRG_EINVAL;
    if (precision < 0 || precision > 2 || nrhs < 1 || nrhs > S->prm.max_rhs)
        return set_error("bad precision or nrhs"), GRG_EINVAL;
    DslashTune t;
    t.SB = info[0];
    t.RG = info[1];
    t.split = info[2];
    t.grid = info[3];
    t.chunk = info[4];
    t.march = info[5];
    t.valid = 1;
    t.ms = 0;
    if (!dc_launch_ok(S->lat->g, precision, nrhs, t))
        return set_error("defect-correction launch {%d, %d, %d, %d, %d, %d} not valid for nrhs %d",
                         info[0], info[1], info[2], info[3], info[4], info[5], nrhs),
               GRG_EINVAL;
    S->dctune[precision][nrhs] = t;
    return GRG_OK;
}

grg_status grg_schur_tune_info(grg_schur S, int precision, int nrhs, int32_t info[6], float *ms)
{
    if (!S || !info || !ms) return set_error("null argument"), GRG_EINVAL;
    if (precision < 0 || precision > 5 || nrhs < 1 || nrhs > kMaxRhs)
        return set_error("bad precision or nrhs"), GRG_EINVAL;
    if (precision >= 3) {  // the half-lattice stencil of the even-odd reduced solve
        Geom gh = S->lat->g;
        gh.V /= 2;
        gh.Vs = S->lat->Vhs;
        const DslashTune &t = S->eotune[precision - 3][nrhs];
        const DslashTune d = t.valid ? t : default_eo_tune(gh, precision - 3, nrhs);
        const int32_t v[6] = {d.SB, d.RG, d.split, d.grid, d.chunk, d.march};
        memcpy(info, v, sizeof(v));
        *ms = t.valid ? t.ms : -1.0f;
        return GRG_OK;
    }
    const DslashTune &t = S->tune[precision][nrhs];
    const DslashTune d = t.valid ? t : default_tune(S->lat->g, precision, nrhs);
    info[0] = d.SB;
    info[1] = d.RG;
    info[2] = d.split;
    info[3] = d.grid;
    info[4] = d.chunk;
    info[5] = d.march;
    *ms = t.valid ? t.ms : -1.0f;
    return GRG_OK;
}

grg_status grg_schur_set_launch(grg_schur S, int precision, int nrhs, const int32_t info[6])
{
    if (!S || !info) return set_error("null argument"), GRG_EINVAL;
    if (precision < 0 || precision > 5 || nrhs < 1 || nrhs > S->prm.max_rhs)
        return set_error("bad precision or nrhs"), GRG_EINVAL;
    DslashTune t;
    t.SB = info[0];
    t.RG = info[1];
    t.split = info[2];
    t.grid = info[3];
    t.chunk = info[4];
    t.march = info[5];
    t.valid = 1;
    t.ms = 0;
    if (precision >= 3) {  // the half-lattice stencil of the even-odd reduced solve
        if (!S->lat->eo_ok) return set_error("the lattice has no even-odd form (odd extent)"), GRG_EINVAL;
        Geom gh = S->lat->g;
        gh.V /= 2;
        gh.Vs = S->lat->Vhs;
        if (!eo_launch_ok(gh, precision - 3, nrhs, t))
            return set_error("half-lattice launch {%d, %d, %d, %d, %d, %d} not valid for precision %d, nrhs %d",
                             info[0], info[1], info[2], info[3], info[4], info[5], precision - 3, nrhs),
                   GRG_EINVAL;
        S->eotune[precision - 3][nrhs] = t;
        return GRG_OK;
    }
    if (!launch_ok(S->lat->g, precision, nrhs, t, false))
        return set_error("launch {%d, %d, %d, %d, %d, %d} not valid for precision %d, nrhs %d",
                         info[0], info[1], info[2], info[3], info[4], info[5], precision, nrhs),
               GRG_EINVAL;
    S->tune[precision][nrhs] = t;
    return GRG_OK;
}

grg_status grg_reduced_apply(grg_schur S, int precision, int parity, const double *in, double *out,
                             int nrhs)
{
    GRG_TRY(check_call(S, in, out, nrhs));
    if (precision < 0 || precision > 2) return set_error("bad precision"), GRG_EINVAL;
    if (parity != 0 && parity != 1) return set_error("parity must be 0 or 1"), GRG_EINVAL;
    if (!S->lat->eo_ok) return set_error("the lattice has no even-odd form (odd extent)"), GRG_EINVAL;
    if (4.0 + S->m0 == 0.0) return set_error("4 + m0 = 0: the reduced operator divides by it"), GRG_EINVAL;
    DeviceGuard dg(S->lat->device);
    grg_status st = reduced_apply_internal(S, precision, parity, in, out, nrhs);
    hipError_t e = hipStreamSynchronize(S->lat->stream);
    if (st == GRG_OK && e != hipSuccess) {
        set_error("stream synchronise failed: %s", hipGetErrorString(e));
        st = GRG_EHIP;
    }
    collect_profile(S);
    return st;
}

grg_status grg_block_apply(grg_schur S, int precision, int rows, int cols, const double *in,
                           double *out, int nrhs)
{
    GRG_TRY(check_call(S, in, out, nrhs));
    if (precision < 0 || precision > 2) return set_error("bad precision"), GRG_EINVAL;
    if (rows < -1 || rows > 1 || cols < -1 || cols > 1)
        return set_error("rows / cols must be -1, 0 or 1"), GRG_EINVAL;
    DeviceGuard dg(S->lat->device);
    grg_status st = block_apply_internal(S, precision, rows, cols, in, out, nrhs);
    hipError_t e = hipStreamSynchronize(S->lat->stream);
    if (st == GRG_OK && e != hipSuccess) {
        set_error("stream synchronise failed: %s", hipGetErrorString(e));
        st = GRG_EHIP;
    }
    collect_profile(S);
    return st;
}

grg_status grg_profile_enable(grg_schur S, int on)
{
    if (!S) return set_error("null argument"), GRG_EINVAL;
    if (on < 0 || on > 2) return set_error("profiling mode %d outside 0..2", on), GRG_EINVAL;
    ProfilePool &P = S->prof;
    if (on && P.start.empty()) {
        const int n = 16384;
        P.start.resize(n);
        P.stop.resize(n);
        P.prec.resize(n);
        for (int i = 0; i < n; ++i) {
            GRG_TRY_HIP(hipEventCreate(&P.start[i]));
            GRG_TRY_HIP(hipEventCreate(&P.stop[i]));
        }
    }
    P.on = on != 0;
    P.phases = P.per_call = on != 2;
    return GRG_OK;
}

// Event pairs not yet read (launch-only profiling reads them here): the
// lattice stream is drained first so that every pair has completed.
static grg_status collect_pending(grg_schur S)
{
    if (S->prof.used == 0) return GRG_OK;
    GRG_TRY_HIP(hipStreamSynchronize(S->lat->stream));
    collect_profile(S);
    return GRG_OK;
}

grg_status grg_profile_read(grg_schur S, int precision, int64_t *count, double *total_ms)
{
    if (!S || !count || !total_ms) return set_error("null argument"), GRG_EINVAL;
    if (precision < 0 || precision >= kProfSlots) return set_error("bad profile slot"), GRG_EINVAL;
    GRG_TRY(collect_pending(S));
    *count = S->prof.count[precision];
    *total_ms = S->prof.total_ms[precision];
    return GRG_OK;
}

grg_status grg_profile_reset(grg_schur S)
{
    if (!S) return set_error("null argument"), GRG_EINVAL;
    GRG_TRY(collect_pending(S));
    for (int p = 0; p < kProfSlots; ++p) {
        S->prof.count[p] = 0;
        S->prof.total_ms[p] = 0;
    }
    return GRG_OK;
}

}  // extern "C"
