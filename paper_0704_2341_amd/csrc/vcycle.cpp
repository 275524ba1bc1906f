// Cyclic-reduction V-cycle (section 4): the hierarchy of levels, one cycle,
// and the BiCGstab solves of whole levels (the top level's "exact" solve and
// the preconditioned solve of D x = f whose average convergence rate section 4
// reports).
//
// Level k is A_k = c_k D_W(lattice k, m_k).  With the all-even coarse set
// (Type I) the Schur complement approximation of A_k is
//     c_k (D_bb - D_br D_rb / d_k) = (c_k / d_k) D_W(V, d_k^2 - 4),
// d_k = 4 + m_k, on the coarse lattice with links V_mu(c) = U_mu(2c) U_mu(2c + mu);
// the coarse sites of level k in the order of its Type I ordering are the
// sites of level k + 1 in lexicographic order.  So level k + 1 is a lattice
// handle of its own with blocked links, m_{k+1} = d_k^2 - 4 and
// c_{k+1} = c_k / d_k, and the A_rr solves of level k are the D_rr solves of a
// Type I coarse-operator handle on lattice k (BiCGstab, FP64, to drr_tol).
//
// Any other ordering of section 2 (Type II, the inverse permutations) gives
// a two-level cycle: level 0 is partitioned by that ordering, and the top
// level is the section 3 approximation S~_bb of its Schur complement on the
// coarse sites (matrix-free through the level-0 handle, in the handle's
// coarse-field layout [nrhs][N_b][12]), solved by BiCGstab to top_tol.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "handles.h"

struct grg_vcycle_s {
    grg_vcycle_params prm;
    int levels = 0;
    bool approx_top = false;  // the top level is S~_bb of level 0's partition (no lattice)
    grg_lattice lat[3] = {nullptr, nullptr, nullptr};  // lat[0] is the caller's
    grg_schur schur[3] = {nullptr, nullptr, nullptr};  // levels below the top
    double m[3] = {0, 0, 0}, c[3] = {1, 1, 1};
    int V[3] = {0, 0, 0}, nb[3] = {0, 0, 0};
    int32_t *d_q[3] = {nullptr, nullptr, nullptr};      // coarse sites of level k, q[0:nb]
    // canonical FP64 fields per level, max_rhs each: the cycle's input and
    // output on that level, and three temporaries
    double *fin[3] = {}, *xout[3] = {}, *t0[3] = {}, *t1[3] = {}, *t2[3] = {};
    // the BiCGstab vectors (sized for level 0; the top level uses them too
    // when it is solved inside a cycle, hence a second set)
    double *bv[2][8] = {};
    double *partials = nullptr, *h_part = nullptr;
    int cycles = 0;
};

namespace grg {

grg_status reusken_apply_internal(grg_schur S, const double *xb, double *yb, int nrhs);

namespace {

struct Dev {
    int prev = -1;
    explicit Dev(int d)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) (void)hipSetDevice(d);
    }
    ~Dev()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

size_t field_bytes(const grg_vcycle_s *v, int k) { return (size_t)v->prm.max_rhs * v->V[k] * 12 * 16; }

grg_status lincomb(grg_vcycle_s *v, int k, int nrhs, double *out, int n, const double *in0,
                   const double2 *c0, const double *in1 = nullptr, const double2 *c1 = nullptr,
                   const double *in2 = nullptr, const double2 *c2 = nullptr)
{
    VcCoef cf;
    cf.n = n;
    const double2 *cs[3] = {c0, c1, c2};
    for (int j = 0; j < 3; ++j)
        for (int r = 0; r < kMaxRhs; ++r) cf.c[j][r] = j < n && r < nrhs ? cs[j][r] : make_double2(0, 0);
    GRG_TRY_HIP(launch_vc_lincomb((size_t)v->V[k] * 12, nrhs, cf, out, in0, in1, in2, v->lat[0]->stream));
    return GRG_OK;
}

// per RHS: <a, b> = sum conj(a) b, and |b|^2
grg_status dots(grg_vcycle_s *v, int k, int nrhs, const double *a, const double *b, double2 *ab, double *bb)
{
    const size_t len = (size_t)v->V[k] * 12;
    const int grid = vc_dot_grid(len);
    hipStream_t st = v->lat[0]->stream;
    GRG_TRY_HIP(launch_vc_dot(len, nrhs, a, b, v->partials, st));
    GRG_TRY_HIP(hipMemcpyAsync(v->h_part, v->partials, sizeof(double) * 3 * grid * nrhs, hipMemcpyDeviceToHost, st));
    GRG_TRY_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int i = 0; i < grid; ++i) {
            const double *p = v->h_part + ((size_t)i * nrhs + r) * 3;
            s0 += p[0];
            s1 += p[1];
            s2 += p[2];
        }
        if (ab) ab[r] = make_double2(s0, s1);
        if (bb) bb[r] = s2;
    }
    return GRG_OK;
}

// out = A_k in (the approximate top level enqueued without the API call's
// synchronisation: the solve's next norm read waits for it)
grg_status apply_level(grg_vcycle_s *v, int k, int nrhs, const double *in, double *out)
{
    if (k > 0 && v->approx_top) return reusken_apply_internal(v->schur[0], in, out, nrhs);
    GRG_TRY(grg_dirac_apply(v->lat[k], v->m[k], GRG_FP64, in, out, nrhs));
    if (v->c[k] != 1.0) {
        double2 s[kMaxRhs];
        for (int r = 0; r < nrhs; ++r) s[r] = make_double2(v->c[k], 0);
        GRG_TRY(lincomb(v, k, nrhs, out, 1, out, s));
    }
    return GRG_OK;
}

grg_status cycle(grg_vcycle_s *v, int k, int nrhs, const double *f, double *x);

inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
inline double2 cdiv(double2 a, double2 b)
{
    const double d = b.x * b.x + b.y * b.y;
    return d > 0 ? make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d) : make_double2(0, 0);
}

// BiCGstab on A_k x = f, x from zero, right-preconditioned by the cycle on
// level k when pre; vector set `set` (0: the outer solve, 1: the top level
// inside a cycle).  Per RHS the residual history gives the rate.
grg_status bicgstab(grg_vcycle_s *v, int k, int set, bool pre, double tol, int nrhs, const double *f,
                    double *x, int *iters, double *rate, bool *converged)
{
    double **w = v->bv[set];
    double *r = w[0], *rh = w[1], *p = w[2], *vv = w[3], *s = w[4], *t = w[5], *ph = w[6], *sh = w[7];
    const size_t bytes = (size_t)nrhs * v->V[k] * 12 * 16;
    hipStream_t st = v->lat[0]->stream;
    double2 one[kMaxRhs], mone[kMaxRhs], zero[kMaxRhs];
    for (int i = 0; i < kMaxRhs; ++i) {
        one[i] = make_double2(1, 0);
        mone[i] = make_double2(-1, 0);
        zero[i] = make_double2(0, 0);
    }
    GRG_TRY_HIP(launch_fill_zero(x, bytes, st));
    GRG_TRY_HIP(hipMemcpyAsync(r, f, bytes, hipMemcpyDeviceToDevice, st));
    GRG_TRY_HIP(hipMemcpyAsync(rh, f, bytes, hipMemcpyDeviceToDevice, st));
    GRG_TRY_HIP(hipMemcpyAsync(p, f, bytes, hipMemcpyDeviceToDevice, st));
    double2 rho[kMaxRhs], alpha[kMaxRhs], omega[kMaxRhs], beta[kMaxRhs], tmp[kMaxRhs];
    double r0n[kMaxRhs], rn[kMaxRhs], tt[kMaxRhs];
    GRG_TRY(dots(v, k, nrhs, f, f, rho, r0n));
    bool act[kMaxRhs];
    for (int i = 0; i < nrhs; ++i) {
        rn[i] = r0n[i];
        act[i] = r0n[i] > 0;
    }
    auto finished = [&]() {
        for (int i = 0; i < nrhs; ++i)
            if (act[i] && rn[i] > tol * tol * r0n[i]) return false;
        return true;
    };
    int it = 0;
    bool done = finished();
    while (!done && it < v->prm.max_iter) {
        const double *pin = p;
        if (pre) {
            GRG_TRY(cycle(v, k, nrhs, p, ph));
            pin = ph;
        }
        GRG_TRY(apply_level(v, k, nrhs, pin, vv));
        GRG_TRY(dots(v, k, nrhs, rh, vv, tmp, nullptr));
        for (int i = 0; i < nrhs; ++i) alpha[i] = act[i] ? cdiv(rho[i], tmp[i]) : make_double2(0, 0);
        for (int i = 0; i < nrhs; ++i) tmp[i] = make_double2(-alpha[i].x, -alpha[i].y);
        GRG_TRY(lincomb(v, k, nrhs, s, 2, r, one, vv, tmp));  // s = r - alpha v
        const double *sin_ = s;
        if (pre) {
            GRG_TRY(cycle(v, k, nrhs, s, sh));
            sin_ = sh;
        }
        GRG_TRY(apply_level(v, k, nrhs, sin_, t));
        GRG_TRY(dots(v, k, nrhs, s, t, tmp, tt));  // <s, t> and |t|^2 in one pass; <t, s> = conj <s, t>
        for (int i = 0; i < nrhs; ++i)
            omega[i] = act[i] && tt[i] > 0 ? make_double2(tmp[i].x / tt[i], -tmp[i].y / tt[i]) : make_double2(0, 0);
        // x += alpha p^ + omega s^ ; r = s - omega t
        GRG_TRY(lincomb(v, k, nrhs, x, 3, x, one, pin, alpha, sin_, omega));
        for (int i = 0; i < nrhs; ++i) tmp[i] = make_double2(-omega[i].x, -omega[i].y);
        GRG_TRY(lincomb(v, k, nrhs, r, 2, s, one, t, tmp));
        double2 rho2[kMaxRhs];
        GRG_TRY(dots(v, k, nrhs, rh, r, rho2, rn));
        for (int i = 0; i < nrhs; ++i) {
            const bool ok = act[i] && (rho[i].x != 0 || rho[i].y != 0) && (omega[i].x != 0 || omega[i].y != 0);
            beta[i] = ok ? cmul(cdiv(rho2[i], rho[i]), cdiv(alpha[i], omega[i])) : make_double2(0, 0);
            rho[i] = rho2[i];
            if (act[i] && rn[i] <= tol * tol * r0n[i]) act[i] = false;
        }
        // p = r + beta (p - omega v)
        for (int i = 0; i < nrhs; ++i) tmp[i] = cmul(make_double2(-beta[i].x, -beta[i].y), omega[i]);
        GRG_TRY(lincomb(v, k, nrhs, p, 3, r, one, p, beta, vv, tmp));
        ++it;
        for (int i = 0; i < nrhs; ++i)
            if (!isfinite(rn[i])) return set_error("non-finite residual in the V-cycle's BiCGstab"), GRG_ENONFINITE;
        done = finished();
    }
    (void)zero;
    (void)mone;
    *iters = it;
    if (converged) *converged = done;
    if (rate) {
        double acc = 0;
        int n = 0;
        for (int i = 0; i < nrhs; ++i)
            if (r0n[i] > 0 && it > 0) {
                acc += pow(sqrt(rn[i] / r0n[i]), 1.0 / it);
                ++n;
            }
        *rate = n ? acc / n : 0.0;
    }
    return GRG_OK;
}

// x = cycle(k) f on level k (canonical fields of lattice k)
grg_status cycle(grg_vcycle_s *v, int k, int nrhs, const double *f, double *x)
{
    hipStream_t st = v->lat[0]->stream;
    double2 one[kMaxRhs], mone[kMaxRhs], ic[kMaxRhs], mc[kMaxRhs];
    for (int i = 0; i < kMaxRhs; ++i) {
        one[i] = make_double2(1, 0);
        mone[i] = make_double2(-1, 0);
        ic[i] = make_double2(1.0 / v->c[k], 0);
        mc[i] = make_double2(-v->c[k], 0);
    }
    if (k == v->levels - 1) {
        // the top level, solved to top_tol
        int it = 0;
        bool conv = false;
        GRG_TRY(bicgstab(v, k, 1, false, v->prm.top_tol, nrhs, f, x, &it, nullptr, &conv));
        if (!conv) return set_error("V-cycle: the top level's solve did not reach top_tol"), GRG_ENOCONV;
        return GRG_OK;
    }
    ++v->cycles;
    grg_schur S = v->schur[k];
    const int V = v->V[k], nb = v->nb[k];
    double *y = v->t0[k], *t = v->t1[k], *u = v->t2[k];
    // y = D_rr^{-1} f_r  (A_rr^{-1} f_r = y / c_k)
    grg_status s = grg_drr_solve(S, f, y, nrhs, nullptr);
    if (s != GRG_OK && s != GRG_ENOCONV) return s;
    // g = f_b - A_br A_rr^{-1} f_r = f_b - (D_br y)_b, restricted to level k + 1
    GRG_TRY(grg_block_apply(S, GRG_FP64, 1, 0, y, t, nrhs));
    GRG_TRY(lincomb(v, k, nrhs, t, 2, f, one, t, mone));
    GRG_TRY_HIP(launch_vc_restrict(t, v->fin[k + 1], v->d_q[k], nb, V, nrhs, st));
    // x_b = cycle(k + 1) g
    GRG_TRY(cycle(v, k + 1, nrhs, v->fin[k + 1], v->xout[k + 1]));
    // u = x_b on the coarse sites; h = f_r - A_rb u = f - c_k (D_rb u)
    GRG_TRY_HIP(launch_fill_zero(u, (size_t)nrhs * V * 12 * 16, st));
    GRG_TRY_HIP(launch_vc_prolong(v->xout[k + 1], u, v->d_q[k], nb, V, nrhs, st));
    GRG_TRY(grg_block_apply(S, GRG_FP64, 0, 1, u, t, nrhs));
    GRG_TRY(lincomb(v, k, nrhs, t, 2, f, one, t, mc));
    // x_r = A_rr^{-1} h = D_rr^{-1} h / c_k ; x = x_r + u
    s = grg_drr_solve(S, t, y, nrhs, nullptr);
    if (s != GRG_OK && s != GRG_ENOCONV) return s;
    GRG_TRY(lincomb(v, k, nrhs, x, 2, y, ic, u, one));
    return GRG_OK;
}

void vfree(void *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

void vcycle_free(grg_vcycle_s *v)
{
    for (int k = 0; k < 3; ++k) {
        if (v->schur[k]) (void)grg_schur_destroy(v->schur[k]);
        if (k > 0 && v->lat[k]) (void)grg_lattice_destroy(v->lat[k]);
        vfree((void *&)v->d_q[k]);
        vfree((void *&)v->fin[k]);
        vfree((void *&)v->xout[k]);
        vfree((void *&)v->t0[k]);
        vfree((void *&)v->t1[k]);
        vfree((void *&)v->t2[k]);
    }
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 8; ++i) vfree((void *&)v->bv[j][i]);
    vfree((void *&)v->partials);
    if (v->h_part) (void)hipHostFree(v->h_part);
    v->h_part = nullptr;
}

}  // namespace

}  // namespace grg

using namespace grg;

extern "C" {

grg_status grg_vcycle_params_default(grg_vcycle_params *p)
{
    if (!p) return set_error("null argument"), GRG_EINVAL;
    p->levels = 3;
    p->drr_tol = 1e-2;
    p->top_tol = 1e-12;
    p->max_rhs = 12;
    p->max_iter = 10000;
    p->perm = GRG_PERM_I;
    p->inverse = 0;
    return GRG_OK;
}

grg_status grg_vcycle_create(grg_lattice L, double m0, const grg_vcycle_params *params, grg_vcycle *out)
{
    if (!L || !out) return set_error("null argument"), GRG_EINVAL;
    *out = nullptr;
    grg_vcycle_params p;
    if (params) p = *params;
    else grg_vcycle_params_default(&p);
    if (p.levels < 2 || p.levels > 3) return set_error("levels must be 2 or 3"), GRG_EINVAL;
    if (!(p.drr_tol > 0 && p.drr_tol < 1) || !(p.top_tol > 0 && p.top_tol < 1))
        return set_error("tolerances must be in (0, 1)"), GRG_EINVAL;
    if (p.max_rhs < 1 || p.max_rhs > kMaxRhs) return set_error("max_rhs must be in 1..%d", kMaxRhs), GRG_EINVAL;
    if (p.max_iter < 1) return set_error("max_iter must be positive"), GRG_EINVAL;
    if (p.perm != GRG_PERM_I && p.perm != GRG_PERM_II) return set_error("unknown perm %d", p.perm), GRG_EINVAL;
    const bool approx_top = !(p.perm == GRG_PERM_I && p.inverse == 0);
    if (approx_top && p.levels != 2)
        return set_error("an ordering other than Type I gives a two-level cycle: levels must be 2"), GRG_EINVAL;
    if (!L->gauge_set) return set_error("gauge field not set"), GRG_EINVAL;
    if (!isfinite(m0) || 4.0 + m0 == 0.0) return set_error("4 + m0 must be finite and nonzero"), GRG_EINVAL;
    // Type I: every level even below the top, the top at least 2 wide;
    // otherwise the partition needs even extents
    const int div = approx_top ? 2 : 1 << p.levels;
    for (int mu = 0; mu < 4; ++mu)
        if (L->g.L[mu] % div)
            return set_error("extent %d of direction %d is not divisible by %d", L->g.L[mu], mu, div), GRG_EINVAL;
    Dev dev(L->device);
    grg_vcycle_s *v = new (std::nothrow) grg_vcycle_s();
    if (!v) return set_error("out of host memory"), GRG_ENOMEM;
    v->prm = p;
    v->levels = p.levels;
    v->approx_top = approx_top;
    v->lat[0] = L;
    v->m[0] = m0;
    v->c[0] = 1.0;
    grg_status s = GRG_OK;
    auto fail = [&](grg_status e) {
        vcycle_free(v);
        delete v;
        return e;
    };
    auto alloc = [&](void **ptr, size_t bytes) -> bool {
        if (hipMalloc(ptr, bytes) != hipSuccess) {
            *ptr = nullptr;
            set_error("V-cycle: hipMalloc of %zu bytes failed", bytes);
            return false;
        }
        return true;
    };
    int dims[4] = {L->g.L[0], L->g.L[1], L->g.L[2], L->g.L[3]};
    for (int k = 0; k < p.levels; ++k) {
        v->V[k] = dims[0] * dims[1] * dims[2] * dims[3];
        if (k + 1 < p.levels) {
            // this level's partition and its D_rr solves
            std::vector<int32_t> q(v->V[k]);
            int32_t nb = 0;
            if ((s = grg_permutation_block(dims, k == 0 ? p.perm : GRG_PERM_I, k == 0 ? p.inverse : 0, q.data(),
                                           &nb)) != GRG_OK)
                return fail(s);
            v->nb[k] = nb;
            grg_solver_params sp;
            grg_solver_params_default(&sp);
            sp.tol = p.drr_tol;
            sp.inner = GRG_FP64;
            sp.method = 1;
            sp.eo = 0;
            sp.max_rhs = p.max_rhs;
            sp.max_iter = p.max_iter;
            if ((s = grg_schur_create(v->lat[k], v->m[k], q.data(), nb, &sp, &v->schur[k])) != GRG_OK)
                return fail(s);
            if (!alloc((void **)&v->d_q[k], sizeof(int32_t) * nb)) return fail(GRG_ENOMEM);
            if (hipMemcpy(v->d_q[k], q.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice) != hipSuccess)
                return set_error("V-cycle: copy of the coarse sites failed"), fail(GRG_EHIP);
            if (approx_top) {
                // the top level: the N_b coarse sites, no lattice of their own
                dims[0] = nb;
                dims[1] = dims[2] = dims[3] = 1;
            } else {
                // the next level: the coarse lattice, its blocked links and mass
                int cd[4] = {dims[0] / 2, dims[1] / 2, dims[2] / 2, dims[3] / 2};
                const int32_t periodic[4] = {1, 1, 1, 1};  // the signs ride in the blocked links
                if ((s = grg_lattice_create(cd, periodic, L->stream, &v->lat[k + 1])) != GRG_OK) return fail(s);
                double *links = nullptr;
                const size_t lb = (size_t)nb * 4 * 9 * 16;
                if (!alloc((void **)&links, lb)) return fail(GRG_ENOMEM);
                if (launch_vc_block_links(v->lat[k]->g, v->lat[k]->U[GRG_FP64], v->lat[k + 1]->g, links, L->stream) !=
                        hipSuccess ||
                    hipStreamSynchronize(L->stream) != hipSuccess) {
                    (void)hipFree(links);
                    return set_error("V-cycle: link blocking failed"), fail(GRG_EHIP);
                }
                s = grg_gauge_set(v->lat[k + 1], links, 1);
                (void)hipFree(links);
                if (s != GRG_OK) return fail(s);
                const double d = 4.0 + v->m[k];
                v->m[k + 1] = d * d - 4.0;
                v->c[k + 1] = v->c[k] / d;
                for (int mu = 0; mu < 4; ++mu) dims[mu] = cd[mu];
            }
        }
        void **f[5] = {(void **)&v->fin[k], (void **)&v->xout[k], (void **)&v->t0[k], (void **)&v->t1[k],
                       (void **)&v->t2[k]};
        for (void **ptr : f)
            if (!alloc(ptr, field_bytes(v, k))) return fail(GRG_ENOMEM);
    }
    for (int i = 0; i < 8; ++i) {
        if (!alloc((void **)&v->bv[0][i], field_bytes(v, 0))) return fail(GRG_ENOMEM);
        if (!alloc((void **)&v->bv[1][i], field_bytes(v, p.levels - 1))) return fail(GRG_ENOMEM);
    }
    const size_t np = (size_t)3 * vc_dot_grid((size_t)v->V[0] * 12) * kMaxRhs;
    if (!alloc((void **)&v->partials, sizeof(double) * np)) return fail(GRG_ENOMEM);
    if (hipHostMalloc((void **)&v->h_part, sizeof(double) * np) != hipSuccess) {
        v->h_part = nullptr;
        return set_error("V-cycle: hipHostMalloc failed"), fail(GRG_ENOMEM);
    }
    *out = v;
    return GRG_OK;
}

grg_status grg_vcycle_destroy(grg_vcycle v)
{
    if (!v) return GRG_OK;
    Dev dev(v->lat[0]->device);
    (void)hipStreamSynchronize(v->lat[0]->stream);
    vcycle_free(v);
    delete v;
    return GRG_OK;
}

grg_status grg_vcycle_apply(grg_vcycle v, const double *f, double *x, int nrhs)
{
    if (!v || !f || !x) return set_error("null argument"), GRG_EINVAL;
    if (nrhs < 1 || nrhs > v->prm.max_rhs) return set_error("nrhs outside 1..max_rhs"), GRG_EINVAL;
    Dev dev(v->lat[0]->device);
    GRG_TRY(cycle(v, 0, nrhs, f, x));
    GRG_TRY_HIP(hipStreamSynchronize(v->lat[0]->stream));
    return GRG_OK;
}

grg_status grg_vcycle_solve(grg_vcycle v, int precondition, double tol, const double *f, double *x, int nrhs,
                            grg_vcycle_stats *stats)
{
    if (!v || !f || !x) return set_error("null argument"), GRG_EINVAL;
    if (nrhs < 1 || nrhs > v->prm.max_rhs) return set_error("nrhs outside 1..max_rhs"), GRG_EINVAL;
    if (!(tol > 0 && tol < 1)) return set_error("tol must be in (0, 1)"), GRG_EINVAL;
    Dev dev(v->lat[0]->device);
    if (stats) memset(stats, 0, sizeof *stats);
    const auto t0 = std::chrono::steady_clock::now();
    v->cycles = 0;
    int it = 0;
    double rate = 0;
    bool conv = false;
    GRG_TRY(bicgstab(v, 0, 0, precondition != 0, tol, nrhs, f, x, &it, &rate, &conv));
    // |f - D x| / |f| from the iterate
    double *t = v->t0[0];
    GRG_TRY(grg_dirac_apply(v->lat[0], v->m[0], GRG_FP64, x, t, nrhs));
    double2 one[kMaxRhs], mone[kMaxRhs];
    for (int i = 0; i < kMaxRhs; ++i) {
        one[i] = make_double2(1, 0);
        mone[i] = make_double2(-1, 0);
    }
    GRG_TRY(lincomb(v, 0, nrhs, t, 2, f, one, t, mone));
    double rr[kMaxRhs], ff[kMaxRhs];
    GRG_TRY(dots(v, 0, nrhs, t, t, nullptr, rr));
    GRG_TRY(dots(v, 0, nrhs, f, f, nullptr, ff));
    double worst = 0;
    for (int i = 0; i < nrhs; ++i) worst = std::max(worst, ff[i] > 0 ? sqrt(rr[i] / ff[i]) : 0.0);
    if (stats) {
        stats->iters = it;
        stats->converged = conv;
        stats->rate = rate;
        stats->true_rel_resid = worst;
        stats->cycles = v->cycles;
        stats->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!conv) {
        set_error("V-cycle BiCGstab: no convergence to %.1e in %d iterations", tol, it);
        return GRG_ENOCONV;
    }
    return GRG_OK;
}

}  // extern "C"
