// Learned preconditioner: handle, inference, loss and gradient, training on
// the GPU, weight files, and its use inside the D_rr solve.
//
// The three layers run as launch_ptc_layer (gather + transport on the vector
// ALUs, channel mixing on the matrix cores).  Backpropagation uses the adjoint
// of each layer, dX = sum_h T_h^+ W_h^H dY, which is again a layer (with the
// hops reversed and the weights conjugate-transposed), and the weight
// gradient dL/dconj(W_h) = sum_x dY(x) (T_h X(x))^+ on the matrix cores.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <random>
#include <vector>

#include "handles.h"
#include "ptc.h"

namespace grg {

BlasShape blas_shape(const Geom &g, int nrhs);
grg_status run_dslash(grg_schur S, int prec, const void *in, void *out, int sel, int nrhs,
                      double *partials, const void *dot_with = nullptr);
DslashTune default_tune(const Geom &g, int prec, int nrhs);
grg_status eo_training_pair(grg_schur S, void *e, void *r_full, int nrhs, int k, const double *neg_one);

static const int kOff[3] = {0, 9 * 8 * 4, 9 * 8 * 4 + 9 * 8 * 8};

static size_t act_bytes(const Geom &g, int nrhs, int F) { return (size_t)nrhs * 3 * F * g.Vs * 4; }

static grg_status embed_all(grg_precond P)
{
    hipStream_t st = P->schur->lat->stream;
    for (int l = 0; l < 3; ++l) {
        const int fin = kPtcChannels[l], fout = kPtcChannels[l + 1];
        GRG_TRY_HIP(launch_ptc_embed(fin, fout, P->w + kOff[l], P->A[l], 0, st));
        GRG_TRY_HIP(launch_ptc_embed(fin, fout, P->w + kOff[l], P->Aadj[l], 1, st));
    }
    return GRG_OK;
}

// act_out = M act_in (bf16 Dirac-field tiles), output zero where mask is not
// 0 (default: the coarse sites)
static grg_status forward(grg_precond P, const void *in, void *out, int nrhs,
                          const uint8_t *mask = nullptr)
{
    grg_schur S = P->schur;
    grg_lattice L = S->lat;
    const void *x = in;
    for (int l = 0; l < 3; ++l) {
        PtcLayerArgs a;
        const int grid = ptc_launch_shape(0, kPtcChannels[l], kPtcChannels[l + 1], L->g, nrhs, &a.rc);
        a.x = x;
        a.y = l == 2 ? out : P->act[l + 1];
        a.U = L->U[GRG_BF16];
        a.A = P->A[l];
        a.mask = l == 2 ? (mask ? mask : S->d_mask) : nullptr;
        a.sel = 0;
        a.g = L->g;
        a.nrhs = nrhs;
        GRG_TRY_HIP(launch_ptc_layer(kPtcChannels[l], kPtcChannels[l + 1], a, grid, L->stream));
        x = a.y;
    }
    return GRG_OK;
}

// gradient of the loss with respect to conj(W) from dact[3] and the stored
// activations act[0..2] (act0: the network input)
static grg_status backward(grg_precond P, const void *act0, int nrhs)
{
    grg_schur S = P->schur;
    grg_lattice L = S->lat;
    for (int l = 2; l >= 0; --l) {
        const int fin = kPtcChannels[l], fout = kPtcChannels[l + 1];
        PtcGradArgs ga;
        const int grid = ptc_launch_shape(1, fin, fout, L->g, nrhs, &ga.rc);
        ga.x = l == 0 ? act0 : P->act[l];
        ga.dy = P->dact[l + 1];
        ga.U = L->U[GRG_BF16];
        ga.g = L->g;
        ga.nrhs = nrhs;
        ga.partials = P->wpart;
        GRG_TRY_HIP(launch_ptc_wgrad(fin, fout, ga, grid, L->stream));
        GRG_TRY_HIP(launch_ptc_wgrad_reduce(fin, fout, P->wpart, grid, P->grad + kOff[l], L->stream));
        if (l > 0) {
            PtcLayerArgs a;
            a.x = P->dact[l + 1];
            a.y = P->dact[l];
            a.U = L->U[GRG_BF16];
            a.A = P->Aadj[l];
            a.mask = nullptr;
            a.sel = 0;
            a.g = L->g;
            a.nrhs = nrhs;
            const int lgrid = ptc_launch_shape(0, fout, fin, L->g, nrhs, &a.rc);
            GRG_TRY_HIP(launch_ptc_layer(fout, fin, a, lgrid, L->stream));
        }
    }
    return GRG_OK;
}

// loss of act[3] against ebuf, and dact[3]
static grg_status loss(grg_precond P, int nrhs, const void *y)
{
    grg_lattice L = P->schur->lat;
    const int grid = std::max(1, std::min((L->g.V + 255) / 256, 1024));
    GRG_TRY_HIP(launch_ptc_loss(y, P->ebuf, L->g, nrhs, P->lpart, grid, P->lsums, P->loss,
                                P->dact[3], L->stream));
    return GRG_OK;
}

// p = M r for the inner solve in precision prec (device fields, internal tiles)
grg_status precond_apply_inner(grg_schur S, int prec, const void *r, void *p, int nrhs)
{
    grg_precond P = S->precond;
    grg_lattice L = S->lat;
    const BlasShape sh = blas_shape(L->g, nrhs);
    const void *in = r;
    if (prec != GRG_BF16) {
        GRG_TRY_HIP(launch_axpy_convert(prec, GRG_BF16, sh, r, P->act[0], nullptr, 0, 0, nullptr,
                                        L->stream));
        in = P->act[0];
    }
    if (prec == GRG_BF16) return forward(P, in, p, nrhs);
    GRG_TRY(forward(P, in, P->act[3], nrhs));
    GRG_TRY_HIP(launch_axpy_convert(GRG_BF16, prec, sh, P->act[3], p, nullptr, 0, 0, nullptr,
                                    L->stream));
    return GRG_OK;
}

static void precond_free(grg_precond P)
{
    auto f = [](void *q) {
        if (q) (void)hipFree(q);
    };
    f(P->w);
    f(P->grad);
    f(P->adam_m);
    f(P->adam_v);
    for (int l = 0; l < 3; ++l) {
        f(P->A[l]);
        f(P->Aadj[l]);
    }
    for (int k = 0; k < 4; ++k) {
        f(P->act[k]);
        f(P->dact[k]);
    }
    f(P->ebuf);
    for (int k = 0; k < 3; ++k) f(P->gen[k]);
    f(P->wpart);
    f(P->lpart);
    f(P->lsums);
    f(P->loss);
    f(P->neg_one);
    if (P->h_buf) (void)hipHostFree(P->h_buf);
}

static grg_status read_weights(grg_precond P, std::vector<double> &w)
{
    w.resize(2 * kPtcWeights);
    GRG_TRY_HIP(hipMemcpy(w.data(), P->w, sizeof(double) * 2 * kPtcWeights, hipMemcpyDeviceToHost));
    return GRG_OK;
}

static grg_status write_weights(grg_precond P, const double *w)
{
    for (int i = 0; i < 2 * kPtcWeights; ++i) P->weights_finite = P->weights_finite && isfinite(w[i]);
    GRG_TRY_HIP(hipMemcpy(P->w, w, sizeof(double) * 2 * kPtcWeights, hipMemcpyHostToDevice));
    GRG_TRY(embed_all(P));
    GRG_TRY_HIP(hipStreamSynchronize(P->schur->lat->stream));
    return GRG_OK;
}

}  // namespace grg

using namespace grg;

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceScope()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

extern "C" {

grg_status grg_precond_create(grg_schur S, grg_precond *out)
{
    if (!S || !out) return set_error("null argument"), GRG_EINVAL;
    *out = nullptr;
    DeviceScope ds(S->lat->device);
    grg_precond P = new (std::nothrow) grg_precond_s();
    if (!P) return set_error("out of host memory"), GRG_ENOMEM;
    P->schur = S;
    P->max_rhs = S->prm.max_rhs;
    const Geom &g = S->lat->g;
    const int R = P->max_rhs;
    bool ok = true;
    auto al = [&](void **p, size_t bytes) {
        if (ok && hipMalloc(p, bytes) != hipSuccess) {
            *p = nullptr;
            ok = false;
        }
    };
    al((void **)&P->w, sizeof(double2) * kPtcWeights);
    al((void **)&P->grad, sizeof(double2) * kPtcWeights);
    al((void **)&P->adam_m, sizeof(double) * 2 * kPtcWeights);
    al((void **)&P->adam_v, sizeof(double) * 2 * kPtcWeights);
    for (int l = 0; l < 3; ++l) {
        al((void **)&P->A[l], sizeof(__bf16) * 16 * ptc_kp(kPtcChannels[l]));
        al((void **)&P->Aadj[l], sizeof(__bf16) * 16 * ptc_kp(kPtcChannels[l + 1]));
    }
    for (int k = 0; k < 4; ++k) {
        al(&P->act[k], act_bytes(g, R, kPtcChannels[k]));
        al(&P->dact[k], act_bytes(g, R, kPtcChannels[k]));
    }
    al(&P->ebuf, act_bytes(g, R, 4));
    for (int k = 0; k < 3; ++k) al(&P->gen[k], act_bytes(g, R, 4));
    al((void **)&P->wpart, sizeof(float) * (size_t)kPtcMaxGrid * 16 * ptc_np(8));
    al((void **)&P->lpart, sizeof(double) * 1024 * kMaxRhs * 2);
    al((void **)&P->lsums, sizeof(double) * kMaxRhs * 2);
    al((void **)&P->loss, sizeof(double) * 2);
    al((void **)&P->neg_one, sizeof(double) * kMaxRhs);
    if (ok && hipHostMalloc((void **)&P->h_buf, sizeof(double) * 4 * kMaxRhs) != hipSuccess) {
        P->h_buf = nullptr;
        ok = false;
    }
    if (!ok) {
        precond_free(P);
        delete P;
        return set_error("preconditioner workspaces: allocation failed"), GRG_ENOMEM;
    }
    // zero everything (activations pad tiles beyond V), identity weights
    hipStream_t st = S->lat->stream;
    for (int k = 0; k < 4; ++k) {
        GRG_TRY_HIP(launch_fill_zero(P->act[k], act_bytes(g, R, kPtcChannels[k]), st));
        GRG_TRY_HIP(launch_fill_zero(P->dact[k], act_bytes(g, R, kPtcChannels[k]), st));
    }
    GRG_TRY_HIP(launch_fill_zero(P->ebuf, act_bytes(g, R, 4), st));
    for (int k = 0; k < 3; ++k) GRG_TRY_HIP(launch_fill_zero(P->gen[k], act_bytes(g, R, 4), st));
    GRG_TRY_HIP(launch_fill_zero(P->adam_m, sizeof(double) * 2 * kPtcWeights, st));
    GRG_TRY_HIP(launch_fill_zero(P->adam_v, sizeof(double) * 2 * kPtcWeights, st));
    std::vector<double> w(2 * kPtcWeights, 0.0);
    for (int l = 0; l < 3; ++l) {
        const int fin = kPtcChannels[l], fout = kPtcChannels[l + 1];
        for (int f = 0; f < std::min(fin, fout); ++f) w[2 * (kOff[l] + f * fin + f)] = 1.0;
    }
    grg_status s = write_weights(P, w.data());
    if (s != GRG_OK) {
        precond_free(P);
        delete P;
        return s;
    }
    *out = P;
    return GRG_OK;
}

grg_status grg_precond_destroy(grg_precond P)
{
    if (!P) return GRG_OK;
    DeviceScope ds(P->schur->lat->device);
    (void)hipStreamSynchronize(P->schur->lat->stream);
    if (P->schur->precond == P) P->schur->precond = nullptr;
    precond_free(P);
    delete P;
    return GRG_OK;
}

grg_status grg_precond_set_weights(grg_precond P, const double *w)
{
    if (!P || !w) return set_error("null argument"), GRG_EINVAL;
    DeviceScope ds(P->schur->lat->device);
    P->weights_finite = true;
    return write_weights(P, w);
}

grg_status grg_precond_get_weights(grg_precond P, double *w)
{
    if (!P || !w) return set_error("null argument"), GRG_EINVAL;
    DeviceScope ds(P->schur->lat->device);
    GRG_TRY_HIP(hipStreamSynchronize(P->schur->lat->stream));
    GRG_TRY_HIP(hipMemcpy(w, P->w, sizeof(double) * 2 * kPtcWeights, hipMemcpyDeviceToHost));
    return GRG_OK;
}

grg_status grg_precond_apply(grg_precond P, const double *in, double *out, int nrhs)
{
    if (!P || !in || !out) return set_error("null argument"), GRG_EINVAL;
    if (nrhs < 1 || nrhs > P->max_rhs) return set_error("nrhs outside 1..max_rhs"), GRG_EINVAL;
    DeviceScope ds(P->schur->lat->device);
    grg_lattice L = P->schur->lat;
    GRG_TRY_HIP(launch_pack_spinor(GRG_BF16, in, P->act[0], L->g, nrhs, L->stream, P->schur->d_mask, 0));
    GRG_TRY(forward(P, P->act[0], P->act[3], nrhs));
    GRG_TRY_HIP(launch_unpack_spinor(GRG_BF16, P->act[3], out, L->g, nrhs, L->stream));
    GRG_TRY_HIP(hipStreamSynchronize(L->stream));
    return GRG_OK;
}

grg_status grg_precond_loss_grad(grg_precond P, const double *r, const double *e, int nrhs,
                                 double *loss_out, double *grad)
{
    if (!P || !r || !e || !loss_out || !grad) return set_error("null argument"), GRG_EINVAL;
    if (nrhs < 1 || nrhs > P->max_rhs) return set_error("nrhs outside 1..max_rhs"), GRG_EINVAL;
    DeviceScope ds(P->schur->lat->device);
    grg_lattice L = P->schur->lat;
    GRG_TRY_HIP(launch_pack_spinor(GRG_BF16, r, P->act[0], L->g, nrhs, L->stream, P->schur->d_mask, 0));
    GRG_TRY_HIP(launch_pack_spinor(GRG_BF16, e, P->ebuf, L->g, nrhs, L->stream, P->schur->d_mask, 0));
    GRG_TRY(forward(P, P->act[0], P->act[3], nrhs));
    GRG_TRY(loss(P, nrhs, P->act[3]));
    GRG_TRY(backward(P, P->act[0], nrhs));
    GRG_TRY_HIP(hipStreamSynchronize(L->stream));
    GRG_TRY_HIP(hipMemcpy(loss_out, P->loss, sizeof(double), hipMemcpyDeviceToHost));
    GRG_TRY_HIP(hipMemcpy(grad, P->grad, sizeof(double2) * kPtcWeights, hipMemcpyDeviceToHost));
    return GRG_OK;
}

grg_status grg_precond_train(grg_precond P, const grg_train_params *tp, grg_train_stats *out)
{
    if (!P || !tp) return set_error("null argument"), GRG_EINVAL;
    if (tp->steps < 1 || tp->batch < 1 || tp->batch > P->max_rhs || tp->max_mr_steps < 0 ||
        !(tp->lr > 0) || (tp->reduced != 0 && tp->reduced != 1))
        return set_error("bad training parameters"), GRG_EINVAL;
    DeviceScope ds(P->schur->lat->device);
    grg_schur S = P->schur;
    grg_lattice L = S->lat;
    if (tp->reduced && !S->d_mask_par)
        return set_error("reduced training needs even lattice extents"), GRG_EINVAL;
    hipStream_t st = L->stream;
    const int B = tp->batch;
    const BlasShape sh = blas_shape(L->g, B);
    const int dgrid = default_tune(L->g, GRG_BF16, B).grid;
    // the solver's tuned launches with fused dots need this grid for the reduce
    const DslashTune &tt = S->tune[GRG_BF16][B];
    const int agrid = tt.valid ? tt.grid : dgrid;
    std::mt19937_64 rng(tp->seed);
    // -1 per RHS for e = e_0 - x
    std::vector<double> neg(kMaxRhs, -1.0);
    GRG_TRY_HIP(hipMemcpy(P->neg_one, neg.data(), sizeof(double) * kMaxRhs, hipMemcpyHostToDevice));
    const auto t0 = std::chrono::steady_clock::now();
    double first = NAN, acc = 0;
    int nacc = 0;
    const int log_every = tp->log_every > 0 ? tp->log_every : tp->steps;
    void *x = P->gen[0], *r = P->gen[1], *q = P->gen[2];
    for (int step = 1; step <= tp->steps; ++step) {
        const int k = (int)(rng() % (uint64_t)(tp->max_mr_steps + 1));
        // Reduced training starts with a quarter of the steps on pairs of
        // D_rr itself: every hop moves a field to the other parity, so on
        // pairs that live on one parity the gradient of each hop weight
        // pairs fields of opposite parities and vanishes while the hop
        // weights are zero (the identity start), and the hop weights would
        // never leave zero.
        const bool red = tp->reduced && step > tp->steps / 4;
        if (red) {
            // pairs of the reduced system (errors and loss on the reduced
            // parity's rest sites)
            GRG_TRY_HIP(launch_random_field(GRG_BF16, P->ebuf, S->d_mask_par, L->g, B, rng(), st));
            GRG_TRY(eo_training_pair(S, P->ebuf, r, B, k, P->neg_one));
        } else {
            GRG_TRY_HIP(launch_random_field(GRG_BF16, P->ebuf, S->d_mask, L->g, B, rng(), st));
            GRG_TRY(run_dslash(S, GRG_BF16, P->ebuf, r, 0, B, nullptr));
            GRG_TRY_HIP(launch_fill_zero(x, act_bytes(L->g, B, 4), st));
            for (int j = 0; j < k; ++j) {
                GRG_TRY(run_dslash(S, GRG_BF16, r, q, 0, B, S->partials));
                GRG_TRY_HIP(launch_reduce(kAlpha, S->partials, agrid, B, S->alpha, nullptr, nullptr,
                                          nullptr, st));
                GRG_TRY_HIP(launch_mr_update(GRG_BF16, sh, x, r, q, nullptr, S->alpha, S->partials, st));
            }
            // e_k = e_0 - x_k and r_k = D_rr e_k: the pair the solver produced
            // (r_k recomputed from e_k, so that the pair is consistent to rounding)
            GRG_TRY_HIP(launch_axpy_convert(GRG_BF16, GRG_BF16, sh, x, P->ebuf, P->neg_one, 0, 1,
                                            nullptr, st));
            GRG_TRY(run_dslash(S, GRG_BF16, P->ebuf, r, 0, B, nullptr));
        }
        GRG_TRY(forward(P, r, P->act[3], B, red ? S->d_mask_par : nullptr));
        GRG_TRY(loss(P, B, P->act[3]));
        GRG_TRY(backward(P, r, B));
        ++P->adam_step;
        GRG_TRY_HIP(launch_ptc_adam((double *)P->w, (const double *)P->grad, P->adam_m, P->adam_v,
                                    2 * kPtcWeights, tp->lr, 0.9, 0.999, 1e-8, P->adam_step, st));
        GRG_TRY(embed_all(P));
        if (step == 1 || step > tp->steps - log_every) {
            double l;
            GRG_TRY_HIP(hipMemcpyAsync(P->h_buf, P->loss, sizeof(double), hipMemcpyDeviceToHost, st));
            GRG_TRY_HIP(hipStreamSynchronize(st));
            l = P->h_buf[0];
            if (!isfinite(l)) return set_error("non-finite training loss at step %d", step), GRG_ENONFINITE;
            if (step == 1) first = l;
            if (step > tp->steps - log_every) {
                acc += l;
                ++nacc;
            }
        }
    }
    GRG_TRY_HIP(hipStreamSynchronize(st));
    std::vector<double> w;
    GRG_TRY(read_weights(P, w));
    P->weights_finite = true;
    for (double v : w) P->weights_finite = P->weights_finite && isfinite(v);
    if (out) {
        out->steps = tp->steps;
        out->pairs = tp->steps * B;
        out->loss_first = first;
        out->loss_last = nacc ? acc / nacc : NAN;
        out->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return GRG_OK;
}

static const char kMagic[8] = {'G', 'R', 'G', 'P', 'T', 'C', '0', '1'};

grg_status grg_precond_save(grg_precond P, const char *path)
{
    if (!P || !path) return set_error("null argument"), GRG_EINVAL;
    DeviceScope ds(P->schur->lat->device);
    std::vector<double> w;
    GRG_TRY(read_weights(P, w));
    FILE *f = fopen(path, "wb");
    if (!f) return set_error("cannot open %s for writing", path), GRG_EINVAL;
    const int32_t hdr[6] = {1, kPtcChannels[0], kPtcChannels[1], kPtcChannels[2], kPtcChannels[3],
                            P->adam_step};
    bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(hdr, sizeof hdr, 1, f) == 1 &&
              fwrite(w.data(), sizeof(double), w.size(), f) == w.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) return set_error("writing %s failed", path), GRG_EINVAL;
    return GRG_OK;
}

grg_status grg_precond_load(grg_precond P, const char *path)
{
    if (!P || !path) return set_error("null argument"), GRG_EINVAL;
    FILE *f = fopen(path, "rb");
    if (!f) return set_error("cannot open %s", path), GRG_EINVAL;
    char magic[8];
    int32_t hdr[6];
    std::vector<double> w(2 * kPtcWeights);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 &&
              fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == 1 && hdr[1] == 4 && hdr[2] == 8 &&
              hdr[3] == 8 && hdr[4] == 4 && fread(w.data(), sizeof(double), w.size(), f) == w.size();
    fclose(f);
    if (!ok) return set_error("%s is not a weight file of this network", path), GRG_EINVAL;
    DeviceScope ds(P->schur->lat->device);
    P->weights_finite = true;
    GRG_TRY(write_weights(P, w.data()));
    P->adam_step = hdr[5];
    return GRG_OK;
}

grg_status grg_schur_attach_precond(grg_schur S, grg_precond P)
{
    if (!S) return set_error("null argument"), GRG_EINVAL;
    if (P && P->schur != S) return set_error("preconditioner belongs to another operator"), GRG_EINVAL;
    S->precond = P;
    return GRG_OK;
}

}  // extern "C"
