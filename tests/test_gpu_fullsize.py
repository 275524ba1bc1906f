"""Parity at the full benchmark size: 32^4, Type I, m0 = -0.3, links eps 0.5
seed 3, 12 right-hand sides, in the tuned launch configuration that the
benchmark times.  The oracle computes sampled right-hand sides one by one
(each full S_bb apply costs seconds on the host), and the GPU's D_rr
solution is judged by the oracle's own FP64 residual."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_support import Lattice, rel_err, to_dev, to_host
from grg_inputs import gaussian_vectors, point_sources
from oracle import rounding

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DIMS, EPS, SEED, M0, NRHS = (32, 32, 32, 32), 0.5, 3, -0.3, 12
SAMPLE = (0, 7, 11)  # right-hand sides the oracle recomputes
TOL = {"fp64": 1e-14, "fp32": 2e-6, "bf16": 1.5e-2}
# Element-wise bound |y - y*| <= C u sum|terms| against the FP64 oracle, u the
# unit roundoff of the storage format, sum|terms| the oracle's sum of the
# absolute values of the products that make up the entry.  A stencil output
# carries the rounding of its inputs and links (u each, relative, on every
# term) and of its own store (u |y|, |y| <= sum|terms|), so C = 3 (+ FP32
# accumulation, 2^-24 per term); the reduced operator's intermediate field
# is stored as well and enters its second stencil: C = 6.
ELEM_C = {"stencil": 3.2, "reduced": 6.4}


@pytest.fixture(scope="module")
def big():
    lat = Lattice(DIMS, EPS, SEED)
    s = lat.schur(M0, "I", False, tol=1e-10, inner="bf16", inner_tol=1e-2, restart=1,
                  max_rhs=NRHS, max_iter=4000)
    lat.grg.grg_schur_tune(s.h, NRHS)
    # the FP32 stencil launches too (the tuner times the inner precision of
    # the handle's parameters)
    lat.grg.grg_schur_set_params(s.h, lat.grg.grg_solver_params_default(
        tol=1e-10, inner="fp32", inner_tol=1e-5, restart=1, max_rhs=NRHS, max_iter=4000))
    lat.grg.grg_schur_tune(s.h, NRHS)
    lat.grg.grg_schur_set_params(s.h, lat.grg.grg_solver_params_default(
        tol=1e-10, inner="bf16", inner_tol=1e-2, restart=1, max_rhs=NRHS, max_iter=4000))
    yield lat, s
    s.close()
    lat.close()


def rest_only(x, q, nb):
    """Zero the coarse sites of lattice fields (nrhs, 12 V)."""
    y = x.reshape(x.shape[0], -1, 12)
    y[:, np.asarray(q[:nb])] = 0
    return x


@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp64"])
def test_drr_stencil_tuned_launch(big, prec):
    import torch

    from oracle import matfree

    lat, s = big
    grg = lat.grg
    info = grg.grg_schur_tune_info(s.h, prec, NRHS)
    print(f"32^4 D_rr stencil, {prec}, 12 RHS, launch {info}", flush=True)
    assert info["ms"] > 0  # the tuner ran for this (precision, RHS count)
    x = rest_only(gaussian_vectors(12 * lat.V, NRHS, 31), s.q, s.nb)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    grg.grg_block_apply(s.h, prec, 0, 0, xd, yd, NRHS)
    y = to_host(yd)
    del xd, yd
    want = matfree.block_apply(lat.links, DIMS, M0, s.q, s.nb, 0, 0, x[list(SAMPLE)])
    assert rel_err(y[list(SAMPLE)], want) < TOL[prec]
    if prec != "fp64":
        # every entry, not only the norm: a defect confined to a few sites fails here
        terms = matfree.block_apply_abs(lat.links, DIMS, M0, s.q, s.nb, 0, 0, x[list(SAMPLE)])
        bound = ELEM_C["stencil"] * rounding.UNIT_ROUNDOFF[prec] * terms
        worst = np.max(np.abs(y[list(SAMPLE)] - want) / np.maximum(bound, 1e-300))
        print(f"element-wise: worst |y - y*| / bound = {worst:.3f}", flush=True)
        assert np.all(np.abs(y[list(SAMPLE)] - want) <= bound)
    # every RHS of the launch is a stencil output: coarse rows are zero
    assert not np.any(y.reshape(NRHS, -1, 12)[:, np.asarray(s.q[:s.nb])])


def test_schur_apply_mixed_bench_workload(big):
    """The benchmark's apply (BF16 inner, FP64 refinement to 1e-10), then the
    same at 1e-12 for the forward-agreement criterion."""
    from oracle import matfree

    lat, s = big
    grg = lat.grg
    xb = point_sources(s.nb, NRHS)
    y10, st = s.apply(xb)
    print(f"32^4 S_bb bf16-mixed tol 1e-10: {st}", flush=True)
    assert st["converged"] and st["true_rel_resid"] <= 1e-10
    grg.grg_schur_set_params(s.h, grg.grg_solver_params_default(
        tol=1e-12, inner="bf16", inner_tol=1e-2, restart=1, max_rhs=NRHS, max_iter=4000))
    try:
        y12, st12 = s.apply(xb)
    finally:
        grg.grg_schur_set_params(s.h, grg.grg_solver_params_default(
            tol=1e-10, inner="bf16", inner_tol=1e-2, restart=1, max_rhs=NRHS, max_iter=4000))
    assert st12["converged"] and st12["true_rel_resid"] <= 1e-12
    want, it, rr = matfree.schur_apply(lat.links, DIMS, M0, s.q, s.nb, xb[list(SAMPLE)], restart=8,
                                       tol=1e-13)
    assert np.all(rr <= 1e-13)
    e12 = rel_err(y12[list(SAMPLE)], want)
    e10 = rel_err(y10[list(SAMPLE)], want)
    print(f"agreement with the oracle: tol 1e-12 -> {e12:.2e}, tol 1e-10 -> {e10:.2e}", flush=True)
    assert e12 <= 1e-10
    # forward error at the bench tolerance: bounded by tol times the
    # amplification ||D_br|| ||D_rb|| / (s_min(D_rr) s_min(S_bb)) ~ 1 here
    assert e10 <= 1e-9


def test_drr_solve_oracle_residual(big):
    """Backward criterion: the oracle's FP64 residual of the GPU's mixed
    precision D_rr solution, at the benchmark's tolerance."""
    from oracle import matfree

    lat, s = big
    b = rest_only(gaussian_vectors(12 * lat.V, NRHS, 32), s.q, s.nb)
    x, st = s.drr_solve(b)
    print(f"32^4 D_rr solve bf16-mixed: {st}", flush=True)
    assert st["converged"] and st["true_rel_resid"] <= 1e-10
    rr = matfree.drr_residual(lat.links, DIMS, M0, s.q, s.nb, b[list(SAMPLE)], x[list(SAMPLE)])
    print(f"oracle residuals {rr}", flush=True)
    assert np.all(rr <= 1e-10 * (1 + 1e-6))
    assert not np.any(x.reshape(NRHS, -1, 12)[:, np.asarray(s.q[:s.nb])])


def test_reduced_operator_tuned_launch(big):
    """The half-lattice stencils of the reduced operator, in the tuned launch
    the benchmark times (the dominant kernel), at the full size."""
    import torch

    from oracle import matfree

    lat, s = big
    grg = lat.grg
    info = grg.grg_schur_tune_info(s.h, "bf16", NRHS, eo=True)
    print(f"32^4 reduced operator, bf16, 12 RHS, launch {info}", flush=True)
    assert info["ms"] > 0
    x = gaussian_vectors(12 * lat.V, NRHS, 33)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    for parity in (0, 1):
        grg.grg_reduced_apply(s.h, "bf16", parity, xd, yd, NRHS)
        y = to_host(yd)
        want = matfree.reduced_apply(lat.links, DIMS, M0, s.q, s.nb, parity, x[list(SAMPLE)])
        assert rel_err(y[list(SAMPLE)], want) < TOL["bf16"]
        terms = matfree.reduced_apply_abs(lat.links, DIMS, M0, s.q, s.nb, parity, x[list(SAMPLE)])
        bound = ELEM_C["reduced"] * rounding.UNIT_ROUNDOFF["bf16"] * terms
        err = np.abs(y[list(SAMPLE)] - want)
        print(f"parity {parity}: worst |y - y*| / bound = {np.max(err / np.maximum(bound, 1e-300)):.3f}",
              flush=True)
        assert np.all(err <= bound)
        par = matfree.site_parity(DIMS)
        off = par != parity
        off[np.asarray(s.q[: s.nb])] = True
        assert not np.any(y.reshape(NRHS, -1, 12)[:, off])


def test_schur_apply_fp32_inner(big):
    """The FP32 inner path of the mixed solve at the full size (FP32 stencil
    and Krylov vectors, FP64 refinement to 1e-10 and to 1e-12), against the
    oracle on sampled right-hand sides."""
    from oracle import matfree

    lat, s = big
    grg = lat.grg
    xb = point_sources(s.nb, NRHS)
    out = {}
    try:
        for tol in (1e-10, 1e-12):
            grg.grg_schur_set_params(s.h, grg.grg_solver_params_default(
                tol=tol, inner="fp32", inner_tol=1e-5, restart=1, max_rhs=NRHS, max_iter=4000))
            y, st = s.apply(xb)
            print(f"32^4 S_bb fp32-mixed tol {tol:g}: {st}", flush=True)
            assert st["converged"] and st["true_rel_resid"] <= tol
            out[tol] = y
    finally:
        grg.grg_schur_set_params(s.h, grg.grg_solver_params_default(
            tol=1e-10, inner="bf16", inner_tol=1e-2, restart=1, max_rhs=NRHS, max_iter=4000))
    want, it, rr = matfree.schur_apply(lat.links, DIMS, M0, s.q, s.nb, xb[list(SAMPLE[:2])], restart=8,
                                       tol=1e-13)
    assert np.all(rr <= 1e-13)
    e12 = rel_err(out[1e-12][list(SAMPLE[:2])], want)
    e10 = rel_err(out[1e-10][list(SAMPLE[:2])], want)
    print(f"fp32 inner, agreement with the oracle: 1e-12 -> {e12:.2e}, 1e-10 -> {e10:.2e}", flush=True)
    assert e12 <= 1e-10 and e10 <= 1e-9


# ---------------------------------------------------------------- network
@pytest.fixture(scope="module")
def trained():
    """A network trained on the GPU on 16^4 solver pairs (m0 = -0.3, the
    training lattice), as the benchmark trains it but with fewer steps, and
    the 16^4 handles it is bound to."""
    lat = Lattice((16, 16, 16, 16), EPS, 5)
    s = lat.schur(M0, "I", False, tol=1e-10, inner="bf16", inner_tol=1e-2, max_rhs=12)
    grg = lat.grg
    p = grg.grg_precond_create(s.h)
    st = grg.grg_precond_train(p, steps=120, batch=12, max_mr_steps=30, lr=3e-3, seed=5, log_every=20,
                               reduced=True)
    print(f"16^4 training: {st}", flush=True)
    assert st["loss_last"] < st["loss_first"]
    w = grg.grg_precond_get_weights(p)
    yield lat, s, p, w
    grg.grg_precond_destroy(p)
    s.close()
    lat.close()


def _rest_field(lat, s, nrhs, seed):
    v = gaussian_vectors(12 * lat.V, nrhs, seed).reshape(nrhs, lat.V, 12)
    v[:, np.asarray(s.q[: s.nb])] = 0
    rmask = np.ones(lat.V)
    rmask[np.asarray(s.q[: s.nb])] = 0
    return v.reshape(nrhs, -1), rmask


# the network computes in BF16 (activations, weights) with FP32 accumulation
NET_TOL = 3e-2


def test_network_forward_16(trained):
    """The trained network's output at the training lattice, every site of
    two RHS, against the whole-lattice oracle."""
    import torch

    from oracle import ptc

    lat, s, p, w = trained
    ws = ptc.unpack_weights(w)
    x, rmask = _rest_field(lat, s, 2, 51)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    lat.grg.grg_precond_apply(p, xd, yd, 2)
    y = to_host(yd)
    for k in range(2):
        want = ptc.net_forward(ptc.to_channels(x[k], lat.dims), ws, lat.links, lat.dims)[-1]
        want = (want * rmask[:, None, None]).reshape(-1)
        e = rel_err(y[k], want)
        print(f"16^4 forward RHS {k}: rel err {e:.2e}", flush=True)
        assert e < NET_TOL


def test_network_gradients_16(trained):
    """Loss and Wirtinger weight gradients at the training lattice (the
    site reduction in its real shape) against the oracle's analytic backward."""
    from oracle import ptc

    lat, s, p, w = trained
    ws = ptc.unpack_weights(w)
    r, rmask = _rest_field(lat, s, 2, 52)
    e, _ = _rest_field(lat, s, 2, 53)
    loss, grad = lat.grg.grg_precond_loss_grad(p, to_dev(r), to_dev(e), 2)
    rs = np.stack([ptc.to_channels(v, lat.dims) for v in r])
    es = np.stack([ptc.to_channels(v, lat.dims) for v in e])
    lo, go = ptc.loss_and_grads(rs, es, ws, lat.links, lat.dims, out_mask=rmask)
    go = ptc.pack_weights(go)
    cos = np.real(np.vdot(grad, go)) / np.linalg.norm(grad) / np.linalg.norm(go)
    print(f"16^4 loss {loss:.5f} (oracle {lo:.5f}), |dg|/|g| "
          f"{np.linalg.norm(grad - go) / np.linalg.norm(go):.2e}, cos {cos:.6f}", flush=True)
    assert abs(loss - lo) < 3e-2 * lo
    assert np.linalg.norm(grad - go) < 5e-2 * np.linalg.norm(go)
    assert cos > 0.998


def test_network_forward_32(big, trained):
    """The trained weights on the 32^4 bench lattice: two RHS, compared at
    sampled sites (every tile position, both parities, the lattice's edges)
    with the oracle's sampled-site evaluation."""
    import torch

    from oracle import ptc

    lat, s = big
    _, _, _, w = trained
    grg = lat.grg
    ws = ptc.unpack_weights(w)
    p = grg.grg_precond_create(s.h)
    try:
        grg.grg_precond_set_weights(p, w)
        x, rmask = _rest_field(lat, s, 2, 54)
        xd = to_dev(x)
        yd = torch.empty_like(xd)
        grg.grg_precond_apply(p, xd, yd, 2)
        y = to_host(yd).reshape(2, lat.V, 4, 3)
        del xd, yd
    finally:
        grg.grg_precond_destroy(p)
    rng = np.random.default_rng(55)
    sites = np.unique(np.concatenate([rng.integers(0, lat.V, 40), np.arange(64), [lat.V - 1, lat.V // 2],
                                      np.arange(lat.V - 64, lat.V)]))
    for k in range(2):
        want = ptc.net_forward_sites(ptc.to_channels(x[k], DIMS), ws, lat.links, DIMS, sites)
        want = want * rmask[sites, None, None]
        e = rel_err(y[k, sites].reshape(1, -1), want.reshape(1, -1))
        print(f"32^4 forward RHS {k}, {len(sites)} sites: rel err {e:.2e}", flush=True)
        assert e < NET_TOL
        # per site as well: no site may be far off
        per = np.linalg.norm((y[k, sites] - want).reshape(len(sites), -1), axis=1)
        ref = np.linalg.norm(want.reshape(len(sites), -1), axis=1)
        assert np.all(per <= 4 * NET_TOL * np.maximum(ref, 1e-12 * ref.max()))
