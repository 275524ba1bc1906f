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

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DIMS, EPS, SEED, M0, NRHS = (32, 32, 32, 32), 0.5, 3, -0.3, 12
SAMPLE = (0, 7, 11)  # right-hand sides the oracle recomputes
TOL = {"fp64": 1e-14, "bf16": 1.5e-2}


@pytest.fixture(scope="module")
def big():
    lat = Lattice(DIMS, EPS, SEED)
    s = lat.schur(M0, "I", False, tol=1e-10, inner="bf16", inner_tol=1e-2, restart=1,
                  max_rhs=NRHS, max_iter=4000)
    lat.grg.grg_schur_tune(s.h, NRHS)
    yield lat, s
    s.close()
    lat.close()


def rest_only(x, q, nb):
    """Zero the coarse sites of lattice fields (nrhs, 12 V)."""
    y = x.reshape(x.shape[0], -1, 12)
    y[:, np.asarray(q[:nb])] = 0
    return x


@pytest.mark.parametrize("prec", ["bf16", "fp64"])
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
        par = matfree.site_parity(DIMS)
        off = par != parity
        off[np.asarray(s.q[: s.nb])] = True
        assert not np.any(y.reshape(NRHS, -1, 12)[:, off])
