"""GPU S_bb apply, D_rr solve and dense assembly against the oracle.

Tolerances (per RHS, norm-wise relative):
* the D_rr solve is stopped at a relative residual tol; the forward error of
  S x is then at most about tol * ||D_br|| ||D_rb|| / (sigma_min(D_rr)
  sigma_min(S)), which is close to tol for these fields, so the parity runs
  use tol = 1e-12 and require agreement to 1e-10 with the oracle (dense LU,
  or the C oracle at 1e-13);
* independently, the oracle recomputes in FP64 the residual of the GPU's
  D_rr solution, which must meet the tolerance the solve was asked for.
"""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors, point_sources
from oracle import dense, matfree

from gpu_support import Lattice, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

PERMS = [("I", False), ("II", False), ("I", True), ("II", True)]


@pytest.fixture(scope="module")
def c1():
    """4^4, eps 0.4, m0 0.1, seed 1: the dense-comparison workload."""
    lat = Lattice((4, 4, 4, 4), 0.4, 1)
    d = dense.wilson_dense(lat.links, lat.dims, 0.1)
    yield lat, d
    lat.close()


@pytest.mark.parametrize("kind,inv", PERMS)
@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16"])
def test_schur_apply_vs_dense(c1, kind, inv, inner):
    lat, d = c1
    s = lat.schur(0.1, kind, inv, tol=1e-12, inner=inner, inner_tol=1e-2 if inner == "bf16" else 1e-5)
    S = dense.schur_dense(d, s.q, s.nb)
    xb = gaussian_vectors(12 * s.nb, 3, 1)
    y, st = s.apply(xb)
    assert st["converged"] and st["true_rel_resid"] <= 1e-12
    assert rel_err(y, (S @ xb.T).T) < 1e-10
    if inner != "fp64":
        assert st["outer"] >= 2
    s.close()


@pytest.mark.parametrize("kind,inv", PERMS)
def test_schur_assemble_vs_dense(c1, kind, inv):
    lat, d = c1
    s = lat.schur(0.1, kind, inv, tol=1e-12)
    S = dense.schur_dense(d, s.q, s.nb)
    got = lat.grg.grg_schur_assemble(s.h, s.nb)
    assert got.shape == (192, 192)
    assert np.abs(got - S).max() < 1e-10 * np.abs(S).max()
    s.close()


@pytest.mark.parametrize("kind,inv", PERMS)
def test_drr_solve_vs_dense(c1, kind, inv):
    lat, d = c1
    s = lat.schur(0.1, kind, inv, tol=1e-12, restart=4)
    _, _, _, drr = dense.blocks(d, s.q, s.nb)
    o_r = dense.dof_order(s.q)[12 * s.nb:]
    o_b = dense.dof_order(s.q)[: 12 * s.nb]
    b = gaussian_vectors(12 * lat.V, 2, 7)
    x, st = s.drr_solve(b)
    want = np.linalg.solve(drr, b[:, o_r].T).T
    assert rel_err(x[:, o_r], want) < 1e-10
    assert np.abs(x[:, o_b]).max() == 0.0  # zero on the coarse sites
    s.close()


@pytest.mark.parametrize("restart", [1, 3, 8])
def test_restart_lengths_agree(restart):
    lat = Lattice((8, 8, 8, 8), 0.5, 8)
    s = lat.schur(-0.3, "II", True, tol=1e-12, restart=restart)
    xb = gaussian_vectors(12 * s.nb, 2, 8)
    y, st = s.apply(xb)
    want, _, _ = matfree.schur_apply(lat.links, lat.dims, -0.3, s.q, s.nb, xb, restart=8, tol=1e-13)
    assert rel_err(y, want) < 1e-10
    s.close()
    lat.close()


def test_zero_input_and_frozen_rhs(c1):
    lat, _ = c1
    s = lat.schur(0.1, "I", False, tol=1e-12)
    xb = gaussian_vectors(12 * s.nb, 3, 4)
    xb[1] = 0.0
    y, st = s.apply(xb)
    assert np.abs(y[1]).max() == 0.0
    y0, _ = s.apply(xb[[0]])
    assert rel_err(y[[0]], y0) < 1e-11
    s.close()


def test_argument_errors(c1):
    import torch

    lat, _ = c1
    grg = lat.grg
    q, nb = grg.grg_permutation_block(lat.dims, 1, False)
    bad = q.copy()
    bad[3] = bad[4]
    with pytest.raises(grg.GrgError) as e:
        grg.grg_schur_create(lat.h, 0.1, bad, nb, grg.grg_solver_params_default())
    assert e.value.status == grg.GRG_EINVAL
    with pytest.raises(grg.GrgError):
        grg.grg_schur_create(lat.h, 0.1, q, nb, grg.grg_solver_params_default(restart=0))
    s = lat.schur(0.1, "I", False, max_rhs=2)
    x = to_dev(np.zeros((3, 12 * nb)))
    y = torch.empty_like(x)
    with pytest.raises(grg.GrgError) as e:
        grg.grg_schur_apply(s.h, x, y, 3)
    assert e.value.status == grg.GRG_EINVAL
    s.close()


def test_noconvergence_is_reported(c1):
    lat, _ = c1
    s = lat.schur(0.1, "I", True, tol=1e-12, max_iter=3)
    xb = gaussian_vectors(12 * s.nb, 1, 2)
    import paper_0704_2341_amd as grg

    with pytest.raises(grg.GrgError) as e:
        s.apply(xb)
    assert e.value.status == grg.GRG_ENOCONV
    y, st = s.apply(xb, allow_noconv=True)
    assert st["status"] == grg.GRG_ENOCONV and not st["converged"] and np.isfinite(y).all()
    s.close()


@pytest.fixture(scope="module")
def c2():
    """16^4, eps 0.5, m0 -0.2, seed 2, 8 Gaussian right-hand sides."""
    lat = Lattice((16, 16, 16, 16), 0.5, 2)
    yield lat
    lat.close()


@pytest.mark.parametrize("kind,inv", PERMS)
def test_16_4_all_permutations(c2, kind, inv):
    lat = c2
    s = lat.schur(-0.2, kind, inv, tol=1e-10)
    # backward error: the oracle's FP64 residual of the GPU's D_rr solutions
    b = np.zeros((8, 12 * lat.V), np.complex128)
    mask = np.zeros(lat.V, bool)
    mask[s.q[s.nb:]] = True
    g = gaussian_vectors(12 * lat.V, 8, 2)
    b[:, np.repeat(mask, 12)] = g[:, np.repeat(mask, 12)]
    x, st = s.drr_solve(b)
    rr = matfree.drr_residual(lat.links, lat.dims, -0.2, s.q, s.nb, b, x)
    assert st["converged"] and rr.max() <= 1e-10
    # forward error of S x for two of the eight RHS against the C oracle
    p = lat.grg.grg_solver_params_default(tol=1e-12)
    lat.grg.grg_schur_set_params(s.h, p)
    xb = gaussian_vectors(12 * s.nb, 8, 2)
    y, st = s.apply(xb)
    assert st["converged"]
    want, _, _ = matfree.schur_apply(lat.links, lat.dims, -0.2, s.q, s.nb, xb[:2], restart=8, tol=1e-13)
    assert rel_err(y[:2], want) < 1e-10
    s.close()


@pytest.mark.parametrize("inner", ["fp32", "bf16"])
def test_16_4_mixed_matches_fp64(c2, inner):
    lat = c2
    s64 = lat.schur(-0.2, "I", False, tol=1e-12)
    smx = lat.schur(-0.2, "I", False, tol=1e-12, inner=inner, inner_tol=1e-2 if inner == "bf16" else 1e-5)
    xb = point_sources(s64.nb, 12)
    y64, _ = s64.apply(xb)
    ymx, st = smx.apply(xb)
    assert st["converged"] and st["outer"] >= 2
    assert rel_err(ymx, y64) < 1e-10
    s64.close()
    smx.close()


def test_iteration_count_matches_oracle():
    """Minimal residual on D_rr takes as many iterations on the GPU as the
    oracle's GCR (37 on this field), also for a handle created after another
    was destroyed (the defect correction must never see stale norms)."""
    lat = Lattice((8, 8, 8, 8), 0.5, 3)
    xb = point_sources(lat.V // 16, 12)
    _, it_or, _ = matfree.schur_apply(lat.links, lat.dims, -0.3, *lat.grg.grg_permutation_block(lat.dims, 1),
                                      xb[:1], restart=1, tol=1e-10)
    for _ in range(2):
        s = lat.schur(-0.3, "I", False, tol=1e-10, restart=1)
        _, st = s.apply(xb)
        assert st["outer"] == 1 and st["iters"] <= it_or[0] + 2, (st, it_or)
        s.close()
    for inner, tol_in in (("fp32", 1e-5), ("bf16", 1e-2)):
        s = lat.schur(-0.3, "I", False, tol=1e-10, inner=inner, inner_tol=tol_in)
        _, st = s.apply(xb)
        assert st["converged"] and st["iters"] <= 2 * it_or[0], (inner, st)
        s.close()
    lat.close()


@pytest.mark.parametrize("inner", ["fp64", "bf16"])
def test_tuned_launch_same_result(inner):
    lat = Lattice((8, 8, 8, 16), 0.5, 6)
    s = lat.schur(-0.1, "II", False, tol=1e-12, inner=inner, inner_tol=1e-2)
    xb = gaussian_vectors(12 * s.nb, 4, 6)
    y0, _ = s.apply(xb)
    lat.grg.grg_schur_tune(s.h, 4)
    info = lat.grg.grg_schur_tune_info(s.h, inner, 4)
    assert info["ms"] > 0 and info["SB"] in (64, 128, 256) and info["grid"] % 8 == 0
    y1, st = s.apply(xb)
    assert st["converged"] and rel_err(y1, y0) < 1e-11
    s.close()
    lat.close()
