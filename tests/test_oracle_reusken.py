"""Pins of the oracle's Schur complement approximation (section 3):

    S~_bb = D_bb - D_br (d^{-1} + d~^{-1} - d^{-1} D_rr d~^{-1}) D_rb,

d = diag(D_rr), d~ = diag(row sums of D_rr).  Pinned by what the formula
fixes independently of how it is coded: it is exact when D_rr is diagonal,
its approximate inverse M reproduces the constant vector exactly
(M D_rr 1 = 1, the row-sum construction), it is a second-order
approximation (the error of M against D_rr^{-1} falls fourfold when the
off-diagonal part of D_rr is halved), and the matrix-free form equals the
dense one.  A dropped or sign-flipped term fails the last three."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors, su3_links
from oracle import dense, matfree

DIMS = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def wilson():
    links = su3_links(DIMS, 0.4, 1)
    return links, dense.wilson_dense(links, DIMS, 0.1)


def test_exact_when_drr_is_diagonal(wilson):
    _, d = wilson
    q, nb = dense.permutation_block(DIMS, "I")
    o = dense.dof_order(q)
    r = o[12 * nb:]
    dm = d.copy()
    # drop every coupling between distinct rest dof
    sub = dm[np.ix_(r, r)]
    dm[np.ix_(r, r)] = np.diag(np.diag(sub))
    s = dense.schur_dense(dm, q, nb)
    st = dense.reusken_dense(dm, q, nb)
    assert np.abs(st - s).max() <= 1e-13 * np.abs(s).max()


def test_constant_vector_is_reproduced(wilson):
    _, d = wilson
    for kind, inv in (("I", False), ("II", True)):
        q, nb = dense.permutation_block(DIMS, kind, inv)
        drr = dense.blocks(d, q, nb)[3]
        m = dense.reusken_inverse(drr)
        one = np.ones(drr.shape[0])
        assert np.abs(m @ (drr @ one) - one).max() < 1e-12


def test_second_order_in_the_off_diagonal_part(wilson):
    _, d = wilson
    q, nb = dense.permutation_block(DIMS, "I")
    drr = dense.blocks(d, q, nb)[3]
    diag = np.diag(np.diag(drr))
    off = drr - diag
    errs = []
    for eps in (0.08, 0.04, 0.02):
        a = diag + eps * off
        errs.append(np.linalg.norm(dense.reusken_inverse(a) - np.linalg.inv(a)))
    # M - A^{-1} = O(eps^2): halving eps divides the error by ~4, not ~2
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.5 < e1 / e2 < 4.5, errs


def test_first_order_terms_alone_are_not_second_order(wilson):
    """Planted mistake: without the cross term the approximation is only
    first order, which the pin above would reject."""
    _, d = wilson
    q, nb = dense.permutation_block(DIMS, "I")
    drr = dense.blocks(d, q, nb)[3]
    diag = np.diag(np.diag(drr))
    off = drr - diag

    def broken(a):
        dd, dt = np.diag(a), a.sum(axis=1)
        return np.diag(1.0 / dd) + np.diag(1.0 / dt) + (a / dd[:, None]) / dt[None, :]

    errs = [np.linalg.norm(broken(diag + e * off) - np.linalg.inv(diag + e * off)) for e in (0.04, 0.02)]
    assert not 3.5 < errs[0] / errs[1] < 4.5


@pytest.mark.parametrize("kind,inv", [("I", False), ("II", False), ("I", True), ("II", True)])
def test_matrix_free_equals_dense(wilson, kind, inv):
    links, d = wilson
    q, nb = dense.permutation_block(DIMS, kind, inv)
    xb = gaussian_vectors(12 * nb, 2, 5)
    want = (dense.reusken_dense(d, q, nb) @ xb.T).T
    got = matfree.reusken_apply(links, DIMS, 0.1, q, nb, xb)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


def test_approximation_is_close_to_the_exact_complement(wilson):
    """The approximation is a perturbation of S_bb on these fields, not an
    unrelated matrix: the relative distance is well below one."""
    _, d = wilson
    q, nb = dense.permutation_block(DIMS, "I")
    s = dense.schur_dense(d, q, nb)
    st = dense.reusken_dense(d, q, nb)
    assert np.linalg.norm(st - s) < 0.5 * np.linalg.norm(s)
