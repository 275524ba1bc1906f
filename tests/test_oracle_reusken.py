"""Pins of the oracle's Schur complement approximation (section 3):

    S~_bb = D_bb - D_br (d^{-1} + d~^{-1} - d^{-1} D_rr d~^{-1}) D_rb,

d = diag(D_rr), d~ = diag(row sums of D_rr).  Pinned by what the formula
fixes independently of how it is coded: it is exact when D_rr is diagonal,
its approximate inverse M reproduces the constant vector exactly
(M D_rr 1 = 1, the row-sum construction), it is a second-order
approximation (the error of M against D_rr^{-1} falls fourfold when the
off-diagonal part of D_rr is halved), and the matrix-free form equals the
dense one.  A dropped or sign-flipped term fails the last three.

The older approximation that ignores the couplings inside D_rr,
D_bb - D_br diag(D_rr)^{-1} D_rb, is pinned by its free-field spectrum in
closed form, gauge covariance, agreement with the exact complement when D_rr
is diagonal, and matrix-free = dense."""
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


# ------------------------------------------------------------------ ignoring D_rr
# The older approximation that section 3 contrasts with the second-order one:
# the couplings inside D_rr ignored, D_rr^{-1} -> diag(D_rr)^{-1}.


def free_diag_schur_type1_spectrum(dims, m0):
    """Eigenvalues of D_bb - D_br D_rb / d for U = 1 and the all-even coarse
    sublattice (Type I), d = 4 + m0.  From a coarse site x the only rest sites
    one hop away are x +- mu, and from those the only coarse sites one hop
    away are x and x +- 2 mu.  The return paths cancel, (1 - g)(1 + g) = 0,
    and x -> x + mu -> x + 2 mu carries (1/2 (1 - g_mu))^2 = (1 - g_mu) / 2.
    On coarse plane waves (spacing 2, antiperiodic in t) this is
        d - (1/d) sum_mu (cos k_mu - i g_mu sin k_mu),
    with eigenvalues d - (sum cos k)/d +- i sqrt(sum sin^2 k)/d, six-fold."""
    import itertools

    lc = [L // 2 for L in dims]
    ax = [2 * np.pi * np.arange(L) / L for L in lc[:3]]
    ax.append(2 * np.pi * (np.arange(lc[3]) + 0.5) / lc[3])
    d = 4 + m0
    ev = []
    for k in itertools.product(*ax):
        k = np.array(k)
        a = d - np.cos(k).sum() / d
        s = np.sqrt((np.sin(k) ** 2).sum()) / d
        ev += [a + 1j * s] * 6 + [a - 1j * s] * 6
    return np.array(ev)


def test_diag_schur_free_field_closed_form(free_links_4):
    from test_oracle_pins import same_multiset

    d = dense.wilson_dense(free_links_4, DIMS, 0.1)
    q, nb = dense.permutation_block(DIMS, "I")
    s0 = dense.diag_schur_dense(d, q, nb)
    ok, worst = same_multiset(np.linalg.eigvals(s0), free_diag_schur_type1_spectrum(DIMS, 0.1), 1e-10)
    assert ok, worst


def test_diag_schur_gauge_covariant_and_exact_for_diagonal_drr(wilson):
    from test_oracle_pins import gauge_transform, random_omega

    links, d = wilson
    q, nb = dense.permutation_block(DIMS, "II", True)
    s0 = dense.diag_schur_dense(d, q, nb)
    om = random_omega(256, 6)
    d2 = dense.wilson_dense(gauge_transform(links, om, DIMS), DIMS, 0.1)
    s2 = dense.diag_schur_dense(d2, q, nb)
    ob = np.zeros_like(s0)
    for k in range(nb):
        ob[12 * k:12 * k + 12, 12 * k:12 * k + 12] = np.kron(np.eye(4), om[q[k]])
    assert np.abs(s2 - ob @ s0 @ ob.conj().T).max() < 1e-12
    # with the couplings inside D_rr removed, the exact complement, the
    # second-order approximation and this one coincide
    o = dense.dof_order(q)
    r = o[12 * nb:]
    dm = d.copy()
    dm[np.ix_(r, r)] = np.diag(np.diag(dm[np.ix_(r, r)]))
    s = dense.schur_dense(dm, q, nb)
    assert np.abs(dense.diag_schur_dense(dm, q, nb) - s).max() <= 1e-13 * np.abs(s).max()


@pytest.mark.parametrize("kind,inv", [("I", False), ("II", False), ("I", True), ("II", True)])
def test_diag_schur_matrix_free_equals_dense(wilson, kind, inv):
    links, d = wilson
    q, nb = dense.permutation_block(DIMS, kind, inv)
    xb = gaussian_vectors(12 * nb, 2, 6)
    want = (dense.diag_schur_dense(d, q, nb) @ xb.T).T
    got = matfree.diag_schur_apply(links, DIMS, 0.1, q, nb, xb)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("kind", ["I", "II"])
def test_second_order_term_vanishes_on_the_all_even_coarse_set(wilson, kind):
    """From a coarse site with all coordinates even, D_rb reaches sites with
    one odd coordinate and a hop inside D_rr sites with two, one hop from no
    coarse site: D_br (d - D_rr) X D_rb = 0 for any diagonal X, so the
    second-order approximation equals the diagonal one there; on the
    inverse permutations it does not."""
    _, d = wilson
    q, nb = dense.permutation_block(DIMS, kind)
    s0 = dense.diag_schur_dense(d, q, nb)
    assert np.abs(dense.reusken_dense(d, q, nb) - s0).max() <= 1e-13 * np.abs(s0).max()
    qi, nbi = dense.permutation_block(DIMS, kind, True)
    gap = np.abs(dense.reusken_dense(d, qi, nbi) - dense.diag_schur_dense(d, qi, nbi)).max()
    assert gap > 1e-3
