"""Pins of the V-cycle oracle (section 4).

* The level operator defined by block elimination with the couplings inside
  the rest block ignored equals the coarse-lattice Wilson form
  (1/d) D_W(V, d^2 - 4), V_mu(c) = U_mu(2c) U_mu(2c + mu): two independent
  routes (probing and masks on the fine operator, against a Wilson operator on
  blocked links), so a wrong link product, boundary sign, mass or scale fails.
* With the exact Schur complement on the top level, one cycle is the exact
  inverse (the block LU of section 1): D cycle(f) = f.
* Whatever the top level, the rest rows of D cycle(f) - f vanish (x_r solves
  them exactly), and the coarse rows carry (S - S0) x_b."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors, su3_links
from oracle import dense, matfree, vcycle

pytestmark = pytest.mark.slow

DIMS = (8, 8, 8, 8)
M0 = -0.4


@pytest.fixture(scope="module")
def links():
    return su3_links(DIMS, 0.5, 41)


def test_level_one_is_the_coarse_wilson_operator(links):
    lv = vcycle.hierarchy(links, DIMS, M0, 2)
    x = gaussian_vectors(12 * lv[1].n, 2, 41)
    for v in x:
        got = lv[1].apply(v)
        want = vcycle.coarse_wilson_apply(links, DIMS, M0, v[None, :])[0]
        assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
        # and the same as the oracle's approximation that ignores D_rr's couplings
        q, nb = dense.permutation_block(DIMS, "I")
        alt = matfree.diag_schur_apply(links, DIMS, M0, q, nb, v[None, :])[0]
        assert np.linalg.norm(got - alt) <= 1e-12 * np.linalg.norm(alt)


@pytest.mark.parametrize("bc", [(-1, 1, -1, 1), (1, -1, 1, 1)])
def test_level_one_other_boundary_signs(bc):
    """With other boundary signs the blocked operator is the coarse Wilson
    form with the same signs (a coarse hop wraps exactly when a fine one
    does)."""
    dims = (4, 4, 8, 4)
    lk = su3_links(dims, 0.5, 43)
    lv = vcycle.hierarchy(lk, dims, M0, 2, bc)
    x = gaussian_vectors(12 * lv[1].n, 1, 43)[0]
    want = vcycle.coarse_wilson_apply(lk, dims, M0, x[None, :], bc)[0]
    assert np.linalg.norm(lv[1].apply(x) - want) <= 1e-12 * np.linalg.norm(want)
    # not the form with the default signs
    dflt = vcycle.coarse_wilson_apply(lk, dims, M0, x[None, :])[0]
    assert np.linalg.norm(lv[1].apply(x) - dflt) > 1e-3 * np.linalg.norm(want)


def test_level_two_is_the_twice_blocked_wilson_operator(links):
    lv = vcycle.hierarchy(links, DIMS, M0, 3)
    d0 = 4 + M0
    cd = tuple(L // 2 for L in DIMS)
    links1 = vcycle.block_links(links, DIMS)
    x = gaussian_vectors(12 * lv[2].n, 1, 42)[0]
    # A_2 = (1/d0) * (1/d1) D_W(V2, d1^2 - 4) with d1 = 4 + m1 = d0^2, periodic
    # coarse boundary handled by the same bc on every level
    want = vcycle.coarse_wilson_apply(links1, cd, d0 * d0 - 4, x[None, :])[0] / d0
    got = lv[2].apply(x)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


def test_cycle_with_the_exact_complement_inverts_d(links):
    dims = (4, 4, 4, 4)
    lk = su3_links(dims, 0.5, 43)
    lv = vcycle.hierarchy(lk, dims, M0, 2)
    q, nb = dense.permutation_block(dims, "I")
    lv[1].apply = lambda xb: matfree.schur_apply(lk, dims, M0, q, nb, xb[None, :], restart=8, tol=1e-14)[0][0]
    f = gaussian_vectors(12 * lv[0].n, 1, 43)[0]
    x = vcycle.cycle(lv, 0, f)
    r = matfree.dirac_apply(lk, dims, M0, x[None, :])[0] - f
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(f)


def test_cycle_solves_the_rest_rows_exactly(links):
    lv = vcycle.hierarchy(links, DIMS, M0, 2)
    f = gaussian_vectors(12 * lv[0].n, 1, 44)[0]
    x = vcycle.cycle(lv, 0, f)
    r = (matfree.dirac_apply(links, DIMS, M0, x[None, :])[0] - f).reshape(lv[0].n, 12)
    assert np.linalg.norm(r[lv[0].rest]) <= 1e-11 * np.linalg.norm(f)
    # the coarse rows do not vanish: S0 is an approximation
    assert np.linalg.norm(r[~lv[0].rest]) > 1e-3 * np.linalg.norm(f)


# ---------------------------------------------------------------- two levels on any ordering
# Type I, II and their inverses (section 2) at kappa = 1/6 (m0 = -1), 4^4:
# the dense operator is small enough to take every block by LU.
PERMS = [("I", False), ("I", True), ("II", False), ("II", True)]
DIMS4 = (4, 4, 4, 4)
M1 = -1.0


@pytest.fixture(scope="module")
def small():
    lk = su3_links(DIMS4, 0.5, 51)
    return lk, dense.wilson_dense(lk, DIMS4, M1)


@pytest.mark.parametrize("kind,inv", PERMS)
def test_two_level_cycle_with_the_exact_complement_inverts_d(small, kind, inv):
    """Exact S_bb on top: the cycle is the block LU solve of section 1, in
    both the matrix-free and the dense form."""
    lk, d = small
    q, nb = dense.permutation_block(DIMS4, kind, inv)
    f = gaussian_vectors(12 * 256, 1, 52)[0]
    x = vcycle.two_level_cycle(lk, DIMS4, M1, q, nb, f, top="exact")
    assert np.linalg.norm(d @ x - f) <= 1e-10 * np.linalg.norm(f)
    xd = vcycle.two_level_cycle_dense(d, q, nb, f, top="exact")
    assert np.linalg.norm(d @ xd - f) <= 1e-11 * np.linalg.norm(f)


@pytest.mark.parametrize("kind,inv", PERMS)
def test_two_level_cycle_matches_the_dense_cycle(small, kind, inv):
    """Section 3's S~_bb on top: the matrix-free cycle (stencil blocks,
    GCR) against the dense one (explicit blocks, LU)."""
    lk, d = small
    q, nb = dense.permutation_block(DIMS4, kind, inv)
    f = gaussian_vectors(12 * 256, 1, 53)[0]
    x = vcycle.two_level_cycle(lk, DIMS4, M1, q, nb, f)
    xd = vcycle.two_level_cycle_dense(d, q, nb, f)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


@pytest.mark.parametrize("kind,inv", PERMS)
def test_two_level_cycle_residual_is_the_complement_error(small, kind, inv):
    """With exact rest solves the residual of one cycle vanishes on the rest
    rows, and on the coarse rows it is (S_bb - S~_bb) x_b: the error of the
    approximation alone."""
    lk, d = small
    q, nb = dense.permutation_block(DIMS4, kind, inv)
    f = gaussian_vectors(12 * 256, 1, 54)[0]
    x = vcycle.two_level_cycle_dense(d, q, nb, f)
    o = dense.dof_order(q)
    r = d @ x - f
    assert np.linalg.norm(r[o[12 * nb:]]) <= 1e-11 * np.linalg.norm(f)
    xb = x[o[: 12 * nb]]
    want = (dense.schur_dense(d, q, nb) - dense.reusken_dense(d, q, nb)) @ xb
    assert np.linalg.norm(r[o[: 12 * nb]] - want) <= 1e-10 * np.linalg.norm(want)
    assert np.linalg.norm(want) > 1e-3 * np.linalg.norm(f)  # an approximation, not the exact complement
