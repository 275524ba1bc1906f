"""The matrix-free C oracle (O2) against the dense oracle (O1), which is pinned
in test_oracle_pins.py: full D, the four sub-blocks, the D_rr solve and the
Schur-complement apply, on 4^4 and 4^3 x 8 lattices."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors, su3_links
from oracle import dense, matfree

PERMS = [("I", False), ("II", False), ("I", True), ("II", True)]


@pytest.fixture(scope="module")
def setup4():
    dims = (4, 4, 4, 4)
    u = su3_links(dims, 0.4, 1)
    return dims, u, dense.wilson_dense(u, dims, 0.1)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 4, 4, 8), (4, 2, 6, 4)])
def test_dirac_apply_vs_dense(dims):
    u = su3_links(dims, 0.5, 11)
    d = dense.wilson_dense(u, dims, -0.2)
    v = int(np.prod(dims))
    x = gaussian_vectors(12 * v, 3, 11)
    y = matfree.dirac_apply(u, dims, -0.2, x)
    assert np.abs(y - (d @ x.T).T).max() < 1e-13 * np.abs(y).max()


@pytest.mark.parametrize("kind,inv", PERMS)
def test_block_apply_vs_dense(setup4, kind, inv):
    dims, u, d = setup4
    q, nb = dense.permutation_block(dims, kind, inv)
    x = gaussian_vectors(12 * 256, 2, 3)
    mask = np.zeros(256, bool)
    mask[q[:nb]] = True
    dmask = np.repeat(mask, 12)
    for osel in (0, 1):
        for isel in (0, 1):
            want = d.copy()
            want[dmask != bool(osel), :] = 0
            want[:, dmask != bool(isel)] = 0
            got = matfree.block_apply(u, dims, 0.1, q, nb, osel, isel, x)
            assert np.abs(got - (want @ x.T).T).max() < 1e-13 * max(1.0, np.abs(got).max())


@pytest.mark.parametrize("kind,inv", PERMS)
def test_drr_solve_vs_dense(setup4, kind, inv):
    dims, u, d = setup4
    q, nb = dense.permutation_block(dims, kind, inv)
    _, _, _, drr = dense.blocks(d, q, nb)
    o = dense.dof_order(q)[12 * nb:]
    b = np.zeros((2, 12 * 256), np.complex128)
    b[:, o] = gaussian_vectors(len(o), 2, 4)
    x, it, rr = matfree.drr_solve(u, dims, 0.1, q, nb, b, restart=8, tol=1e-13)
    assert (rr <= 1e-13).all() and (it > 0).all()
    xd = np.linalg.solve(drr, b[:, o].T).T
    assert np.abs(x[:, o] - xd).max() < 1e-11 * np.abs(xd).max()
    # nothing leaks onto coarse sites
    ob = dense.dof_order(q)[: 12 * nb]
    assert np.abs(x[:, ob]).max() == 0.0
    rr2 = matfree.drr_residual(u, dims, 0.1, q, nb, b, x)
    assert np.allclose(rr, rr2, rtol=1e-6, atol=1e-16)


@pytest.mark.parametrize("kind,inv", PERMS)
@pytest.mark.parametrize("restart", [1, 8])
def test_schur_apply_vs_dense(setup4, kind, inv, restart):
    dims, u, d = setup4
    q, nb = dense.permutation_block(dims, kind, inv)
    s = dense.schur_dense(d, q, nb)
    xb = gaussian_vectors(12 * nb, 2, 1)
    yb, it, rr = matfree.schur_apply(u, dims, 0.1, q, nb, xb, restart=restart, tol=1e-13)
    want = (s @ xb.T).T
    err = np.linalg.norm(yb - want, axis=1) / np.linalg.norm(want, axis=1)
    assert err.max() < 1e-11, err


def test_restart_does_not_change_the_answer(setup4):
    dims, u, d = setup4
    q, nb = dense.permutation_block(dims, "I")
    xb = gaussian_vectors(12 * nb, 1, 9)
    y1, _, _ = matfree.schur_apply(u, dims, 0.1, q, nb, xb, restart=1, tol=1e-13)
    y2, _, _ = matfree.schur_apply(u, dims, 0.1, q, nb, xb, restart=16, tol=1e-13)
    assert np.linalg.norm(y1 - y2) < 1e-11 * np.linalg.norm(y1)


@pytest.mark.parametrize("kind,inv", PERMS)
@pytest.mark.parametrize("parity", [0, 1])
def test_reduced_apply_is_dense_schur_complement(setup4, kind, inv, parity):
    """The even-odd reduced operator against the Schur complement of the
    dense D_rr on the two parities' rest sites, D_pp - D_pq D_qq^{-1} D_qp,
    with D_qq inverted as a matrix (nothing assumed about its form)."""
    dims, u, d = setup4
    q, nb = dense.permutation_block(dims, kind, inv)
    rest = np.ones(256, bool)
    rest[q[:nb]] = False
    par = np.array([sum(dense.coords(s, dims)) % 2 for s in range(256)])
    ip = np.flatnonzero(np.repeat(rest & (par == parity), 12))
    iq = np.flatnonzero(np.repeat(rest & (par != parity), 12))
    a = d[np.ix_(ip, ip)] - d[np.ix_(ip, iq)] @ np.linalg.solve(d[np.ix_(iq, iq)], d[np.ix_(iq, ip)])
    x = gaussian_vectors(12 * 256, 2, 5)
    got = matfree.reduced_apply(u, dims, 0.1, q, nb, parity, x)
    want = np.zeros_like(x)
    want[:, ip] = (a @ x[:, ip].T).T
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("kind,inv", PERMS)
def test_drr_residual_vs_dense(setup4, kind, inv):
    """The residual routine on an arbitrary x (not a solver iterate) against
    ||b - D_rr x|| / ||b|| formed from the dense blocks, and a zero b."""
    dims, u, d = setup4
    q, nb = dense.permutation_block(dims, kind, inv)
    _, _, _, drr = dense.blocks(d, q, nb)
    o = dense.dof_order(q)[12 * nb:]
    b = np.zeros((3, 12 * 256), np.complex128)
    x = np.zeros_like(b)
    b[:, o] = gaussian_vectors(len(o), 3, 5)
    x[:, o] = gaussian_vectors(len(o), 3, 6) * np.array([1e-3, 0.3, 1.0])[:, None]
    got = matfree.drr_residual(u, dims, 0.1, q, nb, b, x)
    want = np.linalg.norm(b[:, o] - (drr @ x[:, o].T).T, axis=1) / np.linalg.norm(b[:, o], axis=1)
    assert np.allclose(got, want, rtol=1e-13, atol=0)
    # entries of x on coarse sites are outside D_rr's columns: ignored
    x2 = x.copy()
    x2[:, dense.dof_order(q)[: 12 * nb]] = 7.0
    assert np.allclose(matfree.drr_residual(u, dims, 0.1, q, nb, b, x2), want, rtol=1e-13, atol=0)
    # zero right-hand side: the absolute residual
    z = matfree.drr_residual(u, dims, 0.1, q, nb, np.zeros_like(b[:1]), x[:1])
    assert np.isclose(z[0], np.linalg.norm((drr @ x[0, o])), rtol=1e-13)


@pytest.mark.parametrize("kind,inv", [("I", False), ("II", True)])
def test_drr_residual_vs_dense(setup4, kind, inv):
    """The oracle's residual ||b - D_rr x|| / ||b|| for an arbitrary x (not a
    solver's output) against the dense D_rr block: values on the coarse
    sites of x are not columns of D_rr and change nothing, and b = 0 gives
    the absolute norm ||D_rr x||."""
    dims, u, d = setup4
    q, nb = dense.permutation_block(dims, kind, inv)
    _, _, _, drr = dense.blocks(d, q, nb)
    o = dense.dof_order(q)[12 * nb:]
    ob = dense.dof_order(q)[: 12 * nb]
    b = np.zeros((3, 12 * 256), np.complex128)
    b[:2, o] = gaussian_vectors(len(o), 2, 21)
    x = np.zeros((3, 12 * 256), np.complex128)
    x[:, o] = gaussian_vectors(len(o), 3, 22)
    want = np.linalg.norm(b[:, o] - (drr @ x[:, o].T).T, axis=1)
    want[:2] /= np.linalg.norm(b[:2, o], axis=1)
    got = matfree.drr_residual(u, dims, 0.1, q, nb, b, x)
    assert np.allclose(got, want, rtol=1e-13, atol=0), (got, want)
    assert got.min() > 0.1  # not a solution: the comparison is of O(1) values
    x[:, ob] = gaussian_vectors(len(ob), 3, 23)
    assert np.allclose(matfree.drr_residual(u, dims, 0.1, q, nb, b, x), want, rtol=1e-13, atol=0)
