"""Pins of the dense oracle O1 against facts fixed by the paper and by textbook
mathematics (not by the oracle itself).

* gamma algebra of the DeGrand-Rossi basis;
* closed-form free-field spectrum and plane-wave symbol of the Wilson operator;
* gamma_5-hermiticity and gauge covariance of D with random links;
* permutation orthogonality, the coarse sets of Type I/II (brute force) and a
  hand-derived fixture for the inverse permutations;
* the Schur complement identities of section 1: S_bb^{-1} = (D^{-1})_bb,
  det D = det S_bb det D_rr, the block-UL factorisation, and the general
  Gaussian-integration form with the blocking kernels B, Bbar;
* a closed-form free-field spectrum of the Type I coarse operator;
* planted mistakes in the oracle that these pins must catch.
"""
import itertools
import os

import numpy as np
import pytest

from grg_inputs import su3_links, gaussian_vectors
from oracle import dense

DIMS = (4, 4, 4, 4)
M0 = 0.1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_gammas():
    """The DeGrand-Rossi table from tests/golden (independent of the oracle's)."""
    rows = {"x": [], "y": [], "z": [], "t": []}
    with open(os.path.join(GOLDEN, "degrand_rossi_gammas.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *vals = line.split()
                rows[k].append([complex(v) for v in vals])
    return np.array([rows[k] for k in "xyzt"], dtype=np.complex128)


# ------------------------------------------------------------------ helpers
def free_spectrum(dims, m0, bc=(1, 1, 1, -1)):
    """Eigenvalues of the free Wilson operator (U = 1) with boundary signs bc
    (the default: periodic x, y, z and antiperiodic t): (4 + m0 - sum cos p)
    +- i sqrt(sum sin^2 p), each six-fold, with p_mu = 2 pi (n + theta_mu) /
    L_mu, theta_mu = 0 for a periodic and 1/2 for an antiperiodic extent."""
    ax = [2 * np.pi * (np.arange(L) + (0.5 if b < 0 else 0.0)) / L for L, b in zip(dims, bc)]
    ev = []
    for p in itertools.product(*ax):
        p = np.array(p)
        a = 4 + m0 - np.cos(p).sum()
        s = np.sqrt((np.sin(p) ** 2).sum())
        ev += [a + 1j * s] * 6 + [a - 1j * s] * 6
    return np.array(ev)


def free_schur_type1_spectrum(dims, m0):
    """Eigenvalues of S_bb for U = 1 and the all-even coarse sublattice.

    S_bb^{-1} = (D^{-1})_bb; on the coarse lattice (spacing 2) the fine
    propagator aliases to G(P) = 1/16 sum_{n in {0,1}^4} D(P/2 + pi n)^{-1}.
    With a_n = 4 + m0 - sum (-1)^{n_mu} cos(P_mu/2), s^2 = sum sin^2(P_mu/2),
    G = alpha - i sum gamma_mu beta_mu with alpha = <a_n/(a_n^2+s^2)>_n and
    beta_mu = sin(P_mu/2) <(-1)^{n_mu}/(a_n^2+s^2)>_n, so the eigenvalues of
    S_bb are (alpha +- i|beta|)/(alpha^2 + |beta|^2), each six-fold.
    """
    lc = [d // 2 for d in dims]
    ax = [2 * np.pi * np.arange(L) / L for L in lc[:3]]
    ax.append(2 * np.pi * (np.arange(lc[3]) + 0.5) / lc[3])
    ns = np.array(list(itertools.product((0, 1), repeat=4)))
    sg = (-1.0) ** ns
    ev = []
    for P in itertools.product(*ax):
        h = np.array(P) / 2
        a = 4 + m0 - (sg * np.cos(h)).sum(axis=1)
        s2 = (np.sin(h) ** 2).sum()
        den = a ** 2 + s2
        alpha = np.mean(a / den)
        beta = np.sin(h) * np.mean(sg / den[:, None], axis=0)
        nb = np.linalg.norm(beta)
        lam = (alpha + 1j * nb) / (alpha ** 2 + nb ** 2)
        ev += [lam] * 6 + [np.conj(lam)] * 6
    return np.array(ev)


def same_multiset(a, b, tol):
    """Compare two complex multisets by greedy nearest matching."""
    a = list(np.asarray(a))
    b = np.asarray(b).copy()
    used = np.zeros(len(b), bool)
    worst = 0.0
    assert len(a) == len(b)
    for z in a:
        d = np.abs(b - z)
        d[used] = np.inf
        k = int(np.argmin(d))
        used[k] = True
        worst = max(worst, d[k])
    return worst <= tol, worst


def logdet(m):
    sign, ld = np.linalg.slogdet(m)
    return np.log(sign) + ld


def random_omega(v, seed):
    return su3_links((v, 1, 1, 1), 1.0, seed)[:, 0]


def gauge_transform(links, omega, dims):
    out = np.empty_like(links)
    v = len(links)
    for s in range(v):
        for mu in range(4):
            c = list(dense.coords(s, dims))
            c[mu] = (c[mu] + 1) % dims[mu]
            sp = dense.site(c, dims)
            out[s, mu] = omega[s] @ links[s, mu] @ omega[sp].conj().T
    return out


def site_local(op_per_site, v):
    """Block-diagonal matrix with one 12x12 block per site."""
    n = 12 * v
    m = np.zeros((n, n), dtype=np.complex128)
    for s in range(v):
        m[12 * s:12 * s + 12, 12 * s:12 * s + 12] = op_per_site(s)
    return m


# ------------------------------------------------------------------ fixtures
@pytest.fixture(scope="module")
def links():
    return su3_links(DIMS, 0.4, 1)


@pytest.fixture(scope="module")
def dmat(links):
    return dense.wilson_dense(links, DIMS, M0)


@pytest.fixture(scope="module")
def dinv(dmat):
    return np.linalg.inv(dmat)


@pytest.fixture(scope="module")
def dfree(free_links_4):
    return dense.wilson_dense(free_links_4, DIMS, M0)


PERMS = [("I", False), ("II", False), ("I", True), ("II", True)]


# ------------------------------------------------------------------ gamma basis
def test_gamma_table_is_degrand_rossi():
    assert np.array_equal(dense.GAMMA, golden_gammas())


def test_gamma_algebra():
    g = golden_gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * np.eye(4) * (mu == nu))
    assert np.allclose(g[0] @ g[1] @ g[2] @ g[3], np.diag([1, 1, -1, -1]))


def test_links_special_unitary(links):
    u = links.reshape(-1, 3, 3)
    assert np.abs(u @ u.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14


# ------------------------------------------------------------------ Wilson D
def test_free_field_spectrum(dfree):
    ok, worst = same_multiset(np.linalg.eigvals(dfree), free_spectrum(DIMS, M0), 1e-9)
    assert ok, worst


def check_plane_wave(d, dims, m0):
    """D (e^{ipx} chi) = e^{ipx} D(p) chi with D(p) = (4 + m0 - sum cos p)
    + i sum gamma_mu sin p_mu, for the free field."""
    v = int(np.prod(dims))
    gam = golden_gammas()
    rng = np.random.default_rng(7)
    cs = np.array([dense.coords(s, dims) for s in range(v)])
    worst = 0.0
    for n in [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (1, 2, 3, 0), (3, 1, 2, 1)]:
        p = np.array([2 * np.pi * n[mu] / dims[mu] for mu in range(3)]
                     + [2 * np.pi * (n[3] + 0.5) / dims[3]])
        chi = rng.standard_normal(12) + 1j * rng.standard_normal(12)
        phase = np.exp(1j * cs @ p)
        psi = (phase[:, None] * chi[None, :]).reshape(-1)
        dp = (4 + m0 - np.cos(p).sum()) * np.eye(12)
        for mu in range(4):
            dp = dp + 1j * np.sin(p[mu]) * np.kron(gam[mu], np.eye(3))
        want = (phase[:, None] * (dp @ chi)[None, :]).reshape(-1)
        worst = max(worst, np.abs(d @ psi - want).max())
    return worst


def test_free_field_plane_wave(dfree):
    assert check_plane_wave(dfree, DIMS, M0) < 1e-12


@pytest.mark.parametrize("bc", [(-1, 1, -1, 1), (1, -1, -1, -1), (1, 1, 1, 1)])
def test_free_field_spectrum_boundary_signs(bc):
    """Other boundary signs: the momenta shift by half a unit exactly in the
    antiperiodic directions, for the dense operator and the C stencil."""
    from oracle import matfree

    dims = (2, 4, 2, 4)
    v = int(np.prod(dims))
    free = np.broadcast_to(np.eye(3, dtype=np.complex128), (v, 4, 3, 3)).copy()
    d = dense.wilson_dense(free, dims, M0, bc=bc)
    ok, worst = same_multiset(np.linalg.eigvals(d), free_spectrum(dims, M0, bc), 1e-9)
    assert ok, worst
    # the same matrix from the C stencil, column by column
    cols = matfree.dirac_apply(free, dims, M0, np.eye(12 * v, dtype=np.complex128), bc)
    assert np.abs(cols.T - d).max() < 1e-14
    # and the pin tells the boundary signs apart
    other = tuple(-b if k == 0 else b for k, b in enumerate(bc))
    assert not same_multiset(np.linalg.eigvals(d), free_spectrum(dims, M0, other), 1e-6)[0]


@pytest.mark.parametrize("dims", [(1, 4, 3, 2), (2, 1, 2, 3), (3, 2, 1, 1), (2, 2, 2, 2)])
def test_free_field_plane_wave_small_extents(dims):
    """Extents of one and two, where the forward and backward neighbours of
    a site coincide (and with one, are the site itself): the plane-wave
    symbol still holds, for the dense operator and the C stencil alike."""
    from oracle import matfree

    v = int(np.prod(dims))
    free = np.broadcast_to(np.eye(3, dtype=np.complex128), (v, 4, 3, 3)).copy()
    d = dense.wilson_dense(free, dims, M0)
    assert check_plane_wave(d, dims, M0) < 1e-12
    x = gaussian_vectors(12 * v, 2, 5)
    assert np.abs(matfree.dirac_apply(free, dims, M0, x) - (d @ x.T).T).max() < 1e-13


def test_gamma5_hermiticity(dmat):
    v = 256
    g5 = site_local(lambda s: np.kron(np.diag([1, 1, -1, -1]), np.eye(3)), v)
    assert np.abs(g5 @ dmat @ g5 - dmat.conj().T).max() < 1e-14


def test_gauge_covariance(links, dmat):
    om = random_omega(256, 99)
    d2 = dense.wilson_dense(gauge_transform(links, om, DIMS), DIMS, M0)
    big = site_local(lambda s: np.kron(np.eye(4), om[s]), 256)
    assert np.abs(d2 - big @ dmat @ big.conj().T).max() < 1e-13


# ------------------------------------------------------------------ permutations
@pytest.mark.parametrize("kind,inv", PERMS)
def test_permutation_orthogonal(kind, inv):
    q, nb = dense.permutation_block(DIMS, kind, inv)
    assert nb == 16 and sorted(q) == list(range(256))
    p = dense.permutation_matrix(q)
    assert np.allclose(p @ p.T, np.eye(256))
    qf, _ = dense.permutation_block(DIMS, kind, False)
    # the inverse ordering's operator is the transpose of the forward one
    if inv:
        assert np.allclose(p, dense.permutation_matrix(qf).T)


def test_coarse_sets_forward_brute_force():
    v = 256
    even = [s for s in range(v) if all(c % 2 == 0 for c in dense.coords(s, DIMS))]
    qi, nb = dense.permutation_block(DIMS, "I")
    qii, _ = dense.permutation_block(DIMS, "II")
    assert list(qi[:nb]) == even
    assert list(qii[:nb]) == even
    # Type II: r-sites ordered by the first odd direction, x-odd sites last
    x_odd = [s for s in range(v) if dense.coords(s, DIMS)[0] % 2 == 1]
    assert list(qii[-len(x_odd):]) == x_odd


def test_coarse_sets_inverse_golden():
    want = {}
    with open(os.path.join(GOLDEN, "inverse_bsets_4x4x4x4.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *vals = line.split()
                want[k] = sorted(int(x) for x in vals)
    qi, nb = dense.permutation_block(DIMS, "I", True)
    qii, _ = dense.permutation_block(DIMS, "II", True)
    assert sorted(qi[:nb]) == want["I_inv"]
    assert sorted(qii[:nb]) == want["II_inv"]


def test_odd_extent_rejected():
    with pytest.raises(ValueError):
        dense.permutation_block((4, 4, 4, 3), "I")


# ------------------------------------------------------------------ Schur complement
@pytest.mark.parametrize("kind,inv", PERMS)
def test_schur_inverse_is_block_of_inverse(dmat, dinv, kind, inv):
    q, nb = dense.permutation_block(DIMS, kind, inv)
    s = dense.schur_dense(dmat, q, nb)
    o = dense.dof_order(q)[: 12 * nb]
    ginv = dinv[np.ix_(o, o)]
    assert np.abs(s @ ginv - np.eye(12 * nb)).max() < 1e-12


@pytest.mark.parametrize("kind,inv", PERMS)
def test_determinant_factorisation(dmat, kind, inv):
    q, nb = dense.permutation_block(DIMS, kind, inv)
    s = dense.schur_dense(dmat, q, nb)
    _, _, _, drr = dense.blocks(dmat, q, nb)
    ld = logdet(dmat)
    diff = logdet(s) + logdet(drr) - ld
    phase = (diff.imag + np.pi) % (2 * np.pi) - np.pi
    assert abs(diff.real) < 1e-10 * abs(ld.real)
    assert abs(phase) < 1e-9


@pytest.mark.parametrize("kind,inv", PERMS)
def test_block_ul(dmat, kind, inv):
    q, nb = dense.permutation_block(DIMS, kind, inv)
    s = dense.schur_dense(dmat, q, nb)
    dbb, dbr, drb, drr = dense.blocks(dmat, q, nb)
    n, k = dmat.shape[0], 12 * nb
    upper = np.eye(n, dtype=np.complex128)
    upper[:k, k:] = dbr @ np.linalg.inv(drr)
    lower = np.zeros((n, n), dtype=np.complex128)
    lower[:k, :k] = s
    lower[k:, :k] = drb
    lower[k:, k:] = drr
    o = dense.dof_order(q)
    assert np.abs(upper @ lower - dmat[np.ix_(o, o)]).max() < 1e-12


@pytest.mark.parametrize("kind,inv", [("I", False), ("I", True)])
def test_gaussian_rg_form_reduces_to_schur(dmat, kind, inv):
    q, nb = dense.permutation_block(DIMS, kind, inv)
    s_rg, dt = dense.schur_gaussian_rg(dmat, q, nb)
    s = dense.schur_dense(dmat, q, nb)
    assert np.abs(s_rg - s).max() < 1e-11
    dbb, _, _, drr = dense.blocks(dmat, q, nb)
    a, b = logdet(dt), logdet(dbb) + logdet(drr)
    assert abs(a.real - b.real) < 1e-10 * abs(a.real)


def test_type1_dbb_is_diagonal(dmat):
    q, nb = dense.permutation_block(DIMS, "I")
    dbb, _, _, _ = dense.blocks(dmat, q, nb)
    assert np.abs(dbb - (4 + M0) * np.eye(12 * nb)).max() == 0.0


def test_free_field_schur_type1_spectrum(dfree):
    q, nb = dense.permutation_block(DIMS, "I")
    s = dense.schur_dense(dfree, q, nb)
    ok, worst = same_multiset(np.linalg.eigvals(s), free_schur_type1_spectrum(DIMS, M0), 1e-10)
    assert ok, worst


def test_schur_gamma5_hermitian_and_gauge_covariant(links, dmat):
    q, nb = dense.permutation_block(DIMS, "II", True)
    s = dense.schur_dense(dmat, q, nb)
    g5 = np.kron(np.eye(nb), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    assert np.abs(g5 @ s @ g5 - s.conj().T).max() < 1e-12
    om = random_omega(256, 5)
    d2 = dense.wilson_dense(gauge_transform(links, om, DIMS), DIMS, M0)
    s2 = dense.schur_dense(d2, q, nb)
    ob = np.zeros_like(s)
    for k in range(nb):
        ob[12 * k:12 * k + 12, 12 * k:12 * k + 12] = np.kron(np.eye(4), om[q[k]])
    assert np.abs(s2 - ob @ s @ ob.conj().T).max() < 1e-12


# ------------------------------------------------------------------ planted mistakes
def test_pins_catch_planted_mistakes(monkeypatch, free_links_4, links, dmat):
    """Each plausible mistake planted in the oracle must fail at least one pin."""
    # (1) sign of the hopping term flipped -> plane-wave symbol.  (The free
    #     spectrum alone cannot see it: on a lattice with even extents the
    #     staggered sign (-1)^(x+y+z+t) maps one sign onto the other.)
    d = dense.wilson_dense(free_links_4, DIMS, M0)
    d_flip = 2 * (4 + M0) * np.eye(d.shape[0]) - d
    assert check_plane_wave(d_flip, DIMS, M0) > 1e-3
    # (2) antiperiodic boundary dropped -> free spectrum
    d_per = dense.wilson_dense(free_links_4, DIMS, M0, bc=(1, 1, 1, 1))
    assert not same_multiset(np.linalg.eigvals(d_per), free_spectrum(DIMS, M0), 1e-6)[0]
    # (3) 1 - gamma and 1 + gamma exchanged in one direction -> plane-wave symbol
    g = dense.GAMMA.copy()
    g[2] = -g[2]
    monkeypatch.setattr(dense, "GAMMA", g)
    assert check_plane_wave(dense.wilson_dense(free_links_4, DIMS, M0), DIMS, M0) > 1e-3
    monkeypatch.undo()
    # (4) transposed link operand -> gauge covariance
    lt = links.transpose(0, 1, 3, 2)
    om = random_omega(256, 99)
    big = site_local(lambda s: np.kron(np.eye(4), om[s]), 256)
    dt = dense.wilson_dense(lt, DIMS, M0)
    dt2 = dense.wilson_dense(gauge_transform(links, om, DIMS).transpose(0, 1, 3, 2), DIMS, M0)
    assert np.abs(dt2 - big @ dt @ big.conj().T).max() > 1e-3
    # (5) backward hop dropped -> gamma5-hermiticity
    real_hop = dense.hop

    def hop_fwd_only(s, mu, step, dims, bc):
        n, sgn = real_hop(s, mu, step, dims, bc)
        return n, (sgn if step > 0 else 0.0)

    monkeypatch.setattr(dense, "hop", hop_fwd_only)
    d_half = dense.wilson_dense(links, DIMS, M0)
    monkeypatch.undo()
    g5 = site_local(lambda s: np.kron(np.diag([1, 1, -1, -1]), np.eye(3)), 256)
    assert np.abs(g5 @ d_half @ g5 - d_half.conj().T).max() > 1e-3
    # (6) Schur complement with D_br and D_rb exchanged (transposed operands)
    #     -> S^{-1} = (D^{-1})_bb
    q, nb = dense.permutation_block(DIMS, "I", True)
    dbb, dbr, drb, drr = dense.blocks(dmat, q, nb)
    bad = dbb - drb.T @ np.linalg.solve(drr, dbr.T)
    o = dense.dof_order(q)[: 12 * nb]
    ginv = np.linalg.inv(dmat)[np.ix_(o, o)]
    assert np.abs(bad @ ginv - np.eye(12 * nb)).max() > 1e-3
