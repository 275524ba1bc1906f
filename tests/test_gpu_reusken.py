"""The second-order Schur complement approximation of section 3 on the GPU
against the oracle: dense at 4^4 for all four permutations, matrix-free at
larger volumes with several right-hand sides, and the clustering of the
spectrum of S~_bb^{-1} S_bb around one that section 4 uses it for; and the
approximation that ignores the couplings inside D_rr, dense and matrix-free,
with its free-field spectrum in closed form."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors
from oracle import dense, matfree

from gpu_support import Lattice, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

PERMS = [("I", False), ("II", False), ("I", True), ("II", True)]


@pytest.fixture(scope="module")
def small():
    lat = Lattice((4, 4, 4, 4), 0.4, 1)
    yield lat, dense.wilson_dense(lat.links, lat.dims, 0.1)
    lat.close()


@pytest.mark.parametrize("kind,inv", PERMS)
def test_dense_4x4x4x4(small, kind, inv):
    lat, d = small
    s = lat.schur(0.1, kind, inv, tol=1e-13, max_rhs=12)
    got = lat.grg.grg_reusken_assemble(s.h, s.nb)
    want = dense.reusken_dense(d, s.q, s.nb)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # section 4: the spectrum of S~^{-1} S clusters around one
    ex = lat.grg.grg_schur_assemble(s.h, s.nb)
    ev = np.linalg.eigvals(np.linalg.solve(got, ex))
    assert np.abs(ev - 1).max() < 0.25, np.abs(ev - 1).max()
    s.close()


@pytest.mark.parametrize("dims,kind,inv,nrhs", [((8, 8, 8, 8), "II", True, 4),
                                                ((8, 6, 4, 10), "I", False, 3),
                                                ((16, 16, 16, 16), "I", True, 12)])
def test_matrix_free(dims, kind, inv, nrhs):
    import torch

    lat = Lattice(dims, 0.5, 2)
    s = lat.schur(-0.2, kind, inv, max_rhs=nrhs)
    xb = gaussian_vectors(12 * s.nb, nrhs, 2)
    x = to_dev(xb)
    y = torch.empty_like(x)
    lat.grg.grg_reusken_apply(s.h, x, y, nrhs)
    got = to_host(y)
    sample = [0, nrhs - 1]
    want = matfree.reusken_apply(lat.links, dims, -0.2, s.q, s.nb, xb[sample])
    assert rel_err(got[sample], want) < 1e-12
    s.close()
    lat.close()


def test_new_gauge_field_recomputes_row_sums():
    """The row sums d~ = D_rr 1 are kept between applies: a new gauge field
    on the lattice must replace them (the apply after it matches the oracle
    on the new links, not the old)."""
    import torch

    from grg_inputs import su3_links

    dims, nrhs = (8, 8, 4, 8), 2
    lat = Lattice(dims, 0.5, 5)
    s = lat.schur(-0.2, "II", True, max_rhs=nrhs)
    xb = gaussian_vectors(12 * s.nb, nrhs, 6)
    x = to_dev(xb)
    y = torch.empty_like(x)
    lat.grg.grg_reusken_apply(s.h, x, y, nrhs)
    first = to_host(y)
    links2 = su3_links(dims, 0.5, 7)
    lat.grg.grg_gauge_set(lat.h, links2)
    lat.grg.grg_reusken_apply(s.h, x, y, nrhs)
    got = to_host(y)
    want = matfree.reusken_apply(links2, dims, -0.2, s.q, s.nb, xb)
    assert rel_err(got, want) < 1e-12
    assert rel_err(first, want) > 1e-3  # the field did change the operator
    s.close()
    lat.close()


def test_zero_diagonal_rejected():
    import torch

    lat = Lattice((4, 4, 4, 4), 0.4, 1)
    s = lat.schur(-4.0, "I", False, max_rhs=1)
    x = torch.zeros(12 * s.nb, dtype=torch.complex128, device="cuda")
    with pytest.raises(lat.grg.GrgError):
        lat.grg.grg_reusken_apply(s.h, x, torch.empty_like(x), 1)
    with pytest.raises(lat.grg.GrgError):
        lat.grg.grg_diag_schur_apply(s.h, x, torch.empty_like(x), 1)
    s.close()
    lat.close()


# ------------------------------------------------------------------ ignoring D_rr
@pytest.mark.parametrize("kind,inv", PERMS)
def test_diag_schur_dense_4x4x4x4(small, kind, inv):
    """D_bb - D_br D_rb / d assembled on the GPU against the dense oracle.
    On the all-even coarse set (Type I, and forward Type II, which has the
    same set) the second-order correction vanishes identically: D_rb lands on
    sites with one odd coordinate, a hop inside D_rr on sites with two, and no
    coarse site is one hop from those, so S~_bb = S0_bb there."""
    lat, d = small
    s = lat.schur(0.1, kind, inv, tol=1e-13, max_rhs=12)
    got = lat.grg.grg_diag_schur_assemble(s.h, s.nb)
    want = dense.diag_schur_dense(d, s.q, s.nb)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    if not inv:
        second = lat.grg.grg_reusken_assemble(s.h, s.nb)
        assert np.abs(second - got).max() <= 1e-12 * np.abs(got).max()
    s.close()


def test_diag_schur_free_field_spectrum():
    """Free field, Type I: the spectrum of the GPU-assembled operator against
    its closed form d - (sum cos k)/d +- i sqrt(sum sin^2 k)/d."""
    from test_oracle_pins import same_multiset
    from test_oracle_reusken import free_diag_schur_type1_spectrum

    dims = (4, 4, 4, 4)
    links = np.zeros((256, 4, 3, 3), dtype=np.complex128)
    links[:] = np.eye(3)
    lat = Lattice(dims, 0.0, 0, links=links)
    s = lat.schur(0.1, "I", False, max_rhs=12)
    got = lat.grg.grg_diag_schur_assemble(s.h, s.nb)
    ok, worst = same_multiset(np.linalg.eigvals(got), free_diag_schur_type1_spectrum(dims, 0.1), 1e-10)
    assert ok, worst
    s.close()
    lat.close()


@pytest.mark.parametrize("dims,kind,inv,nrhs", [((8, 8, 8, 8), "II", True, 4),
                                                ((8, 6, 4, 10), "I", False, 3),
                                                ((16, 16, 16, 16), "II", False, 12)])
def test_diag_schur_matrix_free(dims, kind, inv, nrhs):
    import torch

    lat = Lattice(dims, 0.5, 3)
    s = lat.schur(-0.2, kind, inv, max_rhs=nrhs)
    xb = gaussian_vectors(12 * s.nb, nrhs, 3)
    x = to_dev(xb)
    y = torch.empty_like(x)
    lat.grg.grg_diag_schur_apply(s.h, x, y, nrhs)
    got = to_host(y)
    sample = [0, nrhs - 1]
    want = matfree.diag_schur_apply(lat.links, dims, -0.2, s.q, s.nb, xb[sample])
    assert rel_err(got[sample], want) < 1e-12
    s.close()
    lat.close()
