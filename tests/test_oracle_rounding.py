"""Pins of the oracle pieces that bound reduced-precision results element by
element: the FP32 / bfloat16 value maps (against torch's own converters on
the CPU) and the absolute-value sums of the stencil's terms (against the
entrywise absolute value of the dense Wilson matrix, which for extents >= 3
has one product per entry)."""
import numpy as np
import pytest
import torch

from grg_inputs import gaussian_vectors, su3_links
from oracle import dense, matfree, rounding

PERMS = [("I", False), ("II", False), ("I", True), ("II", True)]


def test_bf16_value_matches_torch_on_fp32_inputs():
    rng = np.random.default_rng(0)
    f = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
        # exact ties: 8 significant bits plus a half unit, both parities of the last bit
        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 3 * 2 ** -9 + 2 ** -17, 0.0, -0.0]),
    ]).astype(np.float32)
    want = torch.from_numpy(f).to(torch.bfloat16).to(torch.float64).numpy()
    got = rounding.bf16_value(f.astype(np.float64))
    assert np.array_equal(got, want)


def test_bf16_value_goes_through_fp32():
    # an FP64 value just above a bf16 tie whose FP32 rounding lands on the tie:
    # the stored value is the even neighbour, not the one above
    x = 1 + 2 ** -8 + 2 ** -30
    assert np.float32(x) == np.float32(1 + 2 ** -8)
    assert rounding.bf16_value(np.array([x]))[0] == 1.0
    # complex values round their parts separately
    z = np.array([x + 1j * (-x)])
    assert rounding.bf16_value(z)[0] == 1.0 - 1.0j


def test_bf16_relative_error_bound():
    rng = np.random.default_rng(1)
    a = rng.standard_normal(100000)
    r = rounding.bf16_value(a)
    assert np.all(np.abs(r - a) <= rounding.UNIT_ROUNDOFF["bf16"] * (1 + 2 ** -15) * np.abs(a))
    assert np.max(np.abs(r - a) / np.abs(a)) > 0.9 * rounding.UNIT_ROUNDOFF["bf16"]
    f = rounding.fp32_value(a)
    assert np.all(np.abs(f - a) <= rounding.UNIT_ROUNDOFF["fp32"] * np.abs(a))


@pytest.mark.parametrize("kind,inv", PERMS)
def test_block_apply_abs_is_abs_matrix(kind, inv):
    """|D|_{rows,cols} |x| with |D| the entrywise absolute value of the dense
    matrix, with and without its diagonal."""
    dims, m0 = (4, 4, 4, 4), -0.3
    u = su3_links(dims, 0.5, 17)
    d = dense.wilson_dense(u, dims, m0)
    q, nb = dense.permutation_block(dims, kind, inv)
    mask = np.zeros(256, bool)
    mask[q[:nb]] = True
    dmask = np.repeat(mask, 12)
    x = gaussian_vectors(12 * 256, 2, 17)
    for osel in (0, 1):
        for isel in (0, 1):
            for diag in (True, False):
                a = np.abs(d)
                if not diag:
                    a = a - np.diag(np.diag(a))
                a[dmask != bool(osel), :] = 0
                a[:, dmask != bool(isel)] = 0
                got = matfree.block_apply_abs(u, dims, m0, q, nb, osel, isel, x, diag=diag)
                want = (a @ np.abs(x).T).T
                assert np.abs(got - want).max() <= 1e-13 * max(want.max(), 1.0)


def test_block_apply_abs_bounds_the_sum():
    """|D x| <= |D| |x| entrywise, with equality where every term has the
    same phase (a single nonzero input entry and one hop)."""
    dims, m0 = (4, 4, 4, 8), 0.1
    u = su3_links(dims, 0.5, 18)
    v = int(np.prod(dims))
    q, nb = dense.permutation_block(dims, "I", False)
    x = gaussian_vectors(12 * v, 3, 18)
    y = matfree.block_apply(u, dims, m0, q, nb, 0, 0, x)
    a = matfree.block_apply_abs(u, dims, m0, q, nb, 0, 0, x)
    assert np.all(np.abs(y) <= a * (1 + 1e-12))
    e = np.zeros((1, 12 * v), complex)
    e[0, 12 * 5 + 4] = 2.0 - 1.0j  # one entry at a rest site
    y = matfree.block_apply(u, dims, m0, q, nb, 0, 0, e)
    a = matfree.block_apply_abs(u, dims, m0, q, nb, 0, 0, e)
    assert np.allclose(np.abs(y), a, rtol=1e-13, atol=0)


def test_reduced_apply_abs_and_intermediate():
    """The reduced operator's absolute-value sums against the dense Schur
    complement of D_rr built from |D|, and the intermediate H_qp x_p."""
    dims, m0 = (4, 4, 4, 4), -0.2
    u = su3_links(dims, 0.5, 19)
    d = dense.wilson_dense(u, dims, m0)
    q, nb = dense.permutation_block(dims, "II", True)
    rest = np.ones(256, bool)
    rest[q[:nb]] = False
    par = matfree.site_parity(dims)
    x = gaussian_vectors(12 * 256, 2, 19)
    for p in (0, 1):
        on_p = np.repeat(rest & (par == p), 12)
        on_q = np.repeat(rest & (par != p), 12)
        a = np.abs(d)
        h = a - np.diag(np.diag(a))
        got = matfree.reduced_apply_abs(u, dims, m0, q, nb, p, x)
        w = np.zeros_like(got)
        w[:, on_p] = abs(4 + m0) * np.abs(x[:, on_p]) + (h[np.ix_(on_p, on_q)] @ (
            h[np.ix_(on_q, on_p)] @ np.abs(x[:, on_p]).T)).T / abs(4 + m0)
        assert np.abs(got - w).max() < 1e-13 * w.max()
        t = matfree.reduced_intermediate(u, dims, m0, q, nb, p, x)
        tw = np.zeros_like(t)
        tw[:, on_q] = (d[np.ix_(on_q, on_p)] @ x[:, on_p].T).T
        assert np.abs(t - tw).max() < 1e-13 * np.abs(tw).max()
