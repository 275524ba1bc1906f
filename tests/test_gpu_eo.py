"""The even-odd reduced inner solve (D_rr eliminated to one parity) against
the unreduced solve and the oracle: every inner precision, permutations whose
coarse sites lie on one parity (Type I) or on both (the inverses), ragged
volumes, the fallback on lattices with an odd extent, and its autotuned
launch."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors
from oracle import matfree

from gpu_support import Lattice, rel_err

pytestmark = pytest.mark.gpu

INNER_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-2}


def rest_rhs(lat, s, nrhs, seed):
    b = gaussian_vectors(12 * lat.V, nrhs, seed).reshape(nrhs, lat.V, 12)
    b[:, np.asarray(s.q[: s.nb])] = 0
    return b.reshape(nrhs, -1)


@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("kind,inv", [("I", False), ("I", True), ("II", True)])
def test_reduced_equals_unreduced(inner, kind, inv):
    lat = Lattice((8, 8, 8, 8), 0.5, 21)
    kw = dict(tol=1e-12, inner=inner, inner_tol=INNER_TOL[inner], max_rhs=3, max_iter=4000)
    s1 = lat.schur(-0.2, kind, inv, eo=1, **kw)
    s0 = lat.schur(-0.2, kind, inv, eo=0, **kw)
    b = rest_rhs(lat, s1, 3, 21)
    x1, st1 = s1.drr_solve(b)
    x0, st0 = s0.drr_solve(b)
    assert st1["converged"] and st0["converged"]
    assert rel_err(x1, x0) < 1e-10
    # the reduced system converges in fewer iterations
    assert st1["iters"] < st0["iters"], (st1, st0)
    rr = matfree.drr_residual(lat.links, lat.dims, -0.2, s1.q, s1.nb, b, x1)
    assert np.all(rr <= 1e-12 * (1 + 1e-6)), rr
    # zero on the coarse sites
    assert not np.any(x1.reshape(3, lat.V, 12)[:, np.asarray(s1.q[: s1.nb])])
    s1.close()
    s0.close()
    lat.close()


@pytest.mark.parametrize("dims", [(8, 6, 4, 10), (4, 4, 4, 2)])
def test_ragged_volumes(dims):
    lat = Lattice(dims, 0.5, 22)
    s = lat.schur(-0.1, "II", False, tol=1e-12, inner="bf16", inner_tol=1e-2, max_rhs=2, eo=1)
    b = rest_rhs(lat, s, 2, 22)
    x, st = s.drr_solve(b)
    assert st["converged"]
    rr = matfree.drr_residual(lat.links, dims, -0.1, s.q, s.nb, b, x)
    assert np.all(rr <= 1e-12 * (1 + 1e-6)), rr
    s.close()
    lat.close()


def test_odd_extent_falls_back():
    """With an odd extent the lattice is not bipartite: the solve runs on
    D_rr itself and still meets the tolerance."""
    dims = (6, 4, 4, 5)
    lat = Lattice(dims, 0.5, 23)
    V = lat.V
    rng = np.random.default_rng(23)
    q = rng.permutation(V).astype(np.int32)
    nb = V // 16
    grg = lat.grg
    h = grg.grg_schur_create(lat.h, -0.1, q, nb, grg.grg_solver_params_default(
        tol=1e-12, inner="fp32", inner_tol=1e-5, max_rhs=2, eo=1))
    from gpu_support import Schur

    s = Schur(lat, h, q, nb, -0.1)
    b = rest_rhs(lat, s, 2, 23)
    x, st = s.drr_solve(b)
    assert st["converged"]
    rr = matfree.drr_residual(lat.links, dims, -0.1, q, nb, b, x)
    assert np.all(rr <= 1e-12 * (1 + 1e-6)), rr
    s.close()
    lat.close()


def test_tuned_reduced_solve_same_result():
    lat = Lattice((16, 16, 8, 8), 0.5, 24)
    s = lat.schur(-0.3, "I", False, tol=1e-12, inner="bf16", inner_tol=1e-2, max_rhs=4, eo=1)
    xb = gaussian_vectors(12 * s.nb, 4, 24)
    y0, st0 = s.apply(xb)
    lat.grg.grg_schur_tune(s.h, 4)
    y1, st1 = s.apply(xb)
    assert st0["converged"] and st1["converged"]
    assert rel_err(y1, y0) < 1e-11
    want, _, _ = matfree.schur_apply(lat.links, lat.dims, -0.3, s.q, s.nb, xb[:1], restart=8, tol=1e-13)
    assert rel_err(y1[:1], want) < 1e-10
    s.close()
    lat.close()


RA_TOL = {"fp64": 1e-13, "fp32": 2e-6, "bf16": 1.5e-2}
# half-lattice stencil launches {SB, RG, hop schedule, grid, chunk, time slices}:
# one hop per iteration, double-buffered hops, and the t-marching form (whole
# t range, ragged time chunks, a grid smaller than the work items)
RA_LAUNCHES = {
    "one-hop": (256, 2, 1, 64, 0, 0),
    "double-buffered": (128, 3, 2, 56, 4, 0),
    "march-all-t": (256, 3, 3, 64, 0, 8),
    "march-ragged-chunks": (256, 1, 3, 24, 0, 3),
    "march-small-grid": (256, 3, 3, 8, 0, 2),
    "two-rhs-per-hop": (128, 2, 4, 48, 0, 0),
    "three-rhs-per-hop": (64, 3, 5, 40, 8, 0),
    "x-hops-from-lanes": (256, 3, 6, 64, 0, 0),
    "x-hops-from-lanes-sb64": (64, 1, 6, 24, 8, 0),
    "plane-all-t": (64, 1, 7, 64, 0, 8),
    "plane-ragged-chunks": (64, 1, 7, 24, 0, 3),
}


@pytest.mark.parametrize("form", list(RA_LAUNCHES))
@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp64"])
@pytest.mark.parametrize("nrhs", [5, 12])
def test_reduced_apply_vs_oracle(form, prec, nrhs):
    """A_p = d - H_pq H_qp / d on both parities, every launch form of the
    half-lattice stencils, against the oracle's Schur complement of D_rr."""
    launch = RA_LAUNCHES[form]
    dims = (16, 8, 8, 8)  # 512 half-sites per time slice: whole 64-column tiles
    lat = Lattice(dims, 0.5, 25)
    s = lat.schur(-0.3, "I", False, tol=1e-10, inner=prec, max_rhs=12)
    grg = lat.grg
    if launch[2] >= 2 and prec != "bf16":
        # the packed-BF16 hop schedules exist for BF16 fields only: any other
        # precision is refused with GRG_EINVAL and the launch in use is kept
        before = grg.grg_schur_tune_info(s.h, prec, nrhs, eo=True)
        with pytest.raises(grg.GrgError) as ei:
            grg.grg_schur_set_launch(s.h, prec, nrhs, launch, eo=True)
        assert ei.value.status == grg.GRG_EINVAL
        assert grg.grg_schur_tune_info(s.h, prec, nrhs, eo=True) == before
        s.close()
        lat.close()
        return
    grg.grg_schur_set_launch(s.h, prec, nrhs, launch, eo=True)
    assert grg.grg_schur_tune_info(s.h, prec, nrhs, eo=True)["split"] == launch[2]
    x = gaussian_vectors(12 * lat.V, nrhs, 25)
    import torch

    from gpu_support import to_dev, to_host

    xd = to_dev(x)
    yd = torch.empty_like(xd)
    for parity in (0, 1):
        print(f"reduced apply {form} {prec} nrhs {nrhs} parity {parity}", flush=True)
        grg.grg_reduced_apply(s.h, prec, parity, xd, yd, nrhs)
        y = to_host(yd)
        want = matfree.reduced_apply(lat.links, dims, -0.3, s.q, s.nb, parity, x)
        assert rel_err(y, want) < RA_TOL[prec]
        # zero off the parity's rest sites
        par = matfree.site_parity(dims)
        off = (par != parity)
        off[np.asarray(s.q[: s.nb])] = True
        assert not np.any(y.reshape(nrhs, lat.V, 12)[:, off])
    s.close()
    lat.close()


@pytest.mark.parametrize("dims,launch", [
    ((8, 32, 4, 6), (128, 1, 7, 40, 0, 6)),     # two wavefronts per plane
    ((16, 32, 4, 4), (256, 1, 7, 16, 0, 3)),    # four, ragged time chunks
    ((32, 32, 2, 4), (512, 1, 7, 8, 0, 1)),     # eight, one slice per item
    ((16, 8, 16, 6), (64, 2, 7, 24, 0, 4)),     # two planes per workgroup, ragged chunks
    ((16, 16, 32, 4), (128, 2, 7, 16, 0, 2)),   # two planes of two wavefronts, two pairs per XCD
    ((32, 32, 16, 2), (512, 2, 7, 8, 0, 1)),    # two planes of eight wavefronts (1024 lanes)
])
def test_plane_form_vs_oracle(dims, launch):
    """The plane form with several wavefronts per x-y plane (y neighbours
    across wavefronts, read from LDS after the slice's barrier), and with two
    planes per workgroup (the z hop between them read from the other plane's
    slot), both parities, with and without the alpha term, against the
    oracle; the two-plane form bit for bit against the one-plane form."""
    lat = Lattice(dims, 0.5, 28)
    nrhs = 3
    s = lat.schur(-0.3, "I", False, tol=1e-10, inner="bf16", max_rhs=nrhs)
    grg = lat.grg
    grg.grg_schur_set_launch(s.h, "bf16", nrhs, launch, eo=True)
    x = gaussian_vectors(12 * lat.V, nrhs, 28)
    import torch

    from gpu_support import to_dev, to_host

    xd = to_dev(x)
    yd = torch.empty_like(xd)
    outs = []
    for parity in (0, 1):
        print(f"plane form {dims} {launch} parity {parity}", flush=True)
        grg.grg_reduced_apply(s.h, "bf16", parity, xd, yd, nrhs)
        want = matfree.reduced_apply(lat.links, dims, -0.3, s.q, s.nb, parity, x)
        outs.append(to_host(yd))
        assert rel_err(outs[-1], want) < RA_TOL["bf16"]
    if launch[1] == 2:
        one = (launch[0], 1, 7, launch[3], launch[4], launch[5])
        grg.grg_schur_set_launch(s.h, "bf16", nrhs, one, eo=True)
        for parity in (0, 1):
            grg.grg_reduced_apply(s.h, "bf16", parity, xd, yd, nrhs)
            assert np.array_equal(to_host(yd), outs[parity]), parity
    s.close()
    lat.close()


def test_bf16_forms_bit_identical():
    """Every BF16 form of the half-lattice stencil sums the hops of a site in
    the same order with the same arithmetic, so their outputs agree bit for
    bit (the autotuner's choice changes speed only)."""
    import torch

    from gpu_support import to_dev, to_host

    dims = (16, 8, 8, 8)
    lat = Lattice(dims, 0.5, 30)
    nrhs = 5
    s = lat.schur(-0.3, "I", False, tol=1e-10, inner="bf16", max_rhs=nrhs)
    grg = lat.grg
    xd = to_dev(gaussian_vectors(12 * lat.V, nrhs, 30))
    yd = torch.empty_like(xd)
    ref = None
    for form, launch in RA_LAUNCHES.items():
        if launch[1] > nrhs:
            continue
        grg.grg_schur_set_launch(s.h, "bf16", nrhs, launch, eo=True)
        print(f"bit identity {form}", flush=True)
        outs = []
        for parity in (0, 1):
            grg.grg_reduced_apply(s.h, "bf16", parity, xd, yd, nrhs)
            outs.append(to_host(yd))
        if ref is None:
            ref = outs
        else:
            for a, b in zip(outs, ref):
                assert np.array_equal(a, b), form
    s.close()
    lat.close()


def test_plane_launch_rejected_for_wrong_plane():
    """The plane form's workgroup is exactly one x-y plane of at most 512
    half-sites, a multiple of 64."""
    lat = Lattice((16, 8, 8, 8), 0.5, 29)
    s = lat.schur(-0.1, "I", False, tol=1e-10, inner="bf16", max_rhs=2)
    # a wrong plane size, no time slices, a grid not a multiple of 8, two
    # planes per workgroup with Lz = 8 (one plane per XCD), three planes
    for bad in ((128, 1, 7, 8, 0, 4), (64, 1, 7, 8, 0, 0), (64, 1, 7, 12, 0, 4), (64, 2, 7, 8, 0, 4),
                (64, 3, 7, 8, 0, 4)):
        with pytest.raises(lat.grg.GrgError):
            lat.grg.grg_schur_set_launch(s.h, "bf16", 2, bad, eo=True)
    s.close()
    lat.close()
    lat = Lattice((8, 6, 4, 10), 0.5, 29)  # 24 half-sites per plane
    s = lat.schur(-0.1, "II", False, tol=1e-10, inner="bf16", max_rhs=2)
    with pytest.raises(lat.grg.GrgError):
        lat.grg.grg_schur_set_launch(s.h, "bf16", 2, (24, 1, 7, 8, 0, 5), eo=True)
    s.close()
    lat.close()


def test_march_launch_rejected_without_whole_tiles():
    """The t-marching form needs a multiple of 64 half-sites per time slice."""
    lat = Lattice((8, 6, 4, 10), 0.5, 26)
    s = lat.schur(-0.1, "II", False, tol=1e-10, inner="bf16", max_rhs=2)
    with pytest.raises(lat.grg.GrgError):
        lat.grg.grg_schur_set_launch(s.h, "bf16", 2, (256, 1, 3, 8, 0, 5), eo=True)
    s.close()
    lat.close()


@pytest.mark.parametrize("launch", [(256, 3, 3, 40, 0, 3), (64, 1, 7, 40, 0, 3)])
@pytest.mark.parametrize("method", ["gcr", "bicgstab"])
@pytest.mark.parametrize("kind,inv", [("I", False), ("II", True)])
def test_march_full_layout_steps(method, kind, inv, launch):
    """With the t-marching launch pinned before any tuning, the first and
    last steps of every reduced solve (full-layout input, and output with the
    other parity copied in) run that form too: same solution as the
    unreduced solve, including a zero right-hand side that takes no step and
    a ragged last group of four RHS."""
    dims = (16, 8, 8, 8)
    lat = Lattice(dims, 0.5, 27)
    kw = dict(tol=1e-12, inner="bf16", inner_tol=1e-2, max_rhs=5, max_iter=4000, method=method)
    s1 = lat.schur(-0.2, kind, inv, eo=1, **kw)
    s0 = lat.schur(-0.2, kind, inv, eo=0, **kw)
    lat.grg.grg_schur_set_launch(s1.h, "bf16", 5, launch, eo=True)
    assert lat.grg.grg_schur_tune_info(s1.h, "bf16", 5, eo=True)["split"] == launch[2]
    b = rest_rhs(lat, s1, 5, 27)
    b[3] = 0
    print(f"march full-layout steps {launch} {method} {kind} inv={inv}", flush=True)
    x1, st1 = s1.drr_solve(b)
    x0, st0 = s0.drr_solve(b)
    assert st1["converged"] and st0["converged"]
    assert rel_err(x1, x0) < 1e-10
    assert not np.any(x1[3])
    rr = matfree.drr_residual(lat.links, dims, -0.2, s1.q, s1.nb, b, x1)
    assert np.all(rr <= 1e-12 * (1 + 1e-6)), rr
    assert not np.any(x1.reshape(5, lat.V, 12)[:, np.asarray(s1.q[: s1.nb])])
    s1.close()
    s0.close()
    lat.close()
