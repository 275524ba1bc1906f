"""Degenerate partitions and empty calls.

Section 1's split of D holds for any set of coarse sites, not only the
blocking sets of section 2, so the library takes any ordering q with
1 <= N_b <= V - 1.  The extreme and structured cases are checked against the
dense oracle at 4^4:
* one coarse site, and one rest site (D_rr a single 12 x 12 block);
* every even site coarse, or every odd site coarse: the rest sites then have
  no rest neighbour, so D_rr = (4 + m0) 1, and the even-odd reduced solve has
  an empty parity;
* a whole time slice coarse (the rest sites a slab, open in t);
* a random coarse set.
Every inner precision and both forms of the D_rr solve (even-odd reduced or
not) go through each, and the many-lattice batch takes such members too.
At m0 = -4 (a zero diagonal) the reduced form does not exist and the solve
runs on D_rr itself.  An empty batch (nrhs = 0) is an invalid argument for
every apply and solve call, rejected before anything runs."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors
from oracle import dense, matfree

from gpu_support import Lattice, Schur, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

DIMS, M0 = (4, 4, 4, 4), -0.2


@pytest.fixture(scope="module")
def c4():
    lat = Lattice(DIMS, 0.4, 61)
    d = dense.wilson_dense(lat.links, DIMS, M0)
    yield lat, d
    lat.close()


def ordering(case):
    V = int(np.prod(DIMS))
    rng = np.random.default_rng(62)
    par = matfree.site_parity(DIMS)
    if case == "one-coarse":
        return rng.permutation(V), 1
    if case == "one-rest":
        return rng.permutation(V), V - 1
    if case in ("even-coarse", "odd-coarse"):
        p = 0 if case == "even-coarse" else 1
        first = np.flatnonzero(par == p)
        return np.concatenate([first, np.flatnonzero(par != p)]), len(first)
    if case == "t-slice":
        v3 = V // DIMS[3]
        return np.arange(V), v3  # sites of t = 0 come first
    assert case == "random"
    return rng.permutation(V), V // 16


CASES = ["one-coarse", "one-rest", "even-coarse", "odd-coarse", "t-slice", "random"]


def make(lat, case, inner, eo):
    q, nb = ordering(case)
    grg = lat.grg
    tol_in = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-2}[inner]
    p = grg.grg_solver_params_default(tol=1e-12, inner=inner, inner_tol=tol_in, max_rhs=2, eo=eo)
    h = grg.grg_schur_create(lat.h, M0, q.astype(np.int32), nb, p)
    return Schur(lat, h, q, nb, M0)


@pytest.mark.parametrize("eo", [1, 0])
@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("case", CASES)
def test_schur_apply_degenerate_partition(c4, case, inner, eo):
    lat, d = c4
    s = make(lat, case, inner, eo)
    xb = gaussian_vectors(12 * s.nb, 2, 63)
    print(f"S_bb apply, {case}, N_b {s.nb}, inner {inner}, eo {eo}", flush=True)
    y, st = s.apply(xb)
    assert st["converged"]
    want = dense.schur_apply_dense(d, s.q, s.nb, xb)
    assert rel_err(y, want) < 1e-10, (case, inner, eo)
    s.close()


@pytest.mark.parametrize("eo", [1, 0])
@pytest.mark.parametrize("case", CASES)
def test_drr_solve_degenerate_partition(c4, case, eo):
    lat, d = c4
    s = make(lat, case, "bf16", eo)
    V = lat.V
    b = gaussian_vectors(12 * V, 2, 64).reshape(2, V, 12)
    b[:, np.asarray(s.q[: s.nb])] = 0
    b = b.reshape(2, -1)
    x, st = s.drr_solve(b)
    assert st["converged"]
    rr = matfree.drr_residual(lat.links, DIMS, M0, s.q, s.nb, b, x)
    assert np.all(rr <= 1e-12 * (1 + 1e-6)), (case, rr)
    assert not np.any(x.reshape(2, V, 12)[:, np.asarray(s.q[: s.nb])])
    if case in ("even-coarse", "odd-coarse"):
        # no rest site has a rest neighbour: D_rr = (4 + m0) 1
        xr = b.reshape(2, V, 12) / (4.0 + M0)
        assert rel_err(x, xr.reshape(2, -1)) < 1e-13
    s.close()


@pytest.mark.parametrize("case", ["one-coarse", "one-rest", "even-coarse", "t-slice"])
def test_approximations_degenerate_partition(c4, case):
    """Section 3's S~_bb and the approximation ignoring D_rr's couplings; on
    the even-site set D_rr is diagonal, so both equal S_bb there."""
    import torch

    lat, d = c4
    s = make(lat, case, "fp64", 1)
    grg = lat.grg
    xb = gaussian_vectors(12 * s.nb, 2, 65)
    x = to_dev(xb)
    y = torch.empty_like(x)
    grg.grg_reusken_apply(s.h, x, y, 2)
    want = (dense.reusken_dense(d, s.q, s.nb) @ xb.T).T
    assert rel_err(to_host(y), want) < 1e-12
    grg.grg_diag_schur_apply(s.h, x, y, 2)
    want0 = (dense.diag_schur_dense(d, s.q, s.nb) @ xb.T).T
    assert rel_err(to_host(y), want0) < 1e-12
    if case == "even-coarse":
        assert rel_err(want, dense.schur_apply_dense(d, s.q, s.nb, xb)) < 1e-12
    s.close()


def test_empty_batch_is_rejected(c4):
    import torch

    lat, _ = c4
    grg = lat.grg
    s = make(lat, "random", "bf16", 1)
    xb = to_dev(np.zeros((1, 12 * s.nb)))
    yb = torch.empty_like(xb)
    xf = to_dev(np.zeros((1, 12 * lat.V)))
    yf = torch.empty_like(xf)
    calls = [
        lambda: grg.grg_schur_apply(s.h, xb, yb, 0),
        lambda: grg.grg_drr_solve(s.h, xf, yf, 0),
        lambda: grg.grg_reusken_apply(s.h, xb, yb, 0),
        lambda: grg.grg_diag_schur_apply(s.h, xb, yb, 0),
        lambda: grg.grg_dirac_apply(lat.h, M0, "fp64", xf, yf, 0),
    ]
    for call in calls:
        yb.fill_(7.0)
        yf.fill_(7.0)
        with pytest.raises(grg.GrgError) as e:
            call()
        assert e.value.status == grg.GRG_EINVAL
        # nothing was written
        assert torch.all(yb == 7.0) and torch.all(yf == 7.0)
    s.close()


def test_partition_bounds_are_checked(c4):
    lat, _ = c4
    grg = lat.grg
    q = np.arange(lat.V, dtype=np.int32)
    for nb in (0, lat.V, -1):
        with pytest.raises(grg.GrgError) as e:
            grg.grg_schur_create(lat.h, M0, q, nb, grg.grg_solver_params_default())
        assert e.value.status == grg.GRG_EINVAL


@pytest.mark.parametrize("method", ["gcr", "bicgstab"])
def test_zero_diagonal(method):
    """m0 = -4: D_rr is the hopping term alone (4 + m0 = 0).  The even-odd
    reduction, which divides by the diagonal, does not exist: the reduced
    apply is refused and the solve runs on D_rr itself whatever params.eo
    says.  With every site of the slice t = 0 coarse, D_rr is invertible
    (condition number about 2e3 on this field) but its spectrum is symmetric
    about zero, where minimal residual stagnates and BiCGstab diverges (as
    restarted GCR does in the oracle too): the call reports GRG_ENOCONV and
    returns per RHS the iterate of smallest residual, never worse than
    x = 0."""
    import torch

    lat = Lattice(DIMS, 0.4, 61)
    m0 = -4.0
    q, nb = ordering("t-slice")
    grg = lat.grg
    xb = gaussian_vectors(12 * nb, 2, 66)
    ys = []
    for eo in (1, 0):
        p = grg.grg_solver_params_default(tol=1e-12, inner="fp64", max_rhs=2, eo=eo, method=method,
                                          max_iter=300)
        s = Schur(lat, grg.grg_schur_create(lat.h, m0, q.astype(np.int32), nb, p), q, nb, m0)
        with pytest.raises(grg.GrgError) as e:
            s.apply(xb)
        assert e.value.status == grg.GRG_ENOCONV
        y, st = s.apply(xb, allow_noconv=True)
        assert st["status"] == grg.GRG_ENOCONV and np.isfinite(y).all()
        assert st["true_rel_resid"] <= 1.0
        ys.append(y)
        x = to_dev(np.zeros((1, 12 * lat.V)))
        with pytest.raises(grg.GrgError) as e:
            grg.grg_reduced_apply(s.h, "fp64", 0, x, torch.empty_like(x), 1)
        assert e.value.status == grg.GRG_EINVAL
        s.close()
    assert np.array_equal(ys[0], ys[1])  # the same unreduced solve
    lat.close()


@pytest.mark.parametrize("eo", [1, 0])
def test_batch_degenerate_partitions(c4, eo):
    """The many-lattice batch with members whose partitions are degenerate
    (one rest site; every even site coarse: an empty reduced parity) beside
    a Type I member, each against the dense oracle."""
    import torch

    lat, d = c4
    grg = lat.grg
    qI, nbI = grg.grg_permutation_block(DIMS, 1, False)
    orders = [ordering("one-rest"), ordering("even-coarse"), (qI, nbI)]
    ms = [dict(dims=DIMS, m0=M0, links=lat.links, q=np.asarray(q, np.int32), n_coarse=nb) for q, nb in orders]
    nrhs = 2
    p = grg.grg_solver_params_default(tol=1e-12, inner="fp32", inner_tol=1e-5, check_every=2, eo=eo)
    b = grg.grg_batch_create(ms, nrhs, p)
    total, _ = grg.grg_batch_layout(b, len(ms))
    x = np.zeros(total, np.complex128)
    for i, m in enumerate(ms):
        off, nb = grg.grg_batch_layout(b, i)
        x[off:off + 12 * nb * nrhs] = gaussian_vectors(12 * nb, nrhs, 67 + i).reshape(-1)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    st = grg.grg_batch_apply(b, xd, yd, use_graph=False)
    assert st["converged"] and st["true_rel_resid"] <= 1e-12
    y = to_host(yd)
    for i, m in enumerate(ms):
        off, nb = grg.grg_batch_layout(b, i)
        xi = x[off:off + 12 * nb * nrhs].reshape(nrhs, -1)
        yi = y[off:off + 12 * nb * nrhs].reshape(nrhs, -1)
        assert rel_err(yi, dense.schur_apply_dense(d, m["q"], nb, xi)) < 1e-10, i
    grg.grg_batch_destroy(b)


@pytest.mark.parametrize("dims", [(1, 4, 3, 2), (3, 2, 1, 1), (2, 2, 2, 2)])
@pytest.mark.parametrize("inner", ["fp64", "bf16"])
def test_tiny_lattices(dims, inner):
    """Extents of one (a site is its own neighbour) and two (forward and
    backward neighbours coincide), fewer sites than one 64-site tile, a
    random coarse set: S_bb against the dense oracle (the even-odd form only
    where every extent is even)."""
    lat = Lattice(dims, 0.4, 68)
    V = lat.V
    q = np.random.default_rng(69).permutation(V).astype(np.int32)
    nb = max(1, V // 6)
    tol_in = {"fp64": 1e-12, "bf16": 1e-2}[inner]
    p = lat.grg.grg_solver_params_default(tol=1e-12, inner=inner, inner_tol=tol_in, max_rhs=2)
    s = Schur(lat, lat.grg.grg_schur_create(lat.h, M0, q, nb, p), q, nb, M0)
    xb = gaussian_vectors(12 * nb, 2, 70)
    y, st = s.apply(xb)
    assert st["converged"]
    d = dense.wilson_dense(lat.links, dims, M0)
    assert rel_err(y, dense.schur_apply_dense(d, q, nb, xb)) < 1e-10
    s.close()
    lat.close()


@pytest.mark.parametrize("bc", [(-1, -1, 1, 1), (1, 1, 1, 1)])
def test_other_boundary_signs_tuned(bc):
    """S_bb, S~_bb and the reduced BF16 solve in the tuned launch forms at
    16^4 (where the plane form of the half-lattice stencil applies) with
    other boundary signs, against the C oracle with the same signs."""
    import torch

    dims = (16, 16, 16, 16)
    lat = Lattice(dims, 0.5, 71, bc=bc)
    grg = lat.grg
    q, nb = grg.grg_permutation_block(dims, 1, False)
    p = grg.grg_solver_params_default(tol=1e-10, inner="bf16", inner_tol=1e-2, max_rhs=2)
    s = Schur(lat, grg.grg_schur_create(lat.h, -0.3, q, nb, p), q, nb, -0.3)
    grg.grg_schur_tune(s.h, 2)
    xb = gaussian_vectors(12 * nb, 2, 72)
    print(f"S_bb 16^4 bc {bc}, tuned", flush=True)
    y, st = s.apply(xb)
    assert st["converged"]
    want, _, _ = matfree.schur_apply(lat.links, dims, -0.3, q, nb, xb[:1], tol=1e-12, bc=bc)
    assert rel_err(y[:1], want) < 1e-8
    x = to_dev(xb)
    yr = torch.empty_like(x)
    grg.grg_reusken_apply(s.h, x, yr, 2)
    assert rel_err(to_host(yr), matfree.reusken_apply(lat.links, dims, -0.3, q, nb, xb, bc=bc)) < 1e-12
    s.close()
    lat.close()


def test_batch_members_with_other_boundary_signs():
    """Batch members keep their own boundary signs."""
    import torch
    from grg_inputs import su3_links

    import paper_0704_2341_amd as grg

    dims = (8, 8, 8, 8)
    bcs = [(1, 1, 1, -1), (-1, 1, 1, 1), (1, -1, -1, -1)]
    q, nb = grg.grg_permutation_block(dims, 1, False)
    ms = [dict(dims=dims, bc=bc, m0=-0.2, links=su3_links(dims, 0.5, 73 + i), q=np.asarray(q), n_coarse=nb)
          for i, bc in enumerate(bcs)]
    nrhs = 2
    p = grg.grg_solver_params_default(tol=1e-11, inner="bf16", inner_tol=1e-2, check_every=2)
    b = grg.grg_batch_create(ms, nrhs, p)
    total, _ = grg.grg_batch_layout(b, len(ms))
    x = np.zeros(total, np.complex128)
    for i in range(len(ms)):
        off, n = grg.grg_batch_layout(b, i)
        x[off:off + 12 * n * nrhs] = gaussian_vectors(12 * n, nrhs, 76 + i).reshape(-1)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    st = grg.grg_batch_apply(b, xd, yd, use_graph=True)
    assert st["converged"]
    y = to_host(yd)
    for i, m in enumerate(ms):
        off, n = grg.grg_batch_layout(b, i)
        xi = x[off:off + 12 * n * nrhs].reshape(nrhs, -1)
        want, _, _ = matfree.schur_apply(m["links"], dims, m["m0"], q, nb, xi[:1], tol=1e-13, bc=m["bc"])
        assert rel_err(y[off:off + 12 * n * nrhs].reshape(nrhs, -1)[:1], want) < 1e-9, i
    grg.grg_batch_destroy(b)


@pytest.mark.parametrize("case", ["even-coarse", "one-rest", "random"])
def test_learned_preconditioner_degenerate_partition(c4, case):
    """The flexible inner solve with the network (its initial weights) on
    the reduced parity, where that parity may be empty."""
    lat, d = c4
    s = make(lat, case, "bf16", 1)
    grg = lat.grg
    p = grg.grg_precond_create(s.h)
    grg.grg_schur_attach_precond(s.h, p)
    xb = gaussian_vectors(12 * s.nb, 2, 78)
    y, st = s.apply(xb)
    assert st["converged"]
    assert rel_err(y, dense.schur_apply_dense(d, s.q, s.nb, xb)) < 1e-10
    grg.grg_schur_attach_precond(s.h, None)
    grg.grg_precond_destroy(p)
    s.close()


@pytest.mark.parametrize("dims,inner,tune", [((8, 8, 8, 8), "fp32", False), ((16, 16, 16, 16), "bf16", True)])
def test_sixteen_rhs(dims, inner, tune):
    """The largest RHS count (16) through the solve, the per-RHS sums and, at
    16^4, the tuned launch forms; every RHS against the C oracle."""
    lat = Lattice(dims, 0.5, 79)
    grg = lat.grg
    q, nb = grg.grg_permutation_block(dims, 1, False)
    tol_in = {"fp32": 1e-5, "bf16": 1e-2}[inner]
    p = grg.grg_solver_params_default(tol=1e-10, inner=inner, inner_tol=tol_in, max_rhs=16)
    s = Schur(lat, grg.grg_schur_create(lat.h, -0.2, q, nb, p), q, nb, -0.2)
    if tune:
        grg.grg_schur_tune(s.h, 16)
    xb = gaussian_vectors(12 * nb, 16, 80)
    xb[5] = 0.0  # a zero RHS among them
    print(f"S_bb {dims}, 16 RHS, inner {inner}", flush=True)
    y, st = s.apply(xb)
    assert st["converged"] and st["true_rel_resid"] <= 1e-10
    assert not np.any(y[5])
    idx = [0, 7, 15] if tune else list(range(16))
    want, _, _ = matfree.schur_apply(lat.links, dims, -0.2, q, nb, xb[idx], tol=1e-13)
    assert rel_err(y[idx], want) < 1e-8
    s.close()
    lat.close()


@pytest.mark.parametrize("inner", ["bf16", "fp32"])
def test_extreme_magnitudes(c4, inner):
    """S_bb is linear: inputs scaled by 1e-15 or 1e15 (beyond the range in
    which the inner solve starts from the unscaled right-hand side, so it is
    rescaled first) give the scaled result of the unit-size input."""
    lat, d = c4
    grg = lat.grg
    q, nb = grg.grg_permutation_block(DIMS, 1, False)
    tol_in = {"fp32": 1e-5, "bf16": 1e-2}[inner]
    p = grg.grg_solver_params_default(tol=1e-12, inner=inner, inner_tol=tol_in, max_rhs=3)
    s = Schur(lat, grg.grg_schur_create(lat.h, M0, q, nb, p), q, nb, M0)
    xb = gaussian_vectors(12 * nb, 1, 86)
    want = dense.schur_apply_dense(d, q, nb, xb)
    y1, st = s.apply(xb)
    assert st["converged"] and rel_err(y1, want) < 1e-10
    x3 = np.concatenate([xb * 1e-15, xb, xb * 1e15])
    y3, st = s.apply(x3)
    assert st["converged"]
    for k, f in enumerate((1e-15, 1.0, 1e15)):
        assert rel_err(y3[k:k + 1] / f, want) < 1e-10, f
    s.close()
