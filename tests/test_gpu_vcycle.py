"""The V-cycle of section 4 on the GPU against the oracle: one cycle with
tight inner tolerances (then a deterministic operator) for two and three
levels, and the right-preconditioned BiCGstab solve of D x = f with its
average convergence rate against the unpreconditioned one."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors
from oracle import matfree, vcycle

from gpu_support import Lattice, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

DIMS, M0 = (8, 8, 8, 8), -0.4


@pytest.fixture(scope="module")
def lat():
    lt = Lattice(DIMS, 0.5, 41)
    yield lt
    lt.close()


@pytest.mark.parametrize("levels", [2, 3])
def test_cycle_vs_oracle(lat, levels):
    import torch

    grg = lat.grg
    prm = grg.grg_vcycle_params_default(levels=levels, drr_tol=1e-12, top_tol=1e-13, max_rhs=2)
    v = grg.grg_vcycle_create(lat.h, M0, prm)
    f = gaussian_vectors(12 * lat.V, 2, 45)
    fd = to_dev(f)
    xd = torch.empty_like(fd)
    print(f"V-cycle apply, {levels} levels, 8^4", flush=True)
    grg.grg_vcycle_apply(v, fd, xd, 2)
    x = to_host(xd)
    lv = vcycle.hierarchy(lat.links, DIMS, M0, levels)
    want = vcycle.cycle(lv, 0, f[0], tol=1e-13)
    assert rel_err(x[0], want) < 1e-9
    grg.grg_vcycle_destroy(v)


@pytest.mark.parametrize("levels", [2, 3])
def test_cycle_other_boundary_signs(levels):
    """Boundary signs other than antiperiodic t: every level keeps them."""
    import torch

    bc = (-1, 1, -1, 1)
    lt = Lattice(DIMS, 0.5, 44, bc=bc)
    grg = lt.grg
    prm = grg.grg_vcycle_params_default(levels=levels, drr_tol=1e-12, top_tol=1e-13, max_rhs=1)
    v = grg.grg_vcycle_create(lt.h, M0, prm)
    f = gaussian_vectors(12 * lt.V, 1, 47)
    fd = to_dev(f)
    xd = torch.empty_like(fd)
    print(f"V-cycle apply, {levels} levels, 8^4, bc {bc}", flush=True)
    grg.grg_vcycle_apply(v, fd, xd, 1)
    lv = vcycle.hierarchy(lt.links, DIMS, M0, levels, bc)
    assert rel_err(to_host(xd)[0], vcycle.cycle(lv, 0, f[0], tol=1e-13)) < 1e-9
    grg.grg_vcycle_destroy(v)
    lt.close()


def test_preconditioned_solve(lat):
    import torch

    grg = lat.grg
    v = grg.grg_vcycle_create(lat.h, M0, grg.grg_vcycle_params_default(levels=3, max_rhs=3))
    f = gaussian_vectors(12 * lat.V, 3, 46)
    fd = to_dev(f)
    xd = torch.empty_like(fd)
    print("V-cycle preconditioned BiCGstab, 8^4", flush=True)
    st = grg.grg_vcycle_solve(v, fd, xd, 3, tol=1e-8, precondition=True)
    x = to_host(xd)
    x0 = torch.empty_like(fd)
    st0 = grg.grg_vcycle_solve(v, fd, x0, 3, tol=1e-8, precondition=False)
    print(f"preconditioned: {st}\nplain: {st0}", flush=True)
    assert st["converged"] and st0["converged"]
    assert st["true_rel_resid"] <= 1e-8 * 1.01 and st0["true_rel_resid"] <= 1e-8 * 1.01
    assert st["rate"] < st0["rate"] and st["iters"] < st0["iters"]
    # the oracle's own residual of the GPU's solution
    r = matfree.dirac_apply(lat.links, DIMS, M0, x) - f
    assert np.all(np.linalg.norm(r, axis=1) <= 1.01e-8 * np.linalg.norm(f, axis=1))
    assert rel_err(x, to_host(x0)) < 1e-6
    grg.grg_vcycle_destroy(v)


def test_invalid_parameters(lat):
    grg = lat.grg
    with pytest.raises(grg.GrgError):
        grg.grg_vcycle_create(lat.h, M0, grg.grg_vcycle_params_default(levels=4))
    with pytest.raises(grg.GrgError):
        grg.grg_vcycle_create(lat.h, -4.0, grg.grg_vcycle_params_default(levels=2))
    odd = Lattice((8, 8, 8, 6), 0.5, 47)
    with pytest.raises(grg.GrgError):  # 6 is not divisible by 2^3
        grg.grg_vcycle_create(odd.h, M0, grg.grg_vcycle_params_default(levels=3))
    odd.close()


# ---------------------------------------------------------------- two levels on the other orderings
# Type II and the inverse permutations (section 4's runs used Type I^-1 and
# II^-1): section 3's S~_bb on top, at kappa = 1/6 (m0 = -1).
ORDERINGS = [("I", 1, True), ("II", 2, False), ("II", 2, True)]
M1 = -1.0


@pytest.mark.parametrize("name,perm,inv", ORDERINGS)
def test_two_level_cycle_vs_oracle(lat, name, perm, inv):
    import torch

    from oracle import dense

    grg = lat.grg
    prm = grg.grg_vcycle_params_default(levels=2, drr_tol=1e-12, top_tol=1e-13, max_rhs=2, perm=perm,
                                        inverse=int(inv))
    v = grg.grg_vcycle_create(lat.h, M1, prm)
    f = gaussian_vectors(12 * lat.V, 2, 48)
    fd = to_dev(f)
    xd = torch.empty_like(fd)
    print(f"two-level cycle, Type {name}{'^-1' if inv else ''}, 8^4", flush=True)
    grg.grg_vcycle_apply(v, fd, xd, 2)
    x = to_host(xd)
    q, nb = dense.permutation_block(DIMS, name, inv)
    for r in range(2):
        want = vcycle.two_level_cycle(lat.links, DIMS, M1, q, nb, f[r], top="reusken", tol=1e-13)
        assert rel_err(x[r], want) < 1e-9
    grg.grg_vcycle_destroy(v)


@pytest.mark.parametrize("name,perm,inv", ORDERINGS)
def test_two_level_preconditioned_solve(lat, name, perm, inv):
    import torch

    grg = lat.grg
    v = grg.grg_vcycle_create(lat.h, M1, grg.grg_vcycle_params_default(levels=2, max_rhs=2, perm=perm,
                                                                       inverse=int(inv)))
    f = gaussian_vectors(12 * lat.V, 2, 49)
    fd = to_dev(f)
    xd = torch.empty_like(fd)
    print(f"two-level preconditioned BiCGstab, Type {name}{'^-1' if inv else ''}, 8^4", flush=True)
    st = grg.grg_vcycle_solve(v, fd, xd, 2, tol=1e-8, precondition=True)
    x0 = torch.empty_like(fd)
    st0 = grg.grg_vcycle_solve(v, fd, x0, 2, tol=1e-8, precondition=False)
    print(f"preconditioned: {st}\nplain: {st0}", flush=True)
    assert st["converged"] and st["true_rel_resid"] <= 1e-8 * 1.01
    assert st["rate"] < st0["rate"] and st["iters"] < st0["iters"]
    r = matfree.dirac_apply(lat.links, DIMS, M1, to_host(xd)) - f
    assert np.all(np.linalg.norm(r, axis=1) <= 1.01e-8 * np.linalg.norm(f, axis=1))
    grg.grg_vcycle_destroy(v)


def test_two_level_invalid_parameters(lat):
    grg = lat.grg
    with pytest.raises(grg.GrgError):  # a two-level cycle only
        grg.grg_vcycle_create(lat.h, M1, grg.grg_vcycle_params_default(levels=3, perm=2))
    with pytest.raises(grg.GrgError):
        grg.grg_vcycle_create(lat.h, M1, grg.grg_vcycle_params_default(levels=2, perm=3))
    with pytest.raises(grg.GrgError):
        grg.grg_vcycle_create(lat.h, M1, grg.grg_vcycle_params_default(levels=3, perm=1, inverse=1))
