"""BiCGstab as the D_rr solver (the solver of the paper's section 4
experiment) against the oracle: the solution of D_rr z = b is unique, so the
GPU's BiCGstab result must match the GCR result and the oracle's FP64
residual, in every inner precision, on D_rr itself and on its even-odd
reduced system, with ragged volumes, a zero right-hand side and the full
S_bb apply."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors
from oracle import matfree

from gpu_support import Lattice, rel_err

pytestmark = pytest.mark.gpu

INNER_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-2}


def rest_rhs(lat, s, nrhs, seed, zero=()):
    b = gaussian_vectors(12 * lat.V, nrhs, seed).reshape(nrhs, lat.V, 12)
    b[:, np.asarray(s.q[: s.nb])] = 0
    for k in zero:
        b[k] = 0
    return b.reshape(nrhs, -1)


@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("eo", [0, 1])
@pytest.mark.parametrize("kind,inv", [("I", False), ("II", True)])
def test_bicgstab_drr_solve(inner, eo, kind, inv):
    lat = Lattice((8, 8, 8, 8), 0.5, 31)
    kw = dict(tol=1e-12, inner=inner, inner_tol=INNER_TOL[inner], max_rhs=3, max_iter=4000, eo=eo)
    sb = lat.schur(-0.2, kind, inv, method="bicgstab", **kw)
    sg = lat.schur(-0.2, kind, inv, **kw)
    b = rest_rhs(lat, sb, 3, 31)
    xb_, stb = sb.drr_solve(b)
    xg, stg = sg.drr_solve(b)
    print(f"bicgstab {inner} eo={eo} {kind}{'^-1' if inv else ''}: {stb['iters']} iterations "
          f"({stb['n_dslash']} stencils), GCR {stg['iters']}", flush=True)
    assert stb["converged"] and stg["converged"]
    assert rel_err(xb_, xg) < 1e-10
    rr = matfree.drr_residual(lat.links, lat.dims, -0.2, sb.q, sb.nb, b, xb_)
    assert np.all(rr <= 1e-12 * (1 + 1e-6)), rr
    assert not np.any(xb_.reshape(3, lat.V, 12)[:, np.asarray(sb.q[: sb.nb])])
    sb.close()
    sg.close()
    lat.close()


@pytest.mark.parametrize("dims", [(8, 6, 4, 10), (6, 4, 4, 5)])
def test_bicgstab_ragged_and_odd_extent_with_a_zero_rhs(dims):
    """A ragged last tile, and an odd extent (no even-odd form: BiCGstab on
    D_rr itself, with a random coarse set since the Type I/II patterns need
    even extents)."""
    lat = Lattice(dims, 0.5, 32)
    kw = dict(tol=1e-12, inner="fp32", inner_tol=1e-5, max_rhs=3, method="bicgstab")
    if all(L % 2 == 0 for L in dims):
        s = lat.schur(-0.1, "II", False, **kw)
    else:
        from gpu_support import Schur

        q = np.random.default_rng(32).permutation(lat.V).astype(np.int32)
        nb = lat.V // 16
        h = lat.grg.grg_schur_create(lat.h, -0.1, q, nb, lat.grg.grg_solver_params_default(**kw))
        s = Schur(lat, h, q, nb, -0.1)
    b = rest_rhs(lat, s, 3, 32, zero=(1,))
    x, st = s.drr_solve(b)
    assert st["converged"]
    assert not np.any(x[1])
    rr = matfree.drr_residual(lat.links, dims, -0.1, s.q, s.nb, b[[0, 2]], x[[0, 2]])
    assert np.all(rr <= 1e-12 * (1 + 1e-6)), rr
    s.close()
    lat.close()


def test_bicgstab_schur_apply_vs_oracle():
    lat = Lattice((8, 8, 8, 8), 0.5, 33)
    s = lat.schur(-0.3, "I", True, tol=1e-12, inner="bf16", inner_tol=1e-2, max_rhs=4,
                  method="bicgstab")
    xb = gaussian_vectors(12 * s.nb, 4, 33)
    y, st = s.apply(xb)
    assert st["converged"]
    want, _, rr = matfree.schur_apply(lat.links, lat.dims, -0.3, s.q, s.nb, xb[:2], restart=8, tol=1e-13)
    assert np.all(rr <= 1e-13)
    assert rel_err(y[:2], want) < 1e-10
    s.close()
    lat.close()


def test_bad_method_rejected():
    lat = Lattice((4, 4, 4, 4), 0.5, 34)
    with pytest.raises(lat.grg.GrgError):
        lat.schur(0.1, "I", False, method=2)
    lat.close()
