"""Boundary behaviour that the parity tests do not reach: the gauge field
handed over from device memory or from a torch host tensor, a lattice on a
stream of its own, and the lattice's queries.  Results are compared bit for
bit with the host-numpy path, and the stencil once with the oracle."""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors, su3_links
from oracle import matfree

from gpu_support import ensure_built, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

DIMS, M0 = (8, 4, 6, 8), -0.25


def apply_all(grg, lat, x):
    import torch

    outs = []
    for prec in ("fp64", "fp32", "bf16"):
        y = torch.empty_like(x)
        grg.grg_dirac_apply(lat, M0, prec, x, y, x.shape[0])
        outs.append(to_host(y))
    return outs


def test_gauge_field_from_device_and_torch_host():
    import torch
    import paper_0704_2341_amd as grg

    ensure_built()
    links = su3_links(DIMS, 0.5, 81)
    x = to_dev(gaussian_vectors(12 * int(np.prod(DIMS)), 2, 82))
    ref = grg.grg_lattice_create(DIMS)
    grg.grg_gauge_set(ref, links)
    want = apply_all(grg, ref, x)
    assert rel_err(want[0], matfree.dirac_apply(links, DIMS, M0, to_host(x))) < 1e-14
    for src in (torch.from_numpy(links).to("cuda"), torch.from_numpy(links)):
        lat = grg.grg_lattice_create(DIMS)
        grg.grg_gauge_set(lat, src)
        got = apply_all(grg, lat, x)
        for a, b in zip(got, want):
            assert np.array_equal(a, b)
        grg.grg_lattice_destroy(lat)
    grg.grg_lattice_destroy(ref)


def test_lattice_on_its_own_stream():
    """Work runs on the lattice's stream and the call returns once that
    stream has drained: the output is complete when the call returns."""
    import torch
    import paper_0704_2341_amd as grg

    ensure_built()
    links = su3_links(DIMS, 0.5, 83)
    V = int(np.prod(DIMS))
    x = to_dev(gaussian_vectors(12 * V, 3, 84))
    ref = grg.grg_lattice_create(DIMS)
    grg.grg_gauge_set(ref, links)
    want = apply_all(grg, ref, x)
    s = torch.cuda.Stream()
    lat = grg.grg_lattice_create(DIMS, stream=s.cuda_stream)
    grg.grg_gauge_set(lat, links)
    q, nb = grg.grg_permutation_block(DIMS, 1, False)
    for a, b in zip(apply_all(grg, lat, x), want):
        assert np.array_equal(a, b)
    # the S_bb apply on that stream, against one on the default stream
    p = grg.grg_solver_params_default(tol=1e-11, inner="bf16", inner_tol=1e-2, max_rhs=3)
    xb = to_dev(gaussian_vectors(12 * nb, 3, 85))
    ys = []
    for lt in (ref, lat):
        h = grg.grg_schur_create(lt, M0, q, nb, p)
        y = torch.empty_like(xb)
        st = grg.grg_schur_apply(h, xb, y, 3)
        assert st["converged"]
        ys.append(to_host(y))
        grg.grg_schur_destroy(h)
    assert np.array_equal(ys[0], ys[1])
    grg.grg_lattice_destroy(lat)
    grg.grg_lattice_destroy(ref)


def test_lattice_queries_and_null_handles():
    import paper_0704_2341_amd as grg

    ensure_built()
    lat = grg.grg_lattice_create(DIMS)
    assert grg.grg_lattice_volume(lat) == int(np.prod(DIMS))
    grg.grg_lattice_destroy(lat)
    # destroying nothing is allowed; using nothing is an invalid argument
    grg.grg_lattice_destroy(None)
    grg.grg_schur_destroy(None)
    with pytest.raises(grg.GrgError) as e:
        grg.grg_lattice_volume(None)
    assert e.value.status == grg.GRG_EINVAL
    for bad in ((8, 4, 0, 8), (8, -2, 6, 8)):
        with pytest.raises(grg.GrgError) as e:
            grg.grg_lattice_create(bad)
        assert e.value.status == grg.GRG_EINVAL
    with pytest.raises(grg.GrgError) as e:
        grg.grg_lattice_create(DIMS, bc=(1, 1, 0, -1))
    assert e.value.status == grg.GRG_EINVAL


def test_new_gauge_field_on_existing_handles():
    """A Schur handle reads the lattice's links at every call: after
    grg_gauge_set its S_bb apply (BF16 inner solve on the even-odd reduced
    D_rr, whose links are repacked) and its section 3 approximation (whose
    row sums of D_rr are cached per gauge field) follow the new field."""
    import torch
    import paper_0704_2341_amd as grg

    ensure_built()
    dims, m0 = (8, 8, 8, 8), -0.2
    fields = [su3_links(dims, 0.5, 86), su3_links(dims, 0.3, 87)]
    lat = grg.grg_lattice_create(dims)
    grg.grg_gauge_set(lat, fields[0])
    q, nb = grg.grg_permutation_block(dims, 1, False)
    p = grg.grg_solver_params_default(tol=1e-12, inner="bf16", inner_tol=1e-2, max_rhs=2)
    h = grg.grg_schur_create(lat, m0, q, nb, p)
    xb = gaussian_vectors(12 * nb, 2, 88)
    x = to_dev(xb)
    for k, links in enumerate(fields):
        if k:
            grg.grg_gauge_set(lat, links)
        y = torch.empty_like(x)
        st = grg.grg_schur_apply(h, x, y, 2)
        assert st["converged"]
        want, _, _ = matfree.schur_apply(links, dims, m0, q, nb, xb, restart=8, tol=1e-13)
        assert rel_err(to_host(y), want) < 1e-10, k
        grg.grg_reusken_apply(h, x, y, 2)
        assert rel_err(to_host(y), matfree.reusken_apply(links, dims, m0, q, nb, xb)) < 1e-12, k
    grg.grg_schur_destroy(h)
    grg.grg_lattice_destroy(lat)


def test_profiling_modes():
    """Full profiling times every stencil launch and the solve's phases and
    reads them per call; launch-only profiling times the same stencil
    launches, no phases, reads them when asked, and reports the per-call
    phase times as -1.  Modes outside 0..2 are rejected."""
    import torch
    import paper_0704_2341_amd as grg
    from paper_0704_2341_amd.binding import load

    ensure_built()
    dims = (8, 8, 8, 8)
    lat = grg.grg_lattice_create(dims)
    grg.grg_gauge_set(lat, su3_links(dims, 0.5, 89))
    q, nb = grg.grg_permutation_block(dims, 1, False)
    p = grg.grg_solver_params_default(tol=1e-10, inner="bf16", inner_tol=1e-2, max_rhs=2)
    h = grg.grg_schur_create(lat, M0, q, nb, p)
    x = to_dev(gaussian_vectors(12 * nb, 2, 90))
    y = torch.empty_like(x)
    grg.grg_schur_apply(h, x, y, 2)
    seen = {}
    for only in (False, True):
        grg.grg_profile_enable(h, True, launches_only=only)
        grg.grg_profile_reset(h)
        sts = [grg.grg_schur_apply(h, x, y, 2) for _ in range(2)]
        seen[only] = {k: grg.grg_profile_read(h, k) for k in ("dc", "blas")}
        seen[only]["eo"] = grg.grg_profile_read(h, "bf16", eo=True)
        seen[only]["stats"] = sts
        grg.grg_profile_enable(h, False)
    full, light = seen[False], seen[True]
    assert full["eo"][0] > 0 and full["eo"][1] > 0
    assert full["dc"][0] > 0 and full["blas"][0] > 0
    assert all(st["t_dc_ms"] > 0 and st["t_dslash_ms"] > 0 for st in full["stats"])
    # the same solves: as many stencil launches timed, no phases
    assert light["eo"][0] == full["eo"][0] and light["eo"][1] > 0
    assert light["dc"] == (0, 0.0) and light["blas"] == (0, 0.0)
    for st in light["stats"]:
        assert st["t_dslash_ms"] == st["t_dc_ms"] == st["t_blas_ms"] == st["t_prec_ms"] == -1.0
    for bad in (-1, 3):
        assert load().grg_profile_enable(h, bad) == grg.GRG_EINVAL
    grg.grg_schur_destroy(h)
    grg.grg_lattice_destroy(lat)
