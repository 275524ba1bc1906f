"""Many-lattice batch against the single-lattice path and the oracle: every
member's S_bb apply, graph replays against eager launches, and the 48-lattice
workload (sizes uniform over {8^4, 12^4, 16^4, 8^3x16}, own seeds, m0 in
[-0.3, 0.1], 4 RHS, FP32 inner / FP64 outer)."""
import numpy as np
import pytest

from grg_inputs import batch_instances, gaussian_vectors, su3_links
from oracle import matfree

from gpu_support import Lattice, ensure_built, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def members(descs, kinds):
    import paper_0704_2341_amd as grg

    out = []
    for d, (kind, inv) in zip(descs, kinds):
        q, nb = grg.grg_permutation_block(d["dims"], kind, inv)
        out.append(dict(dims=d["dims"], m0=d["m0"], links=su3_links(d["dims"], 0.5, d["seed"]), q=q,
                        n_coarse=nb, seed=d["seed"]))
    return out


def batch_inputs(b, ms, nrhs, seed):
    import paper_0704_2341_amd as grg

    total, _ = grg.grg_batch_layout(b, len(ms))
    x = np.zeros(total, np.complex128)
    for i, m in enumerate(ms):
        off, nb = grg.grg_batch_layout(b, i)
        x[off:off + 12 * nb * nrhs] = gaussian_vectors(12 * nb, nrhs, seed + i).reshape(-1)
    return x


def split(b, ms, y, nrhs):
    import paper_0704_2341_amd as grg

    out = []
    for i in range(len(ms)):
        off, nb = grg.grg_batch_layout(b, i)
        out.append(y[off:off + 12 * nb * nrhs].reshape(nrhs, 12 * nb))
    return out


@pytest.mark.parametrize("eo", [1, 0])
def test_small_batch_matches_single_and_oracle(eo):
    """eo 1: the inner solve on each lattice's even-odd reduced D_rr (every
    extent even), with the other parity reconstructed; eo 0: on D_rr."""
    import torch
    import paper_0704_2341_amd as grg

    ensure_built()
    descs = [dict(dims=(8, 8, 8, 8), m0=-0.3, seed=4001), dict(dims=(4, 4, 4, 4), m0=0.1, seed=4002),
             dict(dims=(8, 8, 4, 8), m0=-0.1, seed=4003), dict(dims=(4, 8, 8, 4), m0=0.05, seed=4004)]
    kinds = [(1, False), (2, True), (1, True), (2, False)]
    ms = members(descs, kinds)
    nrhs = 3
    p = grg.grg_solver_params_default(tol=1e-12, inner="fp32", inner_tol=1e-5, check_every=3, eo=eo)
    b = grg.grg_batch_create(ms, nrhs, p)
    grg.grg_batch_tune(b)
    x = batch_inputs(b, ms, nrhs, 50)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    st = grg.grg_batch_apply(b, xd, yd, use_graph=True)
    assert st["converged"] and st["true_rel_resid"] <= 1e-12
    ys = split(b, ms, to_host(yd), nrhs)
    xs = split(b, ms, x, nrhs)
    for i, m in enumerate(ms):
        lat = Lattice(m["dims"], 0.5, m["seed"], links=m["links"])
        q = m["q"]
        sh = grg.grg_schur_create(lat.h, m["m0"], q, m["n_coarse"], grg.grg_solver_params_default(tol=1e-12))
        xx = to_dev(xs[i])
        yy = torch.empty_like(xx)
        grg.grg_schur_apply(sh, xx, yy, nrhs)
        assert rel_err(ys[i], to_host(yy)) < 1e-10, i
        grg.grg_schur_destroy(sh)
        lat.close()
    # the 8^4 member against the C oracle
    want, _, _ = matfree.schur_apply(ms[0]["links"], ms[0]["dims"], ms[0]["m0"], ms[0]["q"],
                                     ms[0]["n_coarse"], xs[0][:2], tol=1e-13)
    assert rel_err(ys[0][:2], want) < 1e-10
    grg.grg_batch_destroy(b)


def test_graph_replays_match_eager():
    import torch
    import paper_0704_2341_amd as grg

    ensure_built()
    descs = [dict(dims=(8, 8, 8, 8), m0=-0.2, seed=4011), dict(dims=(8, 8, 8, 16), m0=0.0, seed=4012)]
    ms = members(descs, [(1, False), (1, True)])
    p = grg.grg_solver_params_default(tol=1e-10, inner="bf16", inner_tol=1e-2, check_every=4)
    b = grg.grg_batch_create(ms, 4, p)
    assert grg.grg_batch_graph_info(b) == (0, 0)
    x = to_dev(batch_inputs(b, ms, 4, 60))
    y = torch.empty_like(x)
    st0 = grg.grg_batch_apply(b, x, y, use_graph=False)
    eager = to_host(y)
    for _ in range(3):
        y.zero_()
        torch.cuda.synchronize()
        st = grg.grg_batch_apply(b, x, y, use_graph=True)
        # the captured apply: as many outer steps as the eager one took, and
        # at least its inner iterations per step
        outer, inner = grg.grg_batch_graph_info(b)
        assert outer == st0["outer"] and inner >= 1, (outer, inner, st0)
        assert st["converged"] and st["iters"] == st0["iters"] and st["outer"] == st0["outer"]
        # same systems take the same iterations on the device: same bits
        assert np.array_equal(to_host(y), eager)
        grg.grg_batch_apply(b, x, y, use_graph=False)  # eager work between replays
        assert np.array_equal(to_host(y), eager)
    grg.grg_batch_destroy(b)


@pytest.mark.parametrize("eo", [1, 0])
def test_device_control_edge_cases(eo):
    """Zero inputs (a system with b = 0 never takes a step; an all-zero
    batch takes none and gives zero), and an input that needs more
    iterations than the captured graph holds: the apply continues eagerly
    from the graph's verified residual and the batch is re-captured.  The
    members other than the first are heavy (m0 = 1: few iterations), so the
    counts recorded without the first member are short of what it needs."""
    import torch
    import paper_0704_2341_amd as grg

    ensure_built()
    descs = [dict(dims=(8, 8, 8, 8), m0=-0.3, seed=4021), dict(dims=(4, 4, 4, 4), m0=1.0, seed=4022),
             dict(dims=(8, 8, 4, 8), m0=1.0, seed=4023)]
    ms = members(descs, [(1, False), (2, True), (1, True)])
    nrhs = 2
    p = grg.grg_solver_params_default(tol=1e-10, inner="fp32", inner_tol=1e-5, check_every=2, eo=eo)
    b = grg.grg_batch_create(ms, nrhs, p)
    x = batch_inputs(b, ms, nrhs, 80)
    # all zero: no step, zero output, in both modes
    z = to_dev(np.zeros_like(x))
    y = torch.full_like(z, 1.0)
    st = grg.grg_batch_apply(b, z, y, use_graph=False)
    assert st["converged"] and st["outer"] == 0 and st["iters"] == 0 and not torch.any(y)
    # the slow member (m0 = -0.3) at zero: the recorded counts are the fast members'
    off0, nb0 = grg.grg_batch_layout(b, 0)
    xe = x.copy()
    xe[off0:off0 + 12 * nb0 * nrhs] = 0
    ye = torch.empty_like(z)
    st_e = grg.grg_batch_apply(b, to_dev(xe), ye, use_graph=False)
    assert st_e["converged"]
    assert not torch.any(ye[off0:off0 + 12 * nb0 * nrhs])
    y.fill_(1.0)
    st = grg.grg_batch_apply(b, z, y, use_graph=True)  # a captured apply of zeros
    assert st["converged"] and grg.grg_batch_graph_info(b) != (0, 0) and not torch.any(y)
    captured = grg.grg_batch_graph_info(b)
    # the full input through the short graph, continued eagerly
    yg = torch.empty_like(z)
    st_g = grg.grg_batch_apply(b, to_dev(x), yg, use_graph=True)
    assert st_g["converged"] and st_g["true_rel_resid"] <= 1e-10, st_g
    yf = torch.empty_like(z)
    st_f = grg.grg_batch_apply(b, to_dev(x), yf, use_graph=False)
    assert st_f["converged"]
    assert rel_err(to_host(yg), to_host(yf)) < 1e-9
    want, _, _ = matfree.schur_apply(ms[0]["links"], ms[0]["dims"], ms[0]["m0"], ms[0]["q"], ms[0]["n_coarse"],
                                     split(b, ms, x, nrhs)[0], tol=1e-13)
    assert rel_err(split(b, ms, to_host(yg), nrhs)[0], want) < 1e-9
    # the next captured apply holds more outer steps and runs to the end alone
    st_g2 = grg.grg_batch_apply(b, to_dev(x), yg, use_graph=True)
    assert st_g2["converged"]
    now = grg.grg_batch_graph_info(b)
    assert now[0] > captured[0] or now[1] > captured[1], (captured, now)
    grg.grg_batch_destroy(b)


def test_48_lattice_workload():
    import torch
    import paper_0704_2341_amd as grg

    ensure_built()
    descs = batch_instances(48)
    ms = members(descs, [(1, False)] * 48)
    assert abs(sum(int(np.prod(m["dims"])) for m in ms) - 48 * 24640) < 48 * 24640
    nrhs = 4
    p = grg.grg_solver_params_default(tol=1e-10, inner="fp32", inner_tol=1e-5, check_every=4)
    b = grg.grg_batch_create(ms, nrhs, p)
    grg.grg_batch_tune(b)
    x = batch_inputs(b, ms, nrhs, 70)
    xd = to_dev(x)
    y = torch.empty_like(xd)
    st = grg.grg_batch_apply(b, xd, y, use_graph=True)  # eager: records the counts
    assert st["converged"] and st["true_rel_resid"] <= 1e-10
    first = to_host(y)
    st = grg.grg_batch_apply(b, xd, y, use_graph=True)  # one captured replay
    assert st["converged"] and st["true_rel_resid"] <= 1e-10
    assert grg.grg_batch_graph_info(b) != (0, 0)
    assert np.array_equal(to_host(y), first)
    ys = split(b, ms, to_host(y), nrhs)
    xs = split(b, ms, x, nrhs)
    for i in (0, 17, 47):  # spot members against the oracle
        m = ms[i]
        want, _, _ = matfree.schur_apply(m["links"], m["dims"], m["m0"], m["q"], m["n_coarse"],
                                         xs[i][:1], tol=1e-13)
        assert rel_err(ys[i][:1], want) < 1e-9, i
    grg.grg_batch_destroy(b)


def test_bicgstab_is_rejected():
    """The batch's captured inner loop is minimal residual only."""
    import paper_0704_2341_amd as grg

    ensure_built()
    ms = members([dict(dims=(4, 4, 4, 4), m0=0.1, seed=4005)], [(1, False)])
    p = grg.grg_solver_params_default(tol=1e-10, inner="fp32", inner_tol=1e-5, method="bicgstab")
    with pytest.raises(grg.GrgError):
        grg.grg_batch_create(ms, 2, p)
