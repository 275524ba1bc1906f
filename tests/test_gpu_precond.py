"""The learned preconditioner on the GPU against the network oracle:
forward pass, the Wilson-weights identity, loss and Wirtinger gradients,
training on the GPU, its use inside the D_rr solve (gain and fallback) and
the weight file.

Tolerances: activations and weights enter the matrix cores as bfloat16
(unit roundoff 2^-9) with FP32 accumulation, and each layer rounds its output
to bfloat16, so three layers carry a relative error of a few times 2^-9
(checked at 3e-2 norm-wise); gradients are a product of two such fields
(checked at 5e-2 norm-wise, and by their direction: cosine > 0.998).
"""
import numpy as np
import pytest

from grg_inputs import gaussian_vectors, point_sources
from oracle import ptc

from gpu_support import Lattice, rel_err, to_dev, to_host
from test_oracle_pins import golden_gammas

pytestmark = pytest.mark.gpu

# 4^4: a 64-site tile is one x-y-z slice and every hop wraps; 8^4 and
# 8x4x4x8: tiles and slices no longer coincide, hops stay inside the lattice
SHAPES = [(4, 4, 4, 4), (8, 8, 8, 8), (8, 4, 4, 8)]


def masked_field(lat, s, seed, nrhs):
    v = gaussian_vectors(12 * lat.V, nrhs, seed)
    mask = np.zeros(lat.V, bool)
    mask[s.q[:s.nb]] = True
    v[:, np.repeat(mask, 12)] = 0
    return v, (~mask).astype(float)


def oracle_apply(ws, links, dims, x, rmask):
    out = []
    for v in x:
        y = ptc.net_forward(ptc.to_channels(v, dims), ws, links, dims)[-1]
        out.append((y * rmask[:, None, None]).reshape(-1))
    return np.array(out)


@pytest.fixture(scope="module", params=SHAPES, ids=lambda d: "x".join(map(str, d)))
def setup(request):
    lat = Lattice(request.param, 0.5, 41)
    s = lat.schur(-0.2, "I", True, max_rhs=4)
    p = lat.grg.grg_precond_create(s.h)
    yield lat, s, p
    lat.grg.grg_precond_destroy(p)
    s.close()
    lat.close()


def gpu_apply(lat, p, x):
    import torch

    xd = to_dev(x)
    out = torch.empty_like(xd)
    lat.grg.grg_precond_apply(p, xd, out, x.shape[0])
    return to_host(out)


def test_identity_initialisation(setup):
    lat, s, p = setup
    lat.grg.grg_precond_set_weights(p, ptc.pack_weights(identity_weights()))
    x, rmask = masked_field(lat, s, 1, 2)
    assert rel_err(gpu_apply(lat, p, x), x) < 1e-2


def identity_weights():
    ws = [np.zeros((9, fo, fi), complex) for fi, fo in zip(ptc.CHANNELS[:-1], ptc.CHANNELS[1:])]
    for w in ws:
        for f in range(min(w.shape[1:])):
            w[0, f, f] = 1
    return ws


def test_forward_vs_oracle(setup):
    lat, s, p = setup
    ws = ptc.random_weights(3, scale=0.25)
    lat.grg.grg_precond_set_weights(p, ptc.pack_weights(ws))
    assert np.allclose(lat.grg.grg_precond_get_weights(p), ptc.pack_weights(ws))
    x, rmask = masked_field(lat, s, 2, 3)
    want = oracle_apply(ws, lat.links, lat.dims, x, rmask)
    assert rel_err(gpu_apply(lat, p, x), want) < 3e-2


def test_network_with_wilson_weights_is_d_rr(setup):
    """Layer 1 = Wilson operator (on the first four channels), layers 2-3 =
    identity: M = D_rr on rest-site fields."""
    lat, s, p = setup
    m0 = -0.2
    g = golden_gammas()
    ws = identity_weights()
    ws[0][:] = 0
    ws[0][0, :4, :4] = (4 + m0) * np.eye(4)
    for mu in range(4):
        ws[0][1 + 2 * mu, :4, :4] = -0.5 * (np.eye(4) - g[mu])
        ws[0][2 + 2 * mu, :4, :4] = -0.5 * (np.eye(4) + g[mu])
    lat.grg.grg_precond_set_weights(p, ptc.pack_weights(ws))
    x, rmask = masked_field(lat, s, 4, 2)
    from oracle import matfree

    # D_rr x on rest-site inputs: the rest rows of D x (the oracle's stencil)
    want = matfree.dirac_apply(lat.links, lat.dims, m0, x) * np.repeat(rmask, 12)[None, :]
    assert rel_err(gpu_apply(lat, p, x), want) < 2e-2


def test_loss_and_gradients_vs_oracle(setup):
    lat, s, p = setup
    ws = ptc.random_weights(5, scale=0.25)
    lat.grg.grg_precond_set_weights(p, ptc.pack_weights(ws))
    r, rmask = masked_field(lat, s, 6, 3)
    e, _ = masked_field(lat, s, 7, 3)
    loss, grad = lat.grg.grg_precond_loss_grad(p, to_dev(r), to_dev(e), 3)
    rs = np.stack([ptc.to_channels(v, lat.dims) for v in r])
    es = np.stack([ptc.to_channels(v, lat.dims) for v in e])
    lo, go = ptc.loss_and_grads(rs, es, ws, lat.links, lat.dims, out_mask=rmask)
    go = ptc.pack_weights(go)
    assert abs(loss - lo) < 3e-2 * lo
    assert np.linalg.norm(grad - go) < 5e-2 * np.linalg.norm(go)
    cos = np.real(np.vdot(grad, go)) / np.linalg.norm(grad) / np.linalg.norm(go)
    assert cos > 0.998


@pytest.mark.parametrize("reduced", [False, True])
def test_training_reduces_loss_and_iterations(reduced):
    """Pairs of D_rr itself, or of its even-odd reduced system (the inner
    solve the network then serves)."""
    lat = Lattice((8, 8, 8, 8), 0.5, 5)
    s = lat.schur(-0.3, "I", False, tol=1e-10, inner="bf16", inner_tol=1e-2, max_rhs=12)
    grg = lat.grg
    p = grg.grg_precond_create(s.h)
    st = grg.grg_precond_train(p, steps=200, batch=8, max_mr_steps=20, lr=3e-3, seed=5, log_every=20,
                               reduced=reduced)
    print(f"reduced={reduced}: {st}", flush=True)
    assert st["pairs"] == 1600 and st["loss_last"] < 0.5 * st["loss_first"], st
    xb = point_sources(s.nb, 12)
    y0, st0 = s.apply(xb)
    grg.grg_schur_attach_precond(s.h, p)
    y1, st1 = s.apply(xb)
    assert st1["converged"] and st1["fallbacks"] == 0
    assert rel_err(y1, y0) < 1e-9
    print(f"inner iterations: plain {st0['iters']}, learned {st1['iters']}", flush=True)
    assert st1["iters"] < st0["iters"], (st0, st1)
    grg.grg_schur_attach_precond(s.h, None)
    grg.grg_precond_destroy(p)
    s.close()
    lat.close()


def test_nan_weights_fall_back_to_plain_gcr(setup, tmp_path):
    lat, s, p = setup
    grg = lat.grg
    ws = ptc.pack_weights(ptc.random_weights(8))
    grg.grg_precond_set_weights(p, ws)
    path = str(tmp_path / "w.bin")
    grg.grg_precond_save(p, path)
    bad = ws.copy()
    bad[17] = np.nan
    grg.grg_precond_set_weights(p, bad)
    xb = gaussian_vectors(12 * s.nb, 2, 9)
    y0, _ = s.apply(xb)
    grg.grg_schur_attach_precond(s.h, p)
    y1, st = s.apply(xb)
    grg.grg_schur_attach_precond(s.h, None)
    assert st["converged"] and st["fallbacks"] >= 1 and rel_err(y1, y0) < 1e-9
    grg.grg_precond_load(p, path)
    assert np.array_equal(grg.grg_precond_get_weights(p), ws)
