"""Pins of the network oracle (oracle.ptc): unitary and adjoint transports,
gauge equivariance, one layer with Wilson weights equal to the Dirac operator,
the adjoint layer, and gradients against central finite differences."""
import numpy as np
import pytest

from grg_inputs import su3_links
from oracle import dense, ptc

from test_oracle_pins import golden_gammas, random_omega, gauge_transform

DIMS = (4, 4, 4, 4)
V = 256


@pytest.fixture(scope="module")
def links():
    return su3_links(DIMS, 0.5, 12)


def rfield(seed, f=4):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((V, f, 3)) + 1j * rng.standard_normal((V, f, 3))


@pytest.mark.parametrize("mu", range(4))
def test_transport_unitary_and_adjoint(links, mu):
    a, b = rfield(1), rfield(2)
    tb = ptc.transport(b, links, DIMS, mu, +1)
    assert np.allclose(ptc.transport(tb, links, DIMS, mu, -1), b, atol=1e-13)
    lhs = np.vdot(a, tb)
    rhs = np.vdot(ptc.transport(a, links, DIMS, mu, -1), b)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_layer_is_wilson_operator_with_wilson_weights(links):
    """W_0 = (4 + m0) 1, W_{+mu} = -1/2 (1 - g_mu), W_{-mu} = -1/2 (1 + g_mu)
    acting on the spin index makes one layer the Dirac operator."""
    m0 = -0.2
    g = golden_gammas()
    w = np.zeros((9, 4, 4), complex)
    w[0] = (4 + m0) * np.eye(4)
    for mu in range(4):
        w[1 + 2 * mu] = -0.5 * (np.eye(4) - g[mu])
        w[2 + 2 * mu] = -0.5 * (np.eye(4) + g[mu])
    x = rfield(3)
    y = ptc.layer_forward(x, w, links, DIMS)
    d = dense.wilson_dense(links, DIMS, m0)
    assert np.abs(y.reshape(-1) - d @ x.reshape(-1)).max() < 1e-12


def test_layer_gauge_equivariant(links):
    ws = ptc.random_weights(4)
    om = random_omega(V, 8)
    lo = gauge_transform(links, om, DIMS)
    x = rfield(5)
    ox = np.einsum("vab,vfb->vfa", om, x)
    for w in ws[:1]:
        y = ptc.layer_forward(x, w, links, DIMS)
        y2 = ptc.layer_forward(ox, w, lo, DIMS)
        assert np.abs(y2 - np.einsum("vab,vfb->vfa", om, y)).max() < 1e-12


def test_identity_weights_and_linearity(links):
    w = np.zeros((9, 4, 4), complex)
    w[0] = np.eye(4)
    x = rfield(6)
    assert np.array_equal(ptc.layer_forward(x, w, links, DIMS), x)
    ws = ptc.random_weights(7)
    a, b = rfield(8), rfield(9)
    f = lambda z: ptc.net_forward(z, ws, links, DIMS)[-1]
    assert np.allclose(f(a + 2j * b), f(a) + 2j * f(b), atol=1e-12)


def test_one_parity_pairs_leave_zero_hop_weights_without_gradient(links):
    """Each hop moves a field to the other parity, so at weights without hop
    terms (the identity start) the hop-weight gradients from pairs that live
    on one parity pair fields of opposite parities and vanish; pairs on both
    parities give them a gradient."""
    ws = []
    for fi, fo in zip(ptc.CHANNELS[:-1], ptc.CHANNELS[1:]):
        w = np.zeros((9, fo, fi), complex)
        for f in range(min(fi, fo)):
            w[0, f, f] = 1.0
        ws.append(w)
    c = np.indices(DIMS[::-1]).reshape(4, -1)[::-1]  # (x, y, z, t) of site x + 4 (y + 4 (z + 4 t))
    even = (c.sum(axis=0) % 2 == 0).astype(float)[:, None, None]
    r = np.stack([rfield(31) * even, rfield(32) * even])
    e = np.stack([rfield(33) * even, rfield(34) * even])
    _, g = ptc.loss_and_grads(r, e, ws, links, DIMS, out_mask=even[:, 0, 0])
    for gl in g:
        assert np.abs(gl[1:]).max() < 1e-14 and np.abs(gl[0]).max() > 1e-3
    _, g = ptc.loss_and_grads(np.stack([rfield(35), rfield(36)]), np.stack([rfield(37), rfield(38)]),
                              ws, links, DIMS)
    assert all(np.abs(gl[1:]).max() > 1e-3 for gl in g)


def test_layer_adjoint(links):
    ws = ptc.random_weights(10)
    x, dy = rfield(11, 8), rfield(12, 8)
    w = ws[1]
    lhs = np.vdot(dy, ptc.layer_forward(x, w, links, DIMS))
    rhs = np.vdot(ptc.layer_adjoint(dy, w, links, DIMS), x)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_gradients_match_finite_differences(links):
    ws = ptc.random_weights(13, scale=0.3)
    rs = np.stack([rfield(20 + i) for i in range(2)])
    es = np.stack([rfield(30 + i) for i in range(2)])
    loss, grads = ptc.loss_and_grads(rs, es, ws, links, DIMS)
    rng = np.random.default_rng(14)
    eps = 1e-6
    for _ in range(12):
        l = int(rng.integers(3))
        idx = tuple(int(rng.integers(n)) for n in ws[l].shape)
        for part in (1, 1j):
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += eps * part
            wm[l][idx] -= eps * part
            lp, _ = ptc.loss_and_grads(rs, es, wp, links, DIMS)
            lm, _ = ptc.loss_and_grads(rs, es, wm, links, DIMS)
            fd = (lp - lm) / (2 * eps)
            an = 2 * (grads[l][idx].real if part == 1 else grads[l][idx].imag)
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (l, idx, part, fd, an)


def test_planted_mistake_in_transport_is_caught(links, monkeypatch):
    """Using U instead of U^dag on the backward hop breaks the Wilson pin."""
    real = ptc.transport

    def wrong(x, lk, dims, mu, step, bc=(1, 1, 1, -1)):
        if step < 0:
            return real(x, lk.conj().transpose(0, 1, 3, 2), dims, mu, step, bc)
        return real(x, lk, dims, mu, step, bc)

    monkeypatch.setattr(ptc, "transport", wrong)
    g = golden_gammas()
    w = np.zeros((9, 4, 4), complex)
    w[0] = 4 * np.eye(4)
    for mu in range(4):
        w[1 + 2 * mu] = -0.5 * (np.eye(4) - g[mu])
        w[2 + 2 * mu] = -0.5 * (np.eye(4) + g[mu])
    x = rfield(3)
    y = ptc.layer_forward(x, w, links, DIMS)
    d = dense.wilson_dense(links, DIMS, 0.0)
    assert np.abs(y.reshape(-1) - d @ x.reshape(-1)).max() > 1e-3


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_forward_at_sites_equals_whole_lattice(dims):
    """The sampled-site evaluation (explicit neighbour gathers on the sites
    within three hops) against the whole-lattice evaluation (array shifts),
    on every site and on an unsorted sample with repeats; antiperiodic and
    periodic t."""
    from grg_inputs import su3_links

    v = int(np.prod(dims))
    links = su3_links(dims, 0.5, 3)
    ws = ptc.random_weights(4, scale=0.3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((v, 4, 3)) + 1j * rng.standard_normal((v, 4, 3))
    for bc in ((1, 1, 1, -1), (1, 1, 1, 1)):
        full = ptc.net_forward(x, ws, links, dims, bc)[-1]
        assert np.allclose(ptc.net_forward_sites(x, ws, links, dims, np.arange(v), bc), full,
                           rtol=0, atol=1e-12 * np.abs(full).max())
        smp = np.array([v - 1, 0, 17 % v, 0, v // 2])
        assert np.allclose(ptc.net_forward_sites(x, ws, links, dims, smp, bc), full[smp],
                           rtol=0, atol=1e-12 * np.abs(full).max())
