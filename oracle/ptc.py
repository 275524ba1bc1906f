"""Oracle of the learned preconditioner (test infrastructure only).

A linear gauge-covariant convolution network on the lattice ("parallel
transport convolutions"): every activation is a set of F colour vectors per
site, and one layer is

    Y_f(x) = sum_{h in H} sum_{f'} W_h[f, f'] (T_h X_{f'})(x),
    H = {0, +x, -x, +y, -y, +z, -z, +t, -t},
    T_0 X(x)  = X(x),
    T_+mu X(x) = U_mu(x) X(x + mu),
    T_-mu X(x) = U_mu(x - mu)^dag X(x - mu),

with the boundary sign of the lattice on every hop that wraps (antiperiodic
in t, as in the Dirac operator).  The weights act on the channel index only
and the links on the colour index only, so each layer maps gauge-covariant
fields to gauge-covariant fields.  No bias and no activation function: the
network is linear.  Channels 4 -> 8 -> 8 -> 4; a Dirac field (12 complex per
site) is 4 channels of colour vectors (the spin index is the channel).

Loss over a batch of pairs (r_i, e_i):  L = (1/B) sum_i |M r_i - e_i|^2 / |e_i|^2.
Gradients are Wirtinger derivatives dL/d conj(W) (the real gradient of the
real and imaginary parts is twice their real and imaginary parts).

Layout: fields are complex arrays (V, F, 3); V sites lexicographic, x fastest.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (4, 8, 8, 4)
# hop order: 0, +x, -x, +y, -y, +z, -z, +t, -t
HOPS = [(None, 0)] + [(mu, s) for mu in range(4) for s in (+1, -1)]


def _lat(a, dims):
    lx, ly, lz, lt = dims
    return a.reshape((lt, lz, ly, lx) + a.shape[1:])


def _flat(a, dims):
    return a.reshape((int(np.prod(dims)),) + a.shape[4:])


def _axis(mu):
    return 3 - mu  # lattice arrays are (t, z, y, x)


def _shift(a, dims, mu, step, bc):
    """b(x) = a(x + step*mu), with the boundary sign where the hop wraps."""
    ax = _axis(mu)
    b = np.roll(a, -step, axis=ax)
    if bc[mu] != 1:
        idx = [slice(None)] * b.ndim
        idx[ax] = dims[mu] - 1 if step > 0 else 0
        b[tuple(idx)] *= bc[mu]
    return b


def transport(x, links, dims, mu, step, bc=(1, 1, 1, -1)):
    """T_{step*mu} x for x of shape (V, F, 3)."""
    X = _lat(x, dims)
    Ul = _lat(links, dims)[..., mu, :, :]  # (t, z, y, x, 3, 3)
    if step > 0:
        Xs = _shift(X, dims, mu, +1, bc)
        out = np.einsum("...ab,...fb->...fa", Ul, Xs)
    else:
        Um = np.roll(Ul, 1, axis=_axis(mu))  # U_mu(x - mu)
        Xs = _shift(X, dims, mu, -1, bc)
        out = np.einsum("...ba,...fb->...fa", Um.conj(), Xs)
    return _flat(out, dims)


def hop(x, links, dims, h, bc=(1, 1, 1, -1)):
    mu, step = HOPS[h]
    return x.copy() if mu is None else transport(x, links, dims, mu, step, bc)


def layer_forward(x, w, links, dims, bc=(1, 1, 1, -1)):
    """Y = sum_h W_h T_h X; w: (9, F_out, F_in)."""
    return sum(np.einsum("gf,vfa->vga", w[h], hop(x, links, dims, h, bc)) for h in range(9))


def layer_adjoint(dy, w, links, dims, bc=(1, 1, 1, -1)):
    """The adjoint map: dX = sum_h T_h^dag W_h^H dY (T_{+mu}^dag = T_{-mu})."""
    out = 0
    for h in range(9):
        mu, step = HOPS[h]
        z = np.einsum("gf,vga->vfa", w[h].conj(), dy)
        out = out + (z if mu is None else transport(z, links, dims, mu, -step, bc))
    return out


def layer_weight_grad(dy, x, links, dims, bc=(1, 1, 1, -1)):
    """sum over sites and colours of dY_f conj(T_h X_f'): shape (9, F_out, F_in)."""
    return np.stack([np.einsum("vga,vfa->gf", dy, hop(x, links, dims, h, bc).conj())
                     for h in range(9)])


def net_forward(x, ws, links, dims, bc=(1, 1, 1, -1)):
    """All activations [x, y1, y2, y3] of the three-layer network."""
    acts = [x]
    for w in ws:
        acts.append(layer_forward(acts[-1], w, links, dims, bc))
    return acts


def loss_and_grads(rs, es, ws, links, dims, bc=(1, 1, 1, -1), out_mask=None):
    """Loss over a batch and dL/d conj(W) per layer.  rs, es: (B, V, 4, 3).
    out_mask (V,) of 0/1, if given, multiplies the network output (the
    preconditioner's output lives on the rest sites only)."""
    B = len(rs)
    loss = 0.0
    grads = [np.zeros_like(w) for w in ws]
    m = None if out_mask is None else np.asarray(out_mask, float)[:, None, None]
    for r, e in zip(rs, es):
        acts = net_forward(r, ws, links, dims, bc)
        if m is not None:
            acts[-1] = acts[-1] * m
        en = np.vdot(e, e).real
        d = acts[-1] - e
        loss += np.vdot(d, d).real / en / B
        dy = d / en / B  # dL/d conj(Y)
        if m is not None:
            dy = dy * m
        for l in range(len(ws) - 1, -1, -1):
            grads[l] += layer_weight_grad(dy, acts[l], links, dims, bc)
            dy = layer_adjoint(dy, ws[l], links, dims, bc)
    return loss, grads


def random_weights(seed, scale=0.1, channels=CHANNELS):
    rng = np.random.default_rng(seed)
    return [scale * (rng.standard_normal((9, fo, fi)) + 1j * rng.standard_normal((9, fo, fi)))
            for fi, fo in zip(channels[:-1], channels[1:])]


def pack_weights(ws):
    """Flat complex vector, layer-major, then [hop][f_out][f_in]."""
    return np.concatenate([w.reshape(-1) for w in ws])


def unpack_weights(flat, channels=CHANNELS):
    out, k = [], 0
    for fi, fo in zip(channels[:-1], channels[1:]):
        n = 9 * fo * fi
        out.append(np.asarray(flat[k:k + n]).reshape(9, fo, fi))
        k += n
    return out


def to_channels(field, dims):
    """Dirac field (12 V,) -> (V, 4, 3) channels (spin = channel)."""
    return np.asarray(field).reshape(int(np.prod(dims)), 4, 3)


def _neighbours(sites, dims, mu, step, bc):
    """Lexicographic index of site + step*mu for each site, and the boundary
    sign of the hop (bc[mu] where it wraps, else 1)."""
    c = []
    r = np.asarray(sites, dtype=np.int64)
    for nu in range(4):
        c.append(r % dims[nu])
        r = r // dims[nu]
    n = c[mu] + step
    wrap = (n < 0) | (n >= dims[mu])
    c[mu] = n % dims[mu]
    idx = c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]))
    return idx, np.where(wrap, float(bc[mu]), 1.0)


def net_forward_sites(x, ws, links, dims, sites, bc=(1, 1, 1, -1)):
    """The network output at the given sites only, (len(sites), F, 3).

    Each layer's output at a site needs the previous activation at that site
    and its eight neighbours, so the input is read on the sites within three
    hops.  The activations are evaluated on those shrinking site sets one
    layer after the other, each hop as an explicit neighbour gather with its
    link and boundary sign, for lattices too large for the whole-lattice
    evaluation."""
    links = np.asarray(links)
    sets = [np.unique(np.asarray(sites, dtype=np.int64))]
    for _ in ws:
        s = sets[-1]
        grown = [s] + [_neighbours(s, dims, mu, st, bc)[0] for mu in range(4) for st in (1, -1)]
        sets.append(np.unique(np.concatenate(grown)))
    sets = sets[::-1]  # sets[0]: input sites, sets[-1]: output sites
    act = np.asarray(x)[sets[0]]
    for l, w in enumerate(ws):
        src, dst = sets[l], sets[l + 1]
        pos = {int(s): i for i, s in enumerate(src)}
        out = np.zeros((len(dst), w.shape[1], 3), complex)
        for h, (mu, step) in enumerate(HOPS):
            if mu is None:
                t = act[[pos[int(s)] for s in dst]]
            else:
                n, sign = _neighbours(dst, dims, mu, step, bc)
                xs = act[[pos[int(s)] for s in n]] * sign[:, None, None]
                if step > 0:
                    u = links[dst, mu]                      # U_mu(x)
                    t = np.einsum("vab,vfb->vfa", u, xs)
                else:
                    u = links[n, mu]                        # U_mu(x - mu)
                    t = np.einsum("vba,vfb->vfa", u.conj(), xs)
            out += np.einsum("gf,vfa->vga", w[h], t)
        act = out
    order = np.searchsorted(sets[-1], np.asarray(sites, dtype=np.int64))
    return act[order]
