"""Oracle of the cyclic-reduction V-cycle of section 4 (test infrastructure only).

Written from the block elimination of section 1 applied level by level, with
every level's operator defined through the previous level's blocks, never
through the coarse-lattice Wilson form the GPU builds it from:

    level 0:      A_0 = D (matrix-free C oracle)
    level k + 1:  A_{k+1} = (A_k)_bb - (A_k)_br diag((A_k)_rr)^{-1} (A_k)_rb
                  on the coarse sites of level k (all-even set, Type I), the
                  Schur complement with the couplings inside (A_k)_rr ignored,
                  its diagonal taken by probing
    cycle(k) f:   y = (A_k)_rr^{-1} f_r,  g = f_b - (A_k)_br y,
                  x_b = cycle(k + 1) g  (the top level: solved),
                  x_r = (A_k)_rr^{-1} (f_r - (A_k)_rb x_b)

Solves are plain restarted GCR in numpy to a tight tolerance, so the cycle is
the deterministic operator the GPU's cycle approaches when its own inner
tolerances are tight.  `two_level_cycle` (matrix-free) and `two_level_cycle_dense` take one
level of the same cycle on the partition of any section 2 ordering, with
section 3's S~_bb (or the exact complement) on top.

Also `block_links` and `coarse_wilson_apply`: the
coarse-lattice Wilson form, (1/d) D_W(V, d^2 - 4) with V_mu(c) = U_mu(2c)
U_mu(2c + mu), that the pins compare with the level operator above.
"""
from __future__ import annotations

import numpy as np

from . import dense, matfree


def gcr(apply, b, tol=1e-13, restart=16, maxit=20000):
    """x with |b - A x| <= tol |b| for one vector b (restarted GCR, MGS)."""
    b = np.asarray(b, np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0:
        return x
    it = 0
    while np.linalg.norm(r) > tol * nb and it < maxit:
        ps, qs = [], []
        for _ in range(restart):
            p = r.copy()
            q = apply(p)
            for pj, qj in zip(ps, qs):
                beta = np.vdot(qj, q)
                q = q - beta * qj
                p = p - beta * pj
            nq = np.linalg.norm(q)
            q, p = q / nq, p / nq
            a = np.vdot(q, r)
            x = x + a * p
            r = r - a * q
            ps.append(p)
            qs.append(q)
            it += 1
            if np.linalg.norm(r) <= tol * nb:
                break
        r = b - apply(x)  # recomputed at every restart
    return x


def block_links(links, dims):
    """V_mu(c) = U_mu(2c) U_mu(2c + mu) on the coarse lattice (dims / 2),
    canonical [Vc][4][3][3]; boundary signs are applied by the operator."""
    links = np.asarray(links).reshape(*dims[::-1], 4, 3, 3)  # [t][z][y][x]
    cd = [L // 2 for L in dims]
    out = np.empty((*cd[::-1], 4, 3, 3), np.complex128)
    ev = links[::2, ::2, ::2, ::2]
    for mu in range(4):
        ax = 3 - mu  # x is the last array axis
        nxt = np.roll(links, -1, axis=ax)[::2, ::2, ::2, ::2]
        out[..., mu, :, :] = ev[..., mu, :, :] @ nxt[..., mu, :, :]
    return out.reshape(-1, 4, 3, 3)


def coarse_wilson_apply(links, dims, m0, x, bc=(1, 1, 1, -1)):
    """(1/d) D_W(V, d^2 - 4) x on the coarse lattice, d = 4 + m0."""
    d = 4.0 + m0
    cd = tuple(L // 2 for L in dims)
    return matfree.dirac_apply(block_links(links, dims), cd, d * d - 4.0, x, bc) / d


class Level:
    """A level: apply(x) for vectors of n sites x 12 dof (one RHS), and its
    Type I partition on the site extents `dims`."""

    def __init__(self, apply, dims):
        self.apply = apply
        self.dims = tuple(dims)
        self.n = int(np.prod(dims))
        q, nb = dense.permutation_block(self.dims, "I")
        self.q, self.nb = np.asarray(q), int(nb)
        self.coarse = np.asarray(q[:nb])
        self.rest = np.ones(self.n, bool)
        self.rest[self.coarse] = False

    def mask(self, x, rest):
        y = x.reshape(self.n, 12).copy()
        y[~self.rest if rest else self.rest] = 0
        return y.reshape(-1)

    def rr_solve(self, f, tol):
        return gcr(lambda v: self.mask(self.apply(self.mask(v, True)), True), self.mask(f, True), tol)

    def rest_diagonal(self):
        """Diagonal of A restricted to the rest sites, by probing with the 16
        classes of coordinate parities (sites of one class share no coupling
        when A couples nearest neighbours only) times 12 dof."""
        c = np.indices(self.dims[::-1]).reshape(4, -1)[::-1]
        cls = np.array([1, 2, 4, 8]) @ (c % 2)
        diag = np.zeros((self.n, 12), np.complex128)
        for k in range(16):
            sel = cls == k
            for a in range(12):
                e = np.zeros((self.n, 12), np.complex128)
                e[sel, a] = 1
                diag[sel, a] = self.apply(e.reshape(-1)).reshape(self.n, 12)[sel, a]
        diag[~self.rest] = 0
        return diag.reshape(-1)

    def next_level(self):
        """A_{k+1} on the coarse sites, in their own lexicographic order."""
        dinv = np.zeros(self.n * 12, np.complex128)
        dr = self.rest_diagonal()
        nz = dr != 0
        dinv[nz] = 1.0 / dr[nz]
        cd = [L // 2 for L in self.dims]

        def apply(xb):
            u = np.zeros((self.n, 12), np.complex128)
            u[self.coarse] = xb.reshape(-1, 12)
            y = self.mask(self.apply(u.reshape(-1)), True) * dinv
            w = u.reshape(-1) - y
            return self.apply(w).reshape(self.n, 12)[self.coarse].reshape(-1)

        return Level(apply, cd)


def hierarchy(links, dims, m0, levels, bc=(1, 1, 1, -1)):
    lv = [Level(lambda x: matfree.dirac_apply(links, dims, m0, x[None, :], bc)[0], dims)]
    for _ in range(levels - 1):
        lv.append(lv[-1].next_level())
    return lv


def cycle(lv, k, f, tol=1e-13):
    """One V-cycle on level k for one vector f."""
    L = lv[k]
    if k == len(lv) - 1:
        return gcr(L.apply, f, tol)
    y = L.rr_solve(f, tol)
    t = L.apply(y).reshape(L.n, 12)
    g = (f.reshape(L.n, 12) - t)[L.coarse].reshape(-1)
    xb = cycle(lv, k + 1, g, tol)
    u = np.zeros((L.n, 12), np.complex128)
    u[L.coarse] = xb.reshape(-1, 12)
    h = f - L.apply(u.reshape(-1))
    xr = L.rr_solve(h, tol)
    return L.mask(xr, True) + u.reshape(-1)


# ---------------------------------------------------------------- two levels, any partition
def two_level_cycle(links, dims, m0, q, nb, f, top="reusken", tol=1e-13, bc=(1, 1, 1, -1)):
    """One two-level cycle of section 4 on the partition (q, nb) of any of
    the section 2 orderings (Type I, II and their inverses), for one vector f
    of 12 V entries:

        y = D_rr^{-1} f_r,  g = f_b - D_br y,  x_b = S_top^{-1} g,
        x_r = D_rr^{-1} (f_r - D_rb x_b),  x = x_r + x_b,

    where the top operator S_top is the section 3 approximation S~_bb
    ("reusken", matrix-free) or the exact Schur complement ("exact"), and
    every solve runs GCR to tol (the cycle the GPU approaches when its own
    tolerances are tight)."""
    v = int(np.prod(dims))
    q = np.asarray(q)
    nb = int(nb)
    coarse = q[:nb]
    f = np.asarray(f, np.complex128).reshape(v, 12)
    fr = f.copy()
    fr[coarse] = 0
    y = matfree.drr_solve(links, dims, m0, q, nb, fr.reshape(1, -1), tol=tol, bc=bc)[0][0]
    t = matfree.block_apply(links, dims, m0, q, nb, 1, 0, y[None, :], bc)[0].reshape(v, 12)
    g = (f - t)[coarse].reshape(-1)
    if top == "reusken":
        def apply(xb):
            return matfree.reusken_apply(links, dims, m0, q, nb, xb[None, :], bc)[0]
    elif top == "exact":
        def apply(xb):
            return matfree.schur_apply(links, dims, m0, q, nb, xb[None, :], tol=tol, bc=bc)[0][0]
    else:
        raise ValueError(f"unknown top level {top!r}")
    xb = gcr(apply, g, tol)
    u = np.zeros((v, 12), np.complex128)
    u[coarse] = xb.reshape(nb, 12)
    h = fr - matfree.block_apply(links, dims, m0, q, nb, 0, 1, u.reshape(1, -1), bc)[0].reshape(v, 12)
    xr = matfree.drr_solve(links, dims, m0, q, nb, h.reshape(1, -1), tol=tol, bc=bc)[0][0].reshape(v, 12)
    xr[coarse] = 0
    return (xr + u).reshape(-1)


def two_level_cycle_dense(d, q, nb, f, top="reusken"):
    """The same cycle from the dense operator d (small lattices): the blocks
    of P D P^T, S_top dense (section 3's S~_bb or the exact S_bb), every solve
    by LU."""
    import scipy.linalg as sla

    nb = int(nb)
    dbb, dbr, drb, drr = dense.blocks(d, q, nb)
    s_top = dense.reusken_dense(d, q, nb) if top == "reusken" else dense.schur_dense(d, q, nb)
    o = dense.dof_order(q)
    f = np.asarray(f, np.complex128).reshape(-1)
    fb, fr = f[o[: 12 * nb]], f[o[12 * nb:]]
    lu = sla.lu_factor(drr)
    y = sla.lu_solve(lu, fr)
    xb = np.linalg.solve(s_top, fb - dbr @ y)
    xr = sla.lu_solve(lu, fr - drb @ xb)
    x = np.zeros_like(f)
    x[o[: 12 * nb]] = xb
    x[o[12 * nb:]] = xr
    return x
