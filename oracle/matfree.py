"""ctypes binding of the C oracle O2 (oracle/matfree.c).  Test infrastructure only.

All arrays are numpy complex128 in canonical layout (see oracle/matfree.c).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        cdp = np.ctypeslib.ndpointer(np.complex128, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        L.orc_num_threads.restype = C.c_int
        L.orc_dirac_apply.argtypes = [i32p, i32p, cdp, C.c_double, cdp, cdp, C.c_int]
        L.orc_block_apply.argtypes = [i32p, i32p, cdp, C.c_double, i32p, C.c_int32, C.c_int,
                                      C.c_int, cdp, cdp, C.c_int]
        L.orc_block_apply_abs.argtypes = [i32p, i32p, cdp, C.c_double, i32p, C.c_int32, C.c_int,
                                          C.c_int, C.c_int, cdp, f64p, C.c_int]
        L.orc_drr_solve.argtypes = [i32p, i32p, cdp, C.c_double, i32p, C.c_int32, cdp, cdp,
                                    C.c_int, C.c_int, C.c_double, C.c_int, i32p, f64p]
        L.orc_drr_residual.argtypes = [i32p, i32p, cdp, C.c_double, i32p, C.c_int32, cdp, cdp,
                                       C.c_int, f64p]
        L.orc_schur_apply.argtypes = [i32p, i32p, cdp, C.c_double, i32p, C.c_int32, cdp, cdp,
                                      C.c_int, C.c_int, C.c_double, C.c_int, i32p, f64p]
        _lib = L
    return _lib


def _geom(dims, bc):
    return (np.ascontiguousarray(dims, dtype=np.int32), np.ascontiguousarray(bc, dtype=np.int32))


def _fields(a, per):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.ndim == 1:
        a = a[None, :]
    assert a.shape[1] == per, (a.shape, per)
    return a


def num_threads() -> int:
    return int(lib().orc_num_threads())


def dirac_apply(links, dims, m0, x, bc=(1, 1, 1, -1)):
    """D x for x of shape (nrhs, 12V)."""
    d, b = _geom(dims, bc)
    v = int(np.prod(dims))
    x = _fields(x, 12 * v)
    out = np.empty_like(x)
    lib().orc_dirac_apply(d, b, np.ascontiguousarray(links), float(m0), x, out, x.shape[0])
    return out


def block_apply(links, dims, m0, q, nb, osel, isel, x, bc=(1, 1, 1, -1)):
    """mask_osel D mask_isel x with sel = 1 for coarse sites q[:nb], 0 for the rest."""
    d, b = _geom(dims, bc)
    v = int(np.prod(dims))
    x = _fields(x, 12 * v)
    out = np.empty_like(x)
    lib().orc_block_apply(d, b, np.ascontiguousarray(links), float(m0),
                          np.ascontiguousarray(q, dtype=np.int32), int(nb), int(osel), int(isel),
                          x, out, x.shape[0])
    return out


def block_apply_abs(links, dims, m0, q, nb, osel, isel, x, diag=True, bc=(1, 1, 1, -1)):
    """Per output entry of block_apply, the sum of the absolute values of the
    products it is made of (|1 -/+ gamma| |U| |x|, plus |4 + m0| |x| with
    diag): the scale of the rounding error of any evaluation from inputs with
    a given relative error.  Real array (nrhs, 12 V)."""
    d, b = _geom(dims, bc)
    v = int(np.prod(dims))
    x = _fields(x, 12 * v)
    out = np.empty(x.shape, np.float64)
    lib().orc_block_apply_abs(d, b, np.ascontiguousarray(links), float(m0),
                              np.ascontiguousarray(q, dtype=np.int32), int(nb), int(osel), int(isel),
                              int(bool(diag)), x, out, x.shape[0])
    return out


def drr_solve(links, dims, m0, q, nb, rhs, restart=8, tol=1e-13, maxit=10000, bc=(1, 1, 1, -1)):
    """GCR solve of D_rr x = rhs; returns (x, iters, relres)."""
    d, b = _geom(dims, bc)
    v = int(np.prod(dims))
    rhs = _fields(rhs, 12 * v)
    x = np.empty_like(rhs)
    it = np.zeros(rhs.shape[0], np.int32)
    rr = np.zeros(rhs.shape[0], np.float64)
    lib().orc_drr_solve(d, b, np.ascontiguousarray(links), float(m0),
                        np.ascontiguousarray(q, dtype=np.int32), int(nb), rhs, x, rhs.shape[0],
                        int(restart), float(tol), int(maxit), it, rr)
    return x, it, rr


def drr_residual(links, dims, m0, q, nb, rhs, x, bc=(1, 1, 1, -1)):
    """||rhs - D_rr x|| / ||rhs|| per RHS, recomputed in FP64 by the oracle."""
    d, b = _geom(dims, bc)
    v = int(np.prod(dims))
    rhs = _fields(rhs, 12 * v)
    x = _fields(x, 12 * v)
    rr = np.zeros(rhs.shape[0], np.float64)
    lib().orc_drr_residual(d, b, np.ascontiguousarray(links), float(m0),
                           np.ascontiguousarray(q, dtype=np.int32), int(nb), rhs, x,
                           rhs.shape[0], rr)
    return rr


def schur_apply(links, dims, m0, q, nb, xb, restart=8, tol=1e-13, maxit=10000, bc=(1, 1, 1, -1)):
    """S_bb x_b for x_b of shape (nrhs, 12 nb); returns (y_b, iters, relres)."""
    d, b = _geom(dims, bc)
    xb = _fields(xb, 12 * int(nb))
    yb = np.empty_like(xb)
    it = np.zeros(xb.shape[0], np.int32)
    rr = np.zeros(xb.shape[0], np.float64)
    lib().orc_schur_apply(d, b, np.ascontiguousarray(links), float(m0),
                          np.ascontiguousarray(q, dtype=np.int32), int(nb), xb, yb, xb.shape[0],
                          int(restart), float(tol), int(maxit), it, rr)
    return yb, it, rr


def reusken_apply(links, dims, m0, q, nb, xb, bc=(1, 1, 1, -1)):
    """S~_bb x_b of section 3, matrix-free from the stencil's blocks:
        u = x_b on the coarse sites,  y = D_rb u,  d~ = D_rr 1 (row sums),
        t = y / d~,  M y = y / d + t - (D_rr t) / d   (d = 4 + m0, the
        diagonal of the Wilson operator),  S~ x_b = D_bb x_b - D_br M y.
    Returns (nrhs, 12 nb)."""
    v = int(np.prod(dims))
    q = np.asarray(q)
    xb = _fields(xb, 12 * int(nb))
    nrhs = xb.shape[0]
    u = np.zeros((nrhs, v, 12), np.complex128)
    u[:, q[:nb]] = xb.reshape(nrhs, nb, 12)
    u = u.reshape(nrhs, 12 * v)
    rest = np.ones(v, bool)
    rest[q[:nb]] = False
    ones = np.zeros((1, v, 12), np.complex128)
    ones[:, rest] = 1.0
    dt = block_apply(links, dims, m0, q, nb, 0, 0, ones.reshape(1, -1), bc).reshape(v, 12)
    y = block_apply(links, dims, m0, q, nb, 0, 1, u, bc).reshape(nrhs, v, 12)
    t = np.zeros_like(y)
    t[:, rest] = y[:, rest] / dt[rest]
    z = block_apply(links, dims, m0, q, nb, 0, 0, t.reshape(nrhs, -1), bc).reshape(nrhs, v, 12)
    my = (y - z) / (4.0 + m0) + t
    # D_bb x_b - D_br M y = [D (u - M y)]_b   (u is zero on the rest sites, M y on the coarse)
    w = u - my.reshape(nrhs, -1)
    out = dirac_apply(links, dims, m0, w, bc).reshape(nrhs, v, 12)
    return np.ascontiguousarray(out[:, q[:nb]].reshape(nrhs, 12 * int(nb)))


def site_parity(dims):
    """(x + y + z + t) mod 2 of every site (lexicographic, x fastest)."""
    c = np.indices(tuple(dims)[::-1]).reshape(4, -1)[::-1]
    return c.sum(axis=0) % 2


def reduced_apply(links, dims, m0, q, nb, parity, x, bc=(1, 1, 1, -1)):
    """The even-odd Schur complement of D_rr on the rest sites of one parity,
    A_p x = (D_rr z)_p with z = x_p - (D_rr x_p)_q / d: the hopping term only
    couples sites of opposite parity, so D_qq = d (= 4 + m0) on the rest sites
    and A_p = D_pp - D_pq D_qq^{-1} D_qp = d - H_pq H_qp / d.  x (nrhs, 12 V)
    is read on the rest sites of parity p; the result is zero elsewhere."""
    v = int(np.prod(dims))
    x = _fields(x, 12 * v)
    nrhs = x.shape[0]
    par = site_parity(dims)
    on_p = (par == parity)[None, :, None]
    on_q = ~on_p
    xp = (x.reshape(nrhs, v, 12) * on_p).reshape(nrhs, -1)
    y = block_apply(links, dims, m0, q, nb, 0, 0, xp, bc).reshape(nrhs, v, 12)
    z = xp.reshape(nrhs, v, 12) - y * on_q / (4.0 + m0)
    out = block_apply(links, dims, m0, q, nb, 0, 0, z.reshape(nrhs, -1), bc).reshape(nrhs, v, 12)
    return (out * on_p).reshape(nrhs, -1)


def diag_schur_apply(links, dims, m0, q, nb, xb, bc=(1, 1, 1, -1)):
    """D_bb x_b - D_br (D_rb x_b) / d with d = 4 + m0, the diagonal of D_rr:
    u = x_b on the coarse sites, y = D_rb u, y_b = [D (u - y / d)]_b.
    Returns (nrhs, 12 nb)."""
    v = int(np.prod(dims))
    q = np.asarray(q)
    xb = _fields(xb, 12 * int(nb))
    nrhs = xb.shape[0]
    u = np.zeros((nrhs, v, 12), np.complex128)
    u[:, q[:nb]] = xb.reshape(nrhs, nb, 12)
    u = u.reshape(nrhs, 12 * v)
    y = block_apply(links, dims, m0, q, nb, 0, 1, u, bc)
    w = u - y / (4.0 + m0)
    out = dirac_apply(links, dims, m0, w, bc).reshape(nrhs, v, 12)
    return out[:, q[:nb]].reshape(nrhs, -1)


def reduced_apply_abs(links, dims, m0, q, nb, parity, x, bc=(1, 1, 1, -1)):
    """The absolute-value sums of the reduced operator A_p x = d x_p - H_pq H_qp x_p / d
    (d = 4 + m0, H the hopping part of D_rr): |d| |x_p| + |H_pq| (|H_qp| |x_p|) / |d|
    on the rest sites of parity p, zero elsewhere.  Real (nrhs, 12 V)."""
    v = int(np.prod(dims))
    x = _fields(x, 12 * v)
    nrhs = x.shape[0]
    par = site_parity(dims)
    on_p = (par == parity)[None, :, None]
    ax = (np.abs(x).reshape(nrhs, v, 12) * on_p).reshape(nrhs, -1).astype(np.complex128)
    h1 = block_apply_abs(links, dims, m0, q, nb, 0, 0, ax, diag=False, bc=bc).reshape(nrhs, v, 12)
    h1 = (h1 * ~on_p).reshape(nrhs, -1).astype(np.complex128)
    h2 = block_apply_abs(links, dims, m0, q, nb, 0, 0, h1, diag=False, bc=bc).reshape(nrhs, v, 12)
    d = abs(4.0 + m0)
    rest = np.ones(v, bool)
    rest[np.asarray(q)[:nb]] = False
    out = (d * np.abs(ax.real).reshape(nrhs, v, 12) + h2 / d) * on_p * rest[None, :, None]
    return out.reshape(nrhs, -1)


def reduced_intermediate(links, dims, m0, q, nb, parity, x, bc=(1, 1, 1, -1)):
    """The intermediate field of the reduced operator, H_qp x_p on the rest
    sites of the other parity q (zero elsewhere): the first of its two
    stencil steps."""
    v = int(np.prod(dims))
    x = _fields(x, 12 * v)
    nrhs = x.shape[0]
    par = site_parity(dims)
    on_p = (par == parity)[None, :, None]
    xp = (x.reshape(nrhs, v, 12) * on_p).reshape(nrhs, -1)
    y = block_apply(links, dims, m0, q, nb, 0, 0, xp, bc).reshape(nrhs, v, 12)
    return (y * ~on_p).reshape(nrhs, -1)
