"""O1: dense FP64 oracle for tiny lattices (test infrastructure only).

Everything here is the plain definition, written out entry by entry:

* the Wilson-Dirac matrix
      D = (4 + m0) 1 - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) delta_{x+mu,y}
                                   + (1 + gamma_mu) U_mu(x-mu)^dag delta_{x-mu,y} ]
  in the DeGrand-Rossi basis, periodic in x, y, z and antiperiodic in t
  (the paper names "the Wilson-Dirac operator" in section 2 without writing it;
  this is the standard form, r = 1, no clover term);
* the site permutations of section 2 (Type I, Type II and their inverses),
  with the coarse sites labelled first (the Permutation_block description);
* the 2x2 block partition of section 1 (step 1) and the Schur complement
  S_bb = D_bb - D_br D_rr^{-1} D_rb (section 1, the formula following the
  blocking kernels), by a dense LU solve;
* the general Gaussian-integration form of section 1 (D~ = D + Bbar D_bb B,
  S_bb = D_bb - D_bb B D~^{-1} Bbar D_bb) with the blocking kernels B, Bbar of
  section 1 (step 2), used only to check that it reduces to the Schur
  complement;
* the second-order Schur complement approximation of section 3,
  S~_bb = D_bb - D_br (d_rr^{-1} + d~_rr^{-1} - d_rr^{-1} D_rr d~_rr^{-1}) D_rb,
  with d_rr the diagonal of D_rr and d~_rr the diagonal matrix of the row sums
  of D_rr (read literally: the sum of each scalar row, dof by dof).

Sizes: 12*V dof; at 4^4 the matrix is 3072 x 3072 complex (151 MB).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

# ---------------------------------------------------------------- gamma basis
# DeGrand-Rossi (chiral) basis, rows as written.  gamma_5 = gx gy gz gt
# = diag(1, 1, -1, -1).
GAMMA = np.array(
    [
        [[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]],  # x
        [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],  # y
        [[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]],  # z
        [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],  # t
    ],
    dtype=np.complex128,
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

DEFAULT_BC = (1, 1, 1, -1)


# ---------------------------------------------------------------- geometry
def volume(dims) -> int:
    return int(np.prod([int(d) for d in dims]))


def coords(s: int, dims):
    lx, ly, lz, _ = dims
    return (s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz))


def site(c, dims) -> int:
    lx, ly, lz, _ = dims
    return int(c[0] + lx * (c[1] + ly * (c[2] + lz * c[3])))


def hop(s: int, mu: int, step: int, dims, bc):
    """Neighbour of site s one step (+1 or -1) along mu, and the boundary
    sign picked up when the hop wraps around the lattice."""
    c = list(coords(s, dims))
    n = c[mu] + step
    sign = 1.0
    if n >= dims[mu] or n < 0:
        sign = float(bc[mu])
        n %= dims[mu]
    c[mu] = n
    return site(c, dims), sign


# ---------------------------------------------------------------- Wilson D
def wilson_dense(links: np.ndarray, dims, m0: float, bc=DEFAULT_BC) -> np.ndarray:
    """Dense Wilson-Dirac matrix, complex128 (12V, 12V); dof = 12 s + 3 spin + colour."""
    dims = tuple(int(d) for d in dims)
    v = volume(dims)
    n = 12 * v
    d = np.zeros((n, n), dtype=np.complex128)
    eye4 = np.eye(4)
    d[np.arange(n), np.arange(n)] = 4.0 + m0
    for s in range(v):
        for mu in range(4):
            sp, sgn_p = hop(s, mu, +1, dims, bc)
            # forward hop: -1/2 (1 - gamma_mu) U_mu(x) psi(x + mu)
            d[12 * s:12 * s + 12, 12 * sp:12 * sp + 12] += (
                -0.5 * sgn_p * np.kron(eye4 - GAMMA[mu], links[s, mu])
            )
            sm, sgn_m = hop(s, mu, -1, dims, bc)
            # backward hop: -1/2 (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu)
            d[12 * s:12 * s + 12, 12 * sm:12 * sm + 12] += (
                -0.5 * sgn_m * np.kron(eye4 + GAMMA[mu], links[sm, mu].conj().T)
            )
    return d


# ---------------------------------------------------------------- permutations
def _all_even(c) -> bool:
    return all(int(x) % 2 == 0 for x in c)


def _level(c) -> int:
    """Type II nesting level: the first direction (x, y, z, t order) in which
    the coordinate is odd; 4 if every coordinate is even."""
    for mu in range(4):
        if int(c[mu]) % 2 == 1:
            return mu
    return 4


def permutation_block(dims, kind: str, inverse: bool = False):
    """Ordering vector q (int64, length V) and the number of coarse sites N_b.

    Row k of P(q) D P(q)^T is row q[k] of D (section 2: the permutation
    operator exchanges the rows of D and labels the coarse sites first).

    * Type I  ("block in all directions"): all-even sites first, then the
      rest, each group lexicographic.
    * Type II ("one direction at a time"): nested red-black blocking, x first:
      sites grouped by the first direction with an odd coordinate, the
      all-even group first and the x-odd group last, lexicographic inside.
    * inverse: the inverse permutation q^{-1} (q^{-1}[q[k]] = k), whose
      operator is P(q)^T.

    N_b = V / 16 in every case: the coarse block is the leading N_b entries.
    """
    dims = tuple(int(d) for d in dims)
    if any(d % 2 for d in dims):
        raise ValueError("Type I/II blocking needs even extents")
    v = volume(dims)
    cs = [coords(s, dims) for s in range(v)]
    if kind in ("I", 1):
        key = [0 if _all_even(c) else 1 for c in cs]
    elif kind in ("II", 2):
        key = [4 - _level(c) for c in cs]
    else:
        raise ValueError(f"unknown permutation type {kind!r}")
    q = np.array(sorted(range(v), key=lambda s: (key[s], s)), dtype=np.int64)
    if inverse:
        qi = np.empty_like(q)
        qi[q] = np.arange(v)
        q = qi
    return q, v // 16


def permutation_matrix(q) -> np.ndarray:
    """P(q) = rows q of the identity, at site level."""
    q = np.asarray(q)
    return np.eye(len(q))[q]


def dof_order(q) -> np.ndarray:
    """Expand a site ordering to a dof ordering (12 dof per site)."""
    q = np.asarray(q, dtype=np.int64)
    return (12 * q[:, None] + np.arange(12)[None, :]).reshape(-1)


# ---------------------------------------------------------------- Schur complement
def blocks(d: np.ndarray, q, n_b: int):
    """D_bb, D_br, D_rb, D_rr of P D P^T (section 1, step 1)."""
    o = dof_order(q)
    b, r = o[: 12 * n_b], o[12 * n_b:]
    return d[np.ix_(b, b)], d[np.ix_(b, r)], d[np.ix_(r, b)], d[np.ix_(r, r)]


def schur_dense(d: np.ndarray, q, n_b: int) -> np.ndarray:
    """S_bb = D_bb - D_br D_rr^{-1} D_rb with D_rr^{-1} D_rb by LU."""
    dbb, dbr, drb, drr = blocks(d, q, n_b)
    lu = sla.lu_factor(drr)
    return dbb - dbr @ sla.lu_solve(lu, drb)


def schur_gaussian_rg(d: np.ndarray, q, n_b: int) -> np.ndarray:
    """S_bb from the general Gaussian-integration form of section 1 with the
    gauge-covariant blocking kernels B = (0, D_bb^{-1} D_br) and
    Bbar = (0 ; D_rb D_bb^{-1}), in the permuted basis.  Requires D_bb
    invertible."""
    o = dof_order(q)
    dp = d[np.ix_(o, o)]
    nb = 12 * n_b
    dbb, dbr, drb = dp[:nb, :nb], dp[:nb, nb:], dp[nb:, :nb]
    n = dp.shape[0]
    bmat = np.zeros((nb, n), dtype=np.complex128)
    bmat[:, nb:] = np.linalg.solve(dbb, dbr)
    bbar = np.zeros((n, nb), dtype=np.complex128)
    bbar[nb:, :] = drb @ np.linalg.inv(dbb)
    dt = dp + bbar @ dbb @ bmat
    return dbb - dbb @ bmat @ np.linalg.solve(dt, bbar @ dbb), dt


def schur_apply_dense(d, q, n_b, x_b):
    """S_bb x_b for a batch x_b of shape (nrhs, 12 N_b)."""
    s = schur_dense(d, q, n_b)
    return (s @ np.atleast_2d(x_b).T).T


# ---------------------------------------------------------------- approximation (section 3)
def reusken_inverse(drr: np.ndarray) -> np.ndarray:
    """M = d^{-1} + d~^{-1} - d^{-1} D_rr d~^{-1}, the approximate D_rr^{-1} of
    the section 3 formula: d = diag(D_rr), d~ = diag(row sums of D_rr)."""
    d = np.diag(drr)
    dt = drr.sum(axis=1)
    return np.diag(1.0 / d) + np.diag(1.0 / dt) - (drr / d[:, None]) / dt[None, :]


def reusken_dense(d: np.ndarray, q, n_b: int) -> np.ndarray:
    """S~_bb = D_bb - D_br M D_rb (section 3)."""
    dbb, dbr, drb, drr = blocks(d, q, n_b)
    return dbb - dbr @ reusken_inverse(drr) @ drb


def diag_schur_dense(d: np.ndarray, q, n_b: int) -> np.ndarray:
    """The Schur complement with D_rr replaced by its diagonal (the older
    approximation section 3 contrasts with, which ignores the couplings inside
    D_rr and keeps the coarse operator's sparsity): D_bb - D_br diag(D_rr)^{-1} D_rb."""
    dbb, dbr, drb, drr = blocks(d, q, n_b)
    return dbb - dbr @ (drb / np.diag(drr)[:, None])
