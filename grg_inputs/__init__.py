"""Seeded synthetic inputs shared by the CPU oracle, the GPU tests and the benchmark.

This module only *draws* inputs.  It holds none of the method's arithmetic
(no Dirac operator, no permutation, no Schur complement), so that the oracle
and the GPU path can both consume its output without sharing any code.

Conventions (canonical layout, used at the library boundary as well):

* lattice dims are (Lx, Ly, Lz, Lt); site index s = x + Lx*(y + Ly*(z + Lz*t)),
  x fastest;
* links are complex128 arrays of shape (V, 4, 3, 3): U[s, mu, row, col] with
  mu = x, y, z, t;
* a fermion field is complex128 of length 12*V with dof = 12*s + 3*spin + colour;
  a batch of fields has shape (nrhs, 12*V).

Synthetic gauge field: for every link, H = sum_k a_k lambda_k with a_k ~ N(0,1)
(Gell-Mann lambda_1..lambda_8), U0 = exp(i*eps*H), then reunitarised by
Gram-Schmidt on rows 0 and 1 and row 2 = conj(row0 x row1), which gives a
special-unitary matrix to rounding.  The paper's workloads are SU(3)
plaquette-action ensembles (section 2, section 4); these random fields stand in
for them, since no ensemble is available.
"""
from __future__ import annotations

import os

import numpy as np

__all__ = [
    "gell_mann",
    "su3_links",
    "gaussian_vectors",
    "point_sources",
    "batch_instances",
    "volume",
]


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3), standard normalisation
    tr(lambda_a lambda_b) = 2 delta_ab."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _reunitarise(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0, 1; row 2 = conj(row0 x row1).  u: (..., 3, 3)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def su3_links(dims, eps: float, seed: int, chunk: int = 1 << 16) -> np.ndarray:
    """Random SU(3) links, shape (V, 4, 3, 3) complex128.

    a[t][z][y][x][mu][k] ~ N(0,1) is drawn from numpy.random.default_rng(seed)
    in C order, so that the flattened site index is x-fastest.  exp(i eps H) is
    evaluated from the Hermitian eigendecomposition of H.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    v = lx * ly * lz * lt
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((lt, lz, ly, lx, 4, 8)).reshape(v * 4, 8)
    lam = gell_mann()
    out = np.empty((v * 4, 3, 3), dtype=np.complex128)

    def one(s):
        e = min(s + chunk, v * 4)
        h = (a[s:e] @ lam.reshape(8, 9)).reshape(-1, 3, 3)
        w, vec = np.linalg.eigh(h)
        u0 = (vec * np.exp(1j * eps * w)[:, None, :]) @ np.conj(vec).transpose(0, 2, 1)
        out[s:e] = _reunitarise(u0)

    starts = range(0, v * 4, chunk)
    if v * 4 <= chunk:
        one(0)
    else:
        # chunks are independent and deterministic, so threads do not change the result
        from concurrent.futures import ThreadPoolExecutor

        with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
            list(ex.map(one, starts))
    return out.reshape(v, 4, 3, 3)


def gaussian_vectors(n: int, nrhs: int, seed: int) -> np.ndarray:
    """nrhs complex128 vectors of length n; real and imaginary parts i.i.d.
    N(0,1) from default_rng(seed + 1), drawn as an (nrhs, n, 2) array."""
    rng = np.random.default_rng(seed + 1)
    g = rng.standard_normal((nrhs, n, 2))
    return np.ascontiguousarray(g[..., 0] + 1j * g[..., 1])


def point_sources(n_coarse: int, nrhs: int = 12, index: int = 0) -> np.ndarray:
    """Unit vectors in coarse space (length 12*n_coarse): source j sits on
    coarse index `index`, spin-colour component j (j < nrhs <= 12)."""
    if not 0 < nrhs <= 12:
        raise ValueError("nrhs must be in 1..12")
    x = np.zeros((nrhs, 12 * n_coarse), dtype=np.complex128)
    for j in range(nrhs):
        x[j, 12 * index + j] = 1.0
    return x


_BATCH_SHAPES = ((8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (8, 8, 8, 16))


def batch_instances(count: int = 48, seed: int = 4, base_seed: int = 4000):
    """Descriptors of a many-lattice batch: a list of dicts with dims, m0 and
    the per-lattice seed.  Shapes are uniform over {8^4, 12^4, 16^4, 8^3x16}
    and m0 ~ U[-0.3, 0.1], both from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    pick = rng.integers(0, len(_BATCH_SHAPES), size=count)
    m0 = rng.uniform(-0.3, 0.1, size=count)
    return [
        {"dims": _BATCH_SHAPES[int(pick[i])], "m0": float(m0[i]), "seed": base_seed + i}
        for i in range(count)
    ]
