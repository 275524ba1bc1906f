"""Shared set-up of the GPU tests: seeded inputs, device copies, the library
handles.  Nothing here computes the method; expected values come from the
oracle only."""
from __future__ import annotations

import os

import numpy as np

from grg_inputs import su3_links

PERM_CODES = {"I": 1, "II": 2}


def ensure_built():
    from paper_0704_2341_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        from paper_0704_2341_amd import build

        build.build()


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def to_host(t):
    return t.cpu().numpy()


def rel_err(a, b):
    """Per-RHS ||a - b|| / ||b||, worst RHS."""
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    den = np.where(den == 0, 1.0, den)
    return float((num / den).max())


class Lattice:
    """A lattice handle with a seeded SU(3) field."""

    def __init__(self, dims, eps, seed, bc=(1, 1, 1, -1), links=None):
        import paper_0704_2341_amd as grg

        ensure_built()
        self.grg = grg
        self.dims = tuple(dims)
        self.bc = tuple(bc)
        self.V = int(np.prod(dims))
        self.links = su3_links(dims, eps, seed) if links is None else links
        self.h = grg.grg_lattice_create(dims, bc)
        grg.grg_gauge_set(self.h, self.links)

    def schur(self, m0, kind, inverse, **params):
        q, nb = self.grg.grg_permutation_block(self.dims, PERM_CODES[kind], inverse)
        p = self.grg.grg_solver_params_default(**params)
        return Schur(self, self.grg.grg_schur_create(self.h, m0, q, nb, p), q, nb, m0)

    def close(self):
        self.grg.grg_lattice_destroy(self.h)


class Schur:
    def __init__(self, lat, h, q, nb, m0):
        self.lat, self.h, self.q, self.nb, self.m0 = lat, h, q, nb, m0

    def apply(self, xb, **kw):
        import torch

        x = to_dev(np.atleast_2d(xb))
        y = torch.empty_like(x)
        st = self.lat.grg.grg_schur_apply(self.h, x, y, x.shape[0], **kw)
        return to_host(y), st

    def drr_solve(self, b, **kw):
        import torch

        bd = to_dev(np.atleast_2d(b))
        x = torch.empty_like(bd)
        st = self.lat.grg.grg_drr_solve(self.h, bd, x, bd.shape[0], **kw)
        return to_host(x), st

    def close(self):
        self.lat.grg.grg_schur_destroy(self.h)
