"""Spectra of the coarse operator at small volume (host side, numpy).

The dense S_bb and S~_bb come from the library (grg_schur_assemble,
grg_reusken_assemble: applies to unit vectors on the GPU); their eigenvalues
are then a host LAPACK call.  This is the analysis of section 2 (Figure 2:
the spectrum of S_bb against that of D) and section 4 (the spectrum of
S~_bb^{-1} S_bb, clustered around one when the approximation is good),
including the shifted kernel c - S_bb.
"""
from __future__ import annotations

import numpy as np

from . import binding as _b


def coarse_matrix(schur, n_coarse, approximate: bool = False, shift=None) -> np.ndarray:
    """Dense S_bb (or S~_bb with approximate=True), or shift * 1 - that
    matrix, as complex128 (12 N_b, 12 N_b)."""
    m = (_b.grg_reusken_assemble if approximate else _b.grg_schur_assemble)(schur, n_coarse)
    if shift is not None:
        m = shift * np.eye(m.shape[0]) - m
    return m


def coarse_spectrum(schur, n_coarse, approximate: bool = False, shift=None) -> np.ndarray:
    """Eigenvalues of coarse_matrix(...), sorted by real part then imaginary part."""
    ev = np.linalg.eigvals(coarse_matrix(schur, n_coarse, approximate, shift))
    return ev[np.lexsort((ev.imag, ev.real))]


def approximation_spectrum(schur, n_coarse) -> np.ndarray:
    """Eigenvalues of S~_bb^{-1} S_bb (section 4)."""
    s = coarse_matrix(schur, n_coarse)
    st = coarse_matrix(schur, n_coarse, approximate=True)
    ev = np.linalg.eigvals(np.linalg.solve(st, s))
    return ev[np.lexsort((ev.imag, ev.real))]
