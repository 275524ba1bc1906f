"""Spectra of the GPU-assembled coarse operator at 4^4 (sections 2 and 4):
the free-field Type I spectrum against its closed form, invariance of the
spectrum under a gauge transformation, the conjugate-pair structure that
gamma_5-hermiticity forces, the shifted kernel, and S~^{-1} S near one."""
import numpy as np
import pytest

from gpu_support import Lattice
from test_oracle_pins import free_schur_type1_spectrum, gauge_transform, random_omega, same_multiset

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)


def spectrum(links, kind, inv, m0, approximate=False, shift=None):
    from paper_0704_2341_amd import spectra

    lat = Lattice(DIMS, 0.4, 1, links=links)
    s = lat.schur(m0, kind, inv, tol=1e-13, max_rhs=12)
    ev = spectra.coarse_spectrum(s.h, s.nb, approximate, shift)
    s.close()
    lat.close()
    return ev


def test_free_field_type1_closed_form():
    v = int(np.prod(DIMS))
    unit = np.broadcast_to(np.eye(3, dtype=np.complex128), (v, 4, 3, 3)).copy()
    ev = spectrum(unit, "I", False, 0.1)
    ok, worst = same_multiset(ev, free_schur_type1_spectrum(DIMS, 0.1), 1e-9)
    assert ok, worst


@pytest.mark.parametrize("kind,inv", [("I", False), ("II", True), ("I", True)])
def test_gauge_invariant_and_conjugate_pairs(kind, inv):
    from grg_inputs import su3_links

    links = su3_links(DIMS, 0.4, 1)
    ev = spectrum(links, kind, inv, 0.1)
    omega = random_omega(int(np.prod(DIMS)), 7)
    ev_g = spectrum(gauge_transform(links, omega, DIMS), kind, inv, 0.1)
    ok, worst = same_multiset(ev, ev_g, 1e-9)
    assert ok, worst
    # gamma_5 S gamma_5 = S^+: the spectrum is closed under conjugation
    ok, worst = same_multiset(ev, np.conj(ev), 1e-9)
    assert ok, worst


def test_shifted_kernel():
    from grg_inputs import su3_links

    links = su3_links(DIMS, 0.4, 1)
    ev = spectrum(links, "II", False, 0.1)
    ev_c = spectrum(links, "II", False, 0.1, shift=2.0)
    ok, worst = same_multiset(2.0 - ev, ev_c, 1e-9)
    assert ok, worst


def test_approximation_spectrum_near_one():
    from grg_inputs import su3_links

    from paper_0704_2341_amd import spectra

    lat = Lattice(DIMS, 0.4, 1, links=su3_links(DIMS, 0.4, 1))
    s = lat.schur(0.1, "II", True, tol=1e-13, max_rhs=12)
    ev = spectra.approximation_spectrum(s.h, s.nb)
    assert np.abs(ev - 1).max() < 0.1
    s.close()
    lat.close()
