"""Pins of the oracle's overlap spectrum (D_ov(mu) = 1 + gamma5 sgn(A),
Section 1): the free-field closed form in momentum space, the Ginsparg-Wilson
circle at mu = 0 and the conjugation symmetry between mu and -mu."""
import numpy as np
import pytest

import synth
from oracle import overlap

MW = -1.5


def match_spectra(a, b):
    """Largest distance from an eigenvalue of a to its partner in b, pairing
    each element of a greedily with the nearest unused element of b."""
    used = np.zeros(len(b), dtype=bool)
    worst = 0.0
    for z in a:
        d = np.abs(b - z)
        d[used] = np.inf
        j = int(np.argmin(d))
        used[j] = True
        worst = max(worst, float(d[j]))
    return worst


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_free_field_spectrum(mu):
    """Unit links on 2^3 x 4: the dense position-space operator has the
    spectrum of the closed-form momentum blocks."""
    dims = (2, 2, 2, 4)
    U = synth.unit_links(dims)
    lam = overlap.overlap_eigenvalues(dims, U, MW, mu)
    ref = overlap.free_overlap_eigenvalues(dims, MW, mu)
    assert len(lam) == len(ref) == 12 * 32
    assert match_spectra(lam, ref) < 1e-10


def test_ginsparg_wilson_circle():
    """mu = 0: gamma5 sgn(A) is unitary, so |lambda - 1| = 1; with random links
    the spectrum is not confined to {0, 2} (which a dropped gamma5 would give)."""
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 0.6, seed=31)
    lam = overlap.overlap_eigenvalues(dims, U, MW, 0.0)
    assert np.abs(np.abs(lam - 1.0) - 1.0).max() < 1e-11
    assert np.abs(lam.imag).max() > 0.1


def test_conjugation_symmetry():
    """spec D_ov(-mu) = conj(spec D_ov(mu)) (D_ov(mu)^dagger = gamma5 D_ov(-mu) gamma5),
    and at mu != 0 the circle no longer holds."""
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 0.6, seed=32)
    lp = overlap.overlap_eigenvalues(dims, U, MW, 0.4)
    lm = overlap.overlap_eigenvalues(dims, U, MW, -0.4)
    assert match_spectra(np.conj(lp), lm) < 1e-10
    assert np.abs(np.abs(lp - 1.0) - 1.0).max() > 1e-3
