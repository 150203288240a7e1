"""Spectrum of the overlap operator D_ov(mu) = 1 + gamma5 sgn(gamma5 Dw(mu)).

Section 1 defines D_ov(mu) through the sign function of A = gamma5 Dw(mu);
the closing outlook of Section 5 applies the Krylov methods to its
eigenvalues.  Here the operator is formed densely (the spectral sign of
eq. (1.3)) and its eigenvalues taken with LAPACK, for lattices small enough
to hold N x N matrices (4^4: N = 3072).

Pins (tests/test_oracle_overlap.py):
  - unit links: the eigenvalues equal those of the momentum-space blocks
    1 + gamma5 sgn(A(p)) of the closed form (each three times, for colour);
  - mu = 0: D_ov - 1 is unitary, so every eigenvalue lies on |lambda - 1| = 1;
  - D_ov(mu)^dagger = gamma5 D_ov(-mu) gamma5, so the spectrum at -mu is the
    complex conjugate of the spectrum at mu.

TEST INFRASTRUCTURE: only tests, smoke and the CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np

from . import dirac, sign
from .freefield import free_sign_momentum
from .dirac import gamma_matrices


def dense_overlap(dims, U, m_w, mu, bc=dirac.DEFAULT_BC) -> np.ndarray:
    """D_ov(mu) = 1 + gamma5 sgn(A), dense (Section 1)."""
    a = dirac.dense_A(dims, U, m_w, mu, bc)
    s, _ = sign.sign_eig(a)
    g5 = dirac.gamma5_rows(int(np.prod(dims)))
    return np.eye(a.shape[0]) + g5[:, None] * s


def overlap_eigenvalues(dims, U, m_w, mu, bc=dirac.DEFAULT_BC) -> np.ndarray:
    """All eigenvalues of D_ov(mu), ordered by increasing magnitude."""
    lam = np.linalg.eigvals(dense_overlap(dims, U, m_w, mu, bc))
    return lam[np.argsort(np.abs(lam), kind="stable")]


def free_overlap_eigenvalues(dims, m_w, mu) -> np.ndarray:
    """Unit links: eigenvalues of 1 + gamma5 sgn(A(p)) over all momenta p (closed
    form of the free sign), each repeated three times (colour), ordered by
    increasing magnitude."""
    _, g5 = gamma_matrices()
    s = free_sign_momentum(tuple(dims), m_w, mu).reshape(-1, 4, 4)
    blocks = np.eye(4)[None] + np.einsum("ij,pjk->pik", g5, s)
    lam = np.repeat(np.linalg.eigvals(blocks).reshape(-1), 3)
    return lam[np.argsort(np.abs(lam), kind="stable")]
