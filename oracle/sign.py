"""Matrix sign function of a (possibly non-Hermitian) matrix.

Section 1, eq. (1.3): for diagonalisable A = R diag(lambda_i) R^{-1},
f(A) = R diag(f(lambda_i)) R^{-1}, and eq. (1.4): sgn(z) = z/sqrt(z^2) =
sgn(Re z) with the square-root branch cut on the negative real axis.
Section 2 closes with Roberts' iteration S <- (S + S^{-1})/2, S^0 = H, which
converges quadratically to sgn(H).

Reading for Re z = 0 exactly (the sign is undefined there): return +1.

TEST INFRASTRUCTURE: only tests, smoke and the CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np


def csgn(z):
    """sgn(Re z), with +1 on the imaginary axis (eq. (1.4))."""
    return np.where(np.real(z) >= 0.0, 1.0, -1.0)


def sign_eig(a: np.ndarray):
    """Full sgn(A) by the spectral definition (eq. (1.3)).

    Returns (S, info) with info = {"cond_R", "min_abs_re"}."""
    lam, r = np.linalg.eig(a)
    s = csgn(lam)
    rinv = np.linalg.inv(r)
    out = (r * s[None, :]) @ rinv
    info = {"cond_R": float(np.linalg.cond(r)), "min_abs_re": float(np.min(np.abs(lam.real)))}
    return out, info


def sign_eig_apply(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """sgn(A) b for one or several columns b, by the spectral definition."""
    lam, r = np.linalg.eig(a)
    s = csgn(lam)
    c = np.linalg.solve(r, b)
    if c.ndim == 1:
        return r @ (s * c)
    return r @ (s[:, None] * c)


def sign_newton(a: np.ndarray, tol: float = 1e-14, max_iter: int = 100):
    """Roberts' iteration S <- (S + S^{-1})/2 from S^0 = A, unscaled (Section 2)."""
    s = np.array(a, dtype=np.complex128, copy=True)
    for it in range(max_iter):
        s_new = 0.5 * (s + np.linalg.inv(s))
        diff = np.linalg.norm(s_new - s)
        s = s_new
        if diff <= tol * np.linalg.norm(s):
            return s, it + 1
    return s, max_iter


def sign_eigh(a: np.ndarray) -> np.ndarray:
    """sgn(A) for Hermitian A via the unitary eigendecomposition (mu = 0 case)."""
    lam, q = np.linalg.eigh(a)
    return (q * np.where(lam >= 0.0, 1.0, -1.0)[None, :]) @ q.conj().T


def sign_e1(g: np.ndarray) -> np.ndarray:
    """First column of sgn(G) (Section 2: only f(H_k) e_1 is needed)."""
    e1 = np.zeros(g.shape[0], dtype=np.complex128)
    e1[0] = 1.0
    return sign_eig_apply(g, e1)
