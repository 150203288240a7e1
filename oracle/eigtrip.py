"""Critical eigentriples (Lambda_m, R_m, L_m) for LR deflation.

Section 3: A R_m = R_m Lambda_m, L_m^dagger A = Lambda_m L_m^dagger,
L_m^dagger R_m = I_m.  Section 5: the critical eigenvalues are those of
smallest magnitude (the paper obtains them with ARPACK).

Reading for ties: order by (|lambda|, Re lambda, Im lambda).

TEST INFRASTRUCTURE: only tests, smoke and the CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def _order(lam):
    return np.lexsort((lam.imag, lam.real, np.abs(lam)))


def dense_eigentriples(a: np.ndarray, m: int):
    """From a full eigendecomposition: R columns unit norm, L = columns of R^{-dagger}."""
    lam, r = np.linalg.eig(a)
    l_full = np.linalg.inv(r).conj().T
    idx = _order(lam)[:m]
    return lam[idx].copy(), np.ascontiguousarray(r[:, idx]), np.ascontiguousarray(l_full[:, idx])


def sparse_eigentriples(a_csr, m: int, tol: float = 1e-12, extra: int = 4):
    """Shift-invert ARPACK (sigma = 0, as the paper's ARPACK runs of Section 5)
    for the m eigenvalues of smallest magnitude: the largest-magnitude
    eigenvalues 1/lambda of A^{-1} give R, those of (A^dagger)^{-1} =
    (A^{-1})^dagger give L.  Both use one sparse LU factorisation of A (the
    left problem solves with its conjugate transpose).  Left vectors are
    paired by lambda_L ~ conj(lambda_R) and biorthonormalised so that
    L^dagger R = I (Section 3); clusters of nearly equal eigenvalues
    blockwise.

    Returns (lam, R, L) ordered by (|lambda|, Re, Im); R columns unit norm.
    Pinned against the full eigendecomposition (dense_eigentriples) on small
    lattices."""
    n = a_csr.shape[0]
    nev = m + extra
    lu = spla.splu(a_csr.tocsc(), permc_spec="MMD_AT_PLUS_A")
    inv_r = spla.LinearOperator((n, n), matvec=lambda x: lu.solve(np.asarray(x, np.complex128)),
                                dtype=np.complex128)
    inv_l = spla.LinearOperator((n, n),
                                matvec=lambda x: lu.solve(np.asarray(x, np.complex128), trans="H"),
                                dtype=np.complex128)
    v0 = np.full(n, 1.0 / np.sqrt(n), dtype=np.complex128)  # fixed start: reproducible runs
    th_r, r = spla.eigs(inv_r, k=nev, which="LM", tol=tol, v0=v0)
    th_l, l_ = spla.eigs(inv_l, k=nev, which="LM", tol=tol, v0=v0)
    lam_r, lam_l = 1.0 / th_r, 1.0 / th_l
    ir = _order(lam_r)
    lam_r, r = lam_r[ir], r[:, ir]
    # pair every right eigenvalue with the closest conj(left) eigenvalue
    used = np.zeros(len(lam_l), dtype=bool)
    perm = []
    for lr in lam_r:
        d = np.abs(np.conj(lam_l) - lr)
        d[used] = np.inf
        j = int(np.argmin(d))
        used[j] = True
        perm.append(j)
    l_ = l_[:, perm]
    lam_r, r, l_ = lam_r[:m], r[:, :m], l_[:, :m]
    r = r / np.linalg.norm(r, axis=0)[None, :]
    # blockwise biorthonormalisation: L <- L (R^dagger L)^{-1} over clusters
    out_l = l_.copy()
    i = 0
    while i < m:
        j = i + 1
        while j < m and abs(lam_r[j] - lam_r[i]) <= 1e-8 * max(1.0, abs(lam_r[i])):
            j += 1
        rb = r[:, i:j]
        lb = l_[:, i:j]
        out_l[:, i:j] = lb @ np.linalg.inv(rb.conj().T @ lb)
        i = j
    return lam_r, np.ascontiguousarray(r), np.ascontiguousarray(out_l)
