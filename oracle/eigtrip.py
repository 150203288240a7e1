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


def sparse_eigentriples(a_csr, a_dag_csr, m: int, tol: float = 1e-12, extra: int = 4):
    """Shift-invert ARPACK (sigma = 0) on A for R and on A^dagger for L, paired by
    lambda_L ~ conj(lambda_R) and biorthonormalised so that L^dagger R = I.

    Returns (lam, R, L) ordered by (|lambda|, Re, Im).  Clusters of nearly
    equal eigenvalues are biorthonormalised blockwise."""
    nev = m + extra
    lam_r, r = spla.eigs(a_csr.tocsc(), k=nev, sigma=0, tol=tol)
    lam_l, l_ = spla.eigs(a_dag_csr.tocsc(), k=nev, sigma=0, tol=tol)
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
