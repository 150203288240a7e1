"""Krylov approximations of f(A) b with LR deflation, plain FP64 on the CPU.

Section 3 (LR deflation): with right/left eigenvectors R_m, L_m of the m
critical eigenvalues, L_m^dagger R_m = I, the source is split into an
oblique projection R_m L_m^dagger b, whose f(A) image is exact, and the rest.
Section 4 (two-sided Lanczos, eq. (4.1)-(4.4)): bases V_k of K_k(A, b_R) and
W_k of K_k(A^dagger, b_L) with W^dagger V = I and the tridiagonal
G_k = W^dagger A V, built by the short recurrences
    beta_i v_{i+1}     = (A - alpha_i) v_i - gamma_{i-1} v_{i-1}
    gamma_i^* w_{i+1}  = (A^dagger - alpha_i^*) w_i - beta_{i-1}^* w_{i-1}
with alpha_i = w_i^dagger A v_i and w_{i+1}^dagger v_{i+1} = 1, and
    f(A) b ~= R_m f(Lambda_m) L_m^dagger b + |b_R| V_k f(G_k) e_1   (eq. 2sLapp).
Section 2 (Arnoldi, eq. (2.1)-(2.5)): orthonormal V_k, Hessenberg H_k = V^dagger A V,
    f(A) b ~= R_m f(Lambda_m) L_m^dagger b + |b_R| V_k f(H_k) e_1   (eq. Arnapp).

Readings where the paper leaves a choice:
  * beta_i = ||v~||_2 (unit-norm v) and gamma_i = delta/beta_i with
    delta = w~^dagger v~; only beta_i gamma_i = delta is fixed by the text.
  * Deflated starts: v_1 = b_R/|b_R|, w_1 = b_L |b_R| / (b_L^dagger b_R)^*,
    so that w_1^dagger v_1 = 1; with m = 0 both equal b/|b| as in the text.
  * Breakdowns: lucky if |v~| <= 1e-14 |A v_i| (Krylov space exhausted,
    result exact at that size); serious if |delta| <= 1e-13 |v~||w~|
    (stop and flag, no look-ahead).
  * Arnoldi orthogonalisation by modified Gram-Schmidt.

TEST INFRASTRUCTURE: only tests, smoke and the CPU baseline use this module.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .sign import csgn, sign_e1

LUCKY_TOL = 1e-14
SERIOUS_TOL = 1e-13


@dataclass
class Deflated:
    b_R: np.ndarray
    b_L: np.ndarray
    y_ex: np.ndarray
    C: np.ndarray
    D: np.ndarray


def deflate(b, lam=None, R=None, L=None, f=csgn) -> Deflated:
    """LR deflation of one source (Section 3 and the end of Section 4).

    C = L^dagger b, D = R^dagger b, b_R = b - R C, b_L = b - L D,
    y_ex = R f(Lambda) C."""
    b = np.asarray(b, dtype=np.complex128)
    if R is None or R.shape[1] == 0:
        z = np.zeros(0, dtype=np.complex128)
        return Deflated(b.copy(), b.copy(), np.zeros_like(b), z, z)
    C = L.conj().T @ b
    D = R.conj().T @ b
    b_R = b - R @ C
    b_L = b - L @ D
    y_ex = R @ (f(lam) * C)
    return Deflated(b_R, b_L, y_ex, C, D)


@dataclass
class LanczosResult:
    alpha: np.ndarray
    beta: np.ndarray
    gamma: np.ndarray
    V: list | None
    W: list | None
    k: int
    status: str = "ok"      # "ok", "lucky", "serious"
    n_b: float = 0.0
    extra: dict = field(default_factory=dict)


def two_sided_lanczos(matvec, rmatvec, b_R, b_L, k, store=True) -> LanczosResult:
    """Two-sided Lanczos of Section 4 from the deflated starts b_R, b_L.

    matvec(x) = A x, rmatvec(x) = A^dagger x.  Returns the tridiagonal
    coefficients (alpha_1..alpha_k, beta_1..beta_{k-1}, gamma_1..gamma_{k-1})
    and, if store, the bases V, W as lists of vectors."""
    n_b = float(np.linalg.norm(b_R))
    if n_b == 0.0:
        return LanczosResult(np.zeros(0, complex), np.zeros(0), np.zeros(0, complex),
                             [], [], 0, "empty", 0.0)
    v = b_R / n_b
    sigma = np.vdot(b_L, b_R)
    if sigma == 0:
        return LanczosResult(np.zeros(0, complex), np.zeros(0), np.zeros(0, complex),
                             [], [], 0, "serious", n_b)
    w = b_L * n_b / np.conj(sigma)
    V = [v] if store else None
    W = [w] if store else None
    alpha, beta, gamma = [], [], []
    v_prev = np.zeros_like(v)
    w_prev = np.zeros_like(w)
    beta_prev = 0.0
    gamma_prev = 0.0
    status = "ok"
    for i in range(k):
        t = matvec(v)
        a = np.vdot(w, t)
        alpha.append(a)
        if i == k - 1:
            break
        vt = t - a * v - gamma_prev * v_prev
        wt = rmatvec(w) - np.conj(a) * w - np.conj(beta_prev) * w_prev
        delta = np.vdot(wt, vt)
        bn = np.linalg.norm(vt)
        if bn <= LUCKY_TOL * np.linalg.norm(t):
            status = "lucky"
            break
        wn = np.linalg.norm(wt)
        if abs(delta) <= SERIOUS_TOL * bn * wn:
            status = "serious"
            break
        g = delta / bn
        beta.append(bn)
        gamma.append(g)
        v_prev, w_prev = v, w
        v = vt / bn
        w = wt / np.conj(g)
        beta_prev, gamma_prev = bn, g
        if store:
            V.append(v)
            W.append(w)
    kk = len(alpha)
    if store:
        V = V[:kk]
        W = W[:kk]
    return LanczosResult(np.array(alpha), np.array(beta), np.array(gamma), V, W, kk, status, n_b)


def tridiag(alpha, beta, gamma) -> np.ndarray:
    """G_k of eq. (4.2): alpha on the diagonal, beta below, gamma above."""
    k = len(alpha)
    g = np.diag(np.asarray(alpha, dtype=np.complex128))
    for i in range(k - 1):
        g[i + 1, i] = beta[i]
        g[i, i + 1] = gamma[i]
    return g


def tsl_apply(matvec, rmatvec, b, k, defl=None, inner=sign_e1, two_pass=False,
              f_scalar=csgn, return_info=False):
    """f(A) b by eq. 2sLapp (LR-deflated two-sided Lanczos).

    defl: None or (lam, R, L).  inner(G) -> f(G) e_1.  With two_pass the
    basis is not stored: a second sweep replays the v-recurrence with the
    stored coefficients and accumulates the result (end of Section 5)."""
    d = deflate(b, *(defl if defl is not None else (None, None, None)), f=f_scalar)
    lr = two_sided_lanczos(matvec, rmatvec, d.b_R, d.b_L, k, store=not two_pass)
    y = d.y_ex.copy()
    x = np.zeros(0, dtype=np.complex128)
    if lr.k > 0 and lr.status != "serious":
        g = tridiag(lr.alpha, lr.beta, lr.gamma)
        x = inner(g)
        if two_pass:
            y = y + lr.n_b * replay_combine(matvec, d.b_R / lr.n_b, lr, x)
        else:
            y = y + lr.n_b * (np.array(lr.V).T @ x)
    if return_info:
        return y, {"lanczos": lr, "x": x, "deflated": d}
    return y


def replay_combine(matvec, v1, lr: LanczosResult, x) -> np.ndarray:
    """Second pass: regenerate v_1..v_k from the stored alpha, beta, gamma and
    return sum_i x_i v_i (small-memory evaluation of eq. 2sLapp)."""
    v_prev = np.zeros_like(v1)
    v = v1
    acc = x[0] * v
    for i in range(1, lr.k):
        t = matvec(v)
        g_prev = lr.gamma[i - 2] if i >= 2 else 0.0
        vn = (t - lr.alpha[i - 1] * v - g_prev * v_prev) / lr.beta[i - 1]
        v_prev, v = v, vn
        acc = acc + x[i] * v
    return acc


@dataclass
class ArnoldiResult:
    H: np.ndarray
    V: list
    k: int
    status: str
    n_b: float


def arnoldi(matvec, b_R, k) -> ArnoldiResult:
    """Arnoldi recursion A V_k = V_k H_k + beta_k v_{k+1} e_k^T (Section 2),
    orthogonalised by modified Gram-Schmidt."""
    n_b = float(np.linalg.norm(b_R))
    if n_b == 0.0:
        return ArnoldiResult(np.zeros((0, 0), complex), [], 0, "empty", 0.0)
    V = [b_R / n_b]
    H = np.zeros((k + 1, k), dtype=np.complex128)
    status = "ok"
    kk = k
    for j in range(k):
        t = matvec(V[j])
        tn = np.linalg.norm(t)
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], t)
            t = t - H[i, j] * V[i]
        h = np.linalg.norm(t)
        H[j + 1, j] = h
        if j == k - 1:
            break
        if h <= LUCKY_TOL * tn:
            status = "lucky"
            kk = j + 1
            break
        V.append(t / h)
    return ArnoldiResult(H[:kk, :kk].copy(), V[:kk], kk, status, n_b)


def arnoldi_apply(matvec, b, k, defl=None, inner=sign_e1, f_scalar=csgn, return_info=False):
    """f(A) b by eq. Arnapp (LR-deflated Arnoldi)."""
    d = deflate(b, *(defl if defl is not None else (None, None, None)), f=f_scalar)
    ar = arnoldi(matvec, d.b_R, k)
    y = d.y_ex.copy()
    x = np.zeros(0, dtype=np.complex128)
    if ar.k > 0:
        x = inner(ar.H)
        y = y + ar.n_b * (np.array(ar.V).T @ x)
    if return_info:
        return y, {"arnoldi": ar, "x": x, "deflated": d}
    return y
