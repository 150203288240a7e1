"""Gradients of L = Re <chi, sgn(A) b> (A = gamma5 Dw(mu)) with respect to the
source b, the chemical potential mu and the gauge links U.

Conventions.  For a real L of complex z the gradient is
    zbar = dL/dRe z + i dL/dIm z,   so that   dL = Re <zbar, dz>,
the convention of PyTorch's autograd.  U is differentiated entry by entry as
an unconstrained complex 3x3 matrix (no projection on the Lie algebra).

Two oracles:

* Exact derivative of the spectral sign (eq. (1.3) with f = sgn): the
  Daleckii-Krein formula for A = R diag(lambda) R^{-1},
      dS[E] = R (F o (R^{-1} E R)) R^{-1},
      F_ij = (s_i - s_j) / (lambda_i - lambda_j)  if s_i != s_j, else 0
  (s = sgn(Re lambda), piecewise constant, so f' = 0 on the diagonal),
  gives the matrix gradient G_A with dL = Re tr(G_A^dagger dA), contracted
  with dA/dU and dA/dmu from the hopping formula of Section 1.  Dense, so
  for lattices of at most a few hundred sites.

* Reverse sweep of the two-sided Lanczos approximation of Section 4 without
  deflation (m = 0): y_k = |b| V_k sgn(G_k) e_1 with the recurrences
  (4.1)-(4.4) and the starts v_1 = w_1 = b/|b|.  The derivative of the
  inner sign sgn(G_k) e_1 is again Daleckii-Krein, on the k x k matrix.
  The sweep walks the recurrences backwards, one stencil adjoint per A and
  per A^dagger application, and is the exact gradient of y_k as a function
  of (b, mu, U) at fixed k.

TEST INFRASTRUCTURE: only tests, smoke and the CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np

from . import dirac, krylov
from .sign import csgn, sign_e1


# ---------------------------------------------------------------- exact (DK)

def dk_matrix_grad(a: np.ndarray, u: np.ndarray, w: np.ndarray) -> np.ndarray:
    """G with d Re(u^dagger sgn(a) w) = Re tr(G^dagger da), by Daleckii-Krein.

    With c = R^dagger u, p = R^{-1} w and M_ij = conj(c_i) F_ij p_j,
    Re u^dagger dS[E] w = Re tr(K E) with K = R M^T R^{-1}, so G = K^dagger."""
    lam, r = np.linalg.eig(a)
    s = csgn(lam)
    rinv = np.linalg.inv(r)
    ds = s[:, None] - s[None, :]
    dl = lam[:, None] - lam[None, :]
    F = np.zeros_like(dl)
    nz = ds != 0
    F[nz] = ds[nz] / dl[nz]
    c = r.conj().T @ u
    p = rinv @ w
    M = np.conj(c)[:, None] * F * p[None, :]
    K = r @ M.T @ rinv
    return K.conj().T


def hop_gammas(nu: int):
    """Spin matrices of the two hops of direction nu inside A = gamma5 Dw:
    gamma5 (1 + gamma_nu) (forward, field from x - nu) and gamma5 (1 - gamma_nu)."""
    gam, g5 = dirac.gamma_matrices()
    one = np.eye(4, dtype=np.complex128)
    return g5 @ (one + gam[nu]), g5 @ (one - gam[nu])


def param_grad_from_matrix(dims, U, m_w, mu, G, bc=dirac.DEFAULT_BC):
    """Contract a dense gradient G (dL = Re tr(G^dagger dA)) with dA/dU and dA/dmu.

    A's forward block at (rows x + nu, columns x) is
        -kappa eta+_nu b_nu(x) kron(gamma5 (1 + gamma_nu), U_nu(x))
    and its backward block at (rows x, columns x + nu) is
        -kappa eta-_nu b_nu(x) kron(gamma5 (1 - gamma_nu), U_nu(x)^dagger);
    d/dmu multiplies the forward time blocks by +1 and the backward ones by -1.
    Returns (grad_U [V, 4, 3, 3], grad_mu)."""
    dims = tuple(int(d) for d in dims)
    v = int(np.prod(dims))
    kap = dirac.kappa_of(m_w)
    eta_p, eta_m = dirac.hop_factors(mu)
    gU = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    gmu = 0.0
    for nu in range(4):
        gp, gm = hop_gammas(nu)
        for s in range(v):
            sp_ = dirac.forward(dims, s, nu)
            b = dirac.boundary_sign(dims, s, nu, bc)
            u = U[s, nu]
            blk_f = G[12 * sp_:12 * sp_ + 12, 12 * s:12 * s + 12].reshape(4, 3, 4, 3)
            blk_b = G[12 * s:12 * s + 12, 12 * sp_:12 * sp_ + 12].reshape(4, 3, 4, 3)
            cf = -kap * eta_p[nu] * b
            cb = -kap * eta_m[nu] * b
            # forward: dA_(alpha a),(beta b) = cf gp[alpha, beta] dU[a, b]
            gU[s, nu] += cf * np.einsum("iajb,ij->ab", blk_f, np.conj(gp))
            # backward: dA_(alpha a),(beta b) = cb gm[alpha, beta] conj(dU[b, a])
            gU[s, nu] += cb * np.einsum("iajb,ij->ba", np.conj(blk_b), gm)
            if nu == 3:
                val_f = cf * np.kron(gp, u)
                val_b = cb * np.kron(gm, u.conj().T)
                gmu += np.real(np.vdot(G[12 * sp_:12 * sp_ + 12, 12 * s:12 * s + 12], val_f))
                gmu -= np.real(np.vdot(G[12 * s:12 * s + 12, 12 * sp_:12 * sp_ + 12], val_b))
    return gU, gmu


def dk_gradient(dims, U, m_w, mu, b, chi, bc=dirac.DEFAULT_BC):
    """Exact (grad_b, grad_mu, grad_U) of L = Re chi^dagger sgn(A) b, dense.

    grad_b = sgn(A)^dagger chi; the rest from the Daleckii-Krein matrix gradient."""
    A = dirac.dense_A(dims, U, m_w, mu, bc)
    G = dk_matrix_grad(A, chi, b)
    lam, r = np.linalg.eig(A)
    S = (r * csgn(lam)[None, :]) @ np.linalg.inv(r)
    grad_b = S.conj().T @ chi
    gU, gmu = param_grad_from_matrix(dims, U, m_w, mu, G, bc)
    return grad_b, gmu, gU


# ------------------------------------------------ stencil parameter adjoint

def stencil_param_vjp(dims, m_w, mu, tbar, x, bc=dirac.DEFAULT_BC):
    """grad_U of Re <tbar, A(mu) x> with the links as variables.

    The forward hop into site x + nu gives, for link U_nu(x),
        cf * sum_{alpha beta} conj(gp[alpha, beta]) tbar(x+nu)[alpha, a] conj(x(x)[beta, b])
    and the backward hop into site x gives for entry (i, j)
        cb * sum_{alpha beta} gm[alpha, beta] x(x+nu)[beta, i] conj(tbar(x)[alpha, j]),
    with cf = -kappa eta+ b_nu(x), cb = -kappa eta- b_nu(x).  Vectorised over
    sites; the same formula as param_grad_from_matrix with G = tbar x^dagger."""
    dims = tuple(int(d) for d in dims)
    v = int(np.prod(dims))
    kap = dirac.kappa_of(m_w)
    eta_p, eta_m = dirac.hop_factors(mu)
    tb = np.asarray(tbar).reshape(v, 4, 3)
    xx = np.asarray(x).reshape(v, 4, 3)
    s_all = np.arange(v)
    cc = list(dirac.coords(dims, s_all))
    gU = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    for nu in range(4):
        c2 = list(cc)
        c2[nu] = cc[nu] + 1
        fw = dirac.site_of(dims, *c2)
        bsign = np.where(cc[nu] == dims[nu] - 1, bc[nu], 1.0)
        gp, gm = hop_gammas(nu)
        ff = np.einsum("ij,sia,sjb->sab", np.conj(gp), tb[fw], np.conj(xx))
        fb = np.einsum("ij,sjc,sid->scd", gm, xx[fw], np.conj(tb))
        cf = -kap * eta_p[nu] * bsign
        cb = -kap * eta_m[nu] * bsign
        gU[:, nu] += cf[:, None, None] * ff + cb[:, None, None] * fb
    return gU


def stencil_mu_vjp(dims, U, m_w, mu, tbar, x, bc=dirac.DEFAULT_BC):
    """d/dmu of Re <tbar, A(mu) x>: the forward time hop scaled by +1, the
    backward one by -1 (eta_4^{+-} = e^{+-mu})."""
    dims = tuple(int(d) for d in dims)
    v = int(np.prod(dims))
    kap = dirac.kappa_of(m_w)
    eta_p, eta_m = dirac.hop_factors(mu)
    tb = np.asarray(tbar).reshape(v, 4, 3)
    xx = np.asarray(x).reshape(v, 4, 3)
    s_all = np.arange(v)
    cc = list(dirac.coords(dims, s_all))
    c2 = list(cc)
    c2[3] = cc[3] + 1
    fw = dirac.site_of(dims, *c2)
    bsign = np.where(cc[3] == dims[3] - 1, bc[3], 1.0)
    gp, gm = hop_gammas(3)
    u = U[:, 3]
    # forward: contribution to (A x)(x + 4) from site x
    hf = np.einsum("ij,sab,sjb->sia", gp, u, xx)
    # backward: contribution to (A x)(x) from site x + 4
    hb = np.einsum("ij,sba,sjb->sia", gm, np.conj(u), xx[fw])
    tf = -kap * eta_p[3] * bsign
    tbk = -kap * eta_m[3] * bsign
    val = np.sum(tf * np.einsum("sia,sia->s", np.conj(tb[fw]), hf))
    val -= np.sum(tbk * np.einsum("sia,sia->s", np.conj(tb), hb))
    return float(np.real(val))


# ------------------------------------------- reverse sweep of 2sL (m = 0)

def sign_e1_vjp(g: np.ndarray, xbar: np.ndarray) -> np.ndarray:
    """Gbar with d Re(xbar^dagger sgn(g) e_1) = Re tr(Gbar^dagger dg) (dense k x k)."""
    e1 = np.zeros(g.shape[0], dtype=np.complex128)
    e1[0] = 1.0
    return dk_matrix_grad(g, xbar, e1)


def tsl_vjp(dims, U, m_w, mu, b, chi, k, bc=dirac.DEFAULT_BC):
    """y_k = |b| V_k sgn(G_k) e_1 (two-sided Lanczos, m = 0) and the exact
    gradient of L = Re chi^dagger y_k with respect to (b, mu, U).

    Forward (Section 4, i = 1..k, 0-based below): t_i = A v_i,
    alpha_i = w_i^dagger t_i; for i < k-1: v~ = t_i - alpha_i v_i - gamma_{i-1} v_{i-1},
    w~ = A^dagger w_i - conj(alpha_i) w_i - beta_{i-1} w_{i-1}, delta_i = w~^dagger v~,
    beta_i = |v~|, gamma_i = delta_i/beta_i, v_{i+1} = v~/beta_i, w_{i+1} = w~/conj(gamma_i).
    Returns (y, grad_b, grad_mu, grad_U, info)."""
    A = dirac.csr_A(dims, U, m_w, mu, bc)
    Ad = dirac.csr_A(dims, U, m_w, -mu, bc)       # A(mu)^dagger = A(-mu)
    b = np.asarray(b, dtype=np.complex128)
    lr = krylov.two_sided_lanczos(lambda z: A @ z, lambda z: Ad @ z, b, b, k, store=True)
    if lr.status != "ok" or lr.k != k:
        raise ValueError(f"two-sided Lanczos stopped early ({lr.status}) at k = {lr.k}")
    V, W = lr.V, lr.W
    al, be, ga = lr.alpha, lr.beta, lr.gamma
    n_b = lr.n_b
    G = krylov.tridiag(al, be, ga)
    x = sign_e1(G)
    y = n_b * (np.array(V).T @ x)

    # y = n_b sum_i x_i v_i
    xbar = n_b * np.array([np.vdot(vi, chi) for vi in V])
    Gbar = sign_e1_vjp(G, xbar)
    abar = np.diag(Gbar).copy()
    bbar = np.array([np.real(Gbar[i + 1, i]) for i in range(k - 1)])
    gbar = np.array([Gbar[i, i + 1] for i in range(k - 1)], dtype=np.complex128)
    vbar = [n_b * np.conj(x[i]) * chi for i in range(k)]
    wbar = [np.zeros_like(b) for _ in range(k)]
    nbar = float(np.real(np.vdot(chi, y))) / n_b

    gU = np.zeros((int(np.prod(dims)), 4, 3, 3), dtype=np.complex128)
    gmu = 0.0
    for i in range(k - 1, -1, -1):
        t_i = A @ V[i]
        tbar = np.zeros_like(b)
        sbar = None
        if i < k - 1:
            # w_{i+1} = w~/conj(gamma_i), v_{i+1} = v~/beta_i
            gbar[i] += -np.vdot(wbar[i + 1], W[i + 1]) / np.conj(ga[i])
            bbar[i] += -np.real(np.vdot(vbar[i + 1], V[i + 1])) / be[i]
            # gamma_i = delta_i / beta_i
            dbar = gbar[i] / be[i]
            bbar[i] += -np.real(np.conj(gbar[i]) * ga[i]) / be[i]
            # v~ feeds v_{i+1}, beta_i = |v~| and delta_i; w~ feeds w_{i+1} and delta_i
            vt = be[i] * V[i + 1]
            wt = np.conj(ga[i]) * W[i + 1]
            vtbar = vbar[i + 1] / be[i] + bbar[i] * V[i + 1] + dbar * wt
            wtbar = wbar[i + 1] / ga[i] + np.conj(dbar) * vt
            # w~ = s_i - conj(alpha_i) w_i - beta_{i-1} w_{i-1}
            sbar = wtbar
            wbar[i] += -al[i] * wtbar
            abar[i] += -np.vdot(wtbar, W[i])
            if i >= 1:
                wbar[i - 1] += -be[i - 1] * wtbar
                bbar[i - 1] += -np.real(np.vdot(W[i - 1], wtbar))
            # v~ = t_i - alpha_i v_i - gamma_{i-1} v_{i-1}
            tbar = tbar + vtbar
            vbar[i] += -np.conj(al[i]) * vtbar
            abar[i] += -np.vdot(V[i], vtbar)
            if i >= 1:
                vbar[i - 1] += -np.conj(ga[i - 1]) * vtbar
                gbar[i - 1] += -np.vdot(V[i - 1], vtbar)
        # alpha_i = w_i^dagger t_i
        tbar = tbar + abar[i] * W[i]
        wbar[i] += np.conj(abar[i]) * t_i
        # t_i = A v_i ; s_i = A^dagger w_i = A(-mu) w_i
        vbar[i] += Ad @ tbar
        gU += stencil_param_vjp(dims, m_w, mu, tbar, V[i], bc)
        gmu += stencil_mu_vjp(dims, U, m_w, mu, tbar, V[i], bc)
        if sbar is not None:
            wbar[i] += A @ sbar
            gU += stencil_param_vjp(dims, m_w, -mu, sbar, W[i], bc)
            gmu -= stencil_mu_vjp(dims, U, m_w, -mu, sbar, W[i], bc)
    # v_1 = w_1 = b/n_b, n_b = |b|
    ubar = vbar[0] + wbar[0]
    u0 = b / n_b
    nbar += -np.real(np.vdot(ubar, u0)) / n_b
    grad_b = ubar / n_b + nbar * u0
    info = {"alpha": al, "beta": be, "gamma": ga, "x": x, "n_b": n_b}
    return y, grad_b, gmu, gU, info


# ------------------------------------------------------------ plain helpers

def loss(y, chi) -> float:
    """L = Re <chi, y>."""
    return float(np.real(np.vdot(chi, y)))


# ------------------------------------------------ Lie-algebra force

def lie_force(U: np.ndarray, G: np.ndarray) -> np.ndarray:
    """The su(3) force of a real L(U) from its link gradient G (the convention
    above: G = dL/dRe U + i dL/dIm U, per link [.., 3, 3]).

    For U -> exp(eps X) U with X traceless anti-Hermitian, dL/deps =
    Re tr(G^dagger X U) = Re tr(X U G^dagger) = <F, X> with <A, B> = Re tr(A^dagger B)
    and F = -TA(U G^dagger), TA(M) = (M - M^dagger)/2 - tr(M - M^dagger)/6 * 1
    (the projection onto su(3), orthogonal for that inner product).  Not in the
    paper: the link force a molecular-dynamics update of the gauge field needs.
    Pinned by central differences of the dense exact L along exp(eps X) U."""
    M = U @ np.conj(np.swapaxes(G, -1, -2))
    A = 0.5 * (M - np.conj(np.swapaxes(M, -1, -2)))
    tr = np.trace(A, axis1=-2, axis2=-1)[..., None, None]
    return -(A - tr / 3.0 * np.eye(3))
