"""Closed-form sgn(gamma5 Dw(mu)) for the free field U = 1.

With unit links the operator of Section 1 is translation invariant.  On the
plane wave e^{i p.x} (p_j = 2 pi n_j / L_j in space, p_4 = 2 pi (n_4 + 1/2)/L_t
for antiperiodic time) the hops give

    Dw(p) = 2 kappa [ M(q) + i sum_nu gamma_nu sin q_nu ],
    M(q)  = m_w + sum_nu (1 - cos q_nu),   q_j = p_j,  q_4 = p_4 + i mu,

because e^{mu} e^{-i p_4} = e^{-i q_4}.  Then A(p) = gamma5 Dw(p) squares to
(2 kappa)^2 (M^2 + sum sin^2 q_nu) times the identity, so by eq. (1.4)

    sgn(A(p)) = gamma5 (M + i gamma.sin q) / sqrt(M^2 + sum sin^2 q)

with the principal square root.  This is exact at any lattice size.

TEST INFRASTRUCTURE: only tests, smoke and the CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np

from .dirac import gamma_matrices


def _momenta(dims, mu):
    lx, ly, lz, lt = dims
    px = 2 * np.pi * np.fft.fftfreq(lx) * 1.0
    py = 2 * np.pi * np.fft.fftfreq(ly)
    pz = 2 * np.pi * np.fft.fftfreq(lz)
    pt = 2 * np.pi * np.fft.fftfreq(lt) + np.pi / lt + 1j * mu
    # array axes are [t][z][y][x]
    qt, qz, qy, qx = np.meshgrid(pt, pz, py, px, indexing="ij")
    return [qx, qy, qz, qt]


def _apply_momentum_space(dims, b, mat_of_q):
    lx, ly, lz, lt = dims
    nrhs = b.shape[0]
    psi = b.reshape(nrhs, lt, lz, ly, lx, 4, 3)
    t = np.arange(lt)
    twist = np.exp(-1j * np.pi * t / lt)[None, :, None, None, None, None, None]
    phi = np.fft.fftn(psi * twist, axes=(1, 2, 3, 4))
    m = mat_of_q  # [lt,lz,ly,lx,4,4]
    phi = np.einsum("tzyxij,ntzyxjc->ntzyxic", m, phi)
    out = np.fft.ifftn(phi, axes=(1, 2, 3, 4)) / twist
    return out.reshape(nrhs, -1)


def free_A_momentum(dims, m_w, mu):
    """A(p) = gamma5 Dw(p) per momentum, shape [lt,lz,ly,lx,4,4]."""
    gam, g5 = gamma_matrices()
    kap = 1.0 / (8.0 + 2.0 * m_w)
    q = _momenta(dims, mu)
    mq = m_w + sum(1.0 - np.cos(qn) for qn in q)
    dw = mq[..., None, None] * np.eye(4)
    for nu in range(4):
        dw = dw + 1j * np.sin(q[nu])[..., None, None] * gam[nu]
    return 2.0 * kap * np.einsum("ij,...jk->...ik", g5, dw)


def free_sign_momentum(dims, m_w, mu):
    """sgn(A(p)) per momentum from the closed form, shape [lt,lz,ly,lx,4,4]."""
    gam, g5 = gamma_matrices()
    q = _momenta(dims, mu)
    mq = m_w + sum(1.0 - np.cos(qn) for qn in q)
    s2 = sum(np.sin(qn) ** 2 for qn in q)
    root = np.sqrt(mq * mq + s2 + 0j)
    dw = mq[..., None, None] * np.eye(4)
    for nu in range(4):
        dw = dw + 1j * np.sin(q[nu])[..., None, None] * gam[nu]
    return np.einsum("ij,...jk->...ik", g5, dw) / root[..., None, None]


def free_apply_A(dims, m_w, mu, b):
    """A b for U = 1, via the Fourier transform.  b: complex [nrhs][12V]."""
    b = np.atleast_2d(b)
    return _apply_momentum_space(tuple(dims), b, free_A_momentum(tuple(dims), m_w, mu))


def free_sign_apply(dims, m_w, mu, b):
    """sgn(A) b for U = 1 from the closed form.  b: complex [nrhs][12V]."""
    b = np.atleast_2d(b)
    return _apply_momentum_space(tuple(dims), b, free_sign_momentum(tuple(dims), m_w, mu))
