"""Pin of the oracle's su(3) link force (oracle.grad.lie_force) against
central differences of the dense exact L = Re chi^dagger sgn(A(U)) b along
U -> exp(eps X) U, for random traceless anti-Hermitian X on every link."""
import numpy as np
import scipy.linalg as sl

import synth
from oracle import dirac, grad, sign

MW = -1.5


def random_su3_algebra(rng, shape):
    h = rng.normal(size=shape + (3, 3)) + 1j * rng.normal(size=shape + (3, 3))
    x = 0.5 * (h - np.conj(np.swapaxes(h, -1, -2)))
    tr = np.trace(x, axis1=-2, axis2=-1)[..., None, None]
    return x - tr / 3.0 * np.eye(3)


def loss(dims, U, mu, b, chi):
    A = dirac.dense_A(dims, U, MW, mu)
    S, _ = sign.sign_eig(A)
    return float(np.real(np.vdot(chi, S @ b)))


def test_lie_force_matches_differences():
    dims = (2, 2, 2, 4)
    mu = 0.3
    U = synth.random_links(dims, 0.6, seed=41)
    b = synth.gaussian_sources(dims, 1, seed=42)[0]
    chi = synth.gaussian_sources(dims, 1, seed=43)[0]
    _, _, gU = grad.dk_gradient(dims, U, MW, mu, b, chi)
    F = grad.lie_force(U, gU)
    # F is traceless anti-Hermitian
    assert np.abs(F + np.conj(np.swapaxes(F, -1, -2))).max() < 1e-13
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-13
    rng = np.random.default_rng(44)
    X = random_su3_algebra(rng, U.shape[:2])
    h = 1e-4
    Up = np.stack([np.stack([sl.expm(h * X[s, n]) @ U[s, n] for n in range(4)]) for s in range(U.shape[0])])
    Um = np.stack([np.stack([sl.expm(-h * X[s, n]) @ U[s, n] for n in range(4)]) for s in range(U.shape[0])])
    fd = (loss(dims, Up, mu, b, chi) - loss(dims, Um, mu, b, chi)) / (2 * h)
    pred = float(np.sum(np.real(np.conj(F) * X)))
    assert abs(fd - pred) <= 1e-6 * max(1.0, abs(pred)), (fd, pred)


def test_lie_force_orientation():
    """A planted mistake (the gradient's orientation conj(G) U^dagger instead of
    U G^dagger) changes the directional derivative: the pin above is sensitive."""
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 0.6, seed=45)
    rng = np.random.default_rng(46)
    G = rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape)
    F = grad.lie_force(U, G)
    M = np.conj(G) @ np.conj(np.swapaxes(U, -1, -2))
    A = 0.5 * (M - np.conj(np.swapaxes(M, -1, -2)))
    Fw = -(A - np.trace(A, axis1=-2, axis2=-1)[..., None, None] / 3.0 * np.eye(3))
    assert np.abs(F - Fw).max() > 1e-3
