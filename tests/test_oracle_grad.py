"""Pins of the gradient oracle (oracle/grad.py).

* Daleckii-Krein on a small matrix against central finite differences of
  the spectral sign (eq. (1.3)).
* The lattice contraction (dA/dU, dA/dmu of Section 1's hopping formula)
  against finite differences of the dense exact sign on a 2^4 lattice, in
  random link directions, single link entries (real and imaginary parts) and mu.
* grad_b of L = Re chi^dagger sgn(A) b equals sgn(A(-mu)) chi (A^dagger = A(-mu)).
* The sparse stencil adjoint against finite differences of Re <tbar, A x>.
* The reverse sweep of two-sided Lanczos (m = 0) against central finite
  differences of the oracle's own forward tsl_apply, and, at a k where the
  Krylov space is exhausted, against the exact Daleckii-Krein gradient.
"""
import numpy as np
import pytest

import synth
from oracle import dirac, grad, krylov, sign

MW = -1.5


def rand_c(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def test_dk_matrix_grad_fd():
    """d Re(u^dagger sgn(a) w) in random directions E, against central FD."""
    rng = np.random.default_rng(5)
    n = 7
    a = rand_c(rng, (n, n)) + np.diag([2.0, -1.5, 1.2, -2.2, 0.9, 1.7, -0.8])
    u, w = rand_c(rng, n), rand_c(rng, n)
    G = grad.dk_matrix_grad(a, u, w)

    def L(m):
        return np.real(np.vdot(u, sign.sign_eig_apply(m, w)))

    h = 1e-5
    for _ in range(4):
        E = rand_c(rng, (n, n))
        fd = (L(a + h * E) - L(a - h * E)) / (2 * h)
        an = np.real(np.trace(G.conj().T @ E))
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(fd))


@pytest.fixture(scope="module")
def lat2():
    dims = (2, 2, 2, 2)
    U = synth.random_links(dims, 0.5, seed=41)
    rng = np.random.default_rng(42)
    N = 12 * 16
    b, chi = rand_c(rng, N), rand_c(rng, N)
    return dims, U, 0.3, b, chi


def exact_loss(dims, U, mu, b, chi):
    A = dirac.dense_A(dims, U, MW, mu)
    return np.real(np.vdot(chi, sign.sign_eig_apply(A, b)))


def test_dk_lattice_gradient_fd(lat2):
    dims, U, mu, b, chi = lat2
    gb, gmu, gU = grad.dk_gradient(dims, U, MW, mu, b, chi)
    h = 1e-5
    # mu
    fd = (exact_loss(dims, U, mu + h, b, chi) - exact_loss(dims, U, mu - h, b, chi)) / (2 * h)
    assert abs(fd - gmu) <= 1e-7 * max(1.0, abs(fd))
    # random direction over all links
    rng = np.random.default_rng(7)
    E = rand_c(rng, U.shape)
    fd = (exact_loss(dims, U + h * E, mu, b, chi) - exact_loss(dims, U - h * E, mu, b, chi)) / (2 * h)
    an = np.real(np.vdot(gU, E))
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd))
    # single entries, real and imaginary parts, including time links on the boundary
    for (s, nu, a_, b_) in [(0, 0, 0, 1), (5, 3, 2, 2), (15, 3, 1, 0), (9, 1, 0, 2)]:
        for ph in (1.0, 1j):
            E = np.zeros_like(U)
            E[s, nu, a_, b_] = ph
            fd = (exact_loss(dims, U + h * E, mu, b, chi)
                  - exact_loss(dims, U - h * E, mu, b, chi)) / (2 * h)
            an = np.real(np.conj(gU[s, nu, a_, b_]) * ph)
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd)), (s, nu, a_, b_, ph)
    # random b direction
    db = rand_c(rng, b.shape)
    fd = (exact_loss(dims, U, mu, b + h * db, chi) - exact_loss(dims, U, mu, b - h * db, chi)) / (2 * h)
    assert abs(fd - np.real(np.vdot(gb, db))) <= 1e-7 * max(1.0, abs(fd))


def test_dk_grad_b_is_adjoint_sign(lat2):
    """grad_b = sgn(A)^dagger chi = sgn(A(-mu)) chi."""
    dims, U, mu, b, chi = lat2
    gb, _, _ = grad.dk_gradient(dims, U, MW, mu, b, chi)
    ref = sign.sign_eig_apply(dirac.dense_A(dims, U, MW, -mu), chi)
    assert np.linalg.norm(gb - ref) <= 1e-11 * np.linalg.norm(ref)


def test_stencil_param_vjp_fd(lat2):
    """Re <tbar, A(U, mu) x> is linear in U: FD in random directions, and the mu part."""
    dims, U, mu, b, chi = lat2
    rng = np.random.default_rng(9)
    x = rand_c(rng, b.shape)
    tbar = rand_c(rng, b.shape)

    def L(UU, m):
        return np.real(np.vdot(tbar, dirac.csr_A(dims, UU, MW, m) @ x))

    gU = grad.stencil_param_vjp(dims, MW, mu, tbar, x)
    gmu = grad.stencil_mu_vjp(dims, U, MW, mu, tbar, x)
    h = 1e-4
    for _ in range(3):
        E = rand_c(rng, U.shape)
        fd = (L(U + h * E, mu) - L(U - h * E, mu)) / (2 * h)
        assert abs(fd - np.real(np.vdot(gU, E))) <= 1e-9 * max(1.0, abs(fd))
    fd = (L(U, mu + h) - L(U, mu - h)) / (2 * h)
    assert abs(fd - gmu) <= 1e-8 * max(1.0, abs(fd))
    # the dense contraction with G = tbar x^dagger gives the same
    gU2, gmu2 = grad.param_grad_from_matrix(dims, U, MW, mu, np.outer(tbar, np.conj(x)))
    assert np.allclose(gU, gU2, atol=1e-13)
    assert abs(gmu - gmu2) <= 1e-12


@pytest.fixture(scope="module")
def lat_tsl():
    dims = (2, 2, 4, 4)
    U = synth.random_links(dims, 0.5, seed=51)
    rng = np.random.default_rng(52)
    N = 12 * 64
    return dims, U, 0.25, rand_c(rng, N), rand_c(rng, N)


def tsl_loss(dims, U, mu, b, chi, k):
    A = dirac.csr_A(dims, U, MW, mu)
    Ad = dirac.csr_A(dims, U, MW, -mu)
    y = krylov.tsl_apply(lambda z: A @ z, lambda z: Ad @ z, b, k)
    return np.real(np.vdot(chi, y))


@pytest.mark.parametrize("k", [1, 2, 5, 24])
def test_tsl_vjp_fd(lat_tsl, k):
    """The reverse sweep is the gradient of the oracle's own forward at fixed k."""
    dims, U, mu, b, chi = lat_tsl
    y, gb, gmu, gU, _ = grad.tsl_vjp(dims, U, MW, mu, b, chi, k)
    A = dirac.csr_A(dims, U, MW, mu)
    Ad = dirac.csr_A(dims, U, MW, -mu)
    y_ref = krylov.tsl_apply(lambda z: A @ z, lambda z: Ad @ z, b, k)
    assert np.linalg.norm(y - y_ref) <= 1e-13 * np.linalg.norm(y_ref)
    h = 1e-5
    rng = np.random.default_rng(100 + k)
    scale = abs(tsl_loss(dims, U, mu, b, chi, k)) + 1.0
    fd = (tsl_loss(dims, U, mu + h, b, chi, k) - tsl_loss(dims, U, mu - h, b, chi, k)) / (2 * h)
    assert abs(fd - gmu) <= 1e-7 * max(scale, abs(fd))
    E = rand_c(rng, U.shape)
    fd = (tsl_loss(dims, U + h * E, mu, b, chi, k) - tsl_loss(dims, U - h * E, mu, b, chi, k)) / (2 * h)
    assert abs(fd - np.real(np.vdot(gU, E))) <= 1e-7 * max(scale, abs(fd))
    db = rand_c(rng, b.shape)
    fd = (tsl_loss(dims, U, mu, b + h * db, chi, k) - tsl_loss(dims, U, mu, b - h * db, chi, k)) / (2 * h)
    assert abs(fd - np.real(np.vdot(gb, db))) <= 1e-7 * max(scale, abs(fd))


def test_tsl_vjp_converges_to_dk():
    """On a 2^3 x 4 lattice (N = 384) at k = 260 the Krylov result is converged
    (5e-12) and its exact gradient matches the Daleckii-Krein gradient of sgn(A) b."""
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 0.3, seed=61)
    rng = np.random.default_rng(62)
    N = 12 * 32
    b, chi = rand_c(rng, N), rand_c(rng, N)
    mu = 0.1
    gb_ex, gmu_ex, gU_ex = grad.dk_gradient(dims, U, MW, mu, b, chi)
    y, gb, gmu, gU, _ = grad.tsl_vjp(dims, U, MW, mu, b, chi, 260)
    y_ex = sign.sign_eig_apply(dirac.dense_A(dims, U, MW, mu), b)
    assert np.linalg.norm(y - y_ex) <= 1e-10 * np.linalg.norm(y_ex)
    assert np.linalg.norm(gb - gb_ex) <= 1e-6 * np.linalg.norm(gb_ex)
    assert abs(gmu - gmu_ex) <= 1e-6 * abs(gmu_ex)
    assert np.linalg.norm(gU - gU_ex) <= 1e-6 * np.linalg.norm(gU_ex)


@pytest.mark.parametrize("k", [150, 400])
def test_fixture_8888_gradient_matches_fd(k):
    """Full-size pin (8^4): the stored oracle gradient against the stored
    central finite differences of the oracle's forward y_k, both written by
    tests/golden/make_fixtures.py, in three directions.  The tolerance adds
    the forward's measured rounding noise over the step (stored beside it)."""
    import os
    f = np.load(os.path.join(os.path.dirname(__file__), "golden", f"gradient_8888_k{k}.npz"))
    slack = 4.0 * float(f["noise"]) / float(f["h"])
    for an, fd in (("grad_mu", "fd_mu"), ("vjp_dir_U", "fd_U"), ("vjp_dir_b", "fd_b")):
        a, d = float(f[an]), float(f[fd])
        assert abs(a - d) <= 1e-6 * max(1.0, abs(d)) + slack, (an, a, d, slack)
