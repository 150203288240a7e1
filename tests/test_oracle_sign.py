"""Pins of the oracle's matrix sign (Section 1, eq. (1.3)-(1.4); Roberts'
iteration of Section 2) against closed forms, a Schur-based library square
root, Newton, the Hermitian eigh route, GW and the free-field closed form."""
import numpy as np
import pytest
import scipy.linalg as sl

import synth
from oracle import dirac, freefield, sign

MW = -1.5


def test_csgn_scalar():
    z = np.array([2 + 5j, -0.1 + 3j, 1e-300 - 1j, -4.0, 0.0])
    assert np.array_equal(sign.csgn(z), [1, -1, 1, -1, 1])


def test_triangular_closed_form():
    """sgn([[a, c], [0, b]]) with Re a > 0 > Re b is [[1, 2c/(a-b)], [0, -1]]."""
    a, b, c = 1.3 + 0.4j, -0.7 + 0.2j, 0.9 - 2.1j
    m = np.array([[a, c], [0, b]])
    s, _ = sign.sign_eig(m)
    ref = np.array([[1, 2 * c / (a - b)], [0, -1]])
    assert np.abs(s - ref).max() < 1e-14
    sn, _ = sign.sign_newton(m)
    assert np.abs(sn - ref).max() < 1e-14


@pytest.fixture(scope="module")
def lattice_A():
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 0.6, seed=21)
    return dims, U, dirac.dense_A(dims, U, MW, 0.4)


def test_square_is_identity_and_gw(lattice_A):
    _, _, A = lattice_A
    S, info = sign.sign_eig(A)
    n = A.shape[0]
    assert np.abs(S @ S - np.eye(n)).max() < 1e-12
    # Ginsparg-Wilson: g5 D + D g5 = D g5 D for D = 1 + g5 S
    g5 = np.diag(dirac.gamma5_rows(n // 12))
    D = np.eye(n) + g5 @ S
    assert np.abs(g5 @ D + D @ g5 - D @ g5 @ D).max() < 1e-12


def test_eig_matches_schur_sqrt(lattice_A):
    """sgn(A) = A (A^2)^{-1/2} with the principal root (eq. (1.4) in matrix form),
    evaluated with scipy's Schur-based sqrtm."""
    _, _, A = lattice_A
    S, _ = sign.sign_eig(A)
    ref = A @ sl.inv(sl.sqrtm(A @ A))
    assert np.abs(S - ref).max() < 1e-12


def test_eig_matches_newton(lattice_A):
    _, _, A = lattice_A
    S, _ = sign.sign_eig(A)
    Sn, iters = sign.sign_newton(A)
    assert iters < 40
    assert np.abs(S - Sn).max() < 1e-12


def test_hermitian_eigh():
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 0.6, seed=22)
    A = dirac.dense_A(dims, U, MW, 0.0)
    S, _ = sign.sign_eig(A)
    assert np.abs(S - sign.sign_eigh(A)).max() < 1e-12


def test_eigenvector_source(lattice_A):
    _, _, A = lattice_A
    lam, R = np.linalg.eig(A)
    for j in (0, 17, 200):
        y = sign.sign_eig_apply(A, R[:, j])
        assert np.abs(y - np.sign(lam[j].real) * R[:, j]).max() < 1e-12


@pytest.mark.parametrize("dims,mu", [((2, 2, 2, 4), 0.3), ((2, 2, 4, 4), 0.5)])
def test_free_field_closed_form_sign(dims, mu):
    U = synth.unit_links(dims)
    A = dirac.dense_A(dims, U, MW, mu)
    b = synth.gaussian_sources(dims, 2, seed=13)
    ref = sign.sign_eig_apply(A, b.T).T
    got = freefield.free_sign_apply(dims, MW, mu, b)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12
