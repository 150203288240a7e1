"""Pins of the oracle's Wilson-Dirac operator (Section 1) against facts that do
not depend on the oracle's own assembly: the Clifford algebra, the free-field
Fourier closed form, the zero-momentum mode, hermiticity identities and gauge
covariance."""
import numpy as np
import pytest

import synth
from oracle import dirac, freefield

MW = -1.5


def test_gamma_algebra():
    gam, g5 = dirac.gamma_matrices()
    one = np.eye(4)
    for a in range(4):
        assert np.allclose(gam[a], gam[a].conj().T)
        for b in range(4):
            anti = gam[a] @ gam[b] + gam[b] @ gam[a]
            assert np.allclose(anti, 2.0 * one * (a == b))
    # chiral basis: gamma5 = g1 g2 g3 g4 is diagonal (1, 1, -1, -1)
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    for a in range(4):
        assert np.allclose(g5 @ gam[a] + gam[a] @ g5, 0)


def test_kappa():
    assert dirac.kappa_of(-1.5) == pytest.approx(0.2)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 3, 4, 5), (3, 2, 2, 4)])
def test_dense_equals_csr(dims):
    U = synth.random_links(dims, 0.5, seed=3)
    d = dirac.dense_A(dims, U, MW, 0.37)
    c = dirac.csr_A(dims, U, MW, 0.37).toarray()
    assert np.array_equal(d, c)


def test_sites_equal_rows():
    dims = (2, 3, 2, 4)
    U = synth.random_links(dims, 0.5, seed=4)
    x = synth.gaussian_sources(dims, 1, seed=9)[0]
    A = dirac.dense_A(dims, U, MW, 0.2)
    sites = [0, 1, 7, 47]
    ref = (A @ x).reshape(-1, 12)[sites]
    got = dirac.apply_at_sites(dims, U, MW, 0.2, x, sites, op="A")
    assert np.abs(got - ref).max() < 1e-14


def test_single_forward_time_hop():
    """Column x of Dw, block row x + t_hat, equals -kappa e^{mu} (1 + gamma_4) U_{x,4}
    (literal T_4^+ of Section 1, away from the time boundary)."""
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 0.7, seed=5)
    mu = 0.45
    d = dirac.dense_dw(dims, U, MW, mu)
    gam, _ = dirac.gamma_matrices()
    x = 3  # t = 0
    y = dirac.forward(dims, x, 3)
    blk = d[12 * y:12 * y + 12, 12 * x:12 * x + 12]
    ref = -0.2 * np.exp(mu) * np.kron(np.eye(4) + gam[3], U[x, 3])
    assert np.abs(blk - ref).max() < 1e-15


def test_zero_momentum_periodic_free_mode():
    """U = 1, mu = 0, periodic time: a constant spinor sees A = 2 kappa m_w gamma5,
    i.e. eigenvalues +-0.6 at m_w = -1.5."""
    dims = (2, 2, 2, 2)
    U = synth.unit_links(dims)
    A = dirac.dense_A(dims, U, MW, 0.0, bc=(1, 1, 1, 1))
    v = 16
    for j in range(12):
        u = np.zeros(12)
        u[j] = 1.0
        x = np.tile(u, v)
        y = A @ x
        sign = 1.0 if j < 6 else -1.0
        assert np.abs(y - sign * (-0.6) * x).max() < 1e-14


@pytest.mark.parametrize("dims,mu", [((2, 2, 2, 4), 0.3), ((2, 3, 4, 6), 0.5), ((4, 2, 2, 2), 0.0)])
def test_free_field_fourier_operator(dims, mu):
    U = synth.unit_links(dims)
    A = dirac.csr_A(dims, U, MW, mu)
    b = synth.gaussian_sources(dims, 2, seed=11)
    ref = (A @ b.T).T
    got = freefield.free_apply_A(dims, MW, mu, b)
    assert np.abs(got - ref).max() < 1e-13


def test_adjoint_is_minus_mu():
    dims = (2, 2, 3, 4)
    U = synth.random_links(dims, 0.6, seed=6)
    A = dirac.dense_A(dims, U, MW, 0.3)
    Am = dirac.dense_A(dims, U, MW, -0.3)
    assert np.abs(A.conj().T - Am).max() < 1e-15
    A0 = dirac.dense_A(dims, U, MW, 0.0)
    assert np.abs(A0 - A0.conj().T).max() < 1e-15
    assert np.abs(A - A.conj().T).max() > 1e-3


def test_gauge_covariance():
    """A[U^g] (g psi) = g A[U] psi with U_nu(x) -> g(x+nu) U_nu(x) g(x)^dagger."""
    dims = (2, 3, 2, 4)
    v = synth.volume(dims)
    U = synth.random_links(dims, 0.6, seed=7)
    g = synth.random_gauge(dims, seed=8)
    Ug = np.empty_like(U)
    for s in range(v):
        for nu in range(4):
            sp_ = dirac.forward(dims, s, nu)
            Ug[s, nu] = g[sp_] @ U[s, nu] @ g[s].conj().T
    psi = synth.gaussian_sources(dims, 1, seed=12)[0].reshape(v, 4, 3)
    gpsi = np.einsum("sab,sib->sia", g, psi).reshape(-1)
    A = dirac.csr_A(dims, U, MW, 0.3)
    Ag = dirac.csr_A(dims, Ug, MW, 0.3)
    lhs = Ag @ gpsi
    rhs = np.einsum("sab,sib->sia", g, (A @ psi.reshape(-1)).reshape(v, 4, 3)).reshape(-1)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_links_are_su3():
    U = synth.random_links((2, 2, 2, 2), 0.8, seed=0)
    uu = np.einsum("snab,sncb->snac", U, U.conj())
    assert np.abs(uu - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
