"""Pins of the oracle's Krylov methods (Sections 2-4): polynomial exactness
(Section 2, eq. (2.0)), the biorthogonality and tridiagonal structure of
Section 4, orthonormality of Arnoldi, the Hermitian mu = 0 reduction, exact
deflation identities, breakdown cases, two-pass equivalence and convergence
to the dense spectral sign."""
import numpy as np
import pytest

import synth
from oracle import dirac, eigtrip, krylov, sign

MW = -1.5


@pytest.fixture(scope="module")
def small():
    dims = (2, 2, 4, 4)
    U = synth.random_links(dims, 0.5, seed=31)
    A = dirac.csr_A(dims, U, MW, 0.3)
    Ad = A.conj().T.tocsr()
    b = synth.gaussian_sources(dims, 1, seed=32)[0]
    dense = A.toarray()
    return dims, U, A, Ad, b, dense


def power_inner(j):
    def f(g):
        e1 = np.zeros(g.shape[0], dtype=np.complex128)
        e1[0] = 1.0
        return np.linalg.matrix_power(g, j) @ e1
    return f


@pytest.mark.parametrize("j", [0, 1, 3, 7])
def test_polynomial_exactness_tsl(small, j):
    """With f(z) = z^j, j < k: |b| V_k G_k^j e_1 = A^j b."""
    _, _, A, Ad, b, dense = small
    y = krylov.tsl_apply(lambda x: A @ x, lambda x: Ad @ x, b, 12, inner=power_inner(j),
                         f_scalar=lambda z: z ** j)
    ref = np.linalg.matrix_power(dense, j) @ b
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-11


@pytest.mark.parametrize("j", [1, 4])
def test_polynomial_exactness_arnoldi(small, j):
    _, _, A, _, b, dense = small
    y = krylov.arnoldi_apply(lambda x: A @ x, b, 10, inner=power_inner(j), f_scalar=lambda z: z ** j)
    ref = np.linalg.matrix_power(dense, j) @ b
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-11


def test_biorthogonal_tridiagonal(small):
    _, _, A, Ad, b, dense = small
    lr = krylov.two_sided_lanczos(lambda x: A @ x, lambda x: Ad @ x, b, b, 15)
    V = np.array(lr.V).T
    W = np.array(lr.W).T
    assert np.abs(W.conj().T @ V - np.eye(15)).max() < 1e-10
    G = W.conj().T @ dense @ V
    assert np.abs(G - krylov.tridiag(lr.alpha, lr.beta, lr.gamma)).max() < 1e-10
    # A V_k = V_k G_k + beta_k v_{k+1} e_k^T : residual lives in the last column only
    Gt = krylov.tridiag(lr.alpha, lr.beta, lr.gamma)
    R = dense @ V - V @ Gt
    assert np.abs(R[:, :-1]).max() < 1e-10
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0)


def test_arnoldi_orthonormal(small):
    _, _, A, _, b, dense = small
    ar = krylov.arnoldi(lambda x: A @ x, b, 20)
    V = np.array(ar.V).T
    assert np.abs(V.conj().T @ V - np.eye(20)).max() < 1e-12
    assert np.abs(V.conj().T @ dense @ V - ar.H).max() < 1e-12
    assert np.abs(np.tril(ar.H, -2)).max() == 0.0


def test_mu_zero_is_hermitian_lanczos():
    dims = (2, 2, 4, 4)
    U = synth.random_links(dims, 0.5, seed=33)
    A = dirac.csr_A(dims, U, MW, 0.0)
    b = synth.gaussian_sources(dims, 1, seed=34)[0]
    lr = krylov.two_sided_lanczos(lambda x: A @ x, lambda x: A.conj().T @ x, b, b, 12)
    assert np.abs(np.array(lr.V) - np.array(lr.W)).max() < 1e-12
    assert np.abs(lr.alpha.imag).max() < 1e-12
    assert np.abs(lr.beta - lr.gamma).max() < 1e-12
    # Arnoldi on Hermitian A gives the same tridiagonal matrix
    ar = krylov.arnoldi(lambda x: A @ x, b, 12)
    assert np.abs(ar.H - krylov.tridiag(lr.alpha, lr.beta, lr.gamma)).max() < 1e-10


@pytest.fixture(scope="module")
def dense_eig(small):
    _, _, _, _, b, dense = small
    lam, R = np.linalg.eig(dense)
    return lam, R


def test_deflation_identity_exact(small, dense_eig):
    """sgn(A) b = R_m sgn(Lambda_m) L_m^dagger b + sgn(A) b_R exactly (Section 3)."""
    _, _, A, _, b, dense = small
    lam, R, L = eigtrip.dense_eigentriples(dense, 10)
    assert np.abs(L.conj().T @ R - np.eye(10)).max() < 1e-10
    d = krylov.deflate(b, lam, R, L)
    lhs = sign.sign_eig_apply(dense, b)
    rhs = d.y_ex + sign.sign_eig_apply(dense, d.b_R)
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(lhs) < 1e-11
    # the left-deflated source is free of the right eigen-directions: R^dagger b_L = 0
    assert np.abs(R.conj().T @ d.b_L).max() < 1e-11
    assert np.abs(L.conj().T @ d.b_R).max() < 1e-11


def test_source_in_deflation_space(small):
    _, _, A, Ad, _, dense = small
    lam, R, L = eigtrip.dense_eigentriples(dense, 6)
    b = R @ np.arange(1, 7).astype(np.complex128)
    y, info = krylov.tsl_apply(lambda x: A @ x, lambda x: Ad @ x, b, 20, defl=(lam, R, L),
                               return_info=True)
    assert np.linalg.norm(info["deflated"].b_R) < 1e-12 * np.linalg.norm(b)
    ref = sign.sign_eig_apply(dense, b)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-10


def test_lucky_breakdown_eigenvector(small, dense_eig):
    _, _, A, Ad, _, dense = small
    lam, R = dense_eig
    j = int(np.argmax(np.abs(lam)))
    r = R[:, j]
    # left eigenvector for the same eigenvalue
    lam_l, Lv = np.linalg.eig(dense.conj().T)
    jl = int(np.argmin(np.abs(lam_l - np.conj(lam[j]))))
    y, info = krylov.tsl_apply(lambda x: A @ x, lambda x: Ad @ x, r, 30, return_info=True)
    assert info["lanczos"].status == "lucky"
    assert info["lanczos"].k == 1
    assert np.abs(y - np.sign(lam[j].real) * r).max() < 1e-12
    _ = Lv[:, jl]


def test_two_pass_equals_one_pass(small, dense_eig):
    _, _, A, Ad, b, dense = small
    lam, R, L = eigtrip.dense_eigentriples(dense, 8)
    y1 = krylov.tsl_apply(lambda x: A @ x, lambda x: Ad @ x, b, 60, defl=(lam, R, L))
    y2 = krylov.tsl_apply(lambda x: A @ x, lambda x: Ad @ x, b, 60, defl=(lam, R, L), two_pass=True)
    assert np.linalg.norm(y1 - y2) / np.linalg.norm(y1) < 1e-13


def test_convergence_to_dense(small, dense_eig):
    """Both methods approach sgn(A) b; deflation helps; Arnoldi needs fewer steps."""
    _, _, A, Ad, b, dense = small
    ref = sign.sign_eig_apply(dense, b)
    lam, R, L = eigtrip.dense_eigentriples(dense, 16)
    errs = {}
    for k in (40, 120, 400):
        for m, d in ((0, None), (16, (lam, R, L))):
            y = krylov.tsl_apply(lambda x: A @ x, lambda x: Ad @ x, b, k, defl=d)
            errs[("tsl", k, m)] = np.linalg.norm(y - ref) / np.linalg.norm(ref)
            y = krylov.arnoldi_apply(lambda x: A @ x, b, k, defl=d)
            errs[("arn", k, m)] = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert errs[("tsl", 400, 16)] < 1e-10
    assert errs[("arn", 400, 16)] < 1e-10
    assert errs[("tsl", 400, 16)] < errs[("tsl", 400, 0)]
    assert errs[("tsl", 120, 16)] < errs[("tsl", 40, 16)]
    assert errs[("tsl", 120, 16)] <= errs[("tsl", 120, 0)]
    assert errs[("arn", 120, 16)] <= 1.5 * errs[("tsl", 120, 16)]


def test_arnoldi_exhausts_free_field():
    """Unit links give few distinct eigenvalues: Arnoldi breaks down early and is exact."""
    from oracle import freefield
    dims = (2, 2, 2, 4)
    U = synth.unit_links(dims)
    A = dirac.csr_A(dims, U, MW, 0.3)
    b = synth.gaussian_sources(dims, 1, seed=35)[0]
    y, info = krylov.arnoldi_apply(lambda x: A @ x, b, 40, return_info=True)
    # 32 distinct eigenvalues in N = 384: k = 40 spans the whole Krylov space
    assert info["arnoldi"].k <= 40
    ref = freefield.free_sign_apply(dims, MW, 0.3, b)[0]
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-10


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_sparse_eigentriples_match_full_eigendecomposition(mu):
    """The shift-invert eigentriples (Section 5's route, used where a full
    eigendecomposition is out of reach) against numpy's full eig of the dense
    operator on a 2^3 x 4 lattice (N = 384): the same 12 eigenvalues of
    smallest magnitude, right vectors equal up to a phase, left vectors giving
    L^dagger R = I and satisfying A^dagger l = conj(lambda) l.  A planted
    wrong pairing (left vectors rolled by one) must break L^dagger R = I."""
    dims = (2, 2, 2, 4)
    U = synth.random_links(dims, 0.5, seed=7)
    A = dirac.csr_A(dims, U, MW, mu)
    Ad = dirac.csr_A(dims, U, MW, -mu)
    m = 12
    lam, R, L = eigtrip.sparse_eigentriples(A, m)
    lam_full = np.linalg.eigvals(A.toarray())
    ref = lam_full[np.lexsort((lam_full.imag, lam_full.real, np.abs(lam_full)))][:m]
    assert np.abs(lam - ref).max() <= 1e-12
    ld, Rd, _ = eigtrip.dense_eigentriples(A.toarray(), m)
    for j in range(m):
        if min(abs(lam[j] - lam[i]) for i in range(m) if i != j) > 1e-8:  # simple eigenvalue
            assert abs(abs(np.vdot(Rd[:, j], R[:, j])) - 1.0) <= 1e-10
    assert np.abs(L.conj().T @ R - np.eye(m)).max() <= 1e-10
    assert np.abs(A @ R - R * lam[None, :]).max() <= 1e-12
    assert np.abs(Ad @ L - L * np.conj(lam)[None, :]).max() <= 1e-10 * np.abs(L).max()
    bad = np.roll(L, 1, axis=1)
    assert np.abs(bad.conj().T @ R - np.eye(m)).max() > 0.5
