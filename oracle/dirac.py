"""Wilson-Dirac operator at chemical potential, assembled literally.

Section 1 (eq. for Dw(mu) and the definition of the hopping matrices):
    Dw(mu) = 1 - kappa * sum_{i=1..3} (T_i^+ + T_i^-)
               - kappa * (e^{mu} T_4^+ + e^{-mu} T_4^-)
    (T_nu^{+-})_{yx} = (1 +- gamma_nu) U_{x,+-nu} delta_{y, x +- nu}
    kappa = 1/(8 + 2 m_w)
and the argument of the sign function is A = gamma5 * Dw(mu).

Readings where the text is silent:
  * U_{x,-nu} = U_{x-nu,nu}^dagger (gauge covariant choice).
  * Euclidean chiral gamma basis:  gamma_k = [[0, -i s_k], [i s_k, 0]],
    gamma_4 = [[0, 1], [1, 0]], gamma5 = gamma_1 gamma_2 gamma_3 gamma_4.
  * Periodic space, antiperiodic time: the time link leaving the last
    time slice carries a factor -1 in both hop directions.
  * Site index s = x + Lx*(y + Ly*(z + Lz*t)); vector index 12*s + 3*spin + colour.

TEST INFRASTRUCTURE: only tests, smoke and the CPU baseline use this module.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


def gamma_matrices():
    """gamma_1..gamma_4 (Euclidean, chiral basis) and gamma5 = g1 g2 g3 g4 (Section 1)."""
    z = np.zeros((2, 2), dtype=np.complex128)
    one = np.eye(2, dtype=np.complex128)
    gam = []
    for s in SIGMA:
        gam.append(np.block([[z, -1j * s], [1j * s, z]]))
    gam.append(np.block([[z, one], [one, z]]))
    g5 = gam[0] @ gam[1] @ gam[2] @ gam[3]
    return gam, g5


def kappa_of(m_w: float) -> float:
    """kappa = 1/(8 + 2 m_w) (Section 1)."""
    return 1.0 / (8.0 + 2.0 * m_w)


def coords(dims, s):
    lx, ly, lz, _ = dims
    x = s % lx
    y = (s // lx) % ly
    z = (s // (lx * ly)) % lz
    t = s // (lx * ly * lz)
    return x, y, z, t


def site_of(dims, x, y, z, t):
    lx, ly, lz, lt = dims
    return (x % lx) + lx * ((y % ly) + ly * ((z % lz) + lz * (t % lt)))


def forward(dims, s, nu):
    """Site s + nu_hat (periodic wrap of the index)."""
    c = list(coords(dims, s))
    c[nu] = c[nu] + 1
    return site_of(dims, *c)


def boundary_sign(dims, s, nu, bc):
    """Sign carried by link (s, nu): bc[nu] if the link wraps around the lattice."""
    c = coords(dims, s)
    return bc[nu] if c[nu] == dims[nu] - 1 else 1.0


def hop_factors(mu: float):
    """eta_nu^{+-}: 1 on space hops, e^{+-mu} on time hops (Section 1)."""
    eta_p = np.array([1.0, 1.0, 1.0, np.exp(mu)])
    eta_m = np.array([1.0, 1.0, 1.0, np.exp(-mu)])
    return eta_p, eta_m


DEFAULT_BC = (1.0, 1.0, 1.0, -1.0)


def dense_dw(dims, U, m_w, mu, bc=DEFAULT_BC) -> np.ndarray:
    """Dense Dw(mu), N x N, assembled hop by hop (Section 1).

    Uses '+=' so lattices with extent 2 (forward and backward neighbour are
    the same site) are assembled correctly."""
    dims = tuple(int(d) for d in dims)
    v = int(np.prod(dims))
    n = 12 * v
    gam, _ = gamma_matrices()
    kap = kappa_of(m_w)
    eta_p, eta_m = hop_factors(mu)
    one4 = np.eye(4, dtype=np.complex128)
    d = np.eye(n, dtype=np.complex128)
    for s in range(v):
        for nu in range(4):
            sp_ = forward(dims, s, nu)
            b = boundary_sign(dims, s, nu, bc)
            u = U[s, nu]
            # T^+ : field at x = s arrives at y = s + nu with (1 + gamma) U_{s,nu}
            d[12 * sp_:12 * sp_ + 12, 12 * s:12 * s + 12] += (
                -kap * eta_p[nu] * b * np.kron(one4 + gam[nu], u))
            # T^- : field at x = s + nu arrives at y = s with (1 - gamma) U_{s+nu,-nu}
            #       and U_{s+nu,-nu} = U_{s,nu}^dagger
            d[12 * s:12 * s + 12, 12 * sp_:12 * sp_ + 12] += (
                -kap * eta_m[nu] * b * np.kron(one4 - gam[nu], u.conj().T))
    return d


def gamma5_rows(n_sites: int) -> np.ndarray:
    """Diagonal of gamma5 (x) 1_colour over the whole lattice, length 12V."""
    _, g5 = gamma_matrices()
    diag = np.real(np.diag(g5))
    return np.tile(np.repeat(diag, 3), n_sites)


def dense_A(dims, U, m_w, mu, bc=DEFAULT_BC) -> np.ndarray:
    """A = gamma5 Dw(mu), dense (argument of the sign function in eq. (1.1))."""
    _, g5 = gamma_matrices()
    v = int(np.prod(dims))
    g5full = np.kron(np.eye(v), np.kron(g5, np.eye(3)))
    return g5full @ dense_dw(dims, U, m_w, mu, bc)


def csr_dw(dims, U, m_w, mu, bc=DEFAULT_BC) -> sp.csr_matrix:
    """Sparse Dw(mu) in CSR, same hop formula as dense_dw, vectorised over sites."""
    dims = tuple(int(d) for d in dims)
    v = int(np.prod(dims))
    n = 12 * v
    gam, _ = gamma_matrices()
    kap = kappa_of(m_w)
    eta_p, eta_m = hop_factors(mu)
    one4 = np.eye(4, dtype=np.complex128)
    s_all = np.arange(v)
    cx, cy, cz, ct = coords(dims, s_all)
    cc = [cx, cy, cz, ct]
    loc_r, loc_c = np.meshgrid(np.arange(12), np.arange(12), indexing="ij")
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.ones(n, dtype=np.complex128)]
    for nu in range(4):
        c2 = list(cc)
        c2[nu] = cc[nu] + 1
        sp_ = site_of(dims, *c2)
        bsign = np.where(cc[nu] == dims[nu] - 1, bc[nu], 1.0)
        u = U[:, nu]
        # forward hop block per site: (12,12) = kron(1+g, U_s)
        blk_f = np.einsum("ij,sab->siajb", one4 + gam[nu], u).reshape(v, 12, 12)
        blk_f = blk_f * (-kap * eta_p[nu] * bsign)[:, None, None]
        rows.append((12 * sp_[:, None, None] + loc_r[None]).ravel())
        cols.append((12 * s_all[:, None, None] + loc_c[None]).ravel())
        vals.append(blk_f.ravel())
        udag = np.conj(np.swapaxes(u, -1, -2))
        blk_b = np.einsum("ij,sab->siajb", one4 - gam[nu], udag).reshape(v, 12, 12)
        blk_b = blk_b * (-kap * eta_m[nu] * bsign)[:, None, None]
        rows.append((12 * s_all[:, None, None] + loc_r[None]).ravel())
        cols.append((12 * sp_[:, None, None] + loc_c[None]).ravel())
        vals.append(blk_b.ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    x = np.concatenate(vals)
    keep = x != 0
    m = sp.coo_matrix((x[keep], (r[keep], c[keep])), shape=(n, n)).tocsr()
    m.sum_duplicates()
    return m


def csr_A(dims, U, m_w, mu, bc=DEFAULT_BC) -> sp.csr_matrix:
    """A = gamma5 Dw(mu) in CSR."""
    v = int(np.prod(dims))
    g5 = sp.diags(gamma5_rows(v).astype(np.complex128))
    return (g5 @ csr_dw(dims, U, m_w, mu, bc)).tocsr()


def apply_at_sites(dims, U, m_w, mu, x, sites, op="A", bc=DEFAULT_BC) -> np.ndarray:
    """Evaluate (op x) at the listed sites only, from the hop formula.

    op in {"Dw", "A"}.  x: complex [12V].  Returns complex [len(sites), 12].
    Adjoint operators are obtained by the caller via the literal conjugate
    transpose of csr_dw/csr_A; this routine is for sampled checks of the
    forward operator on lattices too large for a full matrix."""
    dims = tuple(int(d) for d in dims)
    gam, g5 = gamma_matrices()
    kap = kappa_of(m_w)
    eta_p, eta_m = hop_factors(mu)
    one4 = np.eye(4, dtype=np.complex128)
    xs = x.reshape(-1, 4, 3)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for k, s in enumerate(sites):
        acc = xs[s].copy()
        c = list(coords(dims, s))
        for nu in range(4):
            cb = list(c)
            cb[nu] -= 1
            sb = site_of(dims, *cb)          # s - nu
            sf = forward(dims, s, nu)        # s + nu
            bb = boundary_sign(dims, sb, nu, bc)
            bf = boundary_sign(dims, s, nu, bc)
            acc -= kap * eta_p[nu] * bb * ((one4 + gam[nu]) @ xs[sb] @ U[sb, nu].T)
            acc -= kap * eta_m[nu] * bf * ((one4 - gam[nu]) @ xs[sf] @ U[s, nu].conj())
        if op == "A":
            acc = g5 @ acc
        out[k] = acc
    return out.reshape(len(sites), 12)
