"""Writes the stored expected values used by the tests.

Calls only the CPU oracle (oracle/) and the seeded input generators (synth/);
nothing here touches the HIP library.  Re-run with
    python tests/golden/make_fixtures.py [lattice_4444] [gradient_8888] [sign_16x16x16x32]
                                         [sign_16x16x16x16] [overlap_4444] [config2_8888]
(all when no name is given) after any change to the oracle's arithmetic.

lattice_4444.npz -- the 4^4 workload: links P_SU3(1 + 0.4 G) (seed 0),
    m_w = -1.5, mu = 0.3, one Gaussian source (seed 1).  Holds the exact
    sgn(A) b by the spectral definition (Section 1, eq. (1.3)-(1.4)), the 20
    critical eigentriples (Section 3: smallest |lambda|, L^dagger R = I) and
    the full spectrum's smallest |lambda| and |Re lambda|.

gradient_4444_dk.npz -- the exact (Daleckii-Krein) gradient at the 4^4
    workload, for the deflation-aware gradient.

gradient_8888_converged.npz -- references for the k = 400 gradient from the
    converged function (see gradient_8888_converged below).

gradient_8888_k150.npz, gradient_8888_k400.npz -- the gradient workload: 8^4,
    links P_SU3(1 + 0.6 G) (seed 0), m_w = -1.5, mu = 0.3, one Gaussian
    source b (seed 1) and cotangent chi (seed 2), two-sided Lanczos without
    deflation (Section 4) at k = 150 and k = 400.  Each holds the oracle's
    reverse-sweep gradient of L = Re <chi, y_k> (256 sampled entries of y and
    grad_b, 64 sampled links of grad_U, grad_mu, full norms, directional
    derivatives), central finite differences of the oracle's forward y_k in
    three directions (mu, a random link direction E, a random source
    direction db; synth.complex_normal seeds 3 and 4), and the rounding noise
    of the forward: L(mu +- 1e-13) - L(mu).  At k = 400 that noise is ~1e-5
    (biorthogonality is lost), so its differences are central ones at
    h = 1e-3; at k = 150 it is ~1e-12 and the differences are Richardson
    extrapolations (4 D(h/2) - D(h))/3 of central ones at h = 1e-5.

sign_16x16x16x32.npz -- the benchmark workload: 16^3 x 32, links
    P_SU3(1 + 0.6 G) (seed 0), m_w = -1.5, mu = 0.4, the first four of the 12
    Gaussian sources (seed 1).  The oracle's two-sided Lanczos (CSR, FP64,
    two-pass, no deflation) at k = 650 and k = 700 for each source: 16384
    sampled entries of y (fixed positions, default_rng(7)) and the full
    norms; their difference bounds the reference's own error.  The k = 650
    values come from the k = 700 run's first 650 coefficients (the same
    numbers a k = 650 run produces).

config2_8888.npz -- the 8^4 configuration of the Lanczos/Arnoldi comparison:
    links P_SU3(1 + 0.6 G) (seed 0), m_w = -1.5, one Gaussian source (seed 1),
    mu in {0, 0.1, 0.3, 0.5}.  Per mu: the 34 eigenvalues of smallest
    magnitude with their eigentriples' residuals and biorthogonality
    (eigtrip.sparse_eigentriples, the shift-invert route of Section 5); the
    LR-deflated (m = 30, Section 3) two-sided Lanczos (Section 4) and Arnoldi
    (Section 2) results at k = 200, 400 and 800 (4096 sampled entries,
    default_rng(7)) and their relative errors against the reference, the
    deflated two-sided Lanczos at k = 1600 (two-pass), whose own uncertainty
    is its difference from the Arnoldi result at k = 800.  At mu = 0.3 also
    the undeflated Lanczos coefficients to k = 800 and sgn(G_k) e_1 at k = 400
    and 800 by the spectral definition (with the eigenvector condition number
    and the smallest |Re| of the Ritz values).

overlap_4444.npz -- the spectrum of the overlap operator D_ov(mu) = 1 +
    gamma5 sgn(A) (Section 1) on the 4^4 lattice of lattice_4444.npz (links
    P_SU3(1 + 0.4 G), seed 0; m_w = -1.5) at mu = 0 and mu = 0.3: all 3072
    eigenvalues of the dense operator (oracle.overlap), ordered by magnitude.

sign_16x16x16x16.npz -- the 16^4 configuration: links P_SU3(1 + 0.6 G)
    (seed 0), m_w = -1.5, mu = 0.2, point sources 0 and 1 (spin-colour 0 and
    1 at the origin).  As above at k = 550 and k = 600; the sampled entries are
    4096 random ones plus every entry of the 5^4 sites around the origin, where
    the result is concentrated.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import dirac, eigtrip, grad, krylov, overlap, sign  # noqa: E402


def lattice_4444():
    dims = (4, 4, 4, 4)
    m_w, mu, eps = -1.5, 0.3, 0.4
    U = synth.random_links(dims, eps, seed=synth.LINK_SEED)
    b = synth.gaussian_sources(dims, 1, seed=synth.SOURCE_SEED)[0]
    A = dirac.dense_A(dims, U, m_w, mu)
    lam, R = np.linalg.eig(A)
    s = sign.csgn(lam)
    y = R @ (s * np.linalg.solve(R, b))
    Lfull = np.linalg.inv(R).conj().T
    idx = np.lexsort((lam.imag, lam.real, np.abs(lam)))[:20]
    np.savez_compressed(
        os.path.join(HERE, "lattice_4444.npz"),
        dims=np.array(dims), m_w=m_w, mu=mu, eps=eps,
        y=y, lam=lam[idx], R=R[:, idx], L=Lfull[:, idx],
        min_abs_lam=np.abs(lam).min(), min_abs_re=np.abs(lam.real).min(),
        cond_R=np.linalg.cond(R),
    )


def gradient_8888_at(k, h, richardson):
    dims = (8, 8, 8, 8)
    m_w, mu, eps = -1.5, 0.3, 0.6
    U = synth.random_links(dims, eps, seed=synth.LINK_SEED)
    b = synth.gaussian_sources(dims, 1, seed=synth.SOURCE_SEED)[0]
    chi = synth.gaussian_sources(dims, 1, seed=synth.COTANGENT_SEED)[0]
    y, gb, gmu, gU, _ = grad.tsl_vjp(dims, U, m_w, mu, b, chi, k)
    E = synth.complex_normal(U.shape, 3)
    db = synth.complex_normal(b.shape, 4)

    def loss(UU, mm, bb):
        A = dirac.csr_A(dims, UU, m_w, mm)
        Ad = dirac.csr_A(dims, UU, m_w, -mm)
        yy = krylov.tsl_apply(lambda z: A @ z, lambda z: Ad @ z, bb, k)
        return float(np.real(np.vdot(chi, yy)))

    L0 = loss(U, mu, b)
    noise = max(abs(loss(U, mu + 1e-13, b) - L0), abs(loss(U, mu - 1e-13, b) - L0))
    def central(f, hh):
        return (f(hh) - f(-hh)) / (2 * hh)

    def diff(f):
        if not richardson:
            return central(f, h)
        # (4 D(h/2) - D(h)) / 3 cancels the h^2 term of the central difference
        return (4.0 * central(f, h / 2) - central(f, h)) / 3.0

    fd_mu = diff(lambda t: loss(U, mu + t, b))
    fd_U = diff(lambda t: loss(U + t * E, mu, b))
    fd_b = diff(lambda t: loss(U, mu, b + t * db))
    rng = np.random.default_rng(5)
    V = int(np.prod(dims))
    idx_b = np.sort(rng.choice(12 * V, 256, replace=False))
    idx_U = np.sort(rng.choice(4 * V, 64, replace=False))
    np.savez_compressed(
        os.path.join(HERE, f"gradient_8888_k{k}.npz"),
        dims=np.array(dims), m_w=m_w, mu=mu, eps=eps, k=k, h=h, richardson=richardson,
        loss=float(np.real(np.vdot(chi, y))), noise=noise,
        idx_b=idx_b, idx_U=idx_U,
        y_samp=y[idx_b], grad_b_samp=gb[idx_b], grad_U_samp=gU.reshape(4 * V, 9)[idx_U],
        grad_mu=gmu, norm_y=np.linalg.norm(y), norm_grad_b=np.linalg.norm(gb),
        norm_grad_U=np.linalg.norm(gU),
        vjp_dir_U=float(np.real(np.vdot(gU, E))), vjp_dir_b=float(np.real(np.vdot(gb, db))),
        fd_mu=fd_mu, fd_U=fd_U, fd_b=fd_b,
    )


def gradient_8888_converged():
    """References for the k = 400 gradient that its rounding noise cannot
    swamp: the converged function L(mu, U, b) = Re <chi, sgn(A) b> (the
    oracle's 2sL at k = 800, whose y changes by ~7e-12 from k = 800 to 1200,
    against 5e-8 at k = 400), its central differences in mu and along the
    link direction E (Richardson-extrapolated from h = 2e-4 and 1e-4), and
    sgn(A(-mu)) chi = sgn(A)^dagger chi, the b-gradient of the exact function
    (Section 1: A(mu)^dagger = A(-mu)), by the oracle's 2sL at k = 800."""
    dims = (8, 8, 8, 8)
    m_w, mu, eps, kref = -1.5, 0.3, 0.6, 800
    U = synth.random_links(dims, eps, seed=synth.LINK_SEED)
    b = synth.gaussian_sources(dims, 1, seed=synth.SOURCE_SEED)[0]
    chi = synth.gaussian_sources(dims, 1, seed=synth.COTANGENT_SEED)[0]
    E = synth.complex_normal(U.shape, 3)
    db = synth.complex_normal(b.shape, 4)

    def sign_apply(UU, mm, bb):
        A = dirac.csr_A(dims, UU, m_w, mm)
        Ad = dirac.csr_A(dims, UU, m_w, -mm)
        return krylov.tsl_apply(lambda z: A @ z, lambda z: Ad @ z, bb, kref, two_pass=True)

    def loss(UU, mm):
        return float(np.real(np.vdot(chi, sign_apply(UU, mm, b))))

    def richardson(f, h):
        c1 = (f(h) - f(-h)) / (2 * h)
        c2 = (f(h / 2) - f(-h / 2)) / h
        return (4.0 * c2 - c1) / 3.0, c1, c2

    L0 = loss(U, mu)
    fd_mu, fd_mu_h, fd_mu_h2 = richardson(lambda t: loss(U, mu + t), 2e-4)
    fd_U, fd_U_h, fd_U_h2 = richardson(lambda t: loss(U + t * E, mu), 2e-4)
    gb = sign_apply(U, -mu, chi)   # sgn(A(-mu)) chi
    f400 = np.load(os.path.join(HERE, "gradient_8888_k400.npz"))
    idx_b = f400["idx_b"]
    np.savez_compressed(
        os.path.join(HERE, "gradient_8888_converged.npz"),
        dims=np.array(dims), m_w=m_w, mu=mu, eps=eps, kref=kref, loss=L0,
        fd_mu=fd_mu, fd_mu_h=fd_mu_h, fd_mu_h2=fd_mu_h2, fd_U=fd_U, fd_U_h=fd_U_h,
        fd_U_h2=fd_U_h2, idx_b=idx_b, grad_b_samp=gb[idx_b], norm_grad_b=np.linalg.norm(gb),
        dir_b=float(np.real(np.vdot(gb, db))),
    )
    print("converged L", L0, "dL/dmu", fd_mu, fd_mu_h, fd_mu_h2, "dL/dE", fd_U, fd_U_h, fd_U_h2)


def gradient_4444_dk():
    """The exact derivative (Daleckii-Krein, on the full eigendecomposition) of
    L = Re <chi, sgn(A) b> at the 4^4 workload of lattice_4444.npz (links
    P_SU3(1 + 0.4 G) seed 0, m_w = -1.5, mu = 0.3, b seed 1, chi seed 2):
    grad_b (= sgn(A(-mu)) chi), dL/dmu and the link gradient.  The reference
    of the deflation-aware gradient (20 deflated eigentriples)."""
    dims = (4, 4, 4, 4)
    m_w, mu, eps = -1.5, 0.3, 0.4
    U = synth.random_links(dims, eps, seed=synth.LINK_SEED)
    b = synth.gaussian_sources(dims, 1, seed=synth.SOURCE_SEED)[0]
    chi = synth.gaussian_sources(dims, 1, seed=synth.COTANGENT_SEED)[0]
    gb, gmu, gU = grad.dk_gradient(dims, U, m_w, mu, b, chi)
    np.savez_compressed(os.path.join(HERE, "gradient_4444_dk.npz"), dims=np.array(dims), m_w=m_w,
                        mu=mu, eps=eps, grad_b=gb, grad_mu=gmu, grad_U=gU)


def gradient_8888():
    gradient_8888_at(150, 1e-5, True)
    gradient_8888_at(400, 1e-3, False)


def _sign16_source(r):
    """One source of the 16^3 x 32 fixture: the oracle's two-sided Lanczos to
    k = 700 (coefficients only), the inner sign of the leading 650 x 650 and
    the full 700 x 700 tridiagonal matrix, and one replay sweep for each
    (the steps of krylov.tsl_apply with two_pass, both k from one first pass:
    the first 650 coefficients of the k = 700 run are those of a k = 650 run)."""
    dims = (16, 16, 16, 32)
    m_w, mu, eps = -1.5, 0.4, 0.6
    U = synth.random_links(dims, eps, seed=synth.LINK_SEED)
    b = synth.gaussian_sources(dims, 12, seed=synth.SOURCE_SEED)[r]
    A = dirac.csr_A(dims, U, m_w, mu)
    Ad = dirac.csr_A(dims, U, m_w, -mu)
    del U
    lr = krylov.two_sided_lanczos(lambda z: A @ z, lambda z: Ad @ z, b, b, 700, store=False)
    assert lr.k == 700 and lr.status != "serious", (lr.k, lr.status)
    ys = {}
    for k in (650, 700):
        x = np.zeros(700, dtype=np.complex128)
        x[:k] = sign.sign_e1(krylov.tridiag(lr.alpha[:k], lr.beta[:k - 1], lr.gamma[:k - 1]))
        ys[k] = lr.n_b * krylov.replay_combine(lambda z: A @ z, b / lr.n_b, lr, x)
        print("source", r, "k", k, "norm", np.linalg.norm(ys[k]), flush=True)
    return ys


def sign_16x16x16x32():
    from concurrent.futures import ProcessPoolExecutor
    dims = (16, 16, 16, 32)
    N = synth.volume(dims) * 12
    idx = np.sort(np.random.default_rng(7).choice(N, 16384, replace=False))
    out = {"dims": np.array(dims), "m_w": -1.5, "mu": 0.4, "eps": 0.6, "idx": idx,
           "ks": np.array([650, 700]), "sources": np.arange(4)}
    with ProcessPoolExecutor(4) as ex:
        res = list(ex.map(_sign16_source, range(4)))
    for r, ys in enumerate(res):
        for k in (650, 700):
            out[f"y{r}_k{k}"] = ys[k][idx]
            out[f"norm{r}_k{k}"] = np.linalg.norm(ys[k])
        out[f"ydiff{r}"] = np.linalg.norm(ys[700][idx] - ys[650][idx]) / np.linalg.norm(ys[700][idx])
    np.savez_compressed(os.path.join(HERE, "sign_16x16x16x32.npz"), **out)


def _sign16_4_source(r):
    """Point source r (spin-colour r at the origin) of the 16^4 configuration:
    the oracle's two-sided Lanczos to k = 600 (coefficients only) and replays
    for k = 550 and 600, as in _sign16_source."""
    dims = (16, 16, 16, 16)
    m_w, mu, eps = -1.5, 0.2, 0.6
    U = synth.random_links(dims, eps, seed=synth.LINK_SEED)
    b = synth.point_sources(dims)[r]
    A = dirac.csr_A(dims, U, m_w, mu)
    Ad = dirac.csr_A(dims, U, m_w, -mu)
    del U
    lr = krylov.two_sided_lanczos(lambda z: A @ z, lambda z: Ad @ z, b, b, 600, store=False)
    assert lr.k == 600 and lr.status != "serious", (lr.k, lr.status)
    ys = {}
    for k in (550, 600):
        x = np.zeros(600, dtype=np.complex128)
        x[:k] = sign.sign_e1(krylov.tridiag(lr.alpha[:k], lr.beta[:k - 1], lr.gamma[:k - 1]))
        ys[k] = lr.n_b * krylov.replay_combine(lambda z: A @ z, b / lr.n_b, lr, x)
        print("16^4 source", r, "k", k, "norm", np.linalg.norm(ys[k]), flush=True)
    return ys


def _near_origin(dims, half):
    """Vector indices (12 s + spin-colour) of the sites whose every coordinate
    lies within +-half of the origin (periodic): where a point source's
    sgn(A) e_j is concentrated."""
    lx, ly, lz, lt = dims
    rng = range(-half, half + 1)
    sites = sorted({(x % lx) + lx * ((y % ly) + ly * ((z % lz) + lz * (t % lt)))
                    for x in rng for y in rng for z in rng for t in rng})
    return np.array([12 * s + c for s in sites for c in range(12)])


def sign_16x16x16x16():
    from concurrent.futures import ProcessPoolExecutor
    dims = (16, 16, 16, 16)
    N = synth.volume(dims) * 12
    rnd = np.random.default_rng(7).choice(N, 4096, replace=False)
    idx = np.unique(np.concatenate([rnd, _near_origin(dims, 2)]))
    out = {"dims": np.array(dims), "m_w": -1.5, "mu": 0.2, "eps": 0.6, "idx": idx,
           "ks": np.array([550, 600]), "sources": np.array([0, 1])}
    with ProcessPoolExecutor(2) as ex:
        res = list(ex.map(_sign16_4_source, (0, 1)))
    for r, ys in enumerate(res):
        for k in (550, 600):
            out[f"y{r}_k{k}"] = ys[k][idx]
            out[f"norm{r}_k{k}"] = np.linalg.norm(ys[k])
        out[f"ydiff{r}"] = np.linalg.norm(ys[600][idx] - ys[550][idx]) / np.linalg.norm(ys[600][idx])
    np.savez_compressed(os.path.join(HERE, "sign_16x16x16x16.npz"), **out)


def _config2_mu(mu):
    dims = (8, 8, 8, 8)
    m_w, eps, m = -1.5, 0.6, 30
    U = synth.random_links(dims, eps, seed=synth.LINK_SEED)
    b = synth.gaussian_sources(dims, 1, seed=synth.SOURCE_SEED)[0]
    A = dirac.csr_A(dims, U, m_w, mu)
    Ad = dirac.csr_A(dims, U, m_w, -mu)
    del U
    N = A.shape[0]
    idx = np.sort(np.random.default_rng(7).choice(N, 4096, replace=False))
    lam, R, L = eigtrip.sparse_eigentriples(A, m + 4)
    res_r = np.linalg.norm(A @ R - R * lam[None, :], axis=0) / np.abs(lam)
    res_l = np.linalg.norm(Ad @ L - L * np.conj(lam)[None, :], axis=0) / np.abs(lam)
    res_l = res_l / np.linalg.norm(L, axis=0)
    biorth = np.abs(L[:, :m].conj().T @ R[:, :m] - np.eye(m)).max()
    print("mu", mu, "eigentriples", lam[:3], "res", res_r.max(), res_l.max(), biorth, flush=True)
    defl = (lam[:m], R[:, :m], L[:, :m])
    mv = lambda z: A @ z  # noqa: E731
    rmv = lambda z: Ad @ z  # noqa: E731
    yref = krylov.tsl_apply(mv, rmv, b, 1600, defl=defl, two_pass=True)
    out = {f"lam_mu{mu}": lam, f"res_r_mu{mu}": res_r, f"res_l_mu{mu}": res_l,
           f"biorth_mu{mu}": biorth, f"yref_mu{mu}": yref[idx], f"normref_mu{mu}": np.linalg.norm(yref)}
    for k in (200, 400, 800):
        y2 = krylov.tsl_apply(mv, rmv, b, k, defl=defl, two_pass=True)
        ya = krylov.arnoldi_apply(mv, b, k, defl=defl)
        out[f"y2sl_k{k}_mu{mu}"] = y2[idx]
        out[f"yarn_k{k}_mu{mu}"] = ya[idx]
        out[f"e2sl_k{k}_mu{mu}"] = np.linalg.norm(y2 - yref) / np.linalg.norm(yref)
        out[f"earn_k{k}_mu{mu}"] = np.linalg.norm(ya - yref) / np.linalg.norm(yref)
        print("mu", mu, "k", k, out[f"e2sl_k{k}_mu{mu}"], out[f"earn_k{k}_mu{mu}"], flush=True)
        if k == 800:
            out[f"refunc_mu{mu}"] = np.linalg.norm(ya - yref) / np.linalg.norm(yref)
    if mu == 0.3:
        lr = krylov.two_sided_lanczos(mv, rmv, b, b, 800, store=False)
        assert lr.k == 800 and lr.status == "ok", (lr.k, lr.status)
        out["g_alpha"], out["g_beta"], out["g_gamma"] = lr.alpha, lr.beta, lr.gamma
        for k in (400, 800):
            G = krylov.tridiag(lr.alpha[:k], lr.beta[:k - 1], lr.gamma[:k - 1])
            ev, vecs = np.linalg.eig(G)
            out[f"g_x{k}"] = sign.sign_e1(G)
            out[f"g_cond{k}"] = np.linalg.cond(vecs)
            out[f"g_minre{k}"] = np.abs(ev.real).min()
            out[f"g_minangle{k}"] = np.min(np.abs(np.arctan2(ev.real, np.abs(ev.imag))))
    return out


def config2_8888():
    from concurrent.futures import ProcessPoolExecutor
    out = {"dims": np.array((8, 8, 8, 8)), "m_w": -1.5, "eps": 0.6, "m": 30,
           "mus": np.array([0.0, 0.1, 0.3, 0.5]), "ks": np.array([200, 400, 800]),
           "idx": np.sort(np.random.default_rng(7).choice(12 * 8 ** 4, 4096, replace=False))}
    with ProcessPoolExecutor(4) as ex:
        for res in ex.map(_config2_mu, (0.0, 0.1, 0.3, 0.5)):
            out.update(res)
    np.savez_compressed(os.path.join(HERE, "config2_8888.npz"), **out)


def overlap_4444():
    dims = (4, 4, 4, 4)
    m_w, eps = -1.5, 0.4
    U = synth.random_links(dims, eps, seed=synth.LINK_SEED)
    out = {"dims": np.array(dims), "m_w": m_w, "eps": eps}
    for key, mu in (("lam_mu0", 0.0), ("lam_mu03", 0.3)):
        out[key] = overlap.overlap_eigenvalues(dims, U, m_w, mu)
    np.savez_compressed(os.path.join(HERE, "overlap_4444.npz"), **out)


if __name__ == "__main__":
    names = sys.argv[1:] or ["lattice_4444", "gradient_8888", "sign_16x16x16x32",
                             "sign_16x16x16x16", "overlap_4444", "config2_8888"]
    for name in names:
        if name == "gradient_8888_k150":
            gradient_8888_at(150, 1e-5, True)
        elif name == "gradient_8888_k400":
            gradient_8888_at(400, 1e-3, False)
        else:
            globals()[name]()
        print("written", name)
