"""Writes the stored expected values used by the tests.

Calls only the CPU oracle (oracle/) and the seeded input generators (synth/);
nothing here touches the HIP library.  Re-run with
    python tests/golden/make_fixtures.py
after any change to the oracle's arithmetic.

lattice_4444.npz -- the 4^4 workload: links P_SU3(1 + 0.4 G) (seed 0),
    m_w = -1.5, mu = 0.3, one Gaussian source (seed 1).  Holds the exact
    sgn(A) b by the spectral definition (Section 1, eq. (1.3)-(1.4)), the 20
    critical eigentriples (Section 3: smallest |lambda|, L^dagger R = I) and
    the full spectrum's smallest |lambda| and |Re lambda|.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import dirac, sign  # noqa: E402


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


if __name__ == "__main__":
    lattice_4444()
    print("written")
