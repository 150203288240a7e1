"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input generation only: random SU(3) gauge links, Gaussian
and point sources, and random gauge transformations.  It contains none of the
method's arithmetic (no Wilson-Dirac operator, no sign function, no Krylov
step), so both the CPU oracle and the GPU path can take their inputs from
here without sharing any computation.

Layouts (canonical, shared with the C-ABI library):
  * site index      s = x + Lx*(y + Ly*(z + Lz*t))
  * gauge links     complex128 [V][4][3][3]  (direction nu = 0..3, 3 = time)
  * spinor field    complex128 [nrhs][V][4][3]  (flattened: 12*s + 3*spin + colour)

The paper's links are quenched gauge configurations (Section 1 cites quenched
4^4 studies); none are available here, so links are drawn as the SU(3)
projection of 1 + eps*G with G a complex Gaussian 3x3 matrix, which gives a
tunable roughness eps standing in for the coupling.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume",
    "su3_project",
    "random_links",
    "unit_links",
    "gaussian_sources",
    "point_sources",
    "random_gauge",
    "complex_normal",
    "LINK_SEED",
    "SOURCE_SEED",
    "COTANGENT_SEED",
]

LINK_SEED = 0
SOURCE_SEED = 1
COTANGENT_SEED = 2


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def su3_project(m: np.ndarray) -> np.ndarray:
    """Nearest SU(3) matrix: unitary polar factor divided by the principal
    cube root of its determinant.  Works on stacks [..., 3, 3]."""
    u, _, vh = np.linalg.svd(m)
    w = u @ vh
    det = np.linalg.det(w)
    phase = np.exp(-1j * np.angle(det) / 3.0)
    return w * phase[..., None, None]


def random_links(dims, eps: float, seed: int = LINK_SEED) -> np.ndarray:
    """Links U = P_SU3(1 + eps*G), G_ab = (g1 + i g2)/sqrt(2), g ~ N(0,1) i.i.d.

    Draw order is (site, nu, a, b, re/im), site index as in the module doc.
    Returns complex128 [V][4][3][3]."""
    v = volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((v, 4, 3, 3, 2))
    gc = (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)
    m = np.eye(3, dtype=np.complex128) + eps * gc
    return np.ascontiguousarray(su3_project(m))


def unit_links(dims) -> np.ndarray:
    """The free field U = 1."""
    v = volume(dims)
    u = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def gaussian_sources(dims, nrhs: int, seed: int = SOURCE_SEED) -> np.ndarray:
    """Complex Gaussian sources (g1 + i g2)/sqrt(2); complex128 [nrhs][12V]."""
    n = 12 * volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nrhs, n, 2))
    return np.ascontiguousarray((g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0))


def point_sources(dims, site: int = 0) -> np.ndarray:
    """The 12 spin-colour unit sources at one site; complex128 [12][12V]."""
    n = 12 * volume(dims)
    b = np.zeros((12, n), dtype=np.complex128)
    for j in range(12):
        b[j, 12 * site + j] = 1.0
    return b


def random_gauge(dims, seed: int) -> np.ndarray:
    """A random SU(3) matrix per site, complex128 [V][3][3]."""
    v = volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((v, 3, 3, 2))
    return np.ascontiguousarray(su3_project(g[..., 0] + 1j * g[..., 1]))


def complex_normal(shape, seed: int) -> np.ndarray:
    """(x + i y)/sqrt(2) with x, then y, drawn as whole arrays of standard
    normals from default_rng(seed): random test directions."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
