"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and shapes them into lattice fields; it holds
none of the Wilson-Dirac operator or solver arithmetic. Both the CPU oracle side and
the GPU side consume the arrays it returns.

Canonical layouts (interleaved complex128, x fastest):
  gauge field  U[mu][t][z][y][x][a][b]   mu = 0..3 <-> x, y, z, t
  fermion field psi[t][z][y][x][c][s]    c = colour 0..2, s = spin 0..3
The fermion field at one site is a 3x4 colour-by-spin matrix (Sec. 2, eq. 3).

The paper's quenched ensemble is not available; near-Haar random SU(3) links
U = exp(i*eps*H), with H traceless Hermitian and Gaussian entries, stand in for it.
"""
from __future__ import annotations

import numpy as np

LINK_SEED_BASE = 1000
SOURCE_SEED_BASE = 2000


def volume(dims) -> int:
    X, Y, Z, T = dims
    return X * Y * Z * T


def _gaussian_complex(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def random_hermitian_traceless(rng, n):
    """n traceless Hermitian 3x3 matrices H = (G + G^dag)/2 - tr/3, G complex Gaussian."""
    g = _gaussian_complex(rng, (n, 3, 3))
    h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h[:, 0, 0] -= tr
    h[:, 1, 1] -= tr
    h[:, 2, 2] -= tr
    return h


def expi_hermitian(h, eps):
    """exp(i*eps*H) for a batch of Hermitian H, via the eigendecomposition H = V diag(w) V^dag."""
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return np.einsum("nij,nj,nkj->nik", v, ph, np.conj(v))


def random_su3(rng, n, eps):
    return expi_hermitian(random_hermitian_traceless(rng, n), eps)


def random_links(dims, eps, seed, chunk=1 << 20):
    """Random SU(3) gauge field of shape [4, T, Z, Y, X, 3, 3] (complex128).

    Generated in chunks so large lattices stay within memory."""
    X, Y, Z, T = dims
    n = 4 * volume(dims)
    rng = np.random.default_rng(seed)
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = random_su3(rng, hi - lo, eps)
    return out.reshape(4, T, Z, Y, X, 3, 3)


def unit_links(dims):
    X, Y, Z, T = dims
    u = np.zeros((4, T, Z, Y, X, 3, 3), dtype=np.complex128)
    for a in range(3):
        u[..., a, a] = 1.0
    return u


def gaussian_field(dims, seed):
    """Complex Gaussian fermion field [T, Z, Y, X, 3, 4]; each component (N + iN)/sqrt(2)."""
    X, Y, Z, T = dims
    rng = np.random.default_rng(seed)
    return _gaussian_complex(rng, (T, Z, Y, X, 3, 4))


def point_source(dims, spin, colour, site=(0, 0, 0, 0)):
    """Unit source at one site (x, y, z, t) in one spin and colour component."""
    X, Y, Z, T = dims
    b = np.zeros((T, Z, Y, X, 3, 4), dtype=np.complex128)
    x, y, z, t = site
    b[t, z, y, x, colour, spin] = 1.0
    return b


def random_gauge_transform(dims, seed, eps=1.0):
    """A random SU(3) matrix per site, shape [T, Z, Y, X, 3, 3]."""
    X, Y, Z, T = dims
    rng = np.random.default_rng(seed)
    return random_su3(rng, volume(dims), eps).reshape(T, Z, Y, X, 3, 3)
