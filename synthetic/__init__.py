"""Seeded synthetic inputs for the Wilson-clover multigrid path.

This module only draws random numbers and shapes them into inputs: gauge
links, start vectors, right-hand sides.  It holds none of the method's
arithmetic (no Dirac operator, no projection, no solver), so both the GPU
library's tests and the CPU oracle may take their inputs from here.

Conventions of the inputs
-------------------------
* Lattice sites are lexicographic with x fastest:
  ``i = x + Lx*(y + Ly*(z + Lz*t))``.
* Gauge links: complex128 array ``[V][4][3][3]`` (site, direction mu = x,y,z,t,
  row, column), ``U_mu(x)`` connects ``x`` to ``x + mu``.
* Fermion fields: complex128 ``[nrhs][V][4][3]`` (spin, colour).
* Coarse fields: complex128 ``[nrhs][Vc][Nb]``.

All randomness comes from ``numpy.random.Generator(PCG64(seed))`` in FP64.
Seed layout for a workload with base seed ``s``: ``1000*s + 0`` gauge field,
``+1`` start vectors, ``+2`` right-hand sides, ``+3`` network weights,
``+10*level`` offsets the start vectors of deeper levels.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "volume", "gell_mann", "gauge_field", "unit_gauge", "random_gauge_transform",
    "complex_gaussian", "start_vectors", "point_sources", "config_seeds",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape [8][3][3] complex128."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3.0)
    l[7][2, 2] = -2 / np.sqrt(3.0)
    return l


def _reunitarise(u: np.ndarray) -> np.ndarray:
    # polar projection onto U(3), then fix the determinant to 1
    w, _, vh = np.linalg.svd(u)
    u = w @ vh
    det = np.linalg.det(u)
    return u / (det ** (1.0 / 3.0))[..., None, None]


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """SU(3) links U = exp(i*eps*H), H = sum_a w_a lambda_a / 2, w_a ~ N(0,1).

    Draw order: ``standard_normal((V, 4, 8))`` in lexicographic site order,
    then direction, then Gell-Mann index.  The exponential is taken through
    the eigendecomposition of the Hermitian H, then re-unitarised.
    """
    V = volume(dims)
    g = rng(seed)
    w = g.standard_normal((V, 4, 8))
    H = np.einsum("vma,aij->vmij", w, gell_mann() / 2.0)
    e, q = np.linalg.eigh(H)
    U = (q * np.exp(1j * eps * e)[..., None, :]) @ np.conj(np.swapaxes(q, -1, -2))
    return np.ascontiguousarray(_reunitarise(U))


def unit_gauge(dims) -> np.ndarray:
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """One random SU(3) matrix g(x) per site, shape [V][3][3]."""
    V = volume(dims)
    g = rng(seed)
    w = g.standard_normal((V, 8))
    H = np.einsum("va,aij->vij", w, gell_mann() / 2.0)
    e, q = np.linalg.eigh(H)
    G = (q * np.exp(1j * 1.7 * e)[..., None, :]) @ np.conj(np.swapaxes(q, -1, -2))
    return np.ascontiguousarray(_reunitarise(G))


def complex_gaussian(shape, seed: int) -> np.ndarray:
    """Re and Im each N(0,1); draw order is ``shape + (2,)``."""
    g = rng(seed)
    a = g.standard_normal(tuple(shape) + (2,))
    return np.ascontiguousarray(a[..., 0] + 1j * a[..., 1])


def start_vectors(nv: int, n_sites: int, ns: int, seed: int) -> np.ndarray:
    """Gaussian start vectors for the near-null space, shape [nv][n_sites][ns]."""
    return complex_gaussian((nv, n_sites, ns), seed)


def point_sources(V: int, site: int = 0) -> np.ndarray:
    """Twelve point sources b_{s,c}(x) = delta_{x,site} e_{3s+c}: [12][V][4][3]."""
    b = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for k in range(12):
        b[k, site, k // 3, k % 3] = 1.0
    return b


def config_seeds(base: int) -> dict:
    s = 1000 * int(base)
    return {"gauge": s + 0, "start": s + 1, "rhs": s + 2, "net": s + 3}
