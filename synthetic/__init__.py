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
    "rng", "volume", "gell_mann", "gauge_field", "gauge_field_device", "unit_gauge", "random_gauge_transform",
    "complex_gaussian", "start_vectors", "start_vectors_device", "point_sources", "config_seeds",
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


def _mm3(a, b):
    """Batched 3x3 products [..., 3, 3] as broadcast elementwise operations."""
    return (a[..., :, 0, None] * b[..., None, 0, :] + a[..., :, 1, None] * b[..., None, 1, :]
            + a[..., :, 2, None] * b[..., None, 2, :])


def _expi_traceless_hermitian(Q):
    """exp(iQ) for traceless Hermitian Q (torch complex128 [..., 3, 3]).

    Cayley-Hamilton reduces the exponential to exp(iQ) = f0 + f1 Q + f2 Q^2;
    the coefficients follow from the eigenvalues of Q in the parametrisation
    of C. Morningstar and M. Peardon, Phys. Rev. D 69, 054501 (2004):
    c0 = det Q, c1 = tr(Q^2)/2, theta = arccos(|c0| / (2 (c1/3)^(3/2))),
    u = sqrt(c1/3) cos(theta/3), w = sqrt(c1) sin(theta/3), and
    f_j = h_j / (9u^2 - w^2) with
      h0 = (u^2 - w^2) e^{2iu} + e^{-iu} (8u^2 cos w + 2iu (3u^2 + w^2) xi0(w)),
      h1 = 2u e^{2iu} - e^{-iu} (2u cos w - i (3u^2 - w^2) xi0(w)),
      h2 = e^{2iu} - e^{-iu} (cos w + 3iu xi0(w)),   xi0(w) = sin(w)/w;
    for c0 < 0, f_j(-c0) = (-1)^j conj(f_j(c0)).
    """
    import torch
    Q2 = _mm3(Q, Q)
    c1 = 0.5 * (Q2[..., 0, 0] + Q2[..., 1, 1] + Q2[..., 2, 2]).real
    c0 = (Q[..., 0, 0] * (Q[..., 1, 1] * Q[..., 2, 2] - Q[..., 1, 2] * Q[..., 2, 1])
          - Q[..., 0, 1] * (Q[..., 1, 0] * Q[..., 2, 2] - Q[..., 1, 2] * Q[..., 2, 0])
          + Q[..., 0, 2] * (Q[..., 1, 0] * Q[..., 2, 1] - Q[..., 1, 1] * Q[..., 2, 0])).real
    neg = c0 < 0
    c0max = 2.0 * (c1 / 3.0) ** 1.5
    one = torch.ones_like(c0)
    ratio = torch.where(c0max > 0, c0.abs() / torch.where(c0max > 0, c0max, one), one)
    theta = torch.arccos(ratio.clamp(-1.0, 1.0))
    u = torch.sqrt(c1 / 3.0) * torch.cos(theta / 3.0)
    w = torch.sqrt(c1) * torch.sin(theta / 3.0)
    w2 = w * w
    xi0 = torch.where(w.abs() > 0.05, torch.sin(w) / torch.where(w == 0, one, w),
                      1 - w2 / 6 * (1 - w2 / 20 * (1 - w2 / 42)))
    e2iu = torch.exp(2j * u)
    emiu = torch.exp(-1j * u)
    cw = torch.cos(w)
    h0 = (u * u - w2) * e2iu + emiu * (8 * u * u * cw + 2j * u * (3 * u * u + w2) * xi0)
    h1 = 2 * u * e2iu - emiu * (2 * u * cw - 1j * (3 * u * u - w2) * xi0)
    h2 = e2iu - emiu * (cw + 3j * u * xi0)
    den = 9 * u * u - w2
    f0, f1, f2 = h0 / den, h1 / den, h2 / den
    f0 = torch.where(neg, f0.conj(), f0)
    f1 = torch.where(neg, -f1.conj(), f1)
    f2 = torch.where(neg, f2.conj(), f2)
    out = f1[..., None, None] * Q + f2[..., None, None] * Q2
    for i in range(3):
        out[..., i, i] += f0
    return out


def _reunitarise(U):
    """Projection onto SU(3) (torch [..., 3, 3]): Gram-Schmidt of the first two
    rows, third row = conj(row0 x row1), so that det = 1."""
    import torch
    r0 = U[..., 0, :]
    r1 = U[..., 1, :]
    r0 = r0 / torch.sqrt((r0.abs() ** 2).sum(-1))[..., None]
    r1 = r1 - (r0.conj() * r1).sum(-1)[..., None] * r0
    r1 = r1 / torch.sqrt((r1.abs() ** 2).sum(-1))[..., None]
    r2 = torch.stack([r0[..., 1] * r1[..., 2] - r0[..., 2] * r1[..., 1],
                      r0[..., 2] * r1[..., 0] - r0[..., 0] * r1[..., 2],
                      r0[..., 0] * r1[..., 1] - r0[..., 1] * r1[..., 0]], dim=-1).conj()
    return torch.stack([r0, r1, r2], dim=-2)


def _su3_from_algebra(w: np.ndarray, scale: float, device=None):
    """exp(i scale H), H = sum_a w_a lambda_a / 2, for coefficients w [..., 8],
    re-unitarised; evaluated in chunks (the closed form above, in FP64).
    device None: a numpy array from CPU arithmetic; else a torch tensor
    computed on that device from the same coefficients."""
    import torch
    dv = torch.device("cpu") if device is None else torch.device(device)
    gm = torch.from_numpy(gell_mann().reshape(8, 9) / 2.0).to(dv)
    flat = w.reshape(-1, 8)
    out = (np.empty((flat.shape[0], 3, 3), dtype=np.complex128) if device is None
           else torch.empty((flat.shape[0], 3, 3), dtype=torch.complex128, device=dv))
    step = 1 << 20
    for a in range(0, flat.shape[0], step):
        H = (torch.from_numpy(flat[a:a + step]).to(dv).to(torch.complex128) @ gm).reshape(-1, 3, 3)
        u = _reunitarise(_expi_traceless_hermitian(scale * H))
        out[a:a + step] = u.numpy() if device is None else u
    return out.reshape(w.shape[:-1] + (3, 3))


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """SU(3) links U = exp(i*eps*H), H = sum_a w_a lambda_a / 2, w_a ~ N(0,1).

    Draw order: ``standard_normal((V, 4, 8))`` in lexicographic site order,
    then direction, then Gell-Mann index.  The exponential is taken in closed
    form (Cayley-Hamilton with the Morningstar-Peardon coefficients; equal to
    the eigendecomposition route to ~1e-15), then re-unitarised.
    """
    V = volume(dims)
    g = rng(seed)
    w = g.standard_normal((V, 4, 8))
    return np.ascontiguousarray(_su3_from_algebra(w, eps))


def gauge_field_device(dims, eps: float, seed: int, device="cuda"):
    """gauge_field's links (the same draws, the same closed form) evaluated on
    a torch device: complex128 tensor [V][4][3][3]; equal to gauge_field up
    to the device's rounding."""
    V = volume(dims)
    g = rng(seed)
    w = g.standard_normal((V, 4, 8))
    return _su3_from_algebra(w, eps, device).contiguous()


def start_vectors_device(nv: int, n_sites: int, ns: int, seed: int, device="cuda"):
    """Gaussian start vectors drawn on a torch device ([nv][n_sites][ns]
    complex128; Re and Im each N(0,1)) from torch's generator of that device
    seeded with `seed`: reproducible for a device type, not equal to
    start_vectors' numpy draws."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    a = torch.randn((nv, n_sites, ns, 2), dtype=torch.float64, device=device, generator=g)
    return torch.complex(a[..., 0], a[..., 1]).contiguous()


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
    return np.ascontiguousarray(_su3_from_algebra(w, 1.7))


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
