"""Independent dense / closed-form constructions used to pin the oracle.

Nothing here calls the oracle's arithmetic: these are the mathematical facts
the oracle must reproduce (closed forms, explicit dense matrices assembled from
their definitions with numpy, enumerations by coordinates).
"""
from __future__ import annotations

import numpy as np


def coords(L):
    """Coordinates [V][4] of lexicographic sites, x fastest."""
    V = int(np.prod(L))
    idx = np.arange(V)
    return np.stack(np.unravel_index(idx, tuple(L[::-1]))[::-1], axis=1)


def lex(L, x):
    x = np.asarray(x)
    return x[..., 0] + L[0] * (x[..., 1] + L[1] * (x[..., 2] + L[2] * x[..., 3]))


def agg_map(L, block):
    """Brute-force aggregation map by coordinates."""
    X = coords(L)
    b = np.asarray(block)
    Lc = np.asarray(L) // b
    cx = X // b
    ox = X % b
    coarse = lex(Lc, cx)
    offset = ox[:, 0] + b[0] * (ox[:, 1] + b[1] * (ox[:, 2] + b[2] * ox[:, 3]))
    return coarse.astype(np.int32), offset.astype(np.int32)


def neighbour(L, d):
    """Neighbour index of every site in direction d = 1..8 (+x,-x,+y,...)."""
    X = coords(L)
    mu = (d - 1) // 2
    step = 1 if (d - 1) % 2 == 0 else -1
    Y = X.copy()
    Y[:, mu] = (Y[:, mu] + step) % L[mu]
    return lex(L, Y)


def dense_from_blocks(Lc, blocks):
    """Dense matrix of the 9-point block stencil [Vc][9][Nb][Nb]."""
    Vc, _, nb, _ = blocks.shape
    M = np.zeros((Vc * nb, Vc * nb), np.complex128)
    for c in range(Vc):
        M[c * nb:(c + 1) * nb, c * nb:(c + 1) * nb] += blocks[c, 0]
    for d in range(1, 9):
        nbr = neighbour(Lc, d)
        for c in range(Vc):
            y = nbr[c]
            M[c * nb:(c + 1) * nb, y * nb:(y + 1) * nb] += blocks[c, d]
    return M


def sigma3(nb):
    """Coarse chirality grading: +1 on the first Nb/2 components, -1 on the rest."""
    return np.where(np.arange(nb) < nb // 2, 1.0, -1.0)


def sigma3_mirror(Lc, blocks):
    """Blocks [Vc][9][Nb][Nb] with every backward hop replaced by the
    sigma3-conjugated adjoint of the neighbour's forward hop:
    M_{-mu}(c) = s M_{+mu}(c - mu)^dag s."""
    out = np.array(blocks, copy=True)
    s = sigma3(blocks.shape[-1])
    S = s[:, None] * s[None, :]
    for mu in range(4):
        back = neighbour(Lc, 2 * mu + 2)
        out[:, 2 * mu + 2] = S * np.conj(np.swapaxes(blocks[back, 2 * mu + 1], -1, -2))
    return out


def dense_prolongator(L, block, ns, Pv):
    """Dense P: rows (x, k), columns (c, b); column b reads vector b mod nv on
    chirality half b // nv, restricted to aggregate c."""
    nv = Pv.shape[0]
    V = int(np.prod(L))
    coarse, _ = agg_map(L, block)
    Vc = V // int(np.prod(block))
    nb = 2 * nv
    h = ns // 2
    P = np.zeros((V * ns, Vc * nb), np.complex128)
    Pv = Pv.reshape(nv, V, ns)
    for x in range(V):
        c = coarse[x]
        for b in range(nb):
            i, chi = b % nv, b // nv
            for k in range(chi * h, chi * h + h):
                P[x * ns + k, c * nb + b] = Pv[i, x, k]
    return P


def dense_operator(apply, n):
    """Dense matrix of a linear map given as a function on flat vectors."""
    M = np.zeros((n, n), np.complex128)
    e = np.zeros(n, np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = apply(e)
        e[j] = 0.0
    return M


def free_eigenvalues(L, m0, antiperiodic=True):
    """Closed-form spectrum of the free Wilson operator (U = 1, no clover):
    m0 + sum_mu (1 - cos p_mu) +- i sqrt(sum_mu sin^2 p_mu), each sign 6-fold."""
    ev = []
    grids = []
    for mu in range(4):
        n = np.arange(L[mu])
        shift = 0.5 if (mu == 3 and antiperiodic) else 0.0
        grids.append(2 * np.pi * (n + shift) / L[mu])
    P = np.stack(np.meshgrid(*grids, indexing="ij"), axis=-1).reshape(-1, 4)
    re = m0 + np.sum(1 - np.cos(P), axis=1)
    im = np.sqrt(np.sum(np.sin(P) ** 2, axis=1))
    for r, i in zip(re, im):
        ev += [r + 1j * i] * 6 + [r - 1j * i] * 6
    return np.array(ev)


def sort_spectrum(ev, digits=8):
    ev = np.asarray(ev)
    key = np.lexsort((np.round(ev.imag, digits), np.round(ev.real, digits)))
    return ev[key]


def constant_field(L, mu, nu, n_flux=1, phi_pattern=(1, -1, 0)):
    """Abelian constant field in the mu-nu plane embedded as diag(e^{ia}, e^{-ia}, 1).

    U_mu(x) = e^{-i theta x_nu},  U_nu(x) = e^{i theta L_nu x_mu} on the slice
    x_nu = L_nu - 1 (identity elsewhere), theta = 2 pi n / (L_mu L_nu).  Every
    mu-nu plaquette then equals the embedding of e^{i theta}.
    Returns (U, theta)."""
    V = int(np.prod(L))
    X = coords(L)
    theta = 2 * np.pi * n_flux / (L[mu] * L[nu])
    U = np.zeros((V, 4, 3, 3), np.complex128)
    for a in range(3):
        U[:, :, a, a] = 1.0
    pat = np.array(phi_pattern, float)

    def emb(angle):
        return np.exp(1j * np.outer(angle, pat))

    amu = -theta * X[:, nu]
    anu = np.where(X[:, nu] == L[nu] - 1, theta * L[nu] * X[:, mu], 0.0)
    for a in range(3):
        U[:, mu, a, a] = emb(amu)[:, a]
        U[:, nu, a, a] = emb(anu)[:, a]
    return U, theta


def gauge_transform_links(L, U, g):
    """U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag."""
    out = np.empty_like(U)
    for mu in range(4):
        y = neighbour(L, 1 + 2 * mu)
        out[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[y], -1, -2))
    return out


def gauge_transform_fermion(g, psi):
    """(g psi)(x) = g(x) psi(x) on the colour index; psi [V][4][3]."""
    return np.einsum("vab,vsb->vsa", g, psi)


def gamma_chiral():
    """Chiral Euclidean gamma matrices written out from their definition."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]
    z = np.zeros((2, 2), complex)
    one = np.eye(2)
    g = [np.block([[z, -1j * sk], [1j * sk, z]]) for sk in s]
    g.append(np.block([[z, one], [one, z]]))
    return np.array(g)
