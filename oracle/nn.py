"""Oracle of the learned near-null proposal: plain FP64 NumPy.

TEST INFRASTRUCTURE.  Only the tests, the smoke entry point and the benchmark's
CPU baseline may import this module; the library never does.

The network maps the Nv Gaussian start vectors of the setup (channels) to Nv
proposed near-null vectors.  It is built from parallel-transport convolutions,
so it commutes with gauge transformations: weights act on channels only,
the same for every spin and colour component, and every hop carries the link
that transports colour between the two sites.

Layer (hop h = 0 is the site itself; h = 2 mu + 1 the hop from x + mu,
h = 2 mu + 2 the hop from x - mu, mu = x, y, z, t):

    z_o(x) = sum_i sum_h W[h, o, i] (T_h psi_i)(x)
    (T_0 psi)(x)          = psi(x)
    (T_{2mu+1} psi)(x)    = U_mu(x) psi(x + mu)
    (T_{2mu+2} psi)(x)    = U_mu(x - mu)^dag psi(x - mu)

with the fermion boundary sign (-1) on t hops across the lattice end when the
lattice is antiperiodic in t.  Between layers each channel is squashed site
by site, a = z / sqrt(1 + |z(x)|^2) (norm over the 12 spin-colour components);
the last layer is linear.

Loss (how well the outputs Y span the target near-null vectors v_j of the
plain setup, measured where the multigrid uses them: aggregate by aggregate
and chirality by chirality):

    c_j = argmin_c |v_j - Y c|   on each (aggregate, chirality) block,
    L   = sum_blocks sum_j |v_j - Y c_j|^2 / sum_j |v_j|^2.

Gradients are with respect to conjugated arguments (dL/dY* etc.), so that
dL = 2 Re <g, dY>.  At the optimum c_j the loss is stationary in c (envelope
theorem), hence dL/dY* = -r_j c_j^dag / sum_j |v_j|^2 with r_j = v_j - Y c_j.

Parity pins: the tests pin this module to finite differences, to gauge
covariance, to the closed-form angle loss of one vector against one vector,
and to brute-force single-hop layers.

Arrays: fields [C][V][4][3] complex128 (V lexicographic, x fastest); links
[V][4][3][3]; weights per layer [9][C_out][C_in] complex128.
"""
from __future__ import annotations

import numpy as np

N_HOPS = 9


def lattice_tables(L, antiperiodic=True):
    """Neighbour indices nb[h][x] of the site feeding hop h into x, and the
    boundary sign of that hop (+1, or -1 across the t end when antiperiodic)."""
    L = tuple(int(v) for v in L)
    V = int(np.prod(L))
    idx = np.arange(V)
    coords = []
    r = idx.copy()
    for m in range(4):
        coords.append(r % L[m])
        r //= L[m]
    coords = np.array(coords)  # [4][V]

    def lex(c):
        return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]))

    nb = np.zeros((N_HOPS, V), np.int64)
    sign = np.ones((N_HOPS, V))
    nb[0] = idx
    for mu in range(4):
        fwd = coords.copy()
        fwd[mu] = (coords[mu] + 1) % L[mu]
        bwd = coords.copy()
        bwd[mu] = (coords[mu] - 1) % L[mu]
        nb[2 * mu + 1] = lex(fwd)
        nb[2 * mu + 2] = lex(bwd)
        if mu == 3 and antiperiodic:
            sign[2 * mu + 1] = np.where(coords[3] == L[3] - 1, -1.0, 1.0)
            sign[2 * mu + 2] = np.where(coords[3] == 0, -1.0, 1.0)
    return nb, sign


def transport(U, psi, h, tables):
    """T_h psi for psi [..., V, 4, 3]."""
    nb, sign = tables
    if h == 0:
        return psi.copy()
    mu = (h - 1) // 2
    y = nb[h]
    s = sign[h][:, None, None]
    if h % 2 == 1:  # from x + mu through U_mu(x)
        return s * np.einsum("xab,...xsb->...xsa", U[:, mu], psi[..., y, :, :])
    # from x - mu through U_mu(x - mu)^dag
    return s * np.einsum("xba,...xsb->...xsa", np.conj(U[y, mu]), psi[..., y, :, :])


def adjoint_hop(h):
    """T_h^dag = T_{adjoint_hop(h)}."""
    if h == 0:
        return 0
    return h + 1 if h % 2 == 1 else h - 1


def layer(U, psi, W, tables):
    """Pre-activation z [C_out][V][4][3] of one layer."""
    Cout = W.shape[1]
    z = np.zeros((Cout,) + psi.shape[1:], np.complex128)
    for h in range(N_HOPS):
        t = transport(U, psi, h, tables)
        z += np.einsum("oi,ixsa->oxsa", W[h], t)
    return z


def squash(z):
    s = np.sqrt(1.0 + np.sum(np.abs(z) ** 2, axis=(-2, -1), keepdims=True))
    return z / s, s


def forward(U, eta, Ws, tables):
    """Activations [input, a_1, ..., output] and the squash factors s_l."""
    acts, scales = [eta], []
    a = eta
    for l, W in enumerate(Ws):
        z = layer(U, a, W, tables)
        if l + 1 < len(Ws):
            a, s = squash(z)
            scales.append(s)
        else:
            a = z
        acts.append(a)
    return acts, scales


def chiral_blocks(L, block):
    """(site indices, spin range) of every (aggregate, chirality) block, from
    the aggregation of the lattice by the given block (x fastest)."""
    L = tuple(int(v) for v in L)
    V = int(np.prod(L))
    idx = np.arange(V)
    c = []
    r = idx.copy()
    for m in range(4):
        c.append(r % L[m])
        r //= L[m]
    Lc = [L[m] // block[m] for m in range(4)]
    agg = (c[0] // block[0]) + Lc[0] * ((c[1] // block[1]) + Lc[1] * ((c[2] // block[2]) + Lc[2] * (c[3] // block[3])))
    out = []
    for a in range(int(np.prod(Lc))):
        sites = np.nonzero(agg == a)[0]
        for chi in range(2):
            out.append((sites, slice(2 * chi, 2 * chi + 2)))
    return out


def loss(Y, targets, blocks):
    """Loss and dL/dY* (same shape as Y).  Y, targets: [Nv][V][4][3]."""
    norm = float(np.sum(np.abs(targets) ** 2))
    total = 0.0
    g = np.zeros_like(Y)
    for sites, sp in blocks:
        Yb = Y[:, sites, sp, :].reshape(Y.shape[0], -1).T        # [n][Nv]
        Vb = targets[:, sites, sp, :].reshape(targets.shape[0], -1).T
        G = Yb.conj().T @ Yb
        c = np.linalg.solve(G, Yb.conj().T @ Vb)                   # [Nv][Nv]: column j is c_j
        R = Vb - Yb @ c
        total += float(np.sum(np.abs(R) ** 2))
        gb = -(R @ c.conj().T) / norm                              # [n][Nv]
        g[:, sites, sp, :] = gb.T.reshape(Y.shape[0], len(sites), 2, 3)
    return total / norm, g


def squash_backward(gA, a, s):
    """dL/dz* from dL/da* for a = z / s, s = sqrt(1 + |z|^2)."""
    re = np.real(np.sum(np.conj(gA) * a, axis=(-2, -1), keepdims=True))
    return (gA - a * re) / s


def backward(U, acts, scales, Ws, gY, tables):
    """dL/dW* for every layer, given dL/dY* of the output."""
    grads = [None] * len(Ws)
    g = gY
    for l in range(len(Ws) - 1, -1, -1):
        if l + 1 < len(Ws):
            g = squash_backward(g, acts[l + 1], scales[l])
        x = acts[l]
        W = Ws[l]
        gW = np.zeros_like(W)
        gx = np.zeros_like(x)
        for h in range(N_HOPS):
            t = transport(U, x, h, tables)
            gW[h] = np.einsum("ixsa,oxsa->oi", np.conj(t), g)
            gx += np.einsum("oi,oxsa->ixsa", np.conj(W[h]), transport(U, g, adjoint_hop(h), tables))
        grads[l] = gW
        g = gx
    return grads


def loss_and_grads(U, eta, Ws, targets, L, block, antiperiodic=True):
    tables = lattice_tables(L, antiperiodic)
    acts, scales = forward(U, eta, Ws, tables)
    val, gY = loss(acts[-1], targets, chiral_blocks(L, block))
    return val, backward(U, acts, scales, Ws, gY, tables), acts[-1]


def init_weights(n_vec, channels, layers, rng):
    """Weights of the Nv -> C -> ... -> C -> Nv network: the self hop starts
    near the identity map (as far as the shapes allow), the other hops small."""
    dims = [n_vec] + [channels] * (layers - 1) + [n_vec]
    Ws = []
    for l in range(layers):
        ci, co = dims[l], dims[l + 1]
        W = (rng.standard_normal((N_HOPS, co, ci)) + 1j * rng.standard_normal((N_HOPS, co, ci))) * (0.1 / np.sqrt(ci))
        W[0] += np.eye(co, ci)
        Ws.append(W)
    return Ws


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on real parameters w with gradient g (arrays updated in place)."""
    m *= b1
    m += (1 - b1) * g
    v *= b2
    v += (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    w -= lr * mh / (np.sqrt(vh) + eps)
