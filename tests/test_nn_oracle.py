"""Pins of the learned-proposal oracle (oracle/nn.py) to things other than
itself: central finite differences, gauge covariance, the closed-form loss of
one vector against one vector, brute-force single hops written with explicit
site loops, and zero loss when the outputs are the targets."""
import numpy as np
import pytest

import synthetic as syn
from oracle import nn
from tests import brute_force as bf


def small_problem(L=(2, 2, 2, 4), block=(2, 2, 2, 2), nv=2, ch=3, seed=5):
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.4, seed)
    eta = syn.complex_gaussian((nv, V, 4, 3), seed + 1)
    tgt = syn.complex_gaussian((nv, V, 4, 3), seed + 2)
    Ws = nn.init_weights(nv, ch, 3, np.random.default_rng(seed + 3))
    return L, block, U, eta, tgt, Ws


def test_gradients_match_central_differences():
    L, block, U, eta, tgt, Ws = small_problem()
    val, grads, _ = nn.loss_and_grads(U, eta, Ws, tgt, L, block)
    assert 0 < val < 1
    rng = np.random.default_rng(11)
    d = 1e-5  # truncation and rounding both near 1e-11 here
    worst = 0.0
    for l, W in enumerate(Ws):
        for _ in range(6):
            h, o, i = (int(rng.integers(n)) for n in W.shape)
            for part in (1.0, 1j):
                Wp = [w.copy() for w in Ws]
                Wm = [w.copy() for w in Ws]
                Wp[l][h, o, i] += d * part
                Wm[l][h, o, i] -= d * part
                fp = nn.loss_and_grads(U, eta, Wp, tgt, L, block)[0]
                fm = nn.loss_and_grads(U, eta, Wm, tgt, L, block)[0]
                fd = (fp - fm) / (2 * d)
                g = grads[l][h, o, i]
                an = 2 * (g.real if part == 1.0 else g.imag)  # dL = 2 Re(conj(g) dW)
                worst = max(worst, abs(fd - an) / max(abs(an), 1e-3))
    assert worst < 1e-7, worst


def test_gauge_covariance():
    """f(U^g, g eta) = g f(U, eta), and the loss is gauge invariant."""
    L, block, U, eta, tgt, Ws = small_problem(L=(2, 2, 4, 4), block=(2, 2, 2, 2))
    g = syn.random_gauge_transform(L, 21)
    Ug = bf.gauge_transform_links(L, U, g)
    etag = np.stack([bf.gauge_transform_fermion(g, e) for e in eta])
    tgtg = np.stack([bf.gauge_transform_fermion(g, t) for t in tgt])
    tab = nn.lattice_tables(L)
    Y = nn.forward(U, eta, Ws, tab)[0][-1]
    Yg = nn.forward(Ug, etag, Ws, tab)[0][-1]
    gY = np.stack([bf.gauge_transform_fermion(g, y) for y in Y])
    assert np.linalg.norm(Yg - gY) < 1e-12 * np.linalg.norm(Y)
    l0 = nn.loss_and_grads(U, eta, Ws, tgt, L, block)[0]
    l1 = nn.loss_and_grads(Ug, etag, Ws, tgtg, L, block)[0]
    assert abs(l0 - l1) < 1e-12


def test_loss_one_vector_closed_form():
    """With one output y and one target v the optimal c is <y,v>/<y,y> per
    block, and the residual is |v|^2 - |<y,v>|^2/|y|^2 (Pythagoras)."""
    L, block = (2, 2, 2, 4), (2, 2, 2, 2)
    V = 32
    y = syn.complex_gaussian((1, V, 4, 3), 31)
    v = syn.complex_gaussian((1, V, 4, 3), 32)
    val, g = nn.loss(y, v, nn.chiral_blocks(L, block))
    ref = 0.0
    for agg in range(2):
        sites = np.arange(V)[(np.arange(V) // 16) == agg]  # block spans x, y, z and half of t
        for chi in range(2):
            yb = y[0][sites][:, 2 * chi:2 * chi + 2].ravel()
            vb = v[0][sites][:, 2 * chi:2 * chi + 2].ravel()
            ref += np.vdot(vb, vb).real - abs(np.vdot(yb, vb)) ** 2 / np.vdot(yb, yb).real
    assert abs(val - ref / np.vdot(v, v).real) < 1e-13


def test_zero_loss_when_outputs_are_targets():
    L, block, U, eta, tgt, Ws = small_problem()
    Y = nn.forward(U, eta, Ws, nn.lattice_tables(L))[0][-1]
    val, g = nn.loss(Y, Y, nn.chiral_blocks(L, block))
    assert val < 1e-24 and np.max(np.abs(g)) < 1e-12


@pytest.mark.parametrize("h", [1, 2, 7, 8])
def test_single_hop_layer_brute_force(h):
    """A layer whose only nonzero weight is the channel identity on hop h is
    that hop's parallel transport, written out with explicit site loops
    (t hops across the end pick up the antiperiodic sign)."""
    L = (2, 3, 2, 3)
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.5, 41)
    psi = syn.complex_gaussian((2, V, 4, 3), 42)
    W = np.zeros((9, 2, 2), complex)
    W[h] = np.eye(2)
    z = nn.layer(U, psi, W, nn.lattice_tables(L))
    X = bf.coords(L)
    mu = (h - 1) // 2
    fwd = h % 2 == 1
    ref = np.zeros_like(psi)
    for x in range(V):
        y = X[x].copy()
        y[mu] = (y[mu] + (1 if fwd else -1)) % L[mu]
        yi = bf.lex(L, y)
        sgn = 1.0
        if mu == 3 and ((fwd and X[x][3] == L[3] - 1) or (not fwd and X[x][3] == 0)):
            sgn = -1.0
        link = U[x, mu] if fwd else np.conj(U[yi, mu]).T
        for c in range(2):
            for s in range(4):
                ref[c, x, s] = sgn * link @ psi[c, yi, s]
    assert np.linalg.norm(z - ref) < 1e-13 * np.linalg.norm(ref)


def test_self_hop_is_channel_matrix():
    L = (2, 2, 2, 2)
    U = syn.gauge_field(L, 0.5, 51)
    psi = syn.complex_gaussian((3, 16, 4, 3), 52)
    W = np.zeros((9, 2, 3), complex)
    W[0] = syn.complex_gaussian((2, 3), 53)
    z = nn.layer(U, psi, W, nn.lattice_tables(L))
    ref = np.tensordot(W[0], psi, axes=(1, 0))
    assert np.linalg.norm(z - ref) < 1e-13 * np.linalg.norm(ref)


def test_squash_backward_matches_differences():
    rng = np.random.default_rng(61)
    z = rng.standard_normal((1, 2, 4, 3)) + 1j * rng.standard_normal((1, 2, 4, 3))
    gA = rng.standard_normal(z.shape) + 1j * rng.standard_normal(z.shape)

    def f(zz):  # L = Re <gA, a(z)> has dL/da* = gA / 2
        a, _ = nn.squash(zz)
        return np.real(np.vdot(gA, a))

    a, s = nn.squash(z)
    gz = nn.squash_backward(gA / 2, a, s)
    d = 1e-6
    for idx in [(0, 0, 1, 2), (0, 1, 3, 0)]:
        for part in (1.0, 1j):
            zp, zm = z.copy(), z.copy()
            zp[idx] += d * part
            zm[idx] -= d * part
            fd = (f(zp) - f(zm)) / (2 * d)
            an = 2 * (gz[idx].real if part == 1.0 else gz[idx].imag)
            assert abs(fd - an) < 1e-8


def test_adam_first_step_closed_form():
    """At t = 1 the bias corrections make m_hat = g and v_hat = g^2, so the
    step is -lr g / (|g| + eps) per real parameter, whatever b1 and b2 are."""
    from oracle import nn as onn
    g = np.array([0.3, -2.0, 1e-9, 0.0, 5e3], np.float64)
    for b1, b2 in ((0.9, 0.999), (0.5, 0.8)):
        w = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
        w0 = w.copy()
        m = np.zeros_like(w)
        v = np.zeros_like(w)
        onn.adam_step(w, g, m, v, 1, 0.01, b1=b1, b2=b2, eps=1e-8)
        assert np.allclose(w - w0, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        assert np.allclose(m, (1 - b1) * g, rtol=1e-15) and np.allclose(v, (1 - b2) * g * g, rtol=1e-15)


def test_adam_constant_gradient_keeps_the_first_step():
    """With the same gradient at every step, m = (1 - b1^t) g and
    v = (1 - b2^t) g^2 exactly, so every bias-corrected step equals the first:
    after t steps w moved by -t lr g / (|g| + eps)."""
    from oracle import nn as onn
    g = np.array([0.7, -0.2, 3.0])
    w = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    for t in range(1, 8):
        onn.adam_step(w, g, m, v, t, 1e-3)
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)
        assert np.allclose(w, -t * 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-10)


def test_adam_second_step_hand_computed():
    """Two different gradients: the second step from the definitions
    m_2 = b1 (1-b1) g1 + (1-b1) g2, v_2 = b2 (1-b2) g1^2 + (1-b2) g2^2,
    divided by (1 - b^2)."""
    from oracle import nn as onn
    g1, g2 = np.array([1.0, -3.0]), np.array([-0.5, 2.0])
    w = np.zeros(2)
    m = np.zeros(2)
    v = np.zeros(2)
    onn.adam_step(w, g1, m, v, 1, 0.1)
    w1 = w.copy()
    onn.adam_step(w, g2, m, v, 2, 0.1)
    m2 = (0.9 * 0.1 * g1 + 0.1 * g2) / (1 - 0.81)
    v2 = (0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    assert np.allclose(w - w1, -0.1 * m2 / (np.sqrt(v2) + 1e-8), rtol=1e-12)
