"""Learned near-null proposal on the GPU (wcmg_nn_*) against the FP64 oracle
of oracle/nn.py: forward pass, loss and weight gradients (FP32 activations to
FP32 rounding; BF16 activations to their storage error), gauge covariance,
training, and the learned setup with its fallback.

The oracle takes its targets from its own setup (oracle.Hierarchy), which the
FP64 GPU setup reproduces to 1e-12 (test_gpu_parity), never from the GPU."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from oracle import nn
from tests import brute_force as bf
from tests.test_gpu_parity import dev, host, rel, wc

pytestmark = pytest.mark.gpu


def flat(Ws):
    return np.concatenate([np.stack([W.real, W.imag], -1).ravel() for W in Ws]).astype(np.float32)


def unflat(w, nv, ch):
    shapes = [(9, ch, nv), (9, ch, ch), (9, nv, ch)]
    out, off = [], 0
    for s in shapes:
        n = int(np.prod(s))
        x = w[off:off + 2 * n].astype(np.float64).reshape(s + (2,))
        out.append(x[..., 0] + 1j * x[..., 1])
        off += 2 * n
    return out


def problem(L=(4, 4, 4, 8), block=(2, 2, 2, 2), nv=4, ch=8, seed=901, act=None, setup=False):
    w = wc()
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.3, seed)
    start = syn.complex_gaussian((nv, V, 12), seed + 1)
    ctx = w.Context(dims=L, m0=-0.05, c_sw=1.0, n_levels=2, block=(block,), n_vec=(nv,))
    ctx.set_gauge(dev(U))
    ctx.set_null_vectors(0, dev(start))
    H = None
    if setup:
        ctx.setup()
        H = oracle.Hierarchy(L, U, m0=-0.05, csw=1.0, n_levels=2, blocks=(block,), nv=(nv,))
        H.set_start(0, start)
        H.setup()
    net = w.Network(nv, ch, act_prec=w.F32 if act is None else act, seed=seed + 2)
    Ws = unflat(flat(nn.init_weights(nv, ch, 3, np.random.default_rng(seed + 3))), nv, ch)  # FP32-representable
    net.set_weights(flat(Ws))
    return ctx, H, net, U, start.reshape(nv, V, 4, 3), Ws, L, block


def test_weights_roundtrip_and_sizes():
    ctx, H, net, U, eta, Ws, L, block = problem()
    assert net.n_floats == 2 * 9 * (8 * 4 + 8 * 8 + 4 * 8)
    assert np.array_equal(net.weights(), flat(Ws))


@pytest.mark.parametrize("act,tol", [("f32", 1e-5), ("bf16", 3e-2)])
def test_forward_parity(act, tol):
    w = wc()
    ctx, H, net, U, eta, Ws, L, block = problem(act=w.F32 if act == "f32" else w.BF16)
    got = host(net.forward(ctx))
    ref = nn.forward(U, eta, Ws, nn.lattice_tables(L))[0][-1]
    assert rel(got, ref) < tol


@pytest.mark.parametrize("act,tol", [("f32", 1e-4), ("bf16", 8e-2)])
def test_loss_and_gradient_parity(act, tol):
    w = wc()
    ctx, H, net, U, eta, Ws, L, block = problem(act=w.F32 if act == "f32" else w.BF16, setup=True)
    tgt = H.vectors(0).reshape(eta.shape)
    ref_loss, ref_g, _ = nn.loss_and_grads(U, eta, Ws, tgt, L, block)
    loss, g = net.loss_grad(ctx)
    assert abs(loss - ref_loss) < tol * ref_loss
    ref_flat = np.concatenate([np.stack([2 * x.real, 2 * x.imag], -1).ravel() for x in ref_g])
    assert rel(g, ref_flat) < tol
    # layer by layer, so that one small layer's wrong sign cannot hide in the total
    off = 0
    for x in ref_g:
        n = 2 * x.size
        assert rel(g[off:off + n], ref_flat[off:off + n]) < tol
        off += n


def test_forward_gauge_covariance_on_gpu():
    """f(U^g, g eta) = g f(U, eta) for the GPU network (FP32 activations)."""
    w = wc()
    ctx, H, net, U, eta, Ws, L, block = problem()
    y = host(net.forward(ctx))
    g = syn.random_gauge_transform(L, 911)
    Ug = bf.gauge_transform_links(L, U, g)
    etag = np.stack([bf.gauge_transform_fermion(g, e) for e in eta])
    c2 = w.Context(dims=L, m0=-0.05, c_sw=1.0, n_levels=2, block=(block,), n_vec=(4,))
    c2.set_gauge(dev(Ug))
    c2.set_null_vectors(0, dev(etag.reshape(4, -1, 12)))
    yg = host(net.forward(c2))
    gy = np.stack([bf.gauge_transform_fermion(g, v) for v in y])
    assert rel(yg, gy) < 1e-5


def test_training_lowers_the_loss():
    w = wc()
    ctx, H, net, U, eta, Ws, L, block = problem(L=(8, 8, 8, 8), block=(4, 4, 4, 4), nv=8, ch=16, act=w.BF16,
                                                setup=True)
    losses = [net.train_step(ctx, lr=5e-3) for _ in range(25)]
    final, _ = net.loss_grad(ctx, grad=False)
    assert np.all(np.isfinite(losses))
    assert final < 0.9 * losses[0], (losses[0], final)


def test_setup_learned_and_fallback():
    """Zero weights give zero proposals: the quality check fails and the plain
    setup runs.  The initial network passes an infinite threshold; both
    hierarchies solve to 1e-10."""
    w = wc()
    ctx, H, net, U, eta, Ws, L, block = problem(L=(8, 8, 8, 8), block=(4, 4, 4, 4), nv=8, ch=16, act=w.BF16)
    b = syn.complex_gaussian((4096, 4, 3), 921)
    fb, q = ctx.setup_learned(net)
    assert not fb and np.isfinite(q) and q > 0
    x, info, st = ctx.solve(dev(b))
    assert st == 0 and info[0]["true_rel_res"] <= 1e-10
    net.set_weights(np.zeros(net.n_floats, np.float32))
    fb, q = ctx.setup_learned(net, threshold=10.0)
    assert fb
    x, info, st = ctx.solve(dev(b))
    assert st == 0 and info[0]["true_rel_res"] <= 1e-10
    with pytest.raises(w.WcmgError):
        w.Network(6, 16)  # n_vec must be a multiple of 4


def test_held_out_gain_of_trained_network():
    """Train on the plain setup's near-null vectors (20 sweeps + 2 refinement
    iterations) of six 16^4 fields, then on two held-out fields: the loss
    falls, and at equal smoothing effort (5 MR sweeps, no refinement) the
    learned proposals need fewer outer iterations than the plain setup from the
    Gaussian starts, while the untrained network gains nothing."""
    w = wc()
    L, nv, ch = (16, 16, 16, 16), 12, 32
    V = int(np.prod(L))
    eps = np.random.default_rng(931).uniform(0.2, 0.35, 8)

    def ctx_for(f, relax, refine):
        c = w.Context(dims=L, m0=-0.08, c_sw=1.0, n_levels=2, block=((4, 4, 4, 4),), n_vec=(nv,),
                      relax_sweeps=relax, refine_iters=refine, cycle_prec=w.F32, coarse_store_prec=w.F32,
                      setup_prec=w.F32, outer_restart=20, outer_maxit=2000)
        c.set_gauge(dev(syn.gauge_field(L, eps[f], 9400 + f)))
        c.set_null_vectors(0, dev(syn.start_vectors(nv, V, 12, 9500 + f)))
        return c

    train = []
    for f in range(6):
        c = ctx_for(f, 20, 2)
        c.setup()
        train.append(c)
    held = []
    for f in range(6, 8):
        c = ctx_for(f, 20, 2)
        c.setup()
        held.append(c)
    net = w.Network(nv, ch, act_prec=w.BF16, seed=7)
    w0 = net.weights()
    before = [net.loss_grad(c, grad=False)[0] for c in held]
    for _ in range(8):
        for c in train:
            net.train_step(c, lr=5e-3)
    after = [net.loss_grad(c, grad=False)[0] for c in held]
    assert all(a < 0.9 * b for a, b in zip(after, before)), (before, after)
    untrained = w.Network(nv, ch, act_prec=w.BF16, seed=7)
    untrained.set_weights(w0)
    b = dev(syn.complex_gaussian((V, 4, 3), 933))
    for f in range(6, 8):
        its = {}
        c = ctx_for(f, 5, 0)
        c.setup()
        its["plain"] = c.solve(b)[1][0]["outer_iters"]
        for name, n in (("learned", net), ("untrained", untrained)):
            c = ctx_for(f, 5, 0)
            fb, q = c.setup_learned(n, relax_sweeps=5)
            assert not fb
            x, info, st = c.solve(b)
            assert st == 0 and info[0]["true_rel_res"] <= 1e-10
            its[name] = info[0]["outer_iters"]
        assert its["learned"] < its["plain"], its
        assert abs(its["untrained"] - its["plain"]) <= 2, its
