"""GPU against the oracle, stage by stage, for the parts of the method that are
iterations rather than single operators: the iterative refinement setup and
the level recursion (Sec. 2.1), the K-cycle, the FP32 (and BF16-storage)
preconditioner the benchmark runs (Sec. 2.1, double outer solver with a
single-precision preconditioner), the FP32 setup relaxation, the lane-split
coarse apply at the launch sizes of the large lattices, the network's Adam
step, and the hierarchy a setup checkpoint rebuilds.

Both sides get the same inputs (start vectors, vectors, right-hand sides) from
the seeded generators; nothing the oracle sees comes from the GPU except where
a stage is re-synchronised on purpose (then the GPU output of one stage is the
oracle input of the next, and the test says so).

Bars: FP64 chains 1e-12 (cycle outputs 1e-11); FP32 arithmetic against the
FP64 oracle 1e-5 normwise; BF16 block storage against the oracle applied with
the same BF16-rounded blocks 1e-5; FP32 relaxation (20 MR sweeps) 2e-4 (see
the test); iteration counts within one.
"""
import numpy as np
import pytest

import oracle
import synthetic as syn
from oracle import nn as onn
from tests.test_gpu_parity import bf16_round, dev, host, make_pair, rel, wc
from tests.test_oracle_setup_pins import CFG, Levels, _with_coarse, v_cycle

pytestmark = pytest.mark.gpu

FIXED = 8  # coarse GMRES iterations without early exit: the cycle is a fixed map on both sides


def _two_level_pair(L, block, nv, seed, **kw):
    ctx, H, U = make_pair(L, 0.25, seed, m0=-0.05, blocks=(block,), nv=(nv,), coarse_fixed_iters=FIXED, **kw)
    V = int(np.prod(L))
    start = syn.complex_gaussian((nv, V, 12), seed + 1)
    ctx.set_null_vectors(0, dev(start))
    H.set_start(0, start)
    return ctx, H, U, start


def _three_level_pair(seed, kcycle=1, **kw):
    L, blocks, nv = (8, 8, 8, 8), ((2, 2, 2, 2), (2, 2, 2, 2)), (4, 4)
    ctx, H, U = make_pair(L, 0.25, seed, m0=-0.05, n_levels=3, blocks=blocks, nv=nv, kcycle=kcycle,
                          coarse_fixed_iters=FIXED, **kw)
    starts = [syn.complex_gaussian((nv[0], 4096, 12), seed + 1), syn.complex_gaussian((nv[1], 256, 8), seed + 2)]
    for l in range(2):
        ctx.set_null_vectors(l, dev(starts[l]))
        H.set_start(l, starts[l])
    return ctx, H, U, L, blocks, nv


# ---------------------------------------------------------------- refinement setup
@pytest.mark.parametrize("iters", [1, 2])
def test_refine_two_level_fp64_matches_oracle(iters):
    """wcmg_refine against the oracle's refinement (pinned by composition on
    the CPU): near-null vectors, P and D_c after 1 and 2 iterations."""
    ctx, H, U, start = _two_level_pair((4, 4, 4, 8), (2, 2, 2, 2), 6, 1301)
    ctx.setup()
    H.setup()
    assert rel(host(ctx.coarse_op(1)), H.coarse(1)) < 1e-12
    ctx.refine(iters)
    H.refine(iters)
    assert rel(host(ctx.null_vectors(0)), H.vectors(0)) < 1e-12
    assert rel(host(ctx.prolongator(0)), H.P(0)) < 1e-12
    assert rel(host(ctx.coarse_op(1)), H.coarse(1)) < 1e-12


def test_refine_two_level_resynchronised_stage():
    """One refinement stage from identical inputs: the GPU's own pre-refinement
    vectors go into the oracle (re-synchronised), so the comparison isolates
    the refinement from the setup's drift."""
    ctx, H, U, start = _two_level_pair((8, 8, 8, 8), (4, 4, 4, 4), 12, 1311)
    ctx.setup()
    v = host(ctx.null_vectors(0))
    H.set_vectors(0, v)
    ctx.rebuild_from_vectors(0, dev(v))
    ctx.refine(1)
    H.refine(1)
    assert rel(host(ctx.null_vectors(0)), H.vectors(0)) < 1e-12
    assert rel(host(ctx.coarse_op(1)), H.coarse(1)) < 1e-12


def test_three_level_setup_level_two_operator_matches_oracle():
    """Recursive coarsening: level-1 vectors relaxed on D_c1, P_1 and the
    level-2 operator D_c2 = P_1^dag D_c1 P_1 (pinned against the dense product
    on the CPU)."""
    ctx, H, U, L, blocks, nv = _three_level_pair(1321, kcycle=0)
    ctx.setup()
    H.setup()
    assert rel(host(ctx.null_vectors(1)), H.vectors(1)) < 1e-12
    assert rel(host(ctx.prolongator(1)), H.P(1)) < 1e-12
    assert rel(host(ctx.coarse_op(2)), H.coarse(2)) < 1e-12


def test_three_level_refine_matches_oracle():
    ctx, H, U, L, blocks, nv = _three_level_pair(1331, kcycle=1)
    ctx.setup()
    H.setup()
    ctx.refine(1)
    H.refine(1)
    for l in range(2):
        assert rel(host(ctx.null_vectors(l)), H.vectors(l)) < 1e-11, l
        assert rel(host(ctx.prolongator(l)), H.P(l)) < 1e-11, l
    assert rel(host(ctx.coarse_op(1)), H.coarse(1)) < 1e-11
    assert rel(host(ctx.coarse_op(2)), H.coarse(2)) < 1e-11


# ---------------------------------------------------------------- K-cycle
@pytest.mark.parametrize("kmax,ktol", [(3, 0.0), (5, 0.1)])
def test_kcycle_fp64_output_matches_oracle(kmax, ktol):
    """One K-cycle (flexible GMRES on D_c1 preconditioned by the level-1
    V-cycle; pinned as that composition on the CPU), FP64, fixed coarsest
    iterations: the cycle output to 1e-11."""
    ctx, H, U, L, blocks, nv = _three_level_pair(1341, kcycle=1, kcycle_maxit=kmax, kcycle_tol=ktol)
    ctx.setup()
    H.setup()
    r = syn.complex_gaussian((4096, 4, 3), 1344)
    assert rel(host(ctx.cycle(dev(r))), H.cycle(0, r)) < 1e-11


def test_three_level_kcycle_solve_iterations_match_oracle():
    ctx, H, U, L, blocks, nv = _three_level_pair(1351, kcycle=1, outer_restart=20, refine_iters=1)
    ctx.setup()
    H.setup()
    H.refine(1)
    b = syn.complex_gaussian((4096, 4, 3), 1354)
    x, info, st = ctx.solve(dev(b))
    xo, ito, rro, sto = H.solve(b)
    assert st == 0 and sto == 0 and info[0]["true_rel_res"] <= 1e-10
    assert abs(info[0]["outer_iters"] - ito) <= 1, (info[0]["outer_iters"], ito)
    assert rel(host(x), xo) < 1e-8


# ---------------------------------------------------------------- the FP32 preconditioner of the benchmark
@pytest.mark.parametrize("L,store", [((8, 8, 8, 8), "f32"), ((8, 8, 8, 8), "bf16"), ((16, 16, 16, 32), "f32"),
                                     ((16, 16, 16, 32), "bf16")])
def test_fp32_cycle_matches_oracle(L, store, measured):
    """The mixed-precision cycle (FP32 restriction, cooperative coarsest GMRES
    with fixed iterations, FP32 prolongation, FP32 MR post-smoothing whose
    step length is summed from the Dslash's partials, FP64 output) against the
    FP64 oracle cycle on the same hierarchy: FP32 blocks 1e-5; BF16 blocks
    against the oracle cycle composed with the same BF16-rounded blocks, 1e-5.
    16^3 x 32 with 4^4 aggregates and Nv = 12 is the benchmark's shape."""
    w = wc()
    nv, block = 12, (4, 4, 4, 4)
    V = int(np.prod(L))
    sp = w.F32 if store == "f32" else w.BF16
    ctx, H, U = make_pair(L, 0.25, 1361, m0=-0.08, blocks=(block,), nv=(nv,), coarse_fixed_iters=10,
                          cycle_prec=w.F32, coarse_store_prec=sp, setup_prec=w.F32)
    H = oracle.Hierarchy(L, U, m0=-0.08, blocks=(block,), nv=(nv,), coarse_fixed_iters=10)
    v = syn.complex_gaussian((nv, V, 12), 1362)
    ctx.set_null_vectors(0, dev(v))
    ctx.rebuild_from_vectors(0, dev(v))
    H.set_vectors(0, v)
    r = syn.complex_gaussian((V, 4, 3), 1363)
    got = host(ctx.cycle(dev(r)))
    if store == "f32":
        ref = H.cycle(0, r)
    else:
        lv = Levels(H, L, (block,), (nv,))
        cfg = dict(CFG, coarse_fixed_iters=10)
        ref = v_cycle(_with_coarse(lv, 1, bf16_round(lv.Dc[1])), 0, r.reshape(-1), cfg)
    err = rel(got, ref)
    measured("cycle_rel_err", err)
    assert err < 1e-5, err
    if store == "bf16":  # the composition with the rounded blocks explains the BF16 storage error
        e64 = rel(got, H.cycle(0, r))
        measured("cycle_rel_err_vs_unrounded_blocks", e64)
        assert err < 0.25 * e64, (err, e64)


def test_fp32_setup_relaxation_matches_oracle(measured):
    """setup_prec = F32: 20 FP32 MR sweeps per vector on D x = 0, then FP64
    Gram-Schmidt and Galerkin.  Measured differences from the FP64 oracle are
    ~2e-5 (vectors) after 20 sweeps: each sweep adds FP32 rounding (6e-8 x
    the sums) and MR's step lengths feed back; bar 2e-4."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    ctx, H, U = make_pair(L, 0.25, 1371, m0=-0.08, blocks=(block,), nv=(nv,), setup_prec=w.F32)
    start = syn.complex_gaussian((nv, 4096, 12), 1372)
    ctx.set_null_vectors(0, dev(start))
    H.set_start(0, start)
    ctx.setup()
    H.setup()
    ev = rel(host(ctx.null_vectors(0)), H.vectors(0))
    ep = rel(host(ctx.prolongator(0)), H.P(0))
    ec = rel(host(ctx.coarse_op(1)), H.coarse(1))
    measured("vectors_P_Dc_rel_err", [ev, ep, ec])
    assert ev < 2e-4 and ep < 2e-4 and ec < 2e-4, (ev, ep, ec)


def test_mixed_solve_with_refinement_iterations_match_oracle(measured):
    """The benchmark's method on 8^4 (4^4 aggregates, Nv = 12): FP32 setup
    relaxation + 1 refinement iteration, FP32 cycle with FP32 blocks, FP64
    FGMRES(20) to 1e-10, against the oracle's all-FP64 solve: outer iteration
    counts within one, solutions within 1e-8."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    ctx, H, U = make_pair(L, 0.25, 1381, m0=-0.08, blocks=(block,), nv=(nv,), refine_iters=1, outer_restart=20,
                          cycle_prec=w.F32, coarse_store_prec=w.F32, setup_prec=w.F32)
    start = syn.complex_gaussian((nv, 4096, 12), 1382)
    ctx.set_null_vectors(0, dev(start))
    H.set_start(0, start)
    ctx.setup()
    H.setup()
    H.refine(1)
    b = syn.complex_gaussian((4096, 4, 3), 1383)
    x, info, st = ctx.solve(dev(b))
    xo, ito, rro, sto = H.solve(b)
    assert st == 0 and sto == 0 and info[0]["true_rel_res"] <= 1e-10 and rro <= 1e-10
    measured("outer_iters_gpu_oracle", [info[0]["outer_iters"], ito])
    assert abs(info[0]["outer_iters"] - ito) <= 1, (info[0]["outer_iters"], ito)
    assert rel(host(x), xo) < 1e-8


# ---------------------------------------------------------------- coarse apply at the large-lattice launch sizes
@pytest.mark.parametrize("Lc", [(8, 8, 16, 16), (8, 8, 8, 16), (8, 8, 8, 8)])
def test_coarse_apply_lane_split_random_parity(Lc):
    """Nb = 24: 393,216 / 196,608 / 98,304 output rows give 1 / 2 / 4 lanes
    per row (every other random-input test runs 8); random blocks and fields
    in all three storages against the oracle."""
    w = wc()
    nb = 24
    Vc = int(np.prod(Lc))
    blocks = syn.complex_gaussian((Vc, 9, nb, nb), 1391)
    phi = syn.complex_gaussian((2, Vc, nb), 1392)
    ref = oracle.coarse_apply(Lc, blocks, phi)
    refb = oracle.coarse_apply(Lc, bf16_round(blocks), phi)
    for store in (w.F64, w.F32, w.BF16):
        op = w.CoarseOperator(Lc, nb, store)
        op.set(dev(blocks))
        op.set_kernel(1)
        if store == w.F64:
            assert rel(host(op.apply(dev(phi))), ref) < 1e-14
        else:
            got = host(op.apply(dev(phi.astype(np.complex64))))
            assert rel(got, ref if store == w.F32 else refb) < 1e-5
        op.close()


# ---------------------------------------------------------------- network optimiser
def test_nn_adam_steps_match_oracle():
    """Two training steps on the GPU against the oracle's Adam (pinned by its
    t = 1 closed form and the constant-gradient case) fed with the GPU's own
    gradients (re-synchronised: the gradients are compared with the oracle's
    elsewhere): the weights after each step, relative to the step size."""
    from tests.test_gpu_nn import problem
    ctx, H, net, U, eta, Ws, L, block = problem(setup=True)
    w = net.weights().astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    lr = 1e-2
    for t in (1, 2):
        _, g = net.loss_grad(ctx)
        net.train_step(ctx, lr=lr)
        onn.adam_step(w, g.astype(np.float64), m, v, t, lr)
        got = net.weights().astype(np.float64)
        assert np.max(np.abs(got - w)) < 1e-4 * lr, (t, np.max(np.abs(got - w)))


# ---------------------------------------------------------------- setup checkpoint
def test_checkpoint_hierarchy_matches_oracle_from_the_blob_vectors():
    """A context that imports a checkpoint holds the hierarchy the oracle
    builds from the vectors stored in the blob (read from the documented
    layout: complex128 [nv][V][12] after the 128-byte header)."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    V = 4096
    U = syn.gauge_field(L, 0.25, 1401)
    A = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), refine_iters=1)
    A.set_gauge(dev(U))
    A.set_null_vectors(0, dev(syn.complex_gaussian((nv, V, 12), 1402)))
    A.setup()
    blob = A.export_setup()
    vecs = np.frombuffer(bytes(blob[128:128 + nv * V * 12 * 16]), dtype=np.complex128).reshape(nv, V, 12)
    B = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,))
    B.set_gauge(dev(U))
    B.import_setup(blob)
    H = oracle.Hierarchy(L, U, m0=-0.05, blocks=(block,), nv=(nv,))
    H.set_vectors(0, vecs)
    assert rel(host(B.prolongator(0)), H.P(0)) < 1e-12
    assert rel(host(B.coarse_op(1)), H.coarse(1)) < 1e-12


# ---------------------------------------------------------------- singular coarse operator
@pytest.mark.parametrize("mode", ["f64", "f32", "f32_four_kernel"])
def test_cycle_with_a_zero_coarse_operator_stays_finite(mode):
    """A zero coarse operator: the coarsest GMRES meets a vanishing rotated
    Hessenberg column at its first step and must return x_c = 0 (the
    least-squares minimiser), so the cycle is the post-smoother alone, as in
    the oracle's composition; no division by the zero diagonal."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    kw = dict(coarse_fixed_iters=0)
    if mode != "f64":
        kw.update(cycle_prec=w.F32, coarse_store_prec=w.F32, setup_prec=w.F32)
    if mode == "f32_four_kernel":
        kw.update(reserved=(4,))
    ctx, H, U = make_pair(L, 0.25, 1411, m0=-0.08, blocks=(block,), nv=(nv,), **kw)
    v = syn.complex_gaussian((nv, 4096, 12), 1412)
    ctx.set_null_vectors(0, dev(v))
    ctx.rebuild_from_vectors(0, dev(v))
    H.set_vectors(0, v)
    ctx.set_coarse_op(1, dev(np.zeros((16, 9, 24, 24), np.complex128)))
    r = syn.complex_gaussian((4096, 4, 3), 1413)
    got = host(ctx.cycle(dev(r)))
    assert np.all(np.isfinite(got))
    lv = Levels(H, L, (block,), (nv,))
    ref = v_cycle(_with_coarse(lv, 1, np.zeros((16, 9, 24, 24), np.complex128)), 0, r.reshape(-1), CFG)
    assert rel(got, ref) < (1e-12 if mode == "f64" else 1e-5)
