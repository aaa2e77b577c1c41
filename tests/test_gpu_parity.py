"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bars: integer maps bit-exact; FP64 results within 1e-12 normwise relative;
FP32 arithmetic within 1e-5; BF16-stored coarse blocks compared with the
oracle applied to the same BF16-rounded blocks, within 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
import synthetic as syn
from tests import brute_force as bf

pytestmark = pytest.mark.gpu


def wc():
    import paper_1904_08678_amd as w
    return w


def rel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def bf16_round(x):
    """FP64 -> FP32 -> BF16 (round to nearest even), returned as FP64."""
    def r(a):
        f = np.ascontiguousarray(a, dtype=np.float32)
        u = f.view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    return r(x.real) + 1j * r(x.imag)


def make_pair(L, eps, seed, m0=-0.05, csw=1.0, blocks=((2, 2, 2, 2),), nv=(4,), n_levels=2, **kw):
    """GPU context and oracle hierarchy built from the same parameters and inputs."""
    w = wc()
    U = syn.gauge_field(L, eps, seed)
    gkw = dict(dims=L, m0=m0, c_sw=csw, n_levels=n_levels, block=blocks, n_vec=nv)
    okw = dict(m0=m0, csw=csw, n_levels=n_levels, blocks=blocks, nv=nv)
    for k, v in kw.items():
        gkw[k] = v
        if k in oracle.DEFAULTS:
            okw[k] = v
    ctx = w.Context(**gkw)
    ctx.set_gauge(dev(U))
    H = oracle.Hierarchy(L, U, **okw)
    return ctx, H, U


# ---------------------------------------------------------------- aggregation map
@pytest.mark.parametrize("L,block", [((8, 4, 4, 8), (4, 2, 2, 4)), ((4, 6, 4, 8), (2, 3, 2, 2))])
def test_aggregation_map_bit_exact(L, block):
    w = wc()
    ctx = w.Context(dims=L, n_levels=2, block=(block,), n_vec=(4,))
    c, o = ctx.aggregate_map(0)
    oc, oo, _ = oracle.agg_map(L, block)
    assert np.array_equal(c, oc) and np.array_equal(o, oo)


def test_aggregation_map_second_level_bit_exact():
    w = wc()
    L = (8, 8, 8, 16)
    ctx = w.Context(dims=L, n_levels=3, block=((2, 2, 2, 2), (2, 2, 2, 4)), n_vec=(4, 4))
    c, o = ctx.aggregate_map(1)
    oc, oo, _ = oracle.agg_map((4, 4, 4, 8), (2, 2, 2, 4))
    assert np.array_equal(c, oc) and np.array_equal(o, oo)


def test_dims_errors():
    w = wc()
    with pytest.raises(w.WcmgError) as e:
        w.Context(dims=(6, 4, 4, 4), n_levels=2, block=((4, 2, 2, 2),), n_vec=(4,))
    assert e.value.code == 2
    with pytest.raises(w.WcmgError) as e:
        w.Context(dims=(4, 4, 4, 4), n_levels=2, block=((4, 2, 2, 2),), n_vec=(4,))  # coarse extent 1
    assert e.value.code == 2


# ---------------------------------------------------------------- clover term and Wilson-clover operator
def test_clover_fp64_parity():
    L = (4, 4, 4, 8)
    ctx, H, U = make_pair(L, 0.3, 201)
    C = oracle.clover(L, U, 1.0)
    ref = np.stack([C[:, :6, :6], C[:, 6:, 6:]], axis=1)
    got = host(ctx.get_clover())
    assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("L,block", [((4, 4, 4, 8), (2, 2, 2, 2)), ((4, 6, 4, 8), (2, 3, 2, 4))])
def test_dslash_parity(L, block):
    w = wc()
    ctx, H, U = make_pair(L, 0.3, 202, m0=-0.08, blocks=(block,))
    V = int(np.prod(L))
    psi = syn.complex_gaussian((3, V, 4, 3), 203)
    ref = np.stack([H.apply(0, psi[r]).reshape(V, 4, 3) for r in range(3)])
    got64 = host(ctx.apply_D(0, dev(psi), w.F64))
    assert rel(got64, ref) < 1e-13
    got32 = host(ctx.apply_D(0, dev(psi.astype(np.complex64)), w.F32))
    assert rel(got32, ref) < 1e-5


@pytest.mark.parametrize("nrhs", [2, 5, 16])
def test_dslash_multi_rhs_fp32_ragged(nrhs):
    """FP32 Dslash on several right-hand sides in one launch (links and clover
    staged once per workgroup) on a lattice whose volume (210) leaves a ragged
    last workgroup: against the oracle and against one launch per field."""
    w = wc()
    L = (3, 5, 2, 7)
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.3, 211)
    ctx = w.Context(dims=L, m0=-0.08, c_sw=1.0, n_levels=1)
    ctx.set_gauge(dev(U))
    H = oracle.Hierarchy(L, U, m0=-0.08, csw=1.0, n_levels=1, blocks=())
    psi = syn.complex_gaussian((nrhs, V, 4, 3), 212)
    ref = np.stack([H.apply(0, psi[r]).reshape(V, 4, 3) for r in range(nrhs)])
    x32 = psi.astype(np.complex64)
    got = host(ctx.apply_D(0, dev(x32), w.F32))
    assert rel(got, ref) < 1e-5
    one = np.stack([host(ctx.apply_D(0, dev(x32[r:r + 1]), w.F32))[0] for r in range(nrhs)])
    assert rel(got, one) < 1e-6


def test_dslash_single_point_source_response():
    """A point source picks out one column of D: diagonal block plus 8 hops."""
    w = wc()
    L = (4, 4, 4, 4)
    ctx, H, U = make_pair(L, 0.3, 204)
    e = np.zeros((256, 4, 3), np.complex128)
    e[37, 2, 1] = 1.0
    got = host(ctx.apply_D(0, dev(e), w.F64))
    ref = H.apply(0, e).reshape(256, 4, 3)
    assert rel(got, ref) < 1e-14
    assert np.count_nonzero(np.abs(got).sum(axis=(1, 2)) > 1e-15) == 9


# ---------------------------------------------------------------- coarse operator apply
@pytest.mark.parametrize("Lc,nb", [((3, 2, 4, 3), 8), ((2, 2, 2, 2), 16), ((4, 4, 4, 8), 24), ((3, 3, 2, 2), 32),
                                    ((2, 3, 2, 2), 6)])
def test_coarse_apply_parity_all_precisions(Lc, nb):
    w = wc()
    Vc = int(np.prod(Lc))
    blocks = syn.complex_gaussian((Vc, 9, nb, nb), 301)
    phi = syn.complex_gaussian((2, Vc, nb), 302)
    ref = oracle.coarse_apply(Lc, blocks, phi)
    for store in (w.F64, w.F32, w.BF16):
        if store == w.BF16 and nb % 4:
            with pytest.raises(w.WcmgError):
                w.CoarseOperator(Lc, nb, store)
            continue
        op = w.CoarseOperator(Lc, nb, store)
        op.set(dev(blocks))
        if store == w.F64:
            got = host(op.apply(dev(phi)))
            assert rel(got, ref) < 1e-14
        elif store == w.F32:
            got = host(op.apply(dev(phi.astype(np.complex64))))
            assert rel(got, ref) < 1e-5
        else:
            ref_b = oracle.coarse_apply(Lc, bf16_round(blocks), phi)
            got = host(op.apply(dev(phi.astype(np.complex64))))
            assert rel(got, ref_b) < 1e-5
            assert rel(got, ref) < 2e-2  # storage error of BF16 alone


# ---------------------------------------------------------------- setup
@pytest.mark.parametrize("L,block,nv,m0", [((4, 4, 4, 4), (2, 2, 2, 2), 8, -0.05), ((8, 8, 8, 8), (4, 4, 4, 4), 12, -0.08)])
def test_setup_fp64_parity(L, block, nv, m0):
    """Relaxation (MR on D x = 0), chirality-split Gram-Schmidt and Galerkin
    coarsening from identical start vectors: vectors, P and D_c to 1e-12."""
    ctx, H, U = make_pair(L, 0.3, 401, m0=m0, blocks=(block,), nv=(nv,))
    V = int(np.prod(L))
    start = syn.complex_gaussian((nv, V, 12), 402)
    ctx.set_null_vectors(0, dev(start))
    H.set_start(0, start)
    ctx.setup()
    H.setup()
    assert rel(host(ctx.null_vectors(0)), H.vectors(0)) < 1e-12
    assert rel(host(ctx.prolongator(0)), H.P(0)) < 1e-12
    assert rel(host(ctx.coarse_op(1)), H.coarse(1)) < 1e-12


def test_galerkin_from_given_vectors_parity():
    """Coarsening alone: the same near-null vectors in, D_c out (1e-12)."""
    L, block, nv = (4, 4, 4, 8), (2, 2, 2, 4), 6
    ctx, H, U = make_pair(L, 0.3, 403, blocks=(block,), nv=(nv,))
    V = int(np.prod(L))
    vecs = syn.complex_gaussian((nv, V, 12), 404)
    ctx.set_null_vectors(0, dev(vecs))
    ctx.rebuild_from_vectors(0, dev(vecs))
    H.set_start(0, vecs)
    H.setup()
    H.set_vectors(0, vecs)
    assert rel(host(ctx.prolongator(0)), H.P(0)) < 1e-12
    got = host(ctx.coarse_op(1))
    assert rel(got, H.coarse(1)) < 1e-12
    Dc = bf.dense_from_blocks((2, 2, 2, 2), got)
    s3 = np.kron(np.eye(16), np.diag([1.0] * nv + [-1.0] * nv))
    assert np.max(np.abs(s3 @ Dc @ s3 - Dc.conj().T)) < 1e-12 * np.max(np.abs(Dc))


def test_breakdown_reported():
    w = wc()
    L, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    ctx, H, U = make_pair(L, 0.3, 405, blocks=(block,), nv=(nv,))
    vecs = syn.complex_gaussian((nv, 256, 12), 406)
    vecs[2] = 3.0 * vecs[0]
    with pytest.raises(w.WcmgError) as e:
        ctx.rebuild_from_vectors(0, dev(vecs))
    assert e.value.code == 6


# ---------------------------------------------------------------- restriction and prolongation
@pytest.mark.parametrize("L,block,nrhs", [((8, 4, 4, 8), (4, 2, 2, 4), 2), ((6, 4, 4, 6), (3, 2, 2, 2), 5)])
def test_restrict_prolong_parity(L, block, nrhs):
    """GPU and oracle build P from the same start vectors; each restricts and
    prolongs with its own P.  The second case leaves (aggregates x fields) and
    (site blocks x fields) off a multiple of 8 (padded launch grids)."""
    w = wc()
    nv = 6
    ctx, H, U = make_pair(L, 0.3, 501, blocks=(block,), nv=(nv,))
    V = int(np.prod(L))
    start = syn.complex_gaussian((nv, V, 12), 502)
    ctx.set_null_vectors(0, dev(start))
    ctx.setup()
    H.set_start(0, start)
    H.setup()
    Pv = H.P(0)
    v = syn.complex_gaussian((nrhs, V, 12), 503)
    ref = oracle.restrict(L, block, 12, Pv, v)
    assert rel(host(ctx.restrict(0, dev(v), w.F64)), ref) < 1e-12
    assert rel(host(ctx.restrict(0, dev(v.astype(np.complex64)), w.F32)), ref) < 1e-5
    Vc = V // int(np.prod(block))
    phi = syn.complex_gaussian((nrhs, Vc, 2 * nv), 504)
    ref = oracle.prolong(L, block, 12, Pv, phi)
    assert rel(host(ctx.prolong(0, dev(phi), w.F64)), ref) < 1e-12
    assert rel(host(ctx.prolong(0, dev(phi.astype(np.complex64)), w.F32)), ref) < 1e-5
    # R P = 1
    rp = host(ctx.restrict(0, ctx.prolong(0, dev(phi), w.F64), w.F64))
    assert rel(rp, phi) < 1e-13


def test_coarse_level_apply_parity():
    """The level-1 operator: GPU-built D_c applied in FP64/FP32 against the
    oracle's own D_c; BF16 storage with the oracle's blocks injected."""
    w = wc()
    L, block, nv = (4, 4, 4, 8), (2, 2, 2, 2), 8
    ctx, H, U = make_pair(L, 0.3, 505, blocks=(block,), nv=(nv,))
    start = syn.complex_gaussian((nv, 512, 12), 506)
    ctx.set_null_vectors(0, dev(start))
    ctx.setup()
    H.set_start(0, start)
    H.setup()
    blocks = H.coarse(1)
    Lc = (2, 2, 2, 4)
    phi = syn.complex_gaussian((2, 32, 16), 507)
    ref = oracle.coarse_apply(Lc, blocks, phi)
    assert rel(host(ctx.apply_D(1, dev(phi), w.F64)), ref) < 1e-12
    assert rel(host(ctx.apply_D(1, dev(phi.astype(np.complex64)), w.F32)), ref) < 1e-5
    ctx.set_coarse_op(1, dev(blocks))
    refb = oracle.coarse_apply(Lc, bf16_round(blocks), phi)
    assert rel(host(ctx.apply_D(1, dev(phi.astype(np.complex64)), w.BF16)), refb) < 1e-5


# ---------------------------------------------------------------- cycle and solve
def test_cycle_fp64_parity_fixed_coarse_iterations():
    L, block, nv = (4, 4, 4, 8), (2, 2, 2, 2), 8
    ctx, H, U = make_pair(L, 0.3, 601, blocks=(block,), nv=(nv,), coarse_fixed_iters=12)
    V = 512
    start = syn.complex_gaussian((nv, V, 12), 602)
    ctx.set_null_vectors(0, dev(start))
    H.set_start(0, start)
    ctx.setup()
    H.setup()
    r = syn.complex_gaussian((V, 4, 3), 603)
    got = host(ctx.cycle(dev(r)))
    ref = H.cycle(0, r).reshape(V, 4, 3)
    assert rel(got, ref) < 1e-11


def test_solve_fp64_config1():
    """Config 1: 4^4, 2^4 aggregates, Nv 8, MR(4), FGMRES(16) to 1e-10."""
    L = (4, 4, 4, 4)
    ctx, H, U = make_pair(L, 0.3, 101, m0=-0.05, blocks=((2, 2, 2, 2),), nv=(8,), outer_restart=16)
    start = syn.complex_gaussian((8, 256, 12), 102)
    ctx.set_null_vectors(0, dev(start))
    H.set_start(0, start)
    ctx.setup()
    H.setup()
    b = syn.complex_gaussian((256, 4, 3), 103)
    x, info, st = ctx.solve(dev(b))
    xo, ito, rro, sto = H.solve(b)
    assert st == 0 and info[0]["converged"] and info[0]["true_rel_res"] <= 1e-10
    assert abs(info[0]["outer_iters"] - ito) <= 1
    xg = host(x).reshape(-1)
    # both are solutions to 1e-10; their difference is bounded by the conditioning
    assert rel(xg, xo) < 1e-8
    r = b.reshape(-1) - H.apply(0, xg)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)


def test_solve_mixed_precision_bf16_blocks():
    """FP32 cycle with BF16-stored coarse blocks under the FP64 outer FGMRES:
    the true residual still reaches 1e-10 (the outer solver refines)."""
    w = wc()
    L = (8, 8, 8, 8)
    ctx, H, U = make_pair(L, 0.25, 701, m0=-0.05, blocks=((4, 4, 4, 4),), nv=(12,), cycle_prec=w.F32,
                          coarse_store_prec=w.BF16, setup_prec=w.F32)
    ctx.set_null_vectors(0, dev(syn.complex_gaussian((12, 4096, 12), 702)))
    ctx.setup()
    b = syn.complex_gaussian((4096, 4, 3), 703)
    x, info, st = ctx.solve(dev(b))
    assert st == 0 and info[0]["true_rel_res"] <= 1e-10
    r = b.reshape(-1) - H.apply(0, host(x).reshape(-1))
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)


def test_three_level_kcycle_solve():
    w = wc()
    L = (8, 8, 8, 8)
    ctx, H, U = make_pair(L, 0.25, 111, m0=-0.05, n_levels=3, blocks=((2, 2, 2, 2), (2, 2, 2, 2)), nv=(6, 6),
                          kcycle=1, outer_restart=20)
    ctx.set_null_vectors(0, dev(syn.complex_gaussian((6, 4096, 12), 112)))
    ctx.set_null_vectors(1, dev(syn.complex_gaussian((6, 256, 12), 114)))
    ctx.setup()
    ctx.refine(1)
    b = syn.complex_gaussian((4096, 4, 3), 113)
    x, info, st = ctx.solve(dev(b))
    assert st == 0 and info[0]["true_rel_res"] <= 1e-10


def test_state_errors():
    w = wc()
    ctx = w.Context(dims=(4, 4, 4, 4), n_levels=2, block=((2, 2, 2, 2),), n_vec=(4,))
    with pytest.raises(w.WcmgError) as e:
        ctx.setup()  # no gauge field
    assert e.value.code == 3
    ctx.set_gauge(dev(syn.gauge_field((4, 4, 4, 4), 0.3, 1)))
    with pytest.raises(w.WcmgError) as e:
        ctx.solve(dev(np.ones((256, 4, 3), np.complex128)))
    assert e.value.code == 3


@pytest.mark.parametrize("fixed", [0, 9])
def test_fused_coarse_gmres_matches_generic_path(fixed):
    """The four-kernel Arnoldi step of the coarsest GMRES and the generic
    multi-kernel path give the same cycle output (FP64) and solve."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    U = syn.gauge_field(L, 0.25, 801)
    start = syn.complex_gaussian((nv, 4096, 12), 802)
    r = syn.complex_gaussian((4096, 4, 3), 803)
    outs, infos = [], []
    for flags in (0, 2):
        ctx = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), coarse_fixed_iters=fixed,
                        reserved=(flags,))
        ctx.set_gauge(dev(U))
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        outs.append(host(ctx.cycle(dev(r))))
        x, info, st = ctx.solve(dev(r))
        assert st == 0
        infos.append(info[0])
    assert rel(outs[0], outs[1]) < 1e-11
    assert abs(infos[0]["outer_iters"] - infos[1]["outer_iters"]) <= 1
    assert abs(infos[0]["coarse_iters"] - infos[1]["coarse_iters"]) <= max(2, infos[1]["coarse_iters"] // 50)


@pytest.mark.parametrize("L,block,store,nv", [((8, 8, 8, 8), (4, 4, 4, 4), "f32", 12),
                                              ((8, 8, 8, 8), (4, 4, 4, 4), "bf16", 12),
                                              ((8, 8, 8, 8), (4, 4, 4, 4), "bf16", 16),
                                              ((16, 16, 16, 16), (4, 4, 4, 4), "f32", 12),
                                              ((16, 16, 16, 32), (4, 4, 4, 4), "f32", 12),
                                              ((6, 6, 6, 6), (2, 2, 2, 2), "f32", 12)])
def test_cooperative_coarse_gmres_matches_multi_kernel_path(L, block, store, nv):
    """The coarsest GMRES as one cooperative launch (blocks resident in LDS,
    grid barriers) against the multi-kernel form (reserved[0] flag 4): the
    FP32 cycle with 10 fixed coarse iterations agrees to FP32 rounding and
    repeats bit for bit (every grid reduction is summed in a fixed order, so
    a repeat that differs means a workgroup read data of the wrong phase),
    and mixed solves agree in outer and coarse iteration counts (within one
    step).  Coarse lattices of 16 (Nb 24 and, with BF16 blocks, 32), 256,
    512 and 81 sites (the last with a partly filled final workgroup)."""
    w = wc()
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.25, 821)
    start = syn.complex_gaussian((nv, V, 12), 822)
    r = syn.complex_gaussian((V, 4, 3), 823)
    sp = w.F32 if store == "f32" else w.BF16
    outs, infos = [], []
    for flags in (0, 4):
        kw = dict(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), cycle_prec=w.F32, coarse_store_prec=sp,
                  setup_prec=w.F32, reserved=(flags,))
        ctx = w.Context(coarse_fixed_iters=10, **kw)
        ctx.set_gauge(dev(U))
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        outs.append(host(ctx.cycle(dev(r.astype(np.complex128)))))
        assert np.array_equal(host(ctx.cycle(dev(r.astype(np.complex128)))), outs[-1])
        ctx = w.Context(**kw)
        ctx.set_gauge(dev(U))
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        ctx.profile("coarse_gmres_persistent", True)
        x, info, st = ctx.solve(dev(r))
        assert st == 0 and info[0]["true_rel_res"] <= 1e-10
        assert ctx.timers()["coarse_solve_fallbacks"] == 0, w.lib().wcmg_last_error(ctx.h)
        launches = ctx.profile_stats("coarse_gmres_persistent")[0]
        assert (launches > 0) == (flags == 0), launches
        infos.append(info[0])
    assert rel(outs[0], outs[1]) < 2e-5
    assert abs(infos[0]["outer_iters"] - infos[1]["outer_iters"]) <= 1
    assert abs(infos[0]["coarse_iters"] - infos[1]["coarse_iters"]) <= max(2, infos[1]["coarse_iters"] // 50)


@pytest.mark.parametrize("restart,tol,fixed", [(4, 1e-4, 0), (40, 0.05, 0), (6, 0.05, 15)])
def test_cooperative_coarse_gmres_restart_cycles(restart, tol, fixed):
    """Restart cycles inside the cooperative launch (x complete, residual
    recomputed from A x, new shift, y solved per cycle): restart 4 to 1e-4
    (several cycles per coarse solve), restart 40 (every LDS array at its
    largest), and 15 fixed iterations over restarts of 6; the cycle output
    against the four-kernel form to FP32 rounding and bit-identical on repeat,
    solves with the same outer iteration counts (within one)."""
    w = wc()
    L, block, nv = (16, 16, 16, 16), (4, 4, 4, 4), 12
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.25, 1961)
    start = syn.complex_gaussian((nv, V, 12), 1962)
    r = syn.complex_gaussian((V, 4, 3), 1963)
    outs, its = [], []
    for flags in (0, 4):
        kw = dict(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), cycle_prec=w.F32,
                  coarse_store_prec=w.F32, setup_prec=w.F32, reserved=(flags,), coarse_restart=restart,
                  coarse_tol=tol, coarse_maxit=200, coarse_fixed_iters=fixed)
        ctx = w.Context(**kw)
        ctx.set_gauge(dev(U))
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        outs.append(host(ctx.cycle(dev(r.astype(np.complex128)))))
        assert np.array_equal(host(ctx.cycle(dev(r.astype(np.complex128)))), outs[-1])
        x, info, st = ctx.solve(dev(r))
        assert st == 0 and info[0]["true_rel_res"] <= 1e-10
        assert ctx.timers()["coarse_solve_fallbacks"] == 0, w.lib().wcmg_last_error(ctx.h)
        its.append(info[0])
    assert rel(outs[0], outs[1]) < 5e-5
    assert abs(its[0]["outer_iters"] - its[1]["outer_iters"]) <= 1


def test_cooperative_coarse_gmres_timeout_falls_back():
    """Barrier waits that give up at once (reserved[0] flag 16; every kernel
    still exits normally): each cooperative coarsest solve reports no
    completion, the host clears the barrier flags and redoes it with the
    four-kernel form, so the solve equals the four-kernel solve; the
    fallbacks are counted and the last one is described."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.25, 1941)
    start = syn.complex_gaussian((nv, V, 12), 1942)
    b = syn.complex_gaussian((V, 4, 3), 1943)
    res = []
    for flags in (16, 4, 0):
        ctx = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), cycle_prec=w.F32,
                        coarse_store_prec=w.F32, setup_prec=w.F32, reserved=(flags,))
        ctx.set_gauge(dev(U))
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        x, info, st = ctx.solve(dev(b))
        assert st == 0 and info[0]["true_rel_res"] <= 1e-10
        res.append((host(x), info[0], ctx.timers()["coarse_solve_fallbacks"], w.lib().wcmg_last_error(ctx.h)))
    (x16, i16, f16, e16), (x4, i4, f4, _), (x0, i0, f0, _) = res
    assert f16 > 0 and f4 == 0 and f0 == 0
    assert b"timed out" in e16, e16
    assert np.array_equal(x16, x4) and i16["outer_iters"] == i4["outer_iters"]
    assert i16["coarse_iters"] == i4["coarse_iters"]
    # the cooperative form itself agrees with both
    assert abs(i0["outer_iters"] - i4["outer_iters"]) <= 1


def test_persistent_coarse_gmres_launch_forms_agree():
    """The persistent coarsest GMRES launched as an ordinary kernel (the
    default) and through the cooperative-launch API (reserved[0] flag 256):
    the same kernel and grid, so the solves are bit-identical, with the same
    outer and coarse iteration counts and no barrier time-out."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.25, 1951)
    start = syn.complex_gaussian((nv, V, 12), 1952)
    b = syn.complex_gaussian((V, 4, 3), 1953)
    res = []
    for flags in (0, 256):
        ctx = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), cycle_prec=w.F32,
                        coarse_store_prec=w.F32, setup_prec=w.F32, reserved=(flags,))
        ctx.set_gauge(dev(U))
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        x, info, st = ctx.solve(dev(b))
        assert st == 0 and info[0]["true_rel_res"] <= 1e-10
        assert ctx.timers()["coarse_solve_fallbacks"] == 0
        res.append((host(x), info[0]))
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1]["outer_iters"] == res[1][1]["outer_iters"]
    assert res[0][1]["coarse_iters"] == res[1][1]["coarse_iters"] > 0


def test_cooperative_coarse_gmres_late_check_after_timeout():
    """The host checks a cooperative coarsest solve only at the next progress
    check.  reserved[0] flag 128 makes the first launch's waits give up at
    once (every kernel still exits normally): that launch and the ones queued
    after it before the check return x = 0 (a weaker preconditioner for those
    outer steps), the check counts them, clears the barrier words and
    describes the time-out, and the later launches run normally.  The solve
    still reaches 1e-10 in about the iterations of the unforced solve, and a
    second solve on the context has no fallback."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.25, 1941)
    start = syn.complex_gaussian((nv, V, 12), 1942)
    b = syn.complex_gaussian((V, 4, 3), 1943)
    res = []
    for flags in (128, 0):
        ctx = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), cycle_prec=w.F32,
                        coarse_store_prec=w.F32, setup_prec=w.F32, reserved=(flags,))
        ctx.set_gauge(dev(U))
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        x, info, st = ctx.solve(dev(b))
        assert st == 0 and info[0]["true_rel_res"] <= 1e-10
        f1 = ctx.timers()["coarse_solve_fallbacks"]
        err = w.lib().wcmg_last_error(ctx.h)
        x2, info2, st2 = ctx.solve(dev(b))
        assert st2 == 0 and info2[0]["true_rel_res"] <= 1e-10
        f2 = ctx.timers()["coarse_solve_fallbacks"] - f1
        res.append((host(x), info[0], f1, err, f2, info2[0]))
    (x128, i128, f128, e128, g128, j128), (x0, i0, f0, _, g0, j0) = res
    assert f128 >= 1 and f0 == 0 and g128 == 0 and g0 == 0
    assert b"timed out" in e128, e128
    assert i128["outer_iters"] <= i0["outer_iters"] + 3
    # after the recovery the cooperative form runs as in a fresh context
    assert j128["outer_iters"] == j0["outer_iters"]


@pytest.mark.parametrize("levels,mixed,eo,restart", [(2, True, 0, 20), (2, False, 0, 20), (1, False, 0, 20),
                                                     (2, True, 1, 20), (2, True, 0, 5), (1, False, 0, 7)])
def test_single_reduction_outer_step_matches_cgs2(levels, mixed, eo, restart):
    """The outer FGMRES with one reduction per Arnoldi step (shifted vector,
    norm from |w'|^2 - |h|^2, second projection only on heavy cancellation,
    which the unshifted first step of every cycle takes) against classical
    Gram-Schmidt applied twice (reserved[0] flag 8): same outer iteration
    counts, solutions equal to 1e-12, both to the 1e-10 target.  Two-level
    mixed and FP64, one level (unpreconditioned GMRES), even-odd, and short
    restarts (several restart cycles, each with its own shift)."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.25, 1931)
    start = syn.complex_gaussian((nv, V, 12), 1932)
    b = syn.complex_gaussian((V, 4, 3), 1933)
    xs, infos = [], []
    for flags in (0, 8):
        kw = dict(dims=L, m0=-0.05 if levels > 1 else 0.3, n_levels=levels, block=(block,), n_vec=(nv,),
                  even_odd=eo, reserved=(flags,), outer_maxit=4000, outer_restart=restart)
        if mixed:
            kw.update(cycle_prec=w.F32, coarse_store_prec=w.F32, setup_prec=w.F32)
        ctx = w.Context(**kw)
        ctx.set_gauge(dev(U))
        if levels > 1:
            ctx.set_null_vectors(0, dev(start))
            ctx.setup()
        x, info, st = ctx.solve(dev(b))
        assert st == 0 and info[0]["true_rel_res"] <= 1e-10
        xs.append(host(x))
        infos.append(info[0])
    assert infos[0]["outer_iters"] == infos[1]["outer_iters"], (infos[0]["outer_iters"], infos[1]["outer_iters"])
    assert rel(xs[0], xs[1]) < 1e-12


@pytest.mark.parametrize("Lc,nb,nrhs", [((2, 2, 2, 2), 8, 12), ((3, 2, 2, 4), 16, 5), ((4, 4, 4, 8), 24, 12),
                                         ((2, 3, 2, 2), 24, 16), ((3, 3, 2, 2), 32, 12), ((2, 2, 2, 2), 40, 17)])
def test_coarse_apply_matrix_cores_parity(Lc, nb, nrhs):
    """Batched coarse apply on the matrix cores (complex GEMM per site and
    direction) against the oracle, FP32 and BF16 storage; also equal to the
    per-row vector kernel on the same inputs."""
    w = wc()
    Vc = int(np.prod(Lc))
    blocks = syn.complex_gaussian((Vc, 9, nb, nb), 311)
    phi = syn.complex_gaussian((nrhs, Vc, nb), 312)
    for store in (w.F32, w.BF16):
        op = w.CoarseOperator(Lc, nb, store)
        op.set(dev(blocks))
        ref = oracle.coarse_apply(Lc, blocks if store == w.F32 else bf16_round(blocks), phi)
        x = dev(phi.astype(np.complex64))
        op.set_kernel(2)
        got = host(op.apply(x))
        assert rel(got, ref) < 1e-5
        op.set_kernel(1)
        got1 = host(op.apply(x))
        assert rel(got, got1) < 1e-5


@pytest.mark.parametrize("Lc,nb,nrhs", [((16, 2, 2, 2), 24, 12), ((8, 3, 2, 3), 16, 5), ((4, 2, 2, 2), 40, 16),
                                         ((8, 2, 2, 2), 8, 3), ((16, 2, 2, 2), 32, 16), ((8, 2, 2, 3), 24, 1)])
def test_coarse_apply_mfma_tiles(Lc, nb, nrhs):
    """Matrix-core tiles: one wave per site (tile 0) and 4, 8 or 16 sites of an
    x-row per workgroup with the neighbour vectors staged in LDS give the same
    result bit for bit (same products in the same order), with the outputs
    stored through LDS (4, 8, 16) or per wave (5, 9); tile 0 against the
    oracle; tiles that do not divide Lx are refused; the tuned default records
    every tile that fits and picks one of them."""
    w = wc()
    Vc = int(np.prod(Lc))
    blocks = syn.complex_gaussian((Vc, 9, nb, nb), 331)
    phi = syn.complex_gaussian((nrhs, Vc, nb), 332)
    x = dev(phi.astype(np.complex64))
    for store in (w.F32, w.BF16):
        op = w.CoarseOperator(Lc, nb, store)
        op.set(dev(blocks))
        op.set_kernel(2)
        op.set_tile(0)
        base = host(op.apply(x))
        ref = oracle.coarse_apply(Lc, blocks if store == w.F32 else bf16_round(blocks), phi)
        assert rel(base, ref) < 1e-5
        for tile in (4, 8, 16, 5, 9):
            if Lc[0] % (tile & ~1):
                with pytest.raises(w.WcmgError):
                    op.set_tile(tile)
                continue
            op.set_tile(tile)
            got = host(op.apply(x))
            assert np.array_equal(got, base), (store, tile, rel(got, base))
        op.set_tile(-1)
        got = host(op.apply(x))
        assert np.array_equal(got, base)
        table = op.tune_table()
        keys = [k for k in table if "coarse_mfma_tile" in k and ("nrhs=%d" % min(nrhs, 16)) in k]
        assert len(keys) == 1, table
        ent = table[keys[0]]
        fits = [t == 0 or Lc[0] % (t & ~1) == 0 for t in (0, 4, 8, 16, 5, 9)]
        assert [m >= 0 for m in ent["ms"]] == fits and fits[ent["choice"]], ent


@pytest.mark.parametrize("L,block,levels", [((8, 4, 4, 8), (4, 2, 2, 4), 2), ((6, 4, 6, 6), (2, 2, 2, 2), 2),
                                            ((4, 6, 4, 8), (2, 3, 2, 4), 2), ((3, 5, 2, 7), (1, 1, 1, 1), 1)])
def test_dslash_site_arithmetic_equals_neighbour_table(L, block, levels):
    """The Dslash finds its neighbours from the aggregate-major site
    arithmetic; the table form (reserved[0] flag 32) reads them from the
    neighbour table.  Same arithmetic otherwise: bit-identical outputs, FP64
    and FP32, several right-hand sides, and the residual form through a solve."""
    w = wc()
    U = syn.gauge_field(L, 0.3, 231)
    V = int(np.prod(L))
    psi = syn.complex_gaussian((3, V, 4, 3), 232)
    outs = []
    for flags in (64, 32):  # full links: site arithmetic against the table
        ctx = w.Context(dims=L, m0=-0.08, n_levels=levels, block=(block,), n_vec=(4,), reserved=(flags,))
        ctx.set_gauge(dev(U))
        assert ctx.timers()["dslash_link_rows"] == 3
        outs.append((host(ctx.apply_D(0, dev(psi), w.F64)), host(ctx.apply_D(0, dev(psi.astype(np.complex64)), w.F32))))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    H = oracle.Hierarchy(L, U, m0=-0.08, n_levels=1, blocks=())
    ref = np.stack([H.apply(0, psi[r]).reshape(V, 4, 3) for r in range(3)])
    assert rel(outs[0][0], ref) < 1e-13


@pytest.mark.parametrize("antiperiodic", [1, 0])
def test_dslash_two_row_links(antiperiodic):
    """SU(3) links: the Dslash reads two rows per link and rebuilds the third
    (conjugated cross product, the t-boundary sign from the site coordinates);
    FP64 to 1e-13 and FP32 to 1e-5 against the oracle, periodic and
    antiperiodic t, with the residual form inside a solve.  U(3) links (a
    phase on every link) keep all three rows and stay exact."""
    w = wc()
    L, block = (4, 4, 4, 8), (2, 2, 2, 2)
    V = int(np.prod(L))
    psi = syn.complex_gaussian((2, V, 4, 3), 272)
    for U, rows in ((syn.gauge_field(L, 0.3, 271), 2), (syn.gauge_field(L, 0.3, 271) * np.exp(0.3j), 3)):
        ctx = w.Context(dims=L, m0=-0.08, n_levels=2, block=(block,), n_vec=(4,), antiperiodic_t=antiperiodic)
        ctx.set_gauge(dev(U))
        assert ctx.timers()["dslash_link_rows"] == rows
        H = oracle.Hierarchy(L, U, m0=-0.08, n_levels=1, blocks=(), antiperiodic=antiperiodic)
        ref = np.stack([H.apply(0, psi[r]).reshape(V, 4, 3) for r in range(2)])
        assert rel(host(ctx.apply_D(0, dev(psi), w.F64)), ref) < 1e-13
        assert rel(host(ctx.apply_D(0, dev(psi.astype(np.complex64)), w.F32)), ref) < 1e-5


def test_coarse_op_get_set_precisions():
    """wcmg_get_coarse_op in FP64 / FP32 / BF16 equals the FP64 master, its
    FP32 rounding and its BF16 rounding; wcmg_set_coarse_op from FP32 blocks
    widens them (the FP64 master then equals them exactly) and the cycle's
    FP32 coarse apply uses them; BF16 input is refused."""
    w = wc()
    L, block, nv = (4, 4, 4, 8), (2, 2, 2, 2), 8
    ctx, H, U = make_pair(L, 0.3, 241, blocks=(block,), nv=(nv,))
    ctx.set_null_vectors(0, dev(syn.complex_gaussian((nv, 512, 12), 242)))
    ctx.setup()
    m64 = host(ctx.coarse_op(1))
    assert np.array_equal(host(ctx.coarse_op(1, w.F32)), m64.astype(np.complex64))
    assert np.array_equal(host(ctx.coarse_op(1, w.BF16)).astype(np.complex128), bf16_round(m64))
    new = syn.complex_gaussian(m64.shape, 243).astype(np.complex64)
    ctx.set_coarse_op(1, dev(new))
    assert np.array_equal(host(ctx.coarse_op(1)), new.astype(np.complex128))
    phi = syn.complex_gaussian((1, 32, 16), 244)
    ref = oracle.coarse_apply((2, 2, 2, 4), new.astype(np.complex128), phi)
    assert rel(host(ctx.apply_D(1, dev(phi.astype(np.complex64)), w.F32)), ref) < 1e-5
    import ctypes as C
    st = w.lib().wcmg_set_coarse_op(ctx.h, 1, C.c_void_p(dev(new).data_ptr()), w.BF16)
    assert st == 1


@pytest.mark.parametrize("L,block,nv,nrhs", [((6, 6, 4, 4), (3, 3, 1, 1), 12, 12), ((8, 4, 4, 8), (4, 2, 2, 4), 4, 10),
                                           ((8, 4, 4, 8), (4, 2, 2, 4), 6, 16), ((4, 4, 4, 4), (2, 2, 2, 2), 8, 12)])
def test_restrict_multi_rhs_shapes(L, block, nv, nrhs):
    """Restriction of 10..16 FP32 fields in one launch on other aggregate
    shapes and block sizes: 9-site aggregates (3x3x1x1), aggregates of 16
    sites, Nb = 8, 12, 16 and 24, against the oracle."""
    w = wc()
    seed = 281 + nv
    ctx, H, U = make_pair(L, 0.3, seed, blocks=(block,), nv=(nv,))
    V = int(np.prod(L))
    start = syn.complex_gaussian((nv, V, 12), seed + 1)
    ctx.set_null_vectors(0, dev(start))
    ctx.setup()
    H.set_start(0, start)
    H.setup()
    v = syn.complex_gaussian((nrhs, V, 12), seed + 2)
    got = host(ctx.restrict(0, dev(v.astype(np.complex64)), w.F32))
    assert rel(got, oracle.restrict(L, block, 12, H.P(0), v)) < 1e-5


@pytest.mark.parametrize("nrhs", [2, 5, 12, 16])
def test_restrict_prolong_multi_rhs_fp32(nrhs):
    """Several right-hand sides of an FP32 level-0 field in one launch (each
    aggregate's P read once for all of them, waves split by chirality and
    right-hand-side group) against the oracle, and against one launch per
    field; lattice 8x4x4x8 with 4x2x2x4 aggregates (8 aggregates, 64 sites
    each) and 6x4x4x6 with 3x2x2x2 (24 aggregates of 24 sites)."""
    w = wc()
    for L, block, seed in (((8, 4, 4, 8), (4, 2, 2, 4), 251), ((6, 4, 4, 6), (3, 2, 2, 2), 261)):
        nv = 12
        ctx, H, U = make_pair(L, 0.3, seed, blocks=(block,), nv=(nv,))
        V = int(np.prod(L))
        start = syn.complex_gaussian((nv, V, 12), seed + 1)
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        H.set_start(0, start)
        H.setup()
        Pv = H.P(0)
        v = syn.complex_gaussian((nrhs, V, 12), seed + 2)
        got = host(ctx.restrict(0, dev(v.astype(np.complex64)), w.F32))
        assert rel(got, oracle.restrict(L, block, 12, Pv, v)) < 1e-5
        one = np.stack([host(ctx.restrict(0, dev(v[r:r + 1].astype(np.complex64)), w.F32))[0] for r in range(nrhs)])
        assert rel(got, one) < 1e-6
        Vc = V // int(np.prod(block))
        phi = syn.complex_gaussian((nrhs, Vc, 2 * nv), seed + 3)
        got = host(ctx.prolong(0, dev(phi.astype(np.complex64)), w.F32))
        assert rel(got, oracle.prolong(L, block, 12, Pv, phi)) < 1e-5
        one = np.stack([host(ctx.prolong(0, dev(phi[r:r + 1].astype(np.complex64)), w.F32))[0] for r in range(nrhs)])
        assert rel(got, one) < 1e-6
