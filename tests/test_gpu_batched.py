"""Batched solves (wcmg_solve_batched): several right-hand sides advancing
through shared launches, one FP64 FGMRES each, masked once converged.

Every solution is checked against the oracle's own Wilson-clover operator
(true residual to 1e-10), and against the oracle's single-RHS solve or the
library's single-RHS path for iteration counts."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests.test_gpu_parity import dev, host, make_pair, wc

pytestmark = pytest.mark.gpu


def residuals(H, b, x):
    """||b_r - D x_r|| / ||b_r|| for each right-hand side, D from the oracle."""
    out = []
    for br, xr in zip(b, x):
        br = br.reshape(-1)
        r = br - H.apply(0, xr.reshape(-1))
        nb = np.linalg.norm(br)
        out.append(np.linalg.norm(r) / nb if nb > 0 else np.linalg.norm(r))
    return np.array(out)


def test_batched_fp64_matches_oracle_solves():
    """FP64 cycle, 4^4 lattice, 2^4 aggregates, Nv 8: five right-hand sides
    together; each reaches 1e-10 and needs the oracle's iteration count +-1."""
    L = (4, 4, 4, 4)
    ctx, H, U = make_pair(L, 0.3, 121, m0=-0.05, blocks=((2, 2, 2, 2),), nv=(8,), outer_restart=16)
    start = syn.complex_gaussian((8, 256, 12), 122)
    ctx.set_null_vectors(0, dev(start))
    H.set_start(0, start)
    ctx.setup()
    H.setup()
    b = syn.complex_gaussian((5, 256, 4, 3), 123)
    x, info, st = ctx.solve_batched(dev(b))
    assert st == 0
    xs = host(x)
    res = residuals(H, b, xs)
    assert np.all(res <= 1.01e-10), res
    for r in range(5):
        _, ito, _, _ = H.solve(b[r])
        assert info[r]["converged"] and abs(info[r]["outer_iters"] - ito) <= 1, (r, info[r], ito)


def _mixed_pair(L, seed, store, **kw):
    w = wc()
    ctx, H, U = make_pair(L, 0.25, seed, m0=-0.05, blocks=((4, 4, 4, 4),), nv=(12,), cycle_prec=w.F32,
                          coarse_store_prec=store, setup_prec=w.F32, **kw)
    V = int(np.prod(L))
    ctx.set_null_vectors(0, dev(syn.complex_gaussian((12, V, 12), seed + 1)))
    ctx.setup()
    return ctx, H, V


@pytest.mark.parametrize("kernel", ["auto", "vector", "mfma"])
def test_batched_point_sources_match_single_solves(kernel):
    """Twelve point sources (one per spin-colour) on 8^4 with FP32 cycle and
    blocks: batched (matrix-core or vector coarse apply) against twelve single
    solves of the same context."""
    w = wc()
    L = (8, 8, 8, 8)
    ctx, H, V = _mixed_pair(L, 731, w.F32)
    b = syn.point_sources(V, site=37)
    xb, ib, st = ctx.solve_batched(dev(b), kernel=kernel)
    assert st == 0
    res = residuals(H, b, host(xb))
    assert np.all(res <= 1.01e-10), res
    _, isg, st1 = ctx.solve(dev(b))
    assert st1 == 0
    for r in range(12):
        assert ib[r]["converged"]
        assert abs(ib[r]["outer_iters"] - isg[r]["outer_iters"]) <= 1, (r, ib[r], isg[r])


def test_batched_bf16_blocks_and_graph_replay_is_identical():
    """BF16-stored coarse blocks on the matrix cores; the HIP-graph replay of the
    cycle performs the same launches as the eager cycle, so the solutions agree
    bit for bit."""
    w = wc()
    L = (8, 8, 8, 8)
    ctx, H, V = _mixed_pair(L, 741, w.BF16, coarse_maxit=20)
    b = syn.complex_gaussian((6, V, 4, 3), 742)
    xe, ie, st = ctx.solve_batched(dev(b), graph=False, kernel="mfma")
    assert st == 0
    xg, ig, st = ctx.solve_batched(dev(b), graph=True, kernel="mfma")
    assert st == 0
    ae, ag = host(xe), host(xg)
    res = residuals(H, b, ag)
    assert np.all(res <= 1.01e-10), res
    assert [i["outer_iters"] for i in ie] == [i["outer_iters"] for i in ig]
    assert np.array_equal(ae, ag)


def test_batched_masking_zero_rhs_and_converged_guess():
    """A zero right-hand side and one whose initial guess is already the
    solution drop out at once; the others converge as usual; 17 right-hand
    sides run as a group of 16 and a group of 1."""
    w = wc()
    L = (8, 8, 8, 8)
    ctx, H, V = _mixed_pair(L, 751, w.F32)
    b = syn.complex_gaussian((17, V, 4, 3), 752)
    b[3] = 0.0
    x0 = np.zeros_like(b)
    xs, _, st = ctx.solve(dev(b[5:6]))
    assert st == 0
    x0[5] = host(xs)[0]
    x, info, st = ctx.solve_batched(dev(b), dev(x0))
    assert st == 0
    xh = host(x)
    assert np.all(xh[3] == 0) and info[3]["outer_iters"] == 0
    assert info[5]["outer_iters"] <= 1
    res = residuals(H, b, xh)
    assert np.all(res <= 1.01e-10), res


def test_batched_three_level_kcycle():
    """Three levels (Nb 16 on both coarse levels, both on the matrix cores) with
    a K-cycle on the intermediate level: three right-hand sides to 1e-10."""
    w = wc()
    L = (8, 8, 8, 8)
    ctx, H, U = make_pair(L, 0.25, 761, m0=-0.05, n_levels=3, blocks=((2, 2, 2, 2), (2, 2, 2, 2)), nv=(8, 8),
                          kcycle=1, outer_restart=20, cycle_prec=w.F32, setup_prec=w.F32)
    ctx.set_null_vectors(0, dev(syn.complex_gaussian((8, 4096, 12), 762)))
    ctx.set_null_vectors(1, dev(syn.complex_gaussian((8, 256, 16), 763)))
    ctx.setup()
    b = syn.complex_gaussian((4, 4096, 4, 3), 764)
    x, info, st = ctx.solve_batched(dev(b), kernel="mfma")
    assert st == 0
    res = residuals(H, b, host(x))
    assert np.all(res <= 1.01e-10), res


def test_batched_single_reduction_outer_step_matches_cgs2():
    """The batched outer FGMRES with one reduction per Arnoldi step against
    the CGS2 form (reserved[0] flag 8), four right-hand sides, one of them
    zero: same per-right-hand-side iteration counts, solutions to 1e-12, all
    to the 1e-10 target."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.25, 1951)
    start = syn.complex_gaussian((nv, V, 12), 1952)
    b = syn.complex_gaussian((4, V, 4, 3), 1953)
    b[2] = 0.0
    xs, its = [], []
    for flags in (0, 8):
        ctx = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), cycle_prec=w.F32,
                        coarse_store_prec=w.F32, setup_prec=w.F32, reserved=(flags,))
        ctx.set_gauge(dev(U))
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        x, info, st = ctx.solve_batched(dev(b))
        assert st == 0
        for k in (0, 1, 3):
            assert info[k]["true_rel_res"] <= 1e-10
        xs.append(host(x))
        its.append([i["outer_iters"] for i in info])
    assert its[0] == its[1], its
    assert np.array_equal(xs[0][2], np.zeros_like(xs[0][2]))
    for k in (0, 1, 3):
        assert np.linalg.norm(xs[0][k] - xs[1][k]) < 1e-12 * np.linalg.norm(xs[1][k])


def test_batched_flag_errors():
    w = wc()
    ctx = w.Context(dims=(4, 4, 4, 4), n_levels=2, block=((2, 2, 2, 2),), n_vec=(4,))
    ctx.set_gauge(dev(syn.gauge_field((4, 4, 4, 4), 0.3, 1)))
    ctx.set_null_vectors(0, dev(syn.complex_gaussian((4, 256, 12), 2)))
    ctx.setup()
    b = dev(np.ones((2, 256, 4, 3), np.complex128))
    with pytest.raises(w.WcmgError) as e:
        ctx.solve_batched(b, graph=True)  # FP64 cycle cannot be captured
    assert e.value.code == 1


def test_autotuner_table_and_forced_variants():
    """The autotuner records one decision per launch configuration of the
    batched solve; a loaded table forces each variant, and every variant
    solves to 1e-10 with the same iteration counts to within one."""
    w = wc()
    L = (8, 8, 8, 8)
    ctx, H, V = _mixed_pair(L, 771, w.F32)
    b = syn.complex_gaussian((8, V, 4, 3), 772)
    x, info, st = ctx.solve_batched(dev(b))
    assert st == 0
    table = ctx.tune_table()
    # keys name the device architecture first ("gfx950 dslash_f32 V=...")
    dkeys = [k for k in table if k.split(" ")[1] == "dslash_f32"]
    ckeys = [k for k in table if k.split(" ")[1] == "coarse_apply"]
    tkeys = [k for k in table if k.split(" ")[1] == "coarse_mfma_tile"]
    assert dkeys and ckeys, table
    for k in dkeys + ckeys:
        assert table[k]["choice"] in (0, 1) and len(table[k]["ms"]) == 2
    for k in tkeys:  # tiles 0, 4, 8, 16, 5, 9 on the 2^4 coarse lattice: only 0 fits
        assert table[k]["choice"] == 0 and [m >= 0 for m in table[k]["ms"]] == [True] + [False] * 5
    base = [i["outer_iters"] for i in info]
    for v in (0, 1):
        c2, _, _ = _mixed_pair(L, 771, w.F32)
        c2.tune_load({k: {"choice": v} for k in dkeys + ckeys})
        x2, i2, st2 = c2.solve_batched(dev(b))
        assert st2 == 0
        assert all(c2.tune_table()[k]["choice"] == v for k in dkeys + ckeys)
        res = residuals(H, b, host(x2))
        assert np.all(res <= 1.01e-10), res
        assert all(abs(a - c) <= 1 for a, c in zip(base, [i["outer_iters"] for i in i2]))


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_ragged_coarse_apply(store):
    """One launch over three coarse operators of different lattices (the coarse
    lattices of 8^4, 16^4 and 24^3 x 48 under 4^4 aggregates: 16 + 256 + 2592
    sites, Nb = 24) with 12, 5 and 16 right-hand sides: bit-identical to the
    operators applied one by one, and within FP32 rounding of the oracle
    (applied to the BF16-rounded blocks for BF16 storage)."""
    from tests.test_gpu_parity import bf16_round, rel
    w = wc()
    st = w.F32 if store == "f32" else w.BF16
    lats = [(2, 2, 2, 2), (4, 4, 4, 4), (6, 6, 6, 12)]
    nrhs = [12, 5, 16]
    ops, ins, refs = [], [], []
    for q, (Lc, nr) in enumerate(zip(lats, nrhs)):
        Vc = int(np.prod(Lc))
        blocks = syn.complex_gaussian((Vc, 9, 24, 24), 780 + q)
        phi = syn.complex_gaussian((nr, Vc, 24), 790 + q)
        op = w.CoarseOperator(Lc, 24, st)
        op.set(dev(blocks))
        op.set_kernel(2)
        ops.append(op)
        ins.append(dev(phi.astype(np.complex64)))
        refs.append(oracle.coarse_apply(Lc, bf16_round(blocks) if store == "bf16" else blocks, phi))
    outs = w.coarse_apply_ragged(ops, ins)
    for op, x, y, ref in zip(ops, ins, outs, refs):
        one = host(op.apply(x))
        got = host(y)
        assert np.array_equal(got, one)
        assert rel(got, ref) < 1e-5
    assert w.coarse_time_ragged(ops, ins, reps=3) > 0
    with pytest.raises(w.WcmgError):
        w.coarse_apply_ragged([ops[0], w.CoarseOperator((2, 2, 2, 2), 16, st)], ins[:1] * 2)


@pytest.mark.parametrize("tile", [4, 8, 5])
def test_batched_mfma_tile_forced_through_tuning_table(tile):
    """The batched solve with the coarse level's matrix-core tile forced through
    the tuning table (one wave per site against 4 or 8 sites of an x-row per
    workgroup with LDS-staged neighbours), right-hand sides dropping out of the
    launches as they converge: identical iterates, hence identical solutions and
    iteration counts."""
    import torch
    w = wc()
    L, block = (16, 8, 4, 4), (2, 2, 2, 2)
    V = int(np.prod(L))
    Lc = tuple(l // k for l, k in zip(L, block))
    Vc = int(np.prod(Lc))
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    b = syn.complex_gaussian((6, V, 4, 3), 353)
    b[1] = syn.point_sources(V, site=21)[4]  # converges at another iteration than the Gaussian sources
    out = []
    for t in (0, tile):
        ctx, H, U = make_pair(L, 0.3, 351, m0=-0.05, blocks=(block,), nv=(8,), cycle_prec=w.F32,
                              coarse_store_prec=w.F32, setup_prec=w.F32)
        ctx.set_null_vectors(0, dev(syn.complex_gaussian((8, V, 12), 352)))
        ctx.setup()
        key = "%s coarse_mfma_tile prec=%d Vc=%d Lx=%d nb=16 nrhs=6" % (arch, w.F32, Vc, Lc[0])
        ctx.tune_load({key: {"choice": (0, 4, 8, 16, 5, 9).index(t)}})
        x, info, st = ctx.solve_batched(dev(b), kernel="mfma")
        assert st == 0
        assert ctx.tune_table()[key]["choice"] == (0, 4, 8, 16, 5, 9).index(t)
        out.append((host(x), [i["outer_iters"] for i in info]))
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])
    assert np.all(residuals(H, b, out[1][0]) <= 1.01e-10)
