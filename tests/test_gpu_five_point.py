"""Five-point coarse storage on the GPU: Mdiag and the forward blocks stored,
the backward hops applied as sigma3-conjugated adjoints of the neighbours'
forward blocks.  Compared with the oracle's nine-block apply on operators
whose backward blocks satisfy that relation (every Galerkin operator does:
tests/test_oracle_pins.py pins it on the oracle's own coarsening), and inside
the solver against the nine-block path."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests import brute_force as bf
from tests.test_gpu_parity import bf16_round, dev, host, rel, wc

pytestmark = pytest.mark.gpu


def mirrored_blocks(Lc, nb, seed):
    Vc = int(np.prod(Lc))
    return bf.sigma3_mirror(Lc, syn.complex_gaussian((Vc, 9, nb, nb), seed))


# (coarse lattice, Nb, right-hand sides): sub-lanes per row 8, 4, 2 (consumer
# form through LDS) and 1 (owner form with the scatter buffer) on the
# (8,8,8,8) cases; the owner form for every Nb with a partial last workgroup;
# odd extents; extent 2 where c + mu = c - mu
CASES = [((3, 2, 4, 3), 8, 1), ((2, 2, 2, 2), 16, 3), ((5, 3, 2, 3), 12, 2), ((4, 4, 4, 8), 24, 1),
         ((3, 3, 2, 2), 32, 2), ((8, 8, 8, 8), 24, 1), ((8, 8, 8, 8), 24, 2), ((8, 8, 8, 8), 24, 3),
         ((16, 8, 8, 8), 8, 5), ((16, 8, 8, 8), 12, 3), ((8, 8, 8, 16), 16, 2), ((8, 8, 8, 8), 32, 2)]


@pytest.mark.parametrize("Lc,nb,nrhs", CASES)
def test_five_point_apply_parity(Lc, nb, nrhs):
    w = wc()
    Vc = int(np.prod(Lc))
    blocks = mirrored_blocks(Lc, nb, 1501)
    phi = syn.complex_gaussian((nrhs, Vc, nb), 1502)
    ref = oracle.coarse_apply(Lc, blocks, phi)
    for store in (w.F64, w.F32, w.BF16):
        if store == w.BF16 and nb % 4:
            continue
        op = w.CoarseOperator(Lc, nb, store)
        op.set_kernel(3)
        op.set(dev(blocks))
        if store == w.F64:
            got = host(op.apply(dev(phi)))
            assert rel(got, ref) < 1e-13, store
        elif store == w.F32:
            got = host(op.apply(dev(phi.astype(np.complex64))))
            assert rel(got, ref) < 1e-5, store
        else:
            ref_b = oracle.coarse_apply(Lc, bf16_round(blocks), phi)
            got = host(op.apply(dev(phi.astype(np.complex64))))
            assert rel(got, ref_b) < 1e-5, store


def test_five_point_ignores_stored_backward_blocks():
    """Only Mdiag and the forward blocks are read: garbage in the backward
    slots does not change the result."""
    w = wc()
    Lc, nb = (4, 2, 2, 4), 16
    Vc = int(np.prod(Lc))
    blocks = mirrored_blocks(Lc, nb, 1511)
    noisy = blocks.copy()
    for d in (2, 4, 6, 8):
        noisy[:, d] = syn.complex_gaussian((Vc, nb, nb), 1512 + d)
    phi = syn.complex_gaussian((1, Vc, nb), 1513)
    op = w.CoarseOperator(Lc, nb, w.F64)
    op.set_kernel(3)
    op.set(dev(noisy))
    assert rel(host(op.apply(dev(phi))), oracle.coarse_apply(Lc, blocks, phi)) < 1e-13


def test_five_point_errors():
    w = wc()
    op = w.CoarseOperator((2, 2, 2, 2), 6, w.F32)
    with pytest.raises(w.WcmgError) as e:
        op.set_kernel(3)  # Nb = 6 not supported
    assert e.value.code == 1
    op = w.CoarseOperator((2, 2, 2, 2), 8, w.F32)
    op.set(dev(mirrored_blocks((2, 2, 2, 2), 8, 1521)))
    with pytest.raises(w.WcmgError) as e:
        op.set_kernel(3)  # after the blocks were set
    assert e.value.code == 3
    with pytest.raises(w.WcmgError) as e:
        w.Context(dims=(4, 4, 4, 4), n_levels=2, block=((2, 2, 2, 2),), n_vec=(4,), coarse_points=7)
    assert e.value.code == 1


def _context(w, L, nv, U, start, points, **kw):
    ctx = w.Context(dims=L, m0=-0.05, n_levels=2, block=((4, 4, 4, 4),), n_vec=(nv,), coarse_points=points, **kw)
    ctx.set_gauge(dev(U))
    ctx.set_null_vectors(0, dev(start))
    ctx.setup()
    return ctx


@pytest.mark.parametrize("flags", [0, 2])
def test_five_point_cycle_and_solve_match_nine_point(flags):
    """FP64 cycle with a fixed number of coarse iterations: the same output
    to 1e-11 from five- and nine-point storage (fused coarse GMRES, flags 0,
    and the generic multi-kernel GMRES, flags 2); mixed-precision solves to
    1e-10 with outer iteration counts within one."""
    w = wc()
    L, nv = (8, 8, 8, 8), 12
    U = syn.gauge_field(L, 0.25, 1531)
    start = syn.complex_gaussian((nv, 4096, 12), 1532)
    r = syn.complex_gaussian((4096, 4, 3), 1533)
    outs = []
    for points in (9, 5):
        ctx = _context(w, L, nv, U, start, points, coarse_fixed_iters=8, reserved=(flags,))
        outs.append(host(ctx.cycle(dev(r))))
    assert rel(outs[1], outs[0]) < 1e-11
    its = []
    for points in (9, 5):
        ctx = _context(w, L, nv, U, start, points, cycle_prec=w.F32, coarse_store_prec=w.F32, setup_prec=w.F32,
                       reserved=(flags,))
        x, info, st = ctx.solve(dev(r))
        assert st == 0 and info[0]["true_rel_res"] <= 1e-10
        its.append(info[0]["outer_iters"])
    assert abs(its[0] - its[1]) <= 1, its


@pytest.mark.parametrize("L,block,nrhs", [((8, 8, 8, 8), (4, 4, 4, 4), 3), ((16, 16, 16, 16), (2, 2, 2, 2), 3)])
def test_five_point_batched_solve(L, block, nrhs):
    """Batched solve with the per-row five-point kernel for the batch's
    coarse applies (consumer form on the 2^4 coarse lattice, owner form with
    masked right-hand sides on the 8^4 one) against single solves."""
    w = wc()
    nv = 12
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.25, 1541)
    start = syn.complex_gaussian((nv, V, 12), 1542)
    b = syn.complex_gaussian((nrhs, V, 4, 3), 1543)
    ctx = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), coarse_points=5, cycle_prec=w.F32,
                    coarse_store_prec=w.F32, setup_prec=w.F32)
    ctx.set_gauge(dev(U))
    ctx.set_null_vectors(0, dev(start))
    ctx.setup()
    x, info, st = ctx.solve_batched(dev(b), kernel="vector")
    assert st == 0
    for k in range(nrhs):
        xs, i1, s1 = ctx.solve(dev(b[k]))
        assert s1 == 0 and info[k]["true_rel_res"] <= 1e-10
        assert abs(info[k]["outer_iters"] - i1[0]["outer_iters"]) <= 1
