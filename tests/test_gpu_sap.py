"""SAP smoother on the GPU (wcmg_sap and the cycle's level-0 post-smoother)
against the oracle's SAP (oracle.sap, pinned in tests/test_sap_oracle.py):
FP64 to 1e-12, FP32 arithmetic to 1e-5; the cycle with SAP against the
oracle's cycle; solves with SAP, single and batched."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests.test_gpu_parity import dev, host, make_pair, rel, wc

pytestmark = pytest.mark.gpu


# (lattice, aggregate) -> domains of 256, 16, 32 and 24 sites (one, one, one
# and two waves' worth of sites per direction group)
CASES = [((8, 8, 8, 8), (4, 4, 4, 4)), ((4, 4, 4, 8), (2, 2, 2, 2)), ((4, 4, 8, 8), (2, 2, 2, 4)),
         ((6, 4, 4, 4), (3, 2, 2, 2))]


@pytest.mark.parametrize("L,block", CASES)
def test_sap_parity(L, block):
    w = wc()
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.3, 1701)
    Cl = oracle.clover(L, U, 1.0)
    b = syn.complex_gaussian((2, V, 4, 3), 1702)
    x0 = syn.complex_gaussian((2, V, 4, 3), 1703)
    ctx = w.Context(dims=L, m0=-0.05, c_sw=1.0, n_levels=2, block=(block,), n_vec=(4,), sap_block_iters=4)
    ctx.set_gauge(dev(U))
    ref = np.stack([oracle.sap(L, block, U, Cl, b[k], x0[k], 2, 4, m0=-0.05) for k in range(2)]).reshape(b.shape)
    got = host(ctx.sap(dev(b), dev(x0.copy()), 2))
    assert rel(got, ref) < 1e-12
    got32 = host(ctx.sap(dev(b.astype(np.complex64)), dev(x0.astype(np.complex64)), 2))
    assert rel(got32, ref) < 1e-5
    # zero cycles leave x alone
    assert np.array_equal(host(ctx.sap(dev(b), dev(x0.copy()), 0)), x0)


def test_sap_errors():
    w = wc()
    ctx = w.Context(dims=(6, 4, 4, 4), n_levels=2, block=((2, 2, 2, 2),), n_vec=(4,))  # 3 aggregates in x
    ctx.set_gauge(dev(syn.gauge_field((6, 4, 4, 4), 0.3, 1)))
    z = dev(np.zeros((384, 4, 3), np.complex128))
    with pytest.raises(w.WcmgError) as e:
        ctx.sap(z, z.clone(), 1)
    assert e.value.code == 2
    with pytest.raises(w.WcmgError) as e:
        w.Context(dims=(4, 4, 4, 4), n_levels=2, block=((2, 2, 2, 2),), n_vec=(4,), smoother=2)
    assert e.value.code == 1
    ctx = w.Context(dims=(4, 4, 4, 4), n_levels=1, block=((2, 2, 2, 2),), n_vec=(4,))
    ctx.set_gauge(dev(syn.gauge_field((4, 4, 4, 4), 0.3, 1)))
    z = dev(np.zeros((256, 4, 3), np.complex128))
    with pytest.raises(w.WcmgError) as e:
        ctx.sap(z, z.clone(), 1)
    assert e.value.code == 1


def test_cycle_with_sap_smoother_fp64_parity():
    """One FP64 V-cycle with 2 SAP post-smoothing cycles and a fixed number of
    coarse iterations: GPU against oracle."""
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 8
    kw = dict(smoother=1, sap_block_iters=3, post_smooth=2, coarse_fixed_iters=10)
    ctx, H, U = make_pair(L, 0.3, 1711, blocks=(block,), nv=(nv,), **kw)
    start = syn.complex_gaussian((nv, 4096, 12), 1712)
    ctx.set_null_vectors(0, dev(start))
    H.set_start(0, start)
    ctx.setup()
    H.setup()
    r = syn.complex_gaussian((4096, 4, 3), 1713)
    got = host(ctx.cycle(dev(r)))
    ref = H.cycle(0, r).reshape(r.shape)
    assert rel(got, ref) < 1e-11


def test_solves_with_sap_smoother():
    """Mixed-precision solves with the SAP smoother reach 1e-10 with the
    oracle's FP64 outer iteration count (within one); the batched solve
    matches the single solves."""
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    U = syn.gauge_field(L, 0.25, 1721)
    start = syn.complex_gaussian((nv, 4096, 12), 1722)
    b = syn.complex_gaussian((3, 4096, 4, 3), 1723)
    kw = dict(smoother=1, sap_block_iters=4, post_smooth=2)
    ctx = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), cycle_prec=w.F32,
                    coarse_store_prec=w.F32, setup_prec=w.F32, outer_restart=16, **kw)
    ctx.set_gauge(dev(U))
    ctx.set_null_vectors(0, dev(start))
    ctx.setup()
    H = oracle.Hierarchy(L, U, m0=-0.05, blocks=(block,), nv=(nv,), **kw)
    H.set_start(0, start)
    H.setup()
    _, it_ref, res_ref, _ = H.solve(b[0])
    x, info, st = ctx.solve(dev(b[0]))
    assert st == 0 and info[0]["true_rel_res"] <= 1e-10 and res_ref <= 1e-10
    assert abs(info[0]["outer_iters"] - it_ref) <= 1, (info[0]["outer_iters"], it_ref)
    xb, ib, sb = ctx.solve_batched(dev(b))
    assert sb == 0
    for k in range(3):
        xs, i1, s1 = ctx.solve(dev(b[k]))
        assert s1 == 0 and ib[k]["true_rel_res"] <= 1e-10
        assert abs(ib[k]["outer_iters"] - i1[0]["outer_iters"]) <= 1
