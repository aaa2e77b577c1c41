"""Even-odd preconditioning on the GPU against the oracle (pinned in
tests/test_eo_oracle.py): the Schur complement to 1e-12, and the even-odd
outer solve (FP64 cycle: iteration counts and solution against the oracle's
even-odd solve; mixed precision and with the SAP smoother: the same solution
as the plain solve)."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests.test_gpu_parity import dev, host, make_pair, rel, wc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (8, 4, 6, 8)])
def test_schur_complement_parity(L):
    w = wc()
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.3, 1901)
    Cl = oracle.clover(L, U, 1.0)
    x = syn.complex_gaussian((2, V, 4, 3), 1902)
    ctx = w.Context(dims=L, m0=-0.05, c_sw=1.0, n_levels=2, block=((2, 2, 2, 2),), n_vec=(4,))
    ctx.set_gauge(dev(U))
    got = host(ctx.apply_schur(dev(x)))
    for k in range(2):
        ref = oracle.schur_apply(L, -0.05, True, U, Cl, x[k])
        assert rel(got[k], ref) < 1e-12
    even = oracle.parity(L) == 0
    assert np.max(np.abs(got[:, even])) == 0.0


def test_even_odd_solve_fp64_parity():
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 8
    ctx, H, U = make_pair(L, 0.3, 1911, blocks=(block,), nv=(nv,), outer_restart=16)
    start = syn.complex_gaussian((nv, 4096, 12), 1912)
    ctx.set_null_vectors(0, dev(start))
    H.set_start(0, start)
    ctx.setup()
    H.setup()
    b = syn.complex_gaussian((4096, 4, 3), 1913)
    xo, it, rr, st = H.solve_eo(b)
    assert st == 0
    w = wc()
    ctx2 = w.Context(dims=L, m0=-0.05, c_sw=1.0, n_levels=2, block=(block,), n_vec=(nv,), outer_restart=16,
                     even_odd=1)
    ctx2.set_gauge(dev(U))
    ctx2.set_null_vectors(0, dev(start))
    ctx2.setup()
    x, info, s = ctx2.solve(dev(b))
    assert s == 0 and info[0]["true_rel_res"] <= 1e-10
    assert abs(info[0]["outer_iters"] - it) <= 1, (info[0]["outer_iters"], it)
    assert rel(host(x), xo.reshape(b.shape)) < 1e-8


@pytest.mark.parametrize("smoother", [0, 1])
def test_even_odd_mixed_precision_solve(smoother):
    w = wc()
    L, block, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    U = syn.gauge_field(L, 0.25, 1921)
    start = syn.complex_gaussian((nv, 4096, 12), 1922)
    b = dev(syn.complex_gaussian((4096, 4, 3), 1923))
    sols, its = [], []
    for eo in (0, 1):
        ctx = w.Context(dims=L, m0=-0.05, n_levels=2, block=(block,), n_vec=(nv,), cycle_prec=w.F32,
                        coarse_store_prec=w.F32, setup_prec=w.F32, smoother=smoother, post_smooth=2 if smoother
                        else 4, even_odd=eo)
        ctx.set_gauge(dev(U))
        ctx.set_null_vectors(0, dev(start))
        ctx.setup()
        x, info, st = ctx.solve(b)
        assert st == 0 and info[0]["true_rel_res"] <= 1e-10
        sols.append(host(x))
        its.append(info[0]["outer_iters"])
    assert rel(sols[1], sols[0]) < 1e-8
    assert its[1] <= its[0] + 2, its
    with pytest.raises(w.WcmgError):
        w.Context(dims=L, n_levels=2, block=(block,), n_vec=(nv,), even_odd=3)
