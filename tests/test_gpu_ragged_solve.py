"""wcmg_solve_ragged: several two-level problems on different lattices solved
together, their coarse solves sharing one matrix-core launch per Arnoldi step
(the ragged batch of the multi-RHS configuration).  Each problem must reach
1e-10 on every right-hand side with the outer iteration counts of its own
batched solve (within one) and the same solutions (to 1e-8); errors for
mismatched problems."""
import numpy as np
import pytest
import torch

import synthetic as syn
from tests.test_gpu_parity import dev, host, rel, wc

pytestmark = pytest.mark.gpu


def problem(w, L, seed, nrhs, store, m0=-0.08, **kw):
    V = int(np.prod(L))
    ctx = w.Context(dims=L, m0=m0, n_levels=2, block=((4, 4, 4, 4),), n_vec=(12,), refine_iters=1, outer_restart=20,
                    outer_maxit=2000, cycle_prec=w.F32, coarse_store_prec=store, setup_prec=w.F32, **kw)
    ctx.set_gauge(dev(syn.gauge_field(L, 0.25, seed)))
    ctx.set_null_vectors(0, dev(syn.complex_gaussian((12, V, 12), seed + 1)))
    ctx.setup()
    if nrhs == 12:
        b = syn.point_sources(V, site=0)
    else:
        b = syn.complex_gaussian((nrhs, V, 4, 3), seed + 2)
    return ctx, b


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_ragged_solve_matches_each_problems_own_batched_solve(store):
    w = wc()
    sp = w.F32 if store == "f32" else w.BF16
    probs = [problem(w, (8, 8, 8, 8), 1601, 12, sp), problem(w, (8, 8, 8, 16), 1611, 5, sp),
             problem(w, (16, 16, 16, 16), 1621, 3, sp)]
    ctxs = [p[0] for p in probs]
    bs = [dev(p[1]) for p in probs]
    own = [c.solve_batched(b) for c, b in zip(ctxs, bs)]
    xs, infos, st, launches = w.solve_ragged(ctxs, bs)
    assert st == 0
    assert launches > 0
    for k in range(3):
        xo, io, so = own[k]
        assert so == 0
        for r, (a, o) in enumerate(zip(infos[k], io)):
            assert a["converged"] and a["true_rel_res"] <= 1e-10, (k, r, a)
            assert abs(a["outer_iters"] - o["outer_iters"]) <= 1, (k, r, a["outer_iters"], o["outer_iters"])
        assert rel(host(xs[k]), host(xo)) < 1e-8, k
    # one shared launch per coarse Arnoldi step: fewer launches than the
    # problems' coarse iterations summed over problems and right-hand sides
    assert launches < sum(sum(i["coarse_iters"] for i in inf[:1]) for inf in infos)


def test_ragged_solve_errors():
    w = wc()
    a, ba = problem(w, (8, 8, 8, 8), 1631, 2, w.F32)
    c, bc = problem(w, (8, 8, 8, 8), 1641, 2, w.BF16)
    with pytest.raises(w.WcmgError) as e:
        w.solve_ragged([a, c], [dev(ba), dev(bc)])  # different coarse storage
    assert e.value.code == 1
    with pytest.raises(w.WcmgError) as e:
        w.solve_ragged([a, a], [dev(ba), dev(ba)])  # one context twice
    assert e.value.code == 1
    d = w.Context(dims=(8, 8, 8, 8), m0=-0.08, n_levels=2, block=((4, 4, 4, 4),), n_vec=(12,), cycle_prec=w.F32)
    d.set_gauge(dev(syn.gauge_field((8, 8, 8, 8), 0.25, 1651)))
    with pytest.raises(w.WcmgError) as e:
        w.solve_ragged([a, d], [dev(ba), dev(ba)])  # not set up
    assert e.value.code == 3
    f = w.Context(dims=(8, 8, 8, 8), m0=-0.08, n_levels=2, block=((4, 4, 4, 4),), n_vec=(12,))
    f.set_gauge(dev(syn.gauge_field((8, 8, 8, 8), 0.25, 1652)))
    f.set_null_vectors(0, dev(syn.complex_gaussian((12, 4096, 12), 1653)))
    f.setup()
    with pytest.raises(w.WcmgError) as e:
        w.solve_ragged([a, f], [dev(ba), dev(ba)])  # FP64 cycle
    assert e.value.code == 1
