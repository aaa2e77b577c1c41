"""Setup checkpoints (wcmg_setup_export / wcmg_setup_import): a context that
loads another context's checkpoint holds the same hierarchy bit for bit
(prolongators, coarse operators) and solves bit-identically, with no
relaxation or refinement of its own; corrupted, truncated or mismatched
checkpoints are rejected and leave the context as it was."""
import numpy as np
import pytest

import synthetic as syn
from tests.test_gpu_parity import dev, host, wc

pytestmark = pytest.mark.gpu

# (lattice, aggregates per level, n_vec per level, mixed precision)
CASES = [((8, 8, 8, 8), ((4, 4, 4, 4),), (12,), True),
         ((8, 8, 8, 8), ((2, 2, 2, 2), (2, 2, 2, 2)), (8, 8), False)]


def make(w, L, blocks, nv, U, starts, mixed, **extra):
    kw = dict(cycle_prec=w.F32, coarse_store_prec=w.F32, setup_prec=w.F32) if mixed else {}
    kw.update(extra)
    ctx = w.Context(dims=L, m0=-0.05, n_levels=len(blocks) + 1, block=blocks, n_vec=nv, refine_iters=1, **kw)
    ctx.set_gauge(dev(U))
    for l, s in enumerate(starts):
        ctx.set_null_vectors(l, dev(s))
    return ctx


def problem(L, blocks, nv, seed):
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.25, seed)
    starts, n_l, ns = [], V, 12
    for l in range(len(blocks)):
        starts.append(syn.complex_gaussian((nv[l], n_l, ns), seed + 1 + l))
        n_l //= int(np.prod(blocks[l]))
        ns = 2 * nv[l]
    b = syn.complex_gaussian((V, 4, 3), seed + 9)
    return U, starts, b


@pytest.mark.parametrize("L,blocks,nv,mixed", CASES)
def test_checkpoint_round_trip_is_bit_identical(L, blocks, nv, mixed):
    w = wc()
    U, starts, b = problem(L, blocks, nv, 1901)
    A = make(w, L, blocks, nv, U, starts, mixed)
    A.setup()
    blob = A.export_setup()
    payload, n_l, ns = 0, int(np.prod(L)), 12
    for l in range(len(blocks)):
        payload += nv[l] * n_l * ns * 16
        n_l //= int(np.prod(blocks[l]))
        ns = 2 * nv[l]
    assert len(blob) == 128 + payload and bytes(blob[:8]) == b"WCMGSET1"
    # a fresh context with the same gauge field and no start vectors
    B = w.Context(dims=L, m0=-0.05, n_levels=len(blocks) + 1, block=blocks, n_vec=nv, refine_iters=1,
                  **(dict(cycle_prec=w.F32, coarse_store_prec=w.F32, setup_prec=w.F32) if mixed else {}))
    B.set_gauge(dev(U))
    B.import_setup(blob)
    for l in range(len(blocks)):
        assert np.array_equal(host(B.prolongator(l)), host(A.prolongator(l)))
        assert np.array_equal(host(B.coarse_op(l + 1)), host(A.coarse_op(l + 1)))
    xa, ia, sa = A.solve(dev(b))
    xb, ib, sb = B.solve(dev(b))
    assert sa == 0 and sb == 0
    assert np.array_equal(host(xa), host(xb))
    assert ia[0]["outer_iters"] == ib[0]["outer_iters"] and ia[0]["coarse_iters"] == ib[0]["coarse_iters"]
    # the blob survives a bytes copy, and a re-export reproduces it
    B.import_setup(bytes(blob))
    assert B.export_setup() == blob


def test_checkpoint_rejections_leave_the_context_unchanged():
    w = wc()
    L, blocks, nv = (8, 8, 8, 8), ((4, 4, 4, 4),), (12,)
    U, starts, b = problem(L, blocks, nv, 1911)
    A = make(w, L, blocks, nv, U, starts, True)
    with pytest.raises(w.WcmgError) as e:
        A.export_setup()  # before the setup
    assert e.value.code == 3
    A.setup()
    blob = A.export_setup()
    x0, i0, _ = A.solve(dev(b))
    bad = bytearray(blob)
    bad[128 + 1000] ^= 0x10  # one payload bit
    trunc = blob[:-16]
    wrong_magic = bytearray(blob)
    wrong_magic[0:8] = b"WCMGXXXX"
    for blk, code in ((bad, 1), (trunc, 1), (wrong_magic, 1)):
        with pytest.raises(w.WcmgError) as e:
            A.import_setup(blk)
        assert e.value.code == code
    x1, i1, _ = A.solve(dev(b))
    assert np.array_equal(host(x0), host(x1))
    # another operator (m0), another lattice, another hierarchy
    other = w.Context(dims=L, m0=-0.06, n_levels=2, block=blocks, n_vec=nv)
    other.set_gauge(dev(U))
    with pytest.raises(w.WcmgError) as e:
        other.import_setup(blob)
    assert e.value.code == 1
    other = w.Context(dims=L, m0=-0.05, n_levels=2, block=((2, 2, 2, 2),), n_vec=nv)
    other.set_gauge(dev(U))
    with pytest.raises(w.WcmgError) as e:
        other.import_setup(blob)
    assert e.value.code == 1
    # no gauge field yet
    fresh = w.Context(dims=L, m0=-0.05, n_levels=2, block=blocks, n_vec=nv)
    with pytest.raises(w.WcmgError) as e:
        fresh.import_setup(blob)
    assert e.value.code == 3
