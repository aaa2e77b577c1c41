"""Solver status codes forced from the host: an iteration limit below what the
solve needs gives WCMG_ERR_NOCONV with the info filled and the best iterate
written; a NaN in a right-hand side gives WCMG_ERR_NAN.  Every kernel runs to
its normal end (NaN only flows through the arithmetic).

The iterate returned on NOCONV is checked against the oracle's own operator:
its true residual is the one the info reports."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests.test_gpu_parity import dev, host, make_pair, wc

pytestmark = pytest.mark.gpu

NOCONV, NAN = 7, 8
L = (4, 4, 4, 4)
V = 256


def _pair(**kw):
    ctx, H, U = make_pair(L, 0.3, 801, m0=-0.05, blocks=((2, 2, 2, 2),), nv=(4,), **kw)
    ctx.set_null_vectors(0, dev(syn.complex_gaussian((4, V, 12), 802)))
    ctx.setup()
    return ctx, H


def _true_res(H, b, x):
    r = b.reshape(-1) - H.apply(0, x.reshape(-1))
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_noconv_single_and_batched():
    """outer_maxit = 3: status NOCONV, converged False, outer_iters = 3, and the
    returned x has the reported true residual (oracle operator), below that of
    x = 0; single and batched solves."""
    w = wc()
    ctx, H = _pair(outer_maxit=3, outer_restart=20)
    b = syn.complex_gaussian((2, V, 4, 3), 803)
    x, info, st = ctx.solve(dev(b[:1]), check=False)
    assert st == NOCONV
    assert not info[0]["converged"] and info[0]["outer_iters"] == 3
    res = _true_res(H, b[0], host(x)[0])
    assert abs(res - info[0]["true_rel_res"]) <= 1e-10 + 1e-8 * res
    assert 1e-10 < res < 1.0
    xb, ib, st = ctx.solve_batched(dev(b), check=False)
    assert st == NOCONV
    for r in range(2):
        assert not ib[r]["converged"] and ib[r]["outer_iters"] == 3
        res = _true_res(H, b[r], host(xb)[r])
        assert abs(res - ib[r]["true_rel_res"]) <= 1e-10 + 1e-8 * res
    assert "converge" in ctx.last_error()


def test_nan_rhs_single_and_batched():
    """A NaN in a right-hand side: status NAN; in the batched solve the other
    right-hand sides still converge to the tolerance and report so."""
    w = wc()
    ctx, H = _pair(outer_maxit=4)
    b = syn.complex_gaussian((2, V, 4, 3), 804)
    bad = b.copy()
    bad[0, 17, 2, 1] = np.nan
    x, info, st = ctx.solve(dev(bad[:1]), check=False)
    assert st == NAN
    assert not info[0]["converged"]
    assert "NaN" in ctx.last_error()
    ctx2, _ = _pair(outer_maxit=200)
    xb, ib, st = ctx2.solve_batched(dev(bad), check=False)
    assert st == NAN
    assert not ib[0]["converged"]
    assert ib[1]["converged"] and _true_res(H, b[1], host(xb)[1]) <= 1.01e-10
