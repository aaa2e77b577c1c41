"""Pins of the oracle's SAP smoother (oracle.sap) against dense linear algebra:
the domain operator D_B is the dense D (assembled column by column from the
pinned Wilson-clover apply) restricted to the domain's rows and columns, the
exact domain solves come from numpy, and one MR step has a closed form."""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests import brute_force as bf

L, BLOCK = (4, 2, 2, 4), (2, 1, 1, 2)  # 16 domains of 4 sites, coarse lattice 2^4
M0, CSW = 0.5, 1.0


def problem(seed):
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.3, seed)
    Cl = oracle.clover(L, U, CSW)
    n = 12 * V
    D = oracle.wilson_apply(L, M0, True, U, Cl, np.eye(n).reshape(n, V, 4, 3)).reshape(n, n).T
    b = syn.complex_gaussian((V, 4, 3), seed + 1).reshape(-1)
    x0 = syn.complex_gaussian((V, 4, 3), seed + 2).reshape(-1)
    coarse, _ = bf.agg_map(L, BLOCK)
    Lc = tuple(l // bl for l, bl in zip(L, BLOCK))
    colour = bf.coords(Lc).sum(axis=1) % 2
    return U, Cl, D, b, x0, coarse, colour


def domain_rows(coarse, c):
    sites = np.nonzero(coarse == c)[0]
    return (sites[:, None] * 12 + np.arange(12)[None, :]).ravel()


def exact_half_sweep(D, b, x, coarse, colour, which):
    r = b - D @ x
    x = x.copy()
    for c in np.nonzero(colour == which)[0]:
        idx = domain_rows(coarse, c)
        x[idx] += np.linalg.solve(D[np.ix_(idx, idx)], r[idx])
    return x


def test_half_sweep_with_converged_domain_solves():
    U, Cl, D, b, x0, coarse, colour = problem(1601)
    x1 = oracle.sap(L, BLOCK, U, Cl, b, x0, 1, 300, m0=M0, colours=1)
    ref = exact_half_sweep(D, b, x0, coarse, colour, 0)
    assert np.linalg.norm(x1 - ref) < 1e-10 * np.linalg.norm(ref)
    untouched = np.concatenate([domain_rows(coarse, c) for c in np.nonzero(colour == 1)[0]])
    assert np.array_equal(x1[untouched], x0[untouched])


def test_full_cycle_visits_colour_0_then_colour_1():
    U, Cl, D, b, x0, coarse, colour = problem(1611)
    x1 = oracle.sap(L, BLOCK, U, Cl, b, x0, 1, 300, m0=M0)
    ref = exact_half_sweep(D, b, exact_half_sweep(D, b, x0, coarse, colour, 0), coarse, colour, 1)
    assert np.linalg.norm(x1 - ref) < 1e-10 * np.linalg.norm(ref)
    # colour-1 domains were solved last: their residual vanishes
    r = b - D @ x1
    last = np.concatenate([domain_rows(coarse, c) for c in np.nonzero(colour == 1)[0]])
    assert np.linalg.norm(r[last]) < 1e-9 * np.linalg.norm(b)
    assert np.linalg.norm(r) > 1e-3 * np.linalg.norm(b)


def test_one_mr_step_per_domain_closed_form():
    """e_B = alpha r_B with alpha = <D_B r_B, r_B> / |D_B r_B|^2."""
    U, Cl, D, b, x0, coarse, colour = problem(1621)
    x1 = oracle.sap(L, BLOCK, U, Cl, b, x0, 1, 1, m0=M0, colours=1)
    r = b - D @ x0
    ref = x0.copy()
    for c in np.nonzero(colour == 0)[0]:
        idx = domain_rows(coarse, c)
        p = D[np.ix_(idx, idx)] @ r[idx]
        ref[idx] += np.vdot(p, r[idx]) / np.vdot(p, p).real * r[idx]
    assert np.linalg.norm(x1 - ref) < 1e-13 * np.linalg.norm(ref)


def test_sap_lowers_the_residual_and_rejects_odd_coarse_extents():
    U, Cl, D, b, x0, coarse, colour = problem(1631)
    res = [np.linalg.norm(b - D @ oracle.sap(L, BLOCK, U, Cl, b, x0, k, 4, m0=M0)) for k in (0, 1, 2, 3)]
    assert res[0] > res[1] > res[2] > res[3]
    with pytest.raises(ValueError):
        oracle.sap((6, 2, 2, 4), (2, 1, 1, 2), syn.gauge_field((6, 2, 2, 4), 0.3, 1),
                   np.zeros((96, 12, 12), complex), np.zeros(1152, complex), np.zeros(1152, complex), 1, 1)
