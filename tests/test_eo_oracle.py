"""Pins of the oracle's even-odd preconditioning against dense linear algebra:
the Schur complement against numpy's block elimination of the dense D
(assembled from the pinned Wilson-clover apply), the per-site clover inverse
against the dense site blocks, the parity structure of D, and the even-odd
solve against the full system."""
import numpy as np

import oracle
import synthetic as syn

L = (4, 2, 2, 4)
M0 = -0.05


def dense_problem(seed):
    V = int(np.prod(L))
    U = syn.gauge_field(L, 0.3, seed)
    Cl = oracle.clover(L, U, 1.0)
    n = 12 * V
    D = oracle.wilson_apply(L, M0, True, U, Cl, np.eye(n).reshape(n, V, 4, 3)).reshape(n, n).T
    par = np.repeat(oracle.parity(L), 12)
    return U, Cl, D, par, V


def test_parity_structure_of_D():
    """Hops connect opposite parities only: D_ee and D_oo are site-diagonal."""
    U, Cl, D, par, V = dense_problem(1801)
    site = np.repeat(np.arange(V), 12)
    same = (par[:, None] == par[None, :]) & (site[:, None] != site[None, :])
    assert np.max(np.abs(D[same])) == 0.0


def test_clover_inverse_against_dense_site_blocks():
    U, Cl, D, par, V = dense_problem(1811)
    inv = oracle.clover_inverse(L, M0, Cl)
    for x in (0, 7, V - 1):
        A = (4 + M0) * np.eye(12) + Cl[x]
        assert np.max(np.abs(A @ inv[x] - np.eye(12))) < 1e-13
        assert np.max(np.abs(inv[x][:6, 6:])) == 0.0 and np.max(np.abs(inv[x][6:, :6])) == 0.0


def test_schur_complement_against_dense_elimination():
    U, Cl, D, par, V = dense_problem(1821)
    e, o = np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]
    Dhat = D[np.ix_(o, o)] - D[np.ix_(o, e)] @ np.linalg.solve(D[np.ix_(e, e)], D[np.ix_(e, o)])
    x = syn.complex_gaussian((V, 4, 3), 1822).reshape(-1)
    got = oracle.schur_apply(L, M0, True, U, Cl, x.reshape(V, 4, 3)).reshape(-1)
    assert np.linalg.norm(got[o] - Dhat @ x[o]) < 1e-13 * np.linalg.norm(Dhat @ x[o])
    assert np.max(np.abs(got[e])) == 0.0


def test_even_odd_solve_solves_the_full_system():
    Lh, block = (4, 4, 4, 4), (2, 2, 2, 2)
    V = 256
    U = syn.gauge_field(Lh, 0.3, 1831)
    H = oracle.Hierarchy(Lh, U, m0=M0, blocks=(block,), nv=(8,))
    H.set_start(0, syn.complex_gaussian((8, V, 12), 1832))
    H.setup()
    b = syn.complex_gaussian((V, 4, 3), 1833).reshape(-1)
    x, it, rel, st = H.solve_eo(b)
    assert st == 0 and rel <= 1e-10
    Cl = oracle.clover(Lh, U, 1.0)
    r = b - oracle.wilson_apply(Lh, M0, True, U, Cl, x.reshape(V, 4, 3)).reshape(-1)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
    x_full, it_full, rel_full, st_full = H.solve(b)
    assert np.linalg.norm(x - x_full) < 1e-8 * np.linalg.norm(x_full)
    assert 0 < it <= it_full + 2
