"""Pins of the CPU oracle against what the mathematics fixes.

Each test targets a mistake that could hide in the oracle: a dropped term, a
wrong sign, a wrong link placement, a transposed block, a wrong Gram-Schmidt
order.  None compares the oracle with a retyped copy of itself.
"""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests import brute_force as bf

RNG_TOL = 1e-12


def g5_on_fermion(psi):
    """gamma_5 = diag(1,1,-1,-1) on the spin index of [V][4][3] (chiral basis)."""
    out = psi.copy()
    out[..., 2:, :] *= -1
    return out


# ---------------------------------------------------------------- Dirac algebra
def test_gamma_basis_is_the_chiral_euclidean_basis():
    g, g5 = oracle.gammas()
    ref = bf.gamma_chiral()
    assert np.allclose(g, ref, atol=0)
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2 * np.eye(4) * (mu == nu))
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    assert np.allclose(g5, g[0] @ g[1] @ g[2] @ g[3])


# ---------------------------------------------------------------- clover term
def test_clover_vanishes_on_unit_links():
    L = (2, 2, 2, 4)
    C = oracle.clover(L, syn.unit_gauge(L), 1.0)
    assert np.max(np.abs(C)) == 0.0


def test_clover_hermitian_and_chirally_block_diagonal():
    L = (4, 4, 4, 4)
    U = syn.gauge_field(L, 0.3, 11)
    C = oracle.clover(L, U, 1.0)
    assert np.max(np.abs(C - np.conj(np.swapaxes(C, 1, 2)))) < 1e-14
    assert np.max(np.abs(C[:, :6, 6:])) < 1e-15 and np.max(np.abs(C[:, 6:, :6])) < 1e-15
    assert np.max(np.abs(C)) > 0.1


@pytest.mark.parametrize("mu,nu", [(0, 1), (0, 3), (1, 2), (2, 3)])
def test_clover_constant_abelian_field_closed_form(mu, nu):
    """Every mu-nu plaquette equals diag(e^{it}, e^{-it}, 1), so F_{mu nu} = i sin t
    diag(1,-1,0), every other F vanishes, and C = c_sw (i/2) sigma_{mu nu} (x) F."""
    L = (4, 4, 6, 4)
    U, theta = bf.constant_field(L, mu, nu)
    csw = 1.3
    C = oracle.clover(L, U, csw)
    g = bf.gamma_chiral()
    sigma = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
    F = 1j * np.sin(theta) * np.diag([1.0, -1.0, 0.0])
    expect = csw * 0.5j * np.kron(sigma, F)
    assert np.max(np.abs(C - expect[None])) < 1e-14
    # explicit sign in the chiral basis for the x-y plane: sigma_xy = -diag(s3, s3)
    if (mu, nu) == (0, 1):
        assert np.allclose(sigma, -np.diag([1, -1, 1, -1]))


def test_clover_gauge_covariant():
    L = (4, 4, 4, 4)
    U = syn.gauge_field(L, 0.3, 12)
    g = syn.random_gauge_transform(L, 13)
    C = oracle.clover(L, U, 1.0).reshape(-1, 4, 3, 4, 3)
    Cg = oracle.clover(L, bf.gauge_transform_links(L, U, g), 1.0).reshape(-1, 4, 3, 4, 3)
    expect = np.einsum("vab,vsbrc,vdc->vsard", g, C, np.conj(g))
    assert np.max(np.abs(Cg - expect)) < 1e-13


# ---------------------------------------------------------------- Wilson-clover D
def _fine(L, eps, seed, csw=1.0):
    U = syn.gauge_field(L, eps, seed)
    return U, oracle.clover(L, U, csw)


def test_dirac_gamma5_hermiticity():
    L = (4, 4, 4, 4)
    U, Cl = _fine(L, 0.3, 21)
    V = 256
    phi = syn.complex_gaussian((V, 4, 3), 22)
    psi = syn.complex_gaussian((V, 4, 3), 23)
    Dpsi = oracle.wilson_apply(L, -0.05, 1, U, Cl, psi)
    g5Dg5phi = g5_on_fermion(oracle.wilson_apply(L, -0.05, 1, U, Cl, g5_on_fermion(phi)))
    lhs = np.vdot(phi, Dpsi)
    rhs = np.vdot(g5Dg5phi, psi)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(phi) * np.linalg.norm(Dpsi)


@pytest.mark.parametrize("L,antiperiodic", [((2, 2, 2, 4), 1), ((2, 3, 2, 4), 1), ((2, 2, 3, 2), 0)])
def test_dirac_free_field_spectrum_closed_form(L, antiperiodic):
    m0 = -0.05
    V = int(np.prod(L))
    U = syn.unit_gauge(L)
    Cl = np.zeros((V, 12, 12), np.complex128)
    D = bf.dense_operator(lambda v: oracle.wilson_apply(L, m0, antiperiodic, U, Cl, v.reshape(V, 4, 3)).reshape(-1),
                          V * 12)
    ev = bf.sort_spectrum(np.linalg.eigvals(D))
    ref = bf.sort_spectrum(bf.free_eigenvalues(L, m0, bool(antiperiodic)))
    assert np.max(np.abs(ev - ref)) < 1e-12


def test_dirac_free_field_plane_wave():
    """D acting on e^{ipx} u gives [m0 + sum(1-cos p) + i sum gamma_mu sin p_mu] e^{ipx} u."""
    L = (4, 4, 4, 6)
    m0 = 0.1
    V = int(np.prod(L))
    X = bf.coords(L)
    n = np.array([1, 3, 2, 4])
    p = 2 * np.pi * n / np.array(L, float)
    p[3] = 2 * np.pi * (n[3] + 0.5) / L[3]
    u = syn.complex_gaussian((4, 3), 31)
    phase = np.exp(1j * (X @ p))
    psi = phase[:, None, None] * u[None]
    out = oracle.wilson_apply(L, m0, 1, syn.unit_gauge(L), np.zeros((V, 12, 12)), psi)
    g = bf.gamma_chiral()
    K = (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(g[mu] * np.sin(p[mu]) for mu in range(4))
    expect = phase[:, None, None] * (K @ u)[None]
    assert np.max(np.abs(out - expect)) < 1e-13


def test_dirac_gauge_covariant():
    L = (4, 4, 4, 4)
    U, Cl = _fine(L, 0.3, 41)
    g = syn.random_gauge_transform(L, 42)
    Ug = bf.gauge_transform_links(L, U, g)
    Clg = oracle.clover(L, Ug, 1.0)
    psi = syn.complex_gaussian((256, 4, 3), 43)
    lhs = oracle.wilson_apply(L, -0.05, 1, Ug, Clg, bf.gauge_transform_fermion(g, psi))
    rhs = bf.gauge_transform_fermion(g, oracle.wilson_apply(L, -0.05, 1, U, Cl, psi))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_dirac_is_mdiag_plus_eight_mdir():
    L = (2, 2, 4, 4)
    U, Cl = _fine(L, 0.3, 44)
    psi = syn.complex_gaussian((64, 4, 3), 45)
    tot = sum(oracle.wilson_term(L, 0.2, 1, U, Cl, d, psi) for d in range(9))
    assert np.max(np.abs(tot - oracle.wilson_apply(L, 0.2, 1, U, Cl, psi))) < 1e-14
    # Mdiag is (4+m0) plus the clover term, site-local
    diag = oracle.wilson_term(L, 0.2, 1, U, Cl, 0, psi)
    expect = 4.2 * psi.reshape(64, 12) + np.einsum("vij,vj->vi", Cl, psi.reshape(64, 12))
    assert np.max(np.abs(diag.reshape(64, 12) - expect)) < 1e-14


# ---------------------------------------------------------------- aggregation map
@pytest.mark.parametrize("L,block", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 4, 4, 8), (4, 4, 4, 4)),
                                      ((6, 4, 2, 8), (3, 2, 1, 4))])
def test_aggregation_map_bit_exact(L, block):
    c, o, site_of = oracle.agg_map(L, block)
    cb, ob = bf.agg_map(L, block)
    assert np.array_equal(c, cb) and np.array_equal(o, ob)
    A = int(np.prod(block))
    assert np.array_equal(site_of[c, o], np.arange(int(np.prod(L))))
    assert site_of.shape == (int(np.prod(L)) // A, A)


def test_aggregation_rejects_non_divisible():
    with pytest.raises(ValueError):
        oracle.agg_map((6, 4, 4, 4), (4, 2, 2, 2))


# ---------------------------------------------------------------- prolongator
def _aggregate_matrix(L, block, ns, v, c, chi, nv):
    coarse, _ = bf.agg_map(L, block)
    sites = np.nonzero(coarse == c)[0]
    h = ns // 2
    V = int(np.prod(L))
    v = v.reshape(nv, V, ns)
    return np.stack([v[i][sites][:, chi * h:(chi + 1) * h].reshape(-1) for i in range(nv)], axis=1)


@pytest.mark.parametrize("L,block,ns,nv", [((4, 4, 4, 4), (2, 2, 2, 2), 12, 6), ((4, 4, 4, 4), (4, 4, 2, 2), 24, 8)])
def test_prolongator_orthonormal_and_equal_to_qr(L, block, ns, nv):
    V = int(np.prod(L))
    vecs = syn.complex_gaussian((nv, V, ns), 51)
    Pv, st = oracle.orthonormalise(L, block, ns, vecs)
    assert st == 0
    Vc = V // int(np.prod(block))
    for c in range(Vc):
        for chi in range(2):
            X = _aggregate_matrix(L, block, ns, vecs, c, chi, nv)
            Q = _aggregate_matrix(L, block, ns, Pv, c, chi, nv)
            assert np.max(np.abs(Q.conj().T @ Q - np.eye(nv))) < 1e-14
            # Gram-Schmidt in index order = QR with a positive real diagonal of R
            q, r = np.linalg.qr(X)
            ph = np.diag(r) / np.abs(np.diag(r))
            assert np.max(np.abs(Q - q * ph[None, :])) < 1e-12


def test_prolongator_breakdown_flagged():
    L, block = (4, 4, 4, 4), (2, 2, 2, 2)
    vecs = syn.complex_gaussian((4, 256, 12), 52)
    vecs[3] = 2.0 * vecs[1]
    _, st = oracle.orthonormalise(L, block, 12, vecs)
    assert st != 0


def test_restrict_prolong_against_dense_prolongator():
    L, block, ns, nv = (4, 4, 4, 4), (2, 2, 2, 2), 12, 4
    V = 256
    Pv, _ = oracle.orthonormalise(L, block, ns, syn.complex_gaussian((nv, V, ns), 53))
    P = bf.dense_prolongator(L, block, ns, Pv)
    v = syn.complex_gaussian((V, ns), 54)
    rc = oracle.restrict(L, block, ns, Pv, v)
    assert np.max(np.abs(rc.reshape(-1) - P.conj().T @ v.reshape(-1))) < 1e-13
    phi = syn.complex_gaussian((16, 2 * nv), 55)
    pf = oracle.prolong(L, block, ns, Pv, phi)
    assert np.max(np.abs(pf.reshape(-1) - P @ phi.reshape(-1))) < 1e-13
    # R P = 1
    assert np.max(np.abs(P.conj().T @ P - np.eye(P.shape[1]))) < 1e-13
    rp = oracle.restrict(L, block, ns, Pv, oracle.prolong(L, block, ns, Pv, phi))
    assert np.max(np.abs(rp - phi)) < 1e-13


# ---------------------------------------------------------------- coarse operator
def _hierarchy(L, eps, seed, m0=-0.05, **kw):
    U = syn.gauge_field(L, eps, seed)
    H = oracle.Hierarchy(L, U, m0=m0, **kw)
    return H, U


def test_coarse_apply_against_dense_assembly_random_blocks():
    Lc, nb = (3, 2, 4, 3), 6
    Vc = int(np.prod(Lc))
    blocks = syn.complex_gaussian((Vc, 9, nb, nb), 61)
    phi = syn.complex_gaussian((2, Vc, nb), 62)
    out = oracle.coarse_apply(Lc, blocks, phi)
    M = bf.dense_from_blocks(Lc, blocks)
    for r in range(2):
        assert np.max(np.abs(out[r].reshape(-1) - M @ phi[r].reshape(-1))) < 1e-13


def test_galerkin_equals_dense_PdagDP_extent_two():
    L, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    H, U = _hierarchy(L, 0.3, 71, blocks=(block,), nv=(nv,))
    V = 256
    H.set_start(0, syn.complex_gaussian((nv, V, 12), 72))
    H.setup()
    Pv = H.P(0)
    P = bf.dense_prolongator(L, block, 12, Pv)
    D = bf.dense_operator(lambda v: H.apply(0, v), V * 12)
    Dc = bf.dense_from_blocks((2, 2, 2, 2), H.coarse(1))
    assert np.max(np.abs(P.conj().T @ D @ P - Dc)) < 1e-12 * np.max(np.abs(Dc))


def test_galerkin_blocks_distinct_neighbours_column_by_column():
    """On a 6x4x6x6 lattice with 2^4 aggregates the coarse x, z, t extents are 3, so
    every +mu/-mu block is distinct; D_c e_{c,b} = R D P e_{c,b} fixes each block."""
    L, block, nv = (6, 4, 6, 6), (2, 2, 2, 2), 3
    Lc = (3, 2, 3, 3)
    H, U = _hierarchy(L, 0.3, 73, blocks=(block,), nv=(nv,))
    V = int(np.prod(L))
    Vc, nb = int(np.prod(Lc)), 2 * nv
    H.set_start(0, syn.complex_gaussian((nv, V, 12), 74))
    H.setup()
    Pv = H.P(0)
    blocks = H.coarse(1)
    for c in [0, 7, Vc - 1]:
        for b in range(nb):
            e = np.zeros((Vc, nb), np.complex128)
            e[c, b] = 1.0
            col = oracle.restrict(L, block, 12, Pv, H.apply(0, oracle.prolong(L, block, 12, Pv, e)).reshape(V, 12))
            # column (c, b) of D_c: block 0 at c, block d of site c' with nbr(c', d) == c
            expect = np.zeros((Vc, nb), np.complex128)
            expect[c] += blocks[c, 0][:, b]
            for d in range(1, 9):
                nbr = bf.neighbour(Lc, d)
                for cp in np.nonzero(nbr == c)[0]:
                    expect[cp] += blocks[cp, d][:, b]
            assert np.max(np.abs(col - expect)) < 1e-12


def test_coarse_operator_sigma3_hermitian():
    L, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    H, _ = _hierarchy(L, 0.3, 75, blocks=(block,), nv=(nv,))
    H.set_start(0, syn.complex_gaussian((nv, 256, 12), 76))
    H.setup()
    Dc = bf.dense_from_blocks((2, 2, 2, 2), H.coarse(1))
    s3 = np.kron(np.eye(16), np.diag([1.0] * nv + [-1.0] * nv))
    assert np.max(np.abs(s3 @ Dc @ s3 - Dc.conj().T)) < 1e-12


@pytest.mark.parametrize("L,block,Lc", [((4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2)),
                                         ((6, 4, 4, 6), (2, 2, 2, 3), (3, 2, 2, 2)),
                                         ((6, 4, 4, 4), (3, 2, 2, 2), (2, 2, 2, 2))])
def test_coarse_backward_hops_mirror_forward_hops(L, block, Lc):
    """Term by term, the oracle's directly coarsened backward hop equals the
    sigma3-conjugated adjoint of the neighbour's forward hop (the relation the
    five-point storage and the five-term coarsening rely on), also where the
    coarse extent is 2 (c + mu = c - mu) and for odd aggregate extents."""
    nv = 4
    V = int(np.prod(L))
    H, _ = _hierarchy(L, 0.3, 81, blocks=(block,), nv=(nv,))
    H.set_start(0, syn.complex_gaussian((nv, V, 12), 82))
    H.setup()
    blocks = H.coarse(1)
    assert np.max(np.abs(bf.sigma3_mirror(Lc, blocks) - blocks)) < 1e-12 * np.max(np.abs(blocks))
    s = bf.sigma3(2 * nv)
    M0 = blocks[:, 0]
    assert np.max(np.abs(s[:, None] * s[None, :] * np.conj(np.swapaxes(M0, -1, -2)) - M0)) < 1e-12
    # a planted error in one forward block breaks the relation
    bad = blocks.copy()
    bad[0, 1, 0, 1] += 1e-3
    assert np.max(np.abs(bf.sigma3_mirror(Lc, bad) - bad)) > 1e-4


def test_coarse_operator_gauge_invariant():
    L, block, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    U = syn.gauge_field(L, 0.3, 77)
    g = syn.random_gauge_transform(L, 78)
    start = syn.complex_gaussian((nv, 256, 4, 3), 79)
    H1 = oracle.Hierarchy(L, U, blocks=(block,), nv=(nv,))
    H1.set_start(0, start)
    H1.setup()
    H2 = oracle.Hierarchy(L, bf.gauge_transform_links(L, U, g), blocks=(block,), nv=(nv,))
    H2.set_start(0, np.stack([bf.gauge_transform_fermion(g, s) for s in start]))
    H2.setup()
    assert np.max(np.abs(H1.coarse(1) - H2.coarse(1))) < 1e-11


def test_unitary_prolongator_preserves_spectrum_and_solves_in_one_step():
    """Aggregates of one site with Nv = 6 (Nb = 12) make P unitary: D_c is similar
    to D, and a two-grid cycle with an exact coarse solve solves D x = b at once."""
    L = (2, 2, 2, 4)
    V = 32
    kw = dict(blocks=((1, 1, 1, 1),), nv=(6,), coarse_tol=1e-14, coarse_maxit=2000, coarse_restart=400,
              post_smooth=0, outer_restart=4, outer_tol=1e-10)
    H, U = _hierarchy(L, 0.3, 81, **kw)
    H.set_start(0, syn.complex_gaussian((6, V, 12), 82))
    H.setup()
    D = bf.dense_operator(lambda v: H.apply(0, v), V * 12)
    Dc = bf.dense_from_blocks(L, H.coarse(1))
    ev, evc = bf.sort_spectrum(np.linalg.eigvals(D)), bf.sort_spectrum(np.linalg.eigvals(Dc))
    assert np.max(np.abs(ev - evc)) < 1e-10
    b = syn.complex_gaussian((V, 12), 83).reshape(-1)
    x, it, rel, st = H.solve(b)
    assert st == 0 and it == 1 and rel < 1e-10


# ---------------------------------------------------------------- Krylov solvers
def _coarse_problem(Lc=(2, 2, 2, 2), nb=8, seed=91, shift=6.0):
    Vc = int(np.prod(Lc))
    blocks = 0.5 * syn.complex_gaussian((Vc, 9, nb, nb), seed) / np.sqrt(nb)
    blocks[:, 0] += shift * np.eye(nb)
    return Lc, blocks


def test_mr_step_is_the_one_dimensional_residual_minimiser():
    Lc, blocks = _coarse_problem()
    M = bf.dense_from_blocks(Lc, blocks)
    n = M.shape[0]
    b = syn.complex_gaussian((n,), 92)
    x0 = syn.complex_gaussian((n,), 93)
    x1 = oracle.coarse_mr(Lc, blocks, b.reshape(16, 8), x0.reshape(16, 8), 1).reshape(-1)
    r0 = b - M @ x0
    # minimise || r0 - a M r0 || over complex a with a least-squares solve
    a = np.linalg.lstsq((M @ r0)[:, None], r0, rcond=None)[0][0]
    assert np.max(np.abs(x1 - (x0 + a * r0))) < 1e-12
    # residual norms never increase
    prev = np.linalg.norm(r0)
    x = x0
    for _ in range(6):
        x = oracle.coarse_mr(Lc, blocks, b.reshape(16, 8), x.reshape(16, 8), 1).reshape(-1)
        cur = np.linalg.norm(b - M @ x)
        assert cur <= prev * (1 + 1e-14)
        prev = cur


@pytest.mark.parametrize("k", [1, 3, 7])
def test_gmres_iterate_minimises_residual_over_krylov_space(k):
    Lc, blocks = _coarse_problem(seed=94, shift=3.0)
    M = bf.dense_from_blocks(Lc, blocks)
    b = syn.complex_gaussian((16, 8), 95)
    x, it, _ = oracle.coarse_gmres(Lc, blocks, b, restart=20, maxit=k, tol=0.0)
    assert it == k
    bb = b.reshape(-1)
    K = [bb]
    for _ in range(k - 1):
        K.append(M @ K[-1])
    K = np.stack(K, axis=1)
    y = np.linalg.lstsq(M @ K, bb, rcond=None)[0]
    assert np.max(np.abs(x.reshape(-1) - K @ y)) < 1e-10 * np.linalg.norm(K @ y)


def test_gmres_converges_to_dense_solve():
    Lc, blocks = _coarse_problem(seed=96, shift=4.0)
    M = bf.dense_from_blocks(Lc, blocks)
    b = syn.complex_gaussian((16, 8), 97)
    x, it, est = oracle.coarse_gmres(Lc, blocks, b, restart=10, maxit=400, tol=1e-13)
    ref = np.linalg.solve(M, b.reshape(-1))
    assert est <= 1e-13
    assert np.linalg.norm(x.reshape(-1) - ref) <= 1e-11 * np.linalg.norm(ref)
    # fixed-iteration mode runs exactly that many iterations
    _, it2, _ = oracle.coarse_gmres(Lc, blocks, b, restart=10, maxit=400, tol=0.5, fixed=13)
    assert it2 == 13


# ---------------------------------------------------------------- MG solve
def test_two_level_solve_config1():
    """Two-level MG, 4^4, Nv = 8 (Nb = 16), 20 relaxation sweeps, MR(4), FGMRES(16)."""
    L = (4, 4, 4, 4)
    V = 256
    H, U = _hierarchy(L, 0.3, 101, m0=-0.05, blocks=((2, 2, 2, 2),), nv=(8,), outer_restart=16)
    H.set_start(0, syn.complex_gaussian((8, V, 12), 102))
    H.setup()
    b = syn.complex_gaussian((V, 12), 103).reshape(-1)
    x, it, rel, st = H.solve(b)
    assert st == 0 and rel <= 1e-10
    # the residual, recomputed with the dense operator assembled column by column
    D = bf.dense_operator(lambda v: H.apply(0, v), V * 12)
    assert np.linalg.norm(b - D @ x) <= 1.01e-10 * np.linalg.norm(b)
    assert it < 60


def test_relaxation_lowers_the_residual_of_near_null_vectors():
    L = (4, 4, 4, 4)
    V = 256
    H, U = _hierarchy(L, 0.3, 104, blocks=((2, 2, 2, 2),), nv=(4,))
    start = syn.complex_gaussian((4, V, 12), 105)
    H.set_start(0, start)
    H.setup()
    v = H.vectors(0)
    for i in range(4):
        assert abs(np.linalg.norm(v[i]) - 1.0) < 1e-13
        r_after = np.linalg.norm(H.apply(0, v[i]))
        r_before = np.linalg.norm(H.apply(0, start[i].reshape(-1))) / np.linalg.norm(start[i])
        assert r_after < 0.5 * r_before


def test_refinement_trend_and_three_level_kcycle():
    """Outer iterations do not grow with the number of refinement iterations
    (the shape of the paper's Table 2), and a three-level K-cycle converges."""
    L = (8, 8, 8, 8)
    V = 4096
    its = []
    for n in (0, 1, 2):
        H, U = _hierarchy(L, 0.25, 111, m0=-0.05, blocks=((2, 2, 2, 2),), nv=(6,), outer_restart=20)
        H.set_start(0, syn.complex_gaussian((6, V, 12), 112))
        H.setup()
        H.refine(n)
        b = syn.complex_gaussian((V, 12), 113).reshape(-1)
        x, it, rel, st = H.solve(b)
        assert st == 0 and rel <= 1e-10
        its.append(it)
    assert its[1] <= its[0] + 1 and its[2] <= its[1] + 1
    H3, U = _hierarchy(L, 0.25, 111, m0=-0.05, n_levels=3, blocks=((2, 2, 2, 2), (2, 2, 2, 2)), nv=(6, 6),
                       kcycle=1, outer_restart=20)
    H3.set_start(0, syn.complex_gaussian((6, V, 12), 112))
    H3.set_start(1, syn.complex_gaussian((6, 256, 12), 114))
    H3.setup()
    H3.refine(1)
    x, it, rel, st = H3.solve(b)
    assert st == 0 and rel <= 1e-10


def test_gmres_on_a_singular_operator_keeps_the_least_squares_minimiser():
    """A zero operator makes the first rotated Hessenberg column vanish
    exactly: the minimiser over the Krylov space is x = 0 with the residual
    |b| (not a division by zero).  A block-diagonal operator with a null space
    and b inside it gives the same."""
    Lc, nb = (2, 2, 2, 2), 4
    Vc = 16
    b = syn.complex_gaussian((Vc, nb), 98)
    x, it, est = oracle.coarse_gmres(Lc, np.zeros((Vc, 9, nb, nb), np.complex128), b, restart=10, maxit=10, tol=1e-12)
    assert it == 1 and np.all(x == 0) and abs(est - 1.0) < 1e-15
    blocks = np.zeros((Vc, 9, nb, nb), np.complex128)
    blocks[:, 0] = np.diag([1.0, 2.0, 0.0, 0.0])
    bn = np.zeros((Vc, nb), np.complex128)
    bn[:, 2:] = b[:, 2:]
    x, it, est = oracle.coarse_gmres(Lc, blocks, bn, restart=10, maxit=10, tol=1e-12)
    assert it == 1 and np.all(x == 0) and abs(est - 1.0) < 1e-15
