"""Pins of the oracle's iterative setup, K-cycle and deeper coarsening (CPU).

The iterative refinement (Sec. 2.1, the DDalphaAMG-style setup) and the
K-cycle are iterations, not closed forms.  They are pinned by composing them
by hand from pieces that are pinned on their own elsewhere (restriction and
prolongation against the dense P, coarse GMRES against the least-squares
minimiser over the Krylov space, the coarse MR step against its 1-D minimiser,
the Galerkin product against dense P^dag D P, the Gram-Schmidt against numpy
QR) and checking the oracle's hierarchy routine against that composition.  A
plausible mistake in the routine (no normalisation, cycling with a stale or a
fresh P inside one iteration, skipping the re-taken Galerkin product below,
the wrong level's operator, the K-cycle's least-squares step or its
preconditioner) changes the result far above the 1e-12 bars.

The deeper Galerkin product (level 1 -> 2) is pinned against the dense
P_1^dag D_c1 P_1 and, on a lattice with distinct +-mu neighbours, column by
column.
"""
import numpy as np
import pytest

import oracle
import synthetic as syn
from tests import brute_force as bf


def rel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dims(L, block):
    return tuple(int(L[m]) // int(block[m]) for m in range(4))


def mr_steps(apply, b, x, steps):
    """Minimal residual steps from x on A x = b (each step: the 1-D residual
    minimiser along r, pinned in test_oracle_pins)."""
    x = x.copy()
    r = b - apply(x)
    for _ in range(steps):
        p = apply(r)
        a = np.vdot(p, r) / np.vdot(p, p)
        x = x + a * r
        r = r - a * p
    return x


class Levels:
    """Plain description of a hierarchy taken out of the oracle: level
    lattices, blocks, component counts, P and the coarse blocks."""

    def __init__(self, H, L, blocks, nv):
        self.H = H
        self.L = [tuple(L)]
        for b in blocks:
            self.L.append(_dims(self.L[-1], b))
        self.blocks = blocks
        self.nv = nv
        self.ns = [12] + [2 * n for n in nv]
        self.P = [H.P(l) for l in range(len(blocks))]
        self.Dc = [None] + [H.coarse(l) for l in range(1, len(blocks) + 1)]

    def n(self, l):
        return int(np.prod(self.L[l])) * self.ns[l]

    def apply(self, l, v):
        if l == 0:
            return self.H.apply(0, v)
        return oracle.coarse_apply(self.L[l], self.Dc[l], v.reshape(-1, self.ns[l])).reshape(-1)

    def restrict(self, l, v):
        return oracle.restrict(self.L[l], self.blocks[l], self.ns[l], self.P[l],
                               v.reshape(-1, self.ns[l])).reshape(-1)

    def prolong(self, l, e):
        return oracle.prolong(self.L[l], self.blocks[l], self.ns[l], self.P[l],
                              e.reshape(-1, self.ns[l + 1])).reshape(-1)


def v_cycle(lv, l, r, cfg):
    """Two-level cycle rooted at level l onto the coarsest level l+1: coarse
    GMRES on R r, prolong, post-smoothing MR on level l (no pre-smoothing)."""
    rc = lv.restrict(l, r)
    ec, _, _ = oracle.coarse_gmres(lv.L[l + 1], lv.Dc[l + 1], rc.reshape(-1, lv.ns[l + 1]),
                                   cfg["coarse_restart"], cfg["coarse_maxit"], cfg["coarse_tol"],
                                   cfg["coarse_fixed_iters"])
    x = lv.prolong(l, ec.reshape(-1))
    return mr_steps(lambda v: lv.apply(l, v), r, x, cfg["post_smooth"])


def fgmres_min(apply, precond, b, k):
    """k steps of flexible GMRES from x = 0: the Arnoldi vectors v_j, z_j =
    M v_j, and the result Z c with c the least-squares minimiser of
    |b - A Z c| (the defining property of the method)."""
    beta = np.linalg.norm(b)
    V = [b / beta]
    Z, AZ = [], []
    for j in range(k):
        z = precond(V[j])
        w = apply(z)
        Z.append(z)
        AZ.append(w)
        for v in V:  # modified Gram-Schmidt
            w = w - np.vdot(v, w) * v
        V.append(w / np.linalg.norm(w))
    c = np.linalg.lstsq(np.stack(AZ, axis=1), b, rcond=None)[0]
    return np.stack(Z, axis=1) @ c


def k_cycle(lv, r, cfg):
    """Three-level K-cycle rooted at level 0: restrict, kcycle_maxit steps of
    flexible GMRES on D_c1 preconditioned by the level-1 V-cycle, prolong,
    post-smooth on D."""
    rc = lv.restrict(0, r)
    ec = fgmres_min(lambda v: lv.apply(1, v), lambda v: v_cycle(lv, 1, v, cfg), rc, cfg["kcycle_maxit"])
    x = lv.prolong(0, ec)
    return mr_steps(lambda v: lv.apply(0, v), r, x, cfg["post_smooth"])


def normalised(v):
    return v / np.linalg.norm(v)


CFG = dict(coarse_restart=20, coarse_maxit=100, coarse_tol=0.05, coarse_fixed_iters=0, post_smooth=4,
           kcycle_maxit=3, kcycle_tol=0.0)


def _two_level(seed):
    L, block, nv = (4, 4, 4, 8), (2, 2, 2, 2), 4
    U = syn.gauge_field(L, 0.3, seed)
    kw = dict(m0=-0.05, blocks=(block,), nv=(nv,), **{k: CFG[k] for k in
                                                        ("coarse_restart", "coarse_maxit", "coarse_tol",
                                                         "coarse_fixed_iters", "post_smooth")})
    V = int(np.prod(L))
    start = syn.complex_gaussian((nv, V, 12), seed + 1)
    return L, block, nv, U, kw, start


def test_two_level_cycle_is_the_composition_of_its_pinned_steps():
    L, block, nv, U, kw, start = _two_level(1201)
    H = oracle.Hierarchy(L, U, **kw)
    H.set_start(0, start)
    H.setup()
    lv = Levels(H, L, (block,), (nv,))
    r = syn.complex_gaussian((lv.n(0),), 1203)
    assert rel(H.cycle(0, r), v_cycle(lv, 0, r, CFG)) < 1e-12


@pytest.mark.parametrize("iters", [1, 2])
def test_two_level_refinement_equals_its_composition(iters):
    """refine(k): per iteration, every vector becomes the normalised cycle of
    the PRE-iteration hierarchy applied to it; then P and D_c are rebuilt from
    the new vectors (the rebuild of a fresh hierarchy from those vectors)."""
    L, block, nv, U, kw, start = _two_level(1211)
    H = oracle.Hierarchy(L, U, **kw)
    H.set_start(0, start)
    H.setup()
    cur = H
    vecs = H.vectors(0)
    for _ in range(iters):
        lv = Levels(cur, L, (block,), (nv,))
        vecs = np.stack([normalised(v_cycle(lv, 0, vecs[i], CFG)) for i in range(nv)])
        cur = oracle.Hierarchy(L, U, **kw)
        cur.set_vectors(0, vecs)
    H.refine(iters)
    got = H.vectors(0)
    assert rel(got, vecs) < 1e-12
    for i in range(nv):
        assert abs(np.linalg.norm(got[i]) - 1.0) < 1e-13
    assert rel(H.P(0), cur.P(0)) < 1e-12
    assert rel(H.coarse(1), cur.coarse(1)) < 1e-12
    # the rebuilt P is the per-aggregate QR of the new vectors' chirality halves
    Pq, st = oracle.orthonormalise(L, block, 12, vecs)
    assert st == 0 and rel(H.P(0), Pq) < 1e-12


def _three_level(seed, kcycle=1):
    L, blocks, nv = (8, 8, 8, 8), ((2, 2, 2, 2), (2, 2, 2, 2)), (4, 4)
    U = syn.gauge_field(L, 0.25, seed)
    kw = dict(m0=-0.05, n_levels=3, blocks=blocks, nv=nv, kcycle=kcycle,
              **{k: CFG[k] for k in CFG})
    starts = [syn.complex_gaussian((nv[0], 4096, 12), seed + 1), syn.complex_gaussian((nv[1], 256, 8), seed + 2)]
    return L, blocks, nv, U, kw, starts


def test_kcycle_is_flexible_gmres_preconditioned_by_the_v_cycle():
    L, blocks, nv, U, kw, starts = _three_level(1221)
    H = oracle.Hierarchy(L, U, **kw)
    H.set_start(0, starts[0])
    H.set_start(1, starts[1])
    H.setup()
    lv = Levels(H, L, blocks, nv)
    # the level-1 cycle is the two-level cycle on D_c1
    u = syn.complex_gaussian((lv.n(1),), 1224)
    assert rel(H.cycle(1, u), v_cycle(lv, 1, u, CFG)) < 1e-12
    r = syn.complex_gaussian((lv.n(0),), 1225)
    got = H.cycle(0, r)
    assert rel(got, k_cycle(lv, r, CFG)) < 1e-11
    # a V-cycle in its place (a K-cycle that forgot its Krylov step) is far off
    rc = lv.restrict(0, r)
    vc = mr_steps(lambda v: lv.apply(0, v), r, lv.prolong(0, v_cycle(lv, 1, rc, CFG)), CFG["post_smooth"])
    assert rel(got, vc) > 1e-3


def test_kcycle_iteration_limit_and_tolerance():
    """kcycle_maxit bounds the level-1 Krylov steps; a loose kcycle_tol stops
    them early (after one step the estimate is below 0.99)."""
    L, blocks, nv, U, kw, starts = _three_level(1231)
    outs = {}
    for maxit, tol in ((1, 0.0), (3, 0.0), (3, 0.99)):
        kw2 = dict(kw, kcycle_maxit=maxit, kcycle_tol=tol)
        H = oracle.Hierarchy(L, U, **kw2)
        H.set_start(0, starts[0])
        H.set_start(1, starts[1])
        H.setup()
        lv = Levels(H, L, blocks, nv)
        r = syn.complex_gaussian((lv.n(0),), 1235)
        outs[(maxit, tol)] = H.cycle(0, r)
        if tol == 0.0:
            assert rel(outs[(maxit, tol)], k_cycle(lv, r, dict(CFG, kcycle_maxit=maxit))) < 1e-11
    assert rel(outs[(3, 0.99)], outs[(1, 0.0)]) < 1e-14


def test_three_level_refinement_equals_its_composition():
    """One iteration on three levels: level-0 vectors become normalised
    K-cycles of the pre-iteration hierarchy; P_0 and D_c1 are rebuilt, D_c2 is
    re-taken with the OLD P_1; then the level-1 vectors become normalised
    level-1 cycles on that intermediate hierarchy, and P_1, D_c2 are rebuilt."""
    L, blocks, nv, U, kw, starts = _three_level(1241)
    H = oracle.Hierarchy(L, U, **kw)
    H.set_start(0, starts[0])
    H.set_start(1, starts[1])
    H.setup()
    lv = Levels(H, L, blocks, nv)
    v0 = H.vectors(0)
    v1 = H.vectors(1)
    v0n = np.stack([normalised(k_cycle(lv, v0[i], CFG)) for i in range(nv[0])])
    mid = oracle.Hierarchy(L, U, **kw)
    mid.set_vectors(0, v0n)  # P_0, D_c1 from the new vectors (deeper levels not built yet)
    mid.set_vectors(1, v1)   # the old P_1 (same vectors, same Gram-Schmidt) and D_c2 = P_1^dag D_c1' P_1
    assert rel(mid.P(1), lv.P[1]) < 1e-14
    lm = Levels(mid, L, blocks, nv)
    v1n = np.stack([normalised(v_cycle(lm, 1, v1[i], CFG)) for i in range(nv[1])])
    fin = oracle.Hierarchy(L, U, **kw)
    fin.set_vectors(0, v0n)
    fin.set_vectors(1, v1n)
    H.refine(1)
    assert rel(H.vectors(0), v0n) < 1e-12
    assert rel(H.vectors(1), v1n) < 1e-12
    for l in (0, 1):
        assert rel(H.P(l), fin.P(l)) < 1e-12
    assert rel(H.coarse(1), fin.coarse(1)) < 1e-12
    assert rel(H.coarse(2), fin.coarse(2)) < 1e-12
    # level-1 refinement that skipped the re-taken Galerkin product (cycling on
    # the old D_c2) gives other vectors
    stale = _with_coarse(lm, 2, lv.Dc[2])
    v1_stale = np.stack([normalised(v_cycle(stale, 1, v1[i], CFG)) for i in range(nv[1])])
    assert rel(v1_stale, v1n) > 1e-6


def _with_coarse(lv, l, blocks):
    out = Levels.__new__(Levels)
    out.__dict__.update(lv.__dict__)
    out.Dc = list(lv.Dc)
    out.Dc[l] = blocks
    return out


def test_level_two_galerkin_equals_dense_product():
    """D_c2 = P_1^dag D_c1 P_1 on 8^4 -> 4^4 -> 2^4 (coarse extent 2 at level 2:
    the dense product sees the sum of the +-mu blocks) and sigma3-hermiticity
    one level down."""
    L, blocks, nv, U, kw, starts = _three_level(1251, kcycle=0)
    H = oracle.Hierarchy(L, U, **kw)
    H.set_start(0, starts[0])
    H.set_start(1, starts[1])
    H.setup()
    Dc1 = bf.dense_from_blocks((4, 4, 4, 4), H.coarse(1))
    P1 = bf.dense_prolongator((4, 4, 4, 4), blocks[1], 8, H.P(1))
    Dc2 = bf.dense_from_blocks((2, 2, 2, 2), H.coarse(2))
    assert np.max(np.abs(P1.conj().T @ Dc1 @ P1 - Dc2)) < 1e-12 * np.max(np.abs(Dc2))
    s3 = np.kron(np.eye(16), np.diag([1.0] * nv[1] + [-1.0] * nv[1]))
    assert np.max(np.abs(s3 @ Dc2 @ s3 - Dc2.conj().T)) < 1e-12 * np.max(np.abs(Dc2))


def test_level_two_galerkin_blocks_distinct_neighbours_column_by_column():
    """On 12x8x12x12 -> 6x4x6x6 -> 3x2x3x3 every level-2 +mu/-mu block is
    distinct (extent 3) in x, z, t: column (c, b) of D_c2 equals
    R_1 D_c1 P_1 e_{c,b}, block by block."""
    L, blocks, nv = (12, 8, 12, 12), ((2, 2, 2, 2), (2, 2, 2, 2)), (3, 3)
    L1, L2 = (6, 4, 6, 6), (3, 2, 3, 3)
    U = syn.gauge_field(L, 0.3, 1261)
    H = oracle.Hierarchy(L, U, m0=-0.05, n_levels=3, blocks=blocks, nv=nv, relax_sweeps=4)
    V, V1, V2 = int(np.prod(L)), int(np.prod(L1)), int(np.prod(L2))
    H.set_start(0, syn.complex_gaussian((nv[0], V, 12), 1262))
    H.set_start(1, syn.complex_gaussian((nv[1], V1, 6), 1263))
    H.setup()
    D1 = H.coarse(1)
    P1 = H.P(1)
    B2 = H.coarse(2)
    nb = 6
    for c in [0, 5, V2 - 1]:
        for b in range(nb):
            e = np.zeros((V2, nb), np.complex128)
            e[c, b] = 1.0
            col = oracle.restrict(L1, blocks[1], 6, P1, oracle.coarse_apply(L1, D1, oracle.prolong(L1, blocks[1], 6, P1, e)))
            expect = np.zeros((V2, nb), np.complex128)
            expect[c] += B2[c, 0][:, b]
            for d in range(1, 9):
                nbr = bf.neighbour(L2, d)
                for cp in np.nonzero(nbr == c)[0]:
                    expect[cp] += B2[cp, d][:, b]
            assert np.max(np.abs(col - expect)) < 1e-12 * np.max(np.abs(B2))
