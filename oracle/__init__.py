"""CPU oracle for the Wilson-clover multigrid path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does.

The arithmetic lives in ``wcmg_oracle.cpp`` (plain FP64 C++, OpenMP over
sites); this module only builds it with g++ and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wcmg_oracle.cpp")
LIB = os.path.join(HERE, "libwcmg_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2 -fopenmp).  Returns the library path."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O2", "-fopenmp", "-std=c++17", "-shared", "-fPIC", SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [
        ("L", C.c_int * 4), ("m0", C.c_double), ("csw", C.c_double), ("antiperiodic", C.c_int),
        ("n_levels", C.c_int), ("block", (C.c_int * 4) * 3), ("nv", C.c_int * 3),
        ("relax_sweeps", C.c_int), ("refine_iters", C.c_int), ("post_smooth", C.c_int),
        ("coarse_restart", C.c_int), ("coarse_maxit", C.c_int), ("coarse_fixed_iters", C.c_int),
        ("coarse_tol", C.c_double),
        ("kcycle", C.c_int), ("kcycle_maxit", C.c_int), ("kcycle_tol", C.c_double),
        ("outer_restart", C.c_int), ("outer_maxit", C.c_int), ("outer_tol", C.c_double),
        ("smoother", C.c_int), ("sap_block_iters", C.c_int),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        l = C.CDLL(LIB)
        dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p
        l.or_mg_create.restype = vp
        l.or_mg_create.argtypes = [C.POINTER(Params), dp, dp]
        l.or_mg_destroy.argtypes = [vp]
        l.or_mg_error.restype = C.c_char_p
        l.or_mg_error.argtypes = [vp]
        l.or_mg_size.restype = C.c_long
        l.or_mg_size.argtypes = [vp, C.c_int]
        for name in ("or_mg_setup",):
            getattr(l, name).argtypes = [vp]
        l.or_mg_refine.argtypes = [vp, C.c_int]
        l.or_mg_set_start.argtypes = [vp, C.c_int, dp]
        l.or_mg_set_vectors.argtypes = [vp, C.c_int, dp]
        for name in ("or_mg_get_vectors", "or_mg_get_P", "or_mg_get_coarse"):
            getattr(l, name).argtypes = [vp, C.c_int, dp]
        l.or_mg_get_clover.argtypes = [vp, dp]
        l.or_mg_apply.argtypes = [vp, C.c_int, dp, dp]
        l.or_mg_cycle.argtypes = [vp, C.c_int, dp, dp]
        l.or_mg_solve.argtypes = [vp, dp, dp, C.POINTER(C.c_int), dp]
        l.or_clover.argtypes = [ip, dp, C.c_double, dp]
        l.or_agg_map.argtypes = [ip, ip, ip, ip, ip]
        l.or_coarse_apply.argtypes = [ip, C.c_int, dp, dp, dp, C.c_int]
        l.or_wilson_apply.argtypes = [ip, C.c_double, C.c_int, dp, dp, dp, dp, C.c_int]
        l.or_wilson_term.argtypes = [ip, C.c_double, C.c_int, dp, dp, C.c_int, dp, dp]
        l.or_orthonormalise.argtypes = [ip, ip, C.c_int, C.c_int, dp, dp]
        l.or_restrict.argtypes = [ip, ip, C.c_int, C.c_int, dp, dp, dp, C.c_int]
        l.or_prolong.argtypes = [ip, ip, C.c_int, C.c_int, dp, dp, dp, C.c_int]
        l.or_coarse_gmres.argtypes = [ip, C.c_int, dp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_int, dp]
        l.or_coarse_mr.argtypes = [ip, C.c_int, dp, dp, dp, C.c_int]
        l.or_sap.argtypes = [ip, ip, C.c_double, C.c_int, dp, dp, dp, dp, C.c_int, C.c_int, C.c_int]
        l.or_schur_apply.argtypes = [ip, C.c_double, C.c_int, dp, dp, dp, dp]
        l.or_clover_inverse.argtypes = [ip, C.c_double, dp, dp]
        l.or_mg_solve_eo.argtypes = [vp, dp, dp, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        l.or_gamma.argtypes = [dp, dp]
        l.or_num_threads.restype = C.c_int
        _lib = l
    return _lib


def _c(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(seq) -> "C.Array":
    return (C.c_int32 * len(seq))(*[int(s) for s in seq])


def vol(L) -> int:
    return int(np.prod(L))


def num_threads() -> int:
    return lib().or_num_threads()


def gammas():
    g = np.zeros((4, 4, 4), np.complex128)
    g5 = np.zeros((4, 4), np.complex128)
    lib().or_gamma(_dp(g), _dp(g5))
    return g, g5


def clover(L, U, csw) -> np.ndarray:
    """Clover term C(x), shape [V][12][12]."""
    U = _c(U)
    out = np.zeros((vol(L), 12, 12), np.complex128)
    lib().or_clover(_ip(L), _dp(U), float(csw), _dp(out))
    return out


def agg_map(L, block):
    V = vol(L)
    A = int(np.prod(block))
    coarse = np.zeros(V, np.int32)
    offset = np.zeros(V, np.int32)
    site_of = np.zeros(V, np.int32)
    st = lib().or_agg_map(_ip(L), _ip(block), coarse.ctypes.data_as(C.POINTER(C.c_int32)),
                          offset.ctypes.data_as(C.POINTER(C.c_int32)), site_of.ctypes.data_as(C.POINTER(C.c_int32)))
    if st:
        raise ValueError("lattice extent not divisible by the block")
    return coarse, offset, site_of.reshape(V // A, A)


def wilson_apply(L, m0, antiperiodic, U, Cl, psi) -> np.ndarray:
    """D psi for psi of shape [nrhs][V][4][3] (or [V][4][3])."""
    psi = _c(psi)
    single = psi.ndim == 3
    p = psi.reshape(-1, vol(L), 12)
    out = np.zeros_like(p)
    U, Cl = _c(U), _c(Cl)
    lib().or_wilson_apply(_ip(L), float(m0), int(antiperiodic), _dp(U), _dp(Cl), _dp(p), _dp(out), p.shape[0])
    return out.reshape(psi.shape)


def wilson_term(L, m0, antiperiodic, U, Cl, d, psi) -> np.ndarray:
    psi = _c(psi)
    out = np.zeros_like(psi)
    U, Cl = _c(U), _c(Cl)
    lib().or_wilson_term(_ip(L), float(m0), int(antiperiodic), _dp(U), _dp(Cl), int(d), _dp(psi), _dp(out))
    return out


def coarse_apply(Lc, blocks, phi) -> np.ndarray:
    """D_c phi with blocks [Vc][9][Nb][Nb], phi [nrhs][Vc][Nb] or [Vc][Nb]."""
    blocks, phi = _c(blocks), _c(phi)
    nb = blocks.shape[-1]
    p = phi.reshape(-1, vol(Lc), nb)
    out = np.zeros_like(p)
    lib().or_coarse_apply(_ip(Lc), nb, _dp(blocks), _dp(p), _dp(out), p.shape[0])
    return out.reshape(phi.shape)


def orthonormalise(L, block, ns, vecs):
    vecs = _c(vecs)
    nv = vecs.shape[0]
    out = np.zeros_like(vecs)
    st = lib().or_orthonormalise(_ip(L), _ip(block), int(ns), nv, _dp(vecs), _dp(out))
    return out, st


def restrict(L, block, ns, Pv, fine):
    Pv, fine = _c(Pv), _c(fine)
    nv = Pv.shape[0]
    V = vol(L)
    Vc = V // int(np.prod(block))
    f = fine.reshape(-1, V, ns)
    out = np.zeros((f.shape[0], Vc, 2 * nv), np.complex128)
    lib().or_restrict(_ip(L), _ip(block), int(ns), nv, _dp(Pv), _dp(f), _dp(out), f.shape[0])
    return out[0] if fine.size == V * ns else out


def prolong(L, block, ns, Pv, coarse):
    Pv, coarse = _c(Pv), _c(coarse)
    nv = Pv.shape[0]
    V = vol(L)
    Vc = V // int(np.prod(block))
    c = coarse.reshape(-1, Vc, 2 * nv)
    out = np.zeros((c.shape[0], V, ns), np.complex128)
    lib().or_prolong(_ip(L), _ip(block), int(ns), nv, _dp(Pv), _dp(c), _dp(out), c.shape[0])
    return out[0] if coarse.size == Vc * 2 * nv else out


def coarse_gmres(Lc, blocks, b, restart=20, maxit=100, tol=0.05, fixed=0):
    blocks, b = _c(blocks), _c(b)
    x = np.zeros_like(b)
    est = C.c_double(0.0)
    it = lib().or_coarse_gmres(_ip(Lc), blocks.shape[-1], _dp(blocks), _dp(b), _dp(x), int(restart), int(maxit),
                               float(tol), int(fixed), C.byref(est))
    return x, it, est.value


def sap(L, block, U, clover, b, x0, cycles, block_iters, m0=-0.05, antiperiodic=True, colours=2):
    """SAP cycles on the fine operator (domains: the aggregates of `block`,
    red-black by coarse-coordinate parity); x0 is the initial guess.
    colours=1 runs only the colour-0 half of one cycle."""
    U, clover, b = _c(U), _c(clover), _c(b)
    x = _c(x0).copy()
    st = lib().or_sap(_ip(L), _ip(block), float(m0), int(antiperiodic), _dp(U), _dp(clover), _dp(b), _dp(x),
                      int(cycles), int(block_iters), int(colours))
    if st:
        raise ValueError("SAP needs even coarse extents")
    return x


def schur_apply(L, m0, antiperiodic, U, Cl, psi) -> np.ndarray:
    """Even-odd Schur complement Dhat = A_oo - H_oe A_ee^{-1} H_eo applied to the
    odd part of psi [V][4][3]; the even part of the result is zero."""
    psi = _c(psi)
    out = np.zeros_like(psi)
    st = lib().or_schur_apply(_ip(L), float(m0), int(antiperiodic), _dp(_c(U)), _dp(_c(Cl)), _dp(psi), _dp(out))
    if st:
        raise ValueError("singular clover block")
    return out


def clover_inverse(L, m0, Cl) -> np.ndarray:
    """((4 + m0) + C(x))^{-1} per site, [V][12][12]."""
    out = np.zeros((vol(L), 12, 12), np.complex128)
    st = lib().or_clover_inverse(_ip(L), float(m0), _dp(_c(Cl)), _dp(out))
    if st:
        raise ValueError("singular clover block")
    return out


def parity(L) -> np.ndarray:
    """Site parity (x + y + z + t) mod 2 of the lexicographic sites."""
    V = vol(L)
    i = np.arange(V)
    c = [i % L[0], i // L[0] % L[1], i // (L[0] * L[1]) % L[2], i // (L[0] * L[1] * L[2])]
    return (c[0] + c[1] + c[2] + c[3]) % 2


def coarse_mr(Lc, blocks, b, x0, steps):
    blocks, b = _c(blocks), _c(b)
    x = _c(x0).copy()
    lib().or_coarse_mr(_ip(Lc), blocks.shape[-1], _dp(blocks), _dp(b), _dp(x), int(steps))
    return x


DEFAULTS = dict(
    m0=-0.05, csw=1.0, antiperiodic=1, n_levels=2, blocks=((2, 2, 2, 2),), nv=(8,), relax_sweeps=20,
    refine_iters=0, post_smooth=4, coarse_restart=20, coarse_maxit=100, coarse_fixed_iters=0, coarse_tol=0.05,
    kcycle=0, kcycle_maxit=5, kcycle_tol=0.1, outer_restart=16, outer_maxit=500, outer_tol=1e-10,
    smoother=0, sap_block_iters=4,
)


class Hierarchy:
    """Oracle multigrid hierarchy (relaxation setup, refinement, cycle, FGMRES)."""

    def __init__(self, L, U, clover=None, **kw):
        cfg = dict(DEFAULTS)
        cfg.update(kw)
        self.cfg = cfg
        self.L = tuple(int(x) for x in L)
        p = Params()
        for mu in range(4):
            p.L[mu] = self.L[mu]
        p.m0, p.csw, p.antiperiodic = cfg["m0"], cfg["csw"], int(cfg["antiperiodic"])
        p.n_levels = cfg["n_levels"]
        for l, b in enumerate(cfg["blocks"]):
            for mu in range(4):
                p.block[l][mu] = int(b[mu])
        for l, n in enumerate(cfg["nv"]):
            p.nv[l] = int(n)
        for k in ("relax_sweeps", "refine_iters", "post_smooth", "coarse_restart", "coarse_maxit",
                  "coarse_fixed_iters", "kcycle", "kcycle_maxit", "outer_restart", "outer_maxit", "smoother",
                  "sap_block_iters"):
            setattr(p, k, int(cfg[k]))
        for k in ("coarse_tol", "kcycle_tol", "outer_tol"):
            setattr(p, k, float(cfg[k]))
        self.p = p
        self._U = _c(U)
        self._C = None if clover is None else _c(clover)
        h = lib().or_mg_create(C.byref(p), _dp(self._U), None if self._C is None else _dp(self._C))
        if not h:
            raise ValueError("invalid hierarchy parameters")
        self.h = h
        self.nlev = cfg["n_levels"]

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_mg_destroy(self.h)
            self.h = None

    def size(self, l):
        return lib().or_mg_size(self.h, l)

    def nv(self, l):
        return self.cfg["nv"][l]

    def set_start(self, l, v):
        v = _c(v)
        assert v.size == self.nv(l) * self.size(l)
        self._keep = getattr(self, "_keep", {})
        lib().or_mg_set_start(self.h, l, _dp(v))

    def setup(self):
        st = lib().or_mg_setup(self.h)
        if st:
            raise RuntimeError("oracle setup failed: %s (%d)" % (lib().or_mg_error(self.h).decode(), st))

    def refine(self, iters):
        st = lib().or_mg_refine(self.h, int(iters))
        if st:
            raise RuntimeError("oracle refine failed: %s" % lib().or_mg_error(self.h).decode())

    def set_vectors(self, l, v):
        v = _c(v)
        st = lib().or_mg_set_vectors(self.h, l, _dp(v))
        if st:
            raise RuntimeError("oracle rebuild failed: %s" % lib().or_mg_error(self.h).decode())

    def vectors(self, l):
        out = np.zeros(self.nv(l) * self.size(l), np.complex128)
        lib().or_mg_get_vectors(self.h, l, _dp(out))
        return out.reshape(self.nv(l), -1)

    def P(self, l):
        out = np.zeros(self.nv(l) * self.size(l), np.complex128)
        lib().or_mg_get_P(self.h, l, _dp(out))
        return out.reshape(self.nv(l), -1)

    def coarse(self, l):
        """Blocks [Vc][9][Nb][Nb] of the level-l operator (l >= 1)."""
        nb = 2 * self.nv(l - 1)
        n = self.size(l) // nb
        out = np.zeros((n, 9, nb, nb), np.complex128)
        lib().or_mg_get_coarse(self.h, l, _dp(out))
        return out

    def clover(self):
        out = np.zeros((vol(self.L), 12, 12), np.complex128)
        lib().or_mg_get_clover(self.h, _dp(out))
        return out

    def apply(self, l, v):
        v = _c(v).reshape(-1)
        out = np.zeros_like(v)
        lib().or_mg_apply(self.h, l, _dp(v), _dp(out))
        return out

    def cycle(self, l, r):
        r = _c(r).reshape(-1)
        out = np.zeros_like(r)
        lib().or_mg_cycle(self.h, l, _dp(r), _dp(out))
        return out

    def solve_eo(self, b, x0=None):
        """Even-odd preconditioned outer solve (Schur complement on the odd sites)."""
        b = _c(b).reshape(-1)
        x = np.zeros_like(b) if x0 is None else _c(x0).reshape(-1).copy()
        it = C.c_int(0)
        rr = C.c_double(0.0)
        st = lib().or_mg_solve_eo(self.h, _dp(b), _dp(x), C.byref(it), C.byref(rr))
        return x, it.value, rr.value, st

    def solve(self, b, x0=None):
        b = _c(b).reshape(-1)
        x = np.zeros_like(b) if x0 is None else _c(x0).reshape(-1).copy()
        it = C.c_int(0)
        rr = C.c_double(0.0)
        st = lib().or_mg_solve(self.h, _dp(b), _dp(x), C.byref(it), C.byref(rr))
        return x, it.value, rr.value, st
