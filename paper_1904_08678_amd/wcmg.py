"""ctypes binding of the wcmg C ABI (include/wcmg.h).

Torch supplies device memory and the stream; every operation runs in the HIP
kernels of libwcmg.so.
"""
from __future__ import annotations

import atexit
import ctypes as C
import itertools
import json
import os
import sys
import weakref

import numpy as np
import torch

F64, F32, BF16 = 0, 1, 2
BATCH_GRAPH, BATCH_VECTOR, BATCH_MFMA, BATCH_DSLASH_PER_RHS = 1, 2, 4, 8
_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libwcmg.so")
_lib = None

# Every live handle (context, network, standalone coarse operator), so that
# they can be destroyed from an atexit hook: Python runs atexit hooks before
# it tears modules down, while the HIP runtime (and any profiling tool loaded
# into the process) is still fully alive.  Destroying them later, from
# finalizer order during interpreter shutdown, would free pinned host memory
# and streams after the runtime has begun its own teardown.
_live = weakref.WeakValueDictionary()
_order = itertools.count()


def _register(obj):
    _live[next(_order)] = obj


def close_all():
    """Destroy every live wcmg handle, newest first (also run at exit)."""
    for k in sorted(list(_live.keys()), reverse=True):
        obj = _live.get(k)
        if obj is not None:
            obj.close()


atexit.register(close_all)

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_DIMS", 3: "ERR_STATE", 4: "ERR_HIP", 5: "ERR_NOMEM", 6: "ERR_BREAKDOWN",
          7: "ERR_NOCONV", 8: "ERR_NAN"}


class WcmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("dims", C.c_int32 * 4), ("m0", C.c_double), ("c_sw", C.c_double), ("antiperiodic_t", C.c_int32),
        ("n_levels", C.c_int32), ("block", (C.c_int32 * 4) * 3), ("n_vec", C.c_int32 * 3),
        ("relax_sweeps", C.c_int32), ("refine_iters", C.c_int32), ("post_smooth", C.c_int32),
        ("coarse_restart", C.c_int32), ("coarse_maxit", C.c_int32), ("coarse_fixed_iters", C.c_int32),
        ("coarse_tol", C.c_double), ("kcycle", C.c_int32), ("kcycle_maxit", C.c_int32), ("kcycle_tol", C.c_double),
        ("outer_restart", C.c_int32), ("outer_maxit", C.c_int32), ("outer_tol", C.c_double),
        ("cycle_prec", C.c_int32), ("coarse_store_prec", C.c_int32), ("setup_prec", C.c_int32),
        ("coarse_points", C.c_int32), ("smoother", C.c_int32), ("sap_block_iters", C.c_int32),
        ("even_odd", C.c_int32), ("reserved", C.c_int32 * 1),
    ]


class SolveInfo(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("converged", C.c_int32), ("true_rel_res", C.c_double),
                ("t_solve_s", C.c_double), ("coarse_iters", C.c_int64), ("cycles", C.c_int64)]


def lib():
    """Load libwcmg.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError("libwcmg.so is not built; run `python -m paper_1904_08678_amd.build`")
        l = C.CDLL(library_path)
        vp, ip = C.c_void_p, C.c_int
        l.wcmg_default_params.argtypes = [C.POINTER(Params)]
        l.wcmg_create.argtypes = [C.POINTER(Params), vp, C.POINTER(vp)]
        l.wcmg_destroy.argtypes = [vp]
        l.wcmg_last_error.argtypes = [vp]
        l.wcmg_last_error.restype = C.c_char_p
        for name in ("wcmg_set_gauge", "wcmg_set_clover", "wcmg_get_clover"):
            getattr(l, name).argtypes = [vp, vp]
        l.wcmg_set_null_vectors.argtypes = [vp, ip, vp, ip]
        for name in ("wcmg_get_null_vectors", "wcmg_get_prolongator", "wcmg_rebuild_from_vectors"):
            getattr(l, name).argtypes = [vp, ip, vp]
        for name in ("wcmg_get_coarse_op", "wcmg_set_coarse_op"):
            getattr(l, name).argtypes = [vp, ip, vp, ip]
        l.wcmg_setup.argtypes = [vp]
        l.wcmg_setup_export.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
        l.wcmg_setup_import.argtypes = [vp, vp, C.c_size_t]
        l.wcmg_refine.argtypes = [vp, ip]
        l.wcmg_get_aggregate_map.argtypes = [vp, ip, vp, vp]
        for name in ("wcmg_apply_D", "wcmg_restrict", "wcmg_prolong"):
            getattr(l, name).argtypes = [vp, ip, vp, vp, ip, ip]
        l.wcmg_cycle.argtypes = [vp, vp, vp]
        l.wcmg_solve.argtypes = [vp, vp, vp, ip, C.POINTER(SolveInfo)]
        l.wcmg_solve_batched.argtypes = [vp, vp, vp, ip, ip, C.POINTER(SolveInfo)]
        l.wcmg_solve_ragged.argtypes = [C.POINTER(vp), ip, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int),
                                        C.POINTER(SolveInfo)]
        l.wcmg_tune_enable.argtypes = [vp, ip]
        l.wcmg_tune_table.argtypes = [vp, C.c_char_p, ip, C.POINTER(C.c_int)]
        l.wcmg_tune_load.argtypes = [vp, C.c_char_p]
        l.wcmg_timers.argtypes = [vp, C.POINTER(C.c_double), ip]
        l.wcmg_profile_enable.argtypes = [vp, C.c_char_p, ip]
        l.wcmg_profile_stats.argtypes = [vp, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        l.wcmg_coarse_create.argtypes = [C.POINTER(C.c_int32), ip, ip, vp, C.POINTER(vp)]
        l.wcmg_coarse_destroy.argtypes = [vp]
        l.wcmg_coarse_set.argtypes = [vp, vp, ip]
        l.wcmg_coarse_apply.argtypes = [vp, vp, vp, ip]
        l.wcmg_coarse_apply_noalloc.argtypes = [vp, vp, vp, ip]
        l.wcmg_coarse_set_kernel.argtypes = [vp, ip]
        l.wcmg_coarse_set_tile.argtypes = [vp, ip]
        l.wcmg_coarse_tune_table.argtypes = [vp, C.c_char_p, ip, C.POINTER(C.c_int)]
        l.wcmg_coarse_time.argtypes = [vp, vp, vp, ip, ip, C.POINTER(C.c_double)]
        l.wcmg_coarse_last_error.argtypes = [vp]
        l.wcmg_coarse_last_error.restype = C.c_char_p
        l.wcmg_coarse_apply_ragged.argtypes = [C.POINTER(vp), ip, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int)]
        l.wcmg_coarse_time_ragged.argtypes = [C.POINTER(vp), ip, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int), ip,
                                              C.POINTER(C.c_double)]
        l.wcmg_nn_create.argtypes = [ip, ip, ip, C.c_uint64, vp, C.POINTER(vp)]
        l.wcmg_nn_destroy.argtypes = [vp]
        l.wcmg_nn_last_error.argtypes = [vp]
        l.wcmg_nn_last_error.restype = C.c_char_p
        l.wcmg_nn_num_weights.argtypes = [vp, C.POINTER(C.c_int64)]
        l.wcmg_nn_get_weights.argtypes = [vp, vp, C.c_int64]
        l.wcmg_nn_set_weights.argtypes = [vp, vp, C.c_int64]
        l.wcmg_nn_forward.argtypes = [vp, vp, vp]
        l.wcmg_nn_loss_grad.argtypes = [vp, vp, C.POINTER(C.c_double), vp, C.c_int64]
        l.wcmg_nn_train_step.argtypes = [vp, vp, C.c_float, C.POINTER(C.c_double)]
        l.wcmg_setup_learned.argtypes = [vp, vp, C.c_double, ip, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        _lib = l
    return _lib


def default_params(**kw) -> Params:
    p = Params()
    lib().wcmg_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "dims":
            for m in range(4):
                p.dims[m] = int(v[m])
        elif k == "block":
            for l, b in enumerate(v):
                for m in range(4):
                    p.block[l][m] = int(b[m])
        elif k == "n_vec":
            for l, n in enumerate(v):
                p.n_vec[l] = int(n)
        elif k == "reserved":
            for i, n in enumerate(v):
                p.reserved[i] = int(n)
        else:
            setattr(p, k, v)
    return p


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("wcmg takes device tensors")
    if not t.is_contiguous():
        raise ValueError("wcmg takes contiguous tensors")
    return C.c_void_p(t.data_ptr())


def _cdtype(prec):
    return torch.complex128 if prec == F64 else torch.complex64


class Context:
    """Multigrid context for one fine lattice (wcmg_ctx)."""

    def __init__(self, params: Params | None = None, **kw):
        self.p = params if params is not None else default_params(**kw)
        h = C.c_void_p()
        st = lib().wcmg_create(C.byref(self.p), _stream(), C.byref(h))
        if st:
            raise WcmgError(st, lib().wcmg_last_error(None).decode())
        self.h = h
        self.dims = tuple(self.p.dims)
        self.V = int(self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3])
        self.nlev = self.p.n_levels
        self.level_dims = [self.dims]
        for l in range(self.nlev - 1):
            self.level_dims.append(tuple(self.level_dims[-1][m] // self.p.block[l][m] for m in range(4)))
        self.ns = [12] + [2 * self.p.n_vec[l] for l in range(self.nlev - 1)]
        _register(self)

    def close(self):
        """wcmg_destroy: synchronises the context's stream, frees its buffers."""
        if getattr(self, "h", None) and _lib is not None:
            _lib.wcmg_destroy(self.h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if not sys.is_finalizing():
            self.close()

    def _chk(self, st):
        if st:
            raise WcmgError(st, lib().wcmg_last_error(self.h).decode())

    def last_error(self) -> str:
        """wcmg_last_error: the message of the last failed or non-converged call."""
        return lib().wcmg_last_error(self.h).decode()

    def sites(self, level):
        d = self.level_dims[level]
        return int(d[0] * d[1] * d[2] * d[3])

    # ---- fields
    def set_gauge(self, U: torch.Tensor):
        assert U.dtype == torch.complex128 and U.numel() == self.V * 36
        self._chk(lib().wcmg_set_gauge(self.h, _ptr(U)))

    def set_clover(self, blocks: torch.Tensor | None):
        self._chk(lib().wcmg_set_clover(self.h, None if blocks is None else _ptr(blocks)))

    def get_clover(self) -> torch.Tensor:
        out = torch.empty((self.V, 2, 6, 6), dtype=torch.complex128, device="cuda")
        self._chk(lib().wcmg_get_clover(self.h, _ptr(out)))
        return out

    def set_null_vectors(self, level, v: torch.Tensor):
        nv = self.p.n_vec[level]
        assert v.dtype == torch.complex128 and v.numel() == nv * self.sites(level) * self.ns[level]
        self._chk(lib().wcmg_set_null_vectors(self.h, level, _ptr(v), nv))

    def _level_vectors(self, fn, level):
        out = torch.empty((self.p.n_vec[level], self.sites(level) * self.ns[level]), dtype=torch.complex128,
                          device="cuda")
        self._chk(fn(self.h, level, _ptr(out)))
        return out

    def null_vectors(self, level):
        return self._level_vectors(lib().wcmg_get_null_vectors, level)

    def prolongator(self, level):
        return self._level_vectors(lib().wcmg_get_prolongator, level)

    def rebuild_from_vectors(self, level, v: torch.Tensor):
        self._chk(lib().wcmg_rebuild_from_vectors(self.h, level, _ptr(v.contiguous())))

    def setup(self):
        self._chk(lib().wcmg_setup(self.h))

    def refine(self, iters):
        self._chk(lib().wcmg_refine(self.h, int(iters)))

    def export_setup(self):
        """The hierarchy as a setup checkpoint (a bytearray; wcmg_setup_export)."""
        n = C.c_size_t(0)
        self._chk(lib().wcmg_setup_export(self.h, None, 0, C.byref(n)))
        out = bytearray(n.value)
        cbuf = (C.c_char * n.value).from_buffer(out)
        self._chk(lib().wcmg_setup_export(self.h, cbuf, n.value, C.byref(n)))
        return out

    def import_setup(self, blob):
        """Load a setup checkpoint (bytes or bytearray; wcmg_setup_import)."""
        if isinstance(blob, bytearray):
            ptr = (C.c_char * len(blob)).from_buffer(blob)
        else:
            ptr = C.c_char_p(bytes(blob))
        self._chk(lib().wcmg_setup_import(self.h, ptr, len(blob)))

    def aggregate_map(self, level):
        import numpy as np
        n = self.sites(level)
        c = np.zeros(n, np.int32)
        o = np.zeros(n, np.int32)
        self._chk(lib().wcmg_get_aggregate_map(self.h, level, c.ctypes.data_as(C.c_void_p),
                                               o.ctypes.data_as(C.c_void_p)))
        return c, o

    def coarse_op(self, level, prec=F64) -> torch.Tensor:
        """wcmg_get_coarse_op: complex128 for F64, complex64 for F32 and BF16
        (the BF16-rounded values of the cycle's block storage)."""
        nb = self.ns[level]
        out = torch.empty((self.sites(level), 9, nb, nb), dtype=_cdtype(prec), device="cuda")
        self._chk(lib().wcmg_get_coarse_op(self.h, level, _ptr(out), int(prec)))
        return out

    def set_coarse_op(self, level, blocks: torch.Tensor):
        """wcmg_set_coarse_op from complex128 (F64) or complex64 (F32) blocks."""
        prec = F64 if blocks.dtype == torch.complex128 else F32
        assert blocks.dtype in (torch.complex128, torch.complex64)
        self._chk(lib().wcmg_set_coarse_op(self.h, level, _ptr(blocks.contiguous()), prec))

    # ---- operators
    def apply_D(self, level, x: torch.Tensor, prec=F64) -> torch.Tensor:
        nrhs = x.numel() // (self.sites(level) * self.ns[level])
        assert x.dtype == _cdtype(prec)
        out = torch.empty_like(x)
        self._chk(lib().wcmg_apply_D(self.h, level, _ptr(x), _ptr(out), nrhs, prec))
        return out

    def restrict(self, level, fine: torch.Tensor, prec=F64) -> torch.Tensor:
        nrhs = fine.numel() // (self.sites(level) * self.ns[level])
        out = torch.empty((nrhs, self.sites(level + 1), self.ns[level + 1]), dtype=fine.dtype, device="cuda")
        self._chk(lib().wcmg_restrict(self.h, level, _ptr(fine), _ptr(out), nrhs, prec))
        return out

    def prolong(self, level, coarse: torch.Tensor, prec=F64) -> torch.Tensor:
        nrhs = coarse.numel() // (self.sites(level + 1) * self.ns[level + 1])
        out = torch.empty((nrhs, self.sites(level), self.ns[level]), dtype=coarse.dtype, device="cuda")
        self._chk(lib().wcmg_prolong(self.h, level, _ptr(coarse), _ptr(out), nrhs, prec))
        return out

    def apply_schur(self, x: torch.Tensor) -> torch.Tensor:
        """wcmg_apply_schur: the even-odd Schur complement on the odd sites (FP64)."""
        nrhs = x.numel() // (self.V * 12)
        out = torch.empty_like(x)
        self._chk(lib().wcmg_apply_schur(self.h, _ptr(x), _ptr(out), nrhs))
        return out

    def sap(self, b: torch.Tensor, x: torch.Tensor, cycles: int, prec=None) -> torch.Tensor:
        """wcmg_sap: `cycles` SAP cycles on D x = b (x updated in place)."""
        nrhs = b.numel() // (self.V * 12)
        if prec is None:
            prec = F64 if b.dtype == torch.complex128 else F32
        self._chk(lib().wcmg_sap(self.h, _ptr(b), _ptr(x), nrhs, int(cycles), int(prec)))
        return x

    def cycle(self, r: torch.Tensor) -> torch.Tensor:
        out = torch.empty_like(r)
        self._chk(lib().wcmg_cycle(self.h, _ptr(r), _ptr(out)))
        return out

    def solve(self, b: torch.Tensor, x: torch.Tensor | None = None, check=True):
        nrhs = b.numel() // (self.V * 12)
        if x is None:
            x = torch.zeros_like(b)
        info = (SolveInfo * nrhs)()
        st = lib().wcmg_solve(self.h, _ptr(b), _ptr(x), nrhs, info)
        if check and st not in (0,):
            self._chk(st)
        infos = [dict(outer_iters=i.outer_iters, converged=bool(i.converged), true_rel_res=i.true_rel_res,
                      t_solve_s=i.t_solve_s, coarse_iters=i.coarse_iters, cycles=i.cycles) for i in info]
        return x, infos, st

    def solve_batched(self, b: torch.Tensor, x: torch.Tensor | None = None, graph=False, kernel="auto",
                      dslash_per_rhs=False, check=True):
        """wcmg_solve_batched: groups of up to 16 right-hand sides solved together."""
        nrhs = b.numel() // (self.V * 12)
        if x is None:
            x = torch.zeros_like(b)
        flags = (BATCH_GRAPH if graph else 0) | {"auto": 0, "vector": BATCH_VECTOR, "mfma": BATCH_MFMA}[kernel]
        if dslash_per_rhs:
            flags |= BATCH_DSLASH_PER_RHS
        info = (SolveInfo * nrhs)()
        st = lib().wcmg_solve_batched(self.h, _ptr(b), _ptr(x), nrhs, flags, info)
        if check and st not in (0,):
            self._chk(st)
        infos = [dict(outer_iters=i.outer_iters, converged=bool(i.converged), true_rel_res=i.true_rel_res,
                      t_solve_s=i.t_solve_s, coarse_iters=i.coarse_iters, cycles=i.cycles) for i in info]
        return x, infos, st

    def setup_learned(self, net: "Network", threshold=float("inf"), relax_sweeps=0):
        """wcmg_setup_learned: returns (fell_back, quality)."""
        fb = C.c_int(0)
        q = C.c_double(0.0)
        self._chk(lib().wcmg_setup_learned(self.h, net.h, float(threshold), int(relax_sweeps), C.byref(fb),
                                           C.byref(q)))
        return bool(fb.value), q.value

    def tune_enable(self, enable=True):
        self._chk(lib().wcmg_tune_enable(self.h, int(enable)))

    def tune_table(self) -> dict:
        """The autotuner's decisions so far: {configuration: {"choice": v, "ms": [...]}}."""
        need = C.c_int(0)
        lib().wcmg_tune_table(self.h, None, 0, C.byref(need))
        buf = C.create_string_buffer(max(need.value, 1))
        self._chk(lib().wcmg_tune_table(self.h, buf, len(buf), C.byref(need)))
        return json.loads(buf.value.decode())

    def tune_load(self, table: dict):
        self._chk(lib().wcmg_tune_load(self.h, json.dumps(table).encode()))

    def timers(self):
        out = (C.c_double * 8)()
        self._chk(lib().wcmg_timers(self.h, out, 8))
        d = dict(zip(["setup", "relax", "gram_schmidt", "coarsen", "refine", "solve"], list(out)[:6]))
        d["coarse_solve_fallbacks"] = int(out[6])
        d["dslash_link_rows"] = int(out[7])
        return d

    def profile(self, family, enable=True):
        self._chk(lib().wcmg_profile_enable(self.h, family.encode(), int(enable)))

    def profile_stats(self, family):
        n = C.c_int64(0)
        ms = C.c_double(0.0)
        self._chk(lib().wcmg_profile_stats(self.h, family.encode(), C.byref(n), C.byref(ms)))
        return n.value, ms.value


class Network:
    """Learned near-null proposal (wcmg_nn): three parallel-transport
    convolution layers n_vec -> channels -> channels -> n_vec."""

    def __init__(self, n_vec, channels=32, act_prec=BF16, seed=0):
        h = C.c_void_p()
        st = lib().wcmg_nn_create(int(n_vec), int(channels), int(act_prec), int(seed), _stream(), C.byref(h))
        if st:
            raise WcmgError(st, lib().wcmg_nn_last_error(None).decode())
        self.h = h
        self.n_vec, self.channels = n_vec, channels
        n = C.c_int64(0)
        lib().wcmg_nn_num_weights(self.h, C.byref(n))
        self.n_floats = n.value
        _register(self)

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.wcmg_nn_destroy(self.h)
        self.h = None

    def __del__(self):
        if not sys.is_finalizing():
            self.close()

    def _chk(self, st):
        if st:
            raise WcmgError(st, lib().wcmg_nn_last_error(self.h).decode())

    def weights(self) -> np.ndarray:
        w = np.zeros(self.n_floats, np.float32)
        self._chk(lib().wcmg_nn_get_weights(self.h, w.ctypes.data, self.n_floats))
        return w

    def set_weights(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == self.n_floats
        self._chk(lib().wcmg_nn_set_weights(self.h, w.ctypes.data, self.n_floats))

    def forward(self, ctx) -> torch.Tensor:
        out = torch.empty((self.n_vec, ctx.V, 4, 3), dtype=torch.complex128, device="cuda")
        self._chk(lib().wcmg_nn_forward(self.h, ctx.h, _ptr(out)))
        return out

    def loss_grad(self, ctx, grad=True):
        loss = C.c_double(0.0)
        g = np.zeros(self.n_floats, np.float32) if grad else None
        self._chk(lib().wcmg_nn_loss_grad(self.h, ctx.h, C.byref(loss), g.ctypes.data if grad else None,
                                          self.n_floats))
        return loss.value, g

    def train_step(self, ctx, lr=1e-2) -> float:
        loss = C.c_double(0.0)
        self._chk(lib().wcmg_nn_train_step(self.h, ctx.h, float(lr), C.byref(loss)))
        return loss.value


class CoarseOperator:
    """Standalone coarse operator (wcmg_coarse): nine Nb x Nb blocks per site."""

    def __init__(self, dims, nb, store_prec=F32):
        d = (C.c_int32 * 4)(*[int(x) for x in dims])
        h = C.c_void_p()
        st = lib().wcmg_coarse_create(d, int(nb), int(store_prec), _stream(), C.byref(h))
        if st:
            raise WcmgError(st, "wcmg_coarse_create failed")
        self.h = h
        self.dims = tuple(dims)
        self.nb = nb
        self.store = store_prec
        self.Vc = int(dims[0] * dims[1] * dims[2] * dims[3])
        _register(self)

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.wcmg_coarse_destroy(self.h)
        self.h = None

    def __del__(self):
        if not sys.is_finalizing():
            self.close()

    def _chk(self, st):
        if st:
            raise WcmgError(st, lib().wcmg_coarse_last_error(self.h).decode())

    def set(self, blocks: torch.Tensor):
        prec = F64 if blocks.dtype == torch.complex128 else F32
        self._chk(lib().wcmg_coarse_set(self.h, _ptr(blocks), prec))

    def set_kernel(self, kernel: int):
        """0 automatic, 1 per-row vector kernel, 2 matrix cores, 3 per-row
        kernel on five-point storage (set before `set`; the blocks must be
        sigma3-hermitian, as every Galerkin coarse operator is)."""
        self._chk(lib().wcmg_coarse_set_kernel(self.h, int(kernel)))

    def set_tile(self, tile: int):
        """Matrix-core tile: -1 tuned (default), 0 one wave per site, 4/8/16
        sites of one x-row per workgroup with LDS-staged neighbour vectors and
        outputs, 5/9 the 4- and 8-site tiles with per-wave output stores."""
        self._chk(lib().wcmg_coarse_set_tile(self.h, int(tile)))

    def tune_table(self) -> dict:
        """This operator's tile choices: {configuration: {"choice": v, "ms": [...]}},
        v indexing the tiles (0, 4, 8, 16, 5, 9)."""
        need = C.c_int(0)
        lib().wcmg_coarse_tune_table(self.h, None, 0, C.byref(need))
        buf = C.create_string_buffer(max(need.value, 1))
        self._chk(lib().wcmg_coarse_tune_table(self.h, buf, len(buf), C.byref(need)))
        return json.loads(buf.value.decode())

    def apply(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        nrhs = x.numel() // (self.Vc * self.nb)
        out = torch.empty_like(x) if out is None else out
        self._chk(lib().wcmg_coarse_apply(self.h, _ptr(x), _ptr(out), nrhs))
        return out

    def apply_noalloc(self, x: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """wcmg_coarse_apply_noalloc: out = D_c x with no device allocation
        (out is the caller's)."""
        nrhs = x.numel() // (self.Vc * self.nb)
        self._chk(lib().wcmg_coarse_apply_noalloc(self.h, _ptr(x), _ptr(out), nrhs))
        return out

    def time(self, x: torch.Tensor, out: torch.Tensor, reps=20) -> float:
        nrhs = x.numel() // (self.Vc * self.nb)
        ms = C.c_double(0.0)
        self._chk(lib().wcmg_coarse_time(self.h, _ptr(x), _ptr(out), nrhs, int(reps), C.byref(ms)))
        return ms.value


def solve_ragged(ctxs, bs, xs=None, check=True):
    """wcmg_solve_ragged: problem k solves bs[k] ([nrhs_k][V_k][4][3]
    complex128) on context ctxs[k]; all problems together, their coarse
    solves sharing one coarse-operator launch per Arnoldi step.  Returns
    (xs, infos per problem, status, shared coarse launches)."""
    n = len(ctxs)
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    nr = [b.numel() // (c.V * 12) for c, b in zip(ctxs, bs)]
    total = sum(nr)
    info = (SolveInfo * total)()
    h = (C.c_void_p * n)(*[c.h for c in ctxs])
    pb = (C.c_void_p * n)(*[_ptr(b).value for b in bs])
    px = (C.c_void_p * n)(*[_ptr(x).value for x in xs])
    pn = (C.c_int * n)(*nr)
    st = lib().wcmg_solve_ragged(h, n, pb, px, pn, info)
    if check and st != 0:
        ctxs[0]._chk(st)
    infos, k = [], 0
    for q in range(n):
        infos.append([dict(outer_iters=i.outer_iters, converged=bool(i.converged), true_rel_res=i.true_rel_res,
                           t_solve_s=i.t_solve_s, coarse_iters=i.coarse_iters) for i in info[k:k + nr[q]]])
        k += nr[q]
    return xs, infos, st, (info[0].cycles if total else 0)


def _ragged_args(ops, ins):
    n = len(ops)
    outs = [torch.empty_like(x) for x in ins]
    h = (C.c_void_p * n)(*[o.h for o in ops])
    pi = (C.c_void_p * n)(*[x.data_ptr() for x in ins])
    po = (C.c_void_p * n)(*[y.data_ptr() for y in outs])
    nr = (C.c_int * n)(*[x.numel() // (o.Vc * o.nb) for o, x in zip(ops, ins)])
    return n, outs, h, pi, po, nr


def coarse_apply_ragged(ops, ins):
    """wcmg_coarse_apply_ragged: operator p applied to ins[p] ([nrhs][Vc_p][Nb]
    complex64), all operators in one launch.  Returns the outputs."""
    n, outs, h, pi, po, nr = _ragged_args(ops, ins)
    st = lib().wcmg_coarse_apply_ragged(h, n, pi, po, nr)
    if st:
        raise WcmgError(st, lib().wcmg_coarse_last_error(ops[0].h).decode())
    return outs


def coarse_time_ragged(ops, ins, reps=20):
    n, outs, h, pi, po, nr = _ragged_args(ops, ins)
    ms = C.c_double(0.0)
    st = lib().wcmg_coarse_time_ragged(h, n, pi, po, nr, int(reps), C.byref(ms))
    if st:
        raise WcmgError(st, lib().wcmg_coarse_last_error(ops[0].h).decode())
    return ms.value
