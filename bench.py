#!/usr/bin/env python3
"""Benchmark of the Wilson-clover multigrid hot path on one MI355X.

Workload (two-level MG on a 16^3 x 32 lattice): SU(3) links U = exp(i 0.25 H)
with H Gaussian traceless Hermitian (seeded), c_sw = 1, m0 = -0.08,
antiperiodic t, 4^4 aggregates (coarse lattice 4^3 x 8), 12 near-null vectors
split by chirality to Nb = 24, 20 MR relaxation sweeps plus one iteration of the
iterative setup, MR(4) post-smoothing, coarse GMRES(20) to 0.05, outer FP64
FGMRES(20) to a true relative residual of 1e-10, Gaussian right-hand side.

One step = the whole path on that input: setup (relaxation, chirality-split
Gram-Schmidt, Galerkin coarsening, refinement) and the mixed-precision solve
(FP32 smoother, restriction, prolongation and coarse arithmetic with FP32
coarse blocks; FP64 outer solver; each coarsest GMRES solve is one
persistent launch).  `value` is the solve time of the mixed solve (seconds to
1e-10); the plain FP64 solve, the same solve with reference forms of the
coarsest GMRES (four kernels per step) and of the outer Arnoldi step (CGS2),
the coarse-apply bandwidth on a large synthetic coarse lattice (Nb 16, 24,
32), the roofline of the dominant solve kernel, the latency line of the
coarsest GMRES (time per Arnoldi step), the batched and ragged solves of point
sources (24^3 x 48; 8^4 + 16^4 + 24^3 x 48), the three-level workload
(32^3 x 64), the learned setup and the CPU oracle (the whole workload,
unsampled, on the host cores) are reported beside it.  The warmup step times
every kernel family (the kernel table); the timed steps record HIP events only
around the dominant kernel.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MG solve s to 1e-10 rel. residual (mixed/batched vs FP64); coarse-apply GB/s"
HBM_PEAK_GBS = 8000.0

WORKLOAD = dict(
    name="two-level MG, 16^3x32, Nb=24 (4^4 aggregates, 12 vectors), 1 refinement iteration, FGMRES(20) to 1e-10",
    L=(16, 16, 16, 32), eps=0.25, m0=-0.08, csw=1.0, block=(4, 4, 4, 4), nv=12, relax=20, refine=1, seed=102,
)


WORKLOAD_BATCH = dict(
    name="two-level MG, 24^3x48, Nb=24 (4^4 aggregates, 12 vectors), 1 refinement iteration, 12 point sources "
         "(one per spin-colour) solved together, FGMRES(20) to 1e-10",
    L=(24, 24, 24, 48), eps=0.25, m0=-0.08, csw=1.0, block=(4, 4, 4, 4), nv=12, relax=20, refine=1, seed=104,
)


WORKLOAD_THREE = dict(
    name="three-level MG, 32^3x64, Nb=24 then 32 (4^4 then 2^4 aggregates), 3 refinement iterations, BF16 coarse "
         "blocks with FP32 accumulation, K-cycle, FGMRES(20) to 1e-10",
    L=(32, 32, 32, 64), eps=0.25, m0=-0.09, csw=1.0, blocks=((4, 4, 4, 4), (2, 2, 2, 2)), nv=(12, 16), relax=20,
    refine=3, seed=103,
)


def three_level(w, torch, wl=WORKLOAD_THREE, fp64=True):
    """Config 3: three-level hierarchy with BF16-stored coarse blocks and a
    K-cycle on the intermediate level, against the same hierarchy run in FP64."""
    import numpy as np
    import synthetic as syn
    L = wl["L"]
    V = int(np.prod(L))
    s = syn.config_seeds(wl["seed"])
    Ud = torch.from_numpy(syn.gauge_field(L, wl["eps"], s["gauge"])).cuda()
    starts = [torch.from_numpy(syn.start_vectors(wl["nv"][0], V, 12, s["start"])).cuda()]
    V1 = V // int(np.prod(wl["blocks"][0]))
    starts.append(torch.from_numpy(syn.start_vectors(wl["nv"][1], V1, 2 * wl["nv"][0], s["start"] + 500)).cuda())
    b = torch.from_numpy(syn.complex_gaussian((V, 4, 3), s["rhs"])).cuda()
    out = {"workload": wl["name"]}
    for label, mixed in (("mixed_bf16_kcycle", True), ("fp64_kcycle", False)):
        if label.startswith("fp64") and not fp64:
            continue
        kw = dict(dims=L, m0=wl["m0"], c_sw=wl["csw"], n_levels=3, block=wl["blocks"], n_vec=wl["nv"],
                  relax_sweeps=wl["relax"], refine_iters=wl["refine"], outer_restart=20, outer_maxit=2000, kcycle=1)
        if mixed:
            kw.update(cycle_prec=w.F32, coarse_store_prec=w.BF16, setup_prec=w.F32)
        ctx = w.Context(**kw)
        ctx.set_gauge(Ud)
        ctx.set_null_vectors(0, starts[0])
        ctx.set_null_vectors(1, starts[1])
        ctx.setup()
        setup_s = ctx.timers()["setup"]
        ctx.solve(b)
        x, info, st = ctx.solve(b)
        out[label] = {"setup_s": setup_s, "solve_s": info[0]["t_solve_s"], "outer_iters": info[0]["outer_iters"],
                      "coarse_iters": info[0]["coarse_iters"], "true_rel_res": info[0]["true_rel_res"],
                      "converged": bool(info[0]["converged"]) and st == 0}
        print("[bench] three-level %s: setup %.3f s, solve %.3f s, %d outer iterations, res %.2e" % (
            label, setup_s, out[label]["solve_s"], out[label]["outer_iters"], out[label]["true_rel_res"]),
            file=sys.stderr, flush=True)
        del ctx, x
        torch.cuda.empty_cache()
    if fp64:
        out["speedup_mixed_vs_fp64"] = out["fp64_kcycle"]["solve_s"] / out["mixed_bf16_kcycle"]["solve_s"]
    return out


def algorithmic_bytes(family: str, V: int, Vc: int, nb: int, nv: int, nrhs: int = 1, link_rows: int = 3) -> float:
    """Bytes a launch must move at minimum (each operand read once, output written
    once); with nrhs fields per launch the gauge data and P are read once.
    link_rows: rows of each link the Dslash reads (2 when it rebuilds the third)."""
    if family == "dslash_f64":
        # links 4 x 3 rows x 48 B (two rows: 384), clover 576, in 192 + out 192 per field (FP64)
        return (192.0 * link_rows + 576.0 + 384.0 * nrhs) * V
    if family == "dslash_f32":
        # links 4 x 3 rows x 24 B (two rows: 192), clover 288, in 96 + out 96 per field (FP32)
        return (96.0 * link_rows + 288.0 + 192.0 * nrhs) * V
    if family.startswith("coarse_apply"):
        sb = {"coarse_apply_f64": 16, "coarse_apply_f32": 8, "coarse_apply_bf16": 4}[family]
        sv = 16 if family.endswith("f64") else 8
        return (9.0 * nb * nb * sb + 2.0 * nb * sv) * Vc
    if family in ("restrict_f32", "prolong_f32"):
        return (nv * 12 * 8.0 + 12 * 8.0 * nrhs) * V
    if family in ("restrict_f64", "prolong_f64"):
        return (nv * 12 * 16.0 + 12 * 16.0 * nrhs) * V
    return float("nan")


TRAFFIC_SOURCES = {
    "dslash_f32": ("paper_1904_08678_amd/csrc/wilson.hip", "paper_1904_08678_amd/csrc/wilson_ops.h"),
    "coarse_apply_f32_large": ("paper_1904_08678_amd/csrc/coarse.hip", "paper_1904_08678_amd/csrc/coarse_common.h"),
    "coarse_mfma_f32_12rhs": ("paper_1904_08678_amd/csrc/coarse_mfma.hip",),
    "coarse_mfma_bf16_12rhs": ("paper_1904_08678_amd/csrc/coarse_mfma.hip",),
    "dslash_f32_mrhs_12rhs": ("paper_1904_08678_amd/csrc/wilson.hip", "paper_1904_08678_amd/csrc/wilson_ops.h"),
}


def counter_traffic(key: str):
    """Calibrated HBM traffic per launch from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_counters.md")
    try:
        text = open(path).read()
        data = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        rec = data[key]
    except (OSError, IndexError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[key]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest()[:16] != rec["source_sha"]:
        return None
    return rec["traffic_bytes"]


def make_inputs(wl):
    import numpy as np
    import synthetic as syn
    L = wl["L"]
    V = int(np.prod(L))
    s = syn.config_seeds(wl["seed"])
    U = syn.gauge_field(L, wl["eps"], s["gauge"])
    start = syn.start_vectors(wl["nv"], V, 12, s["start"])
    b = syn.complex_gaussian((V, 4, 3), s["rhs"])
    return U, start, b


COARSE_POINTS = 9  # blocks stored per coarse site (set by --coarse-points)


def make_context(w, wl, mixed: bool, reserved: int = 0, **extra):
    kw = dict(dims=wl["L"], m0=wl["m0"], c_sw=wl["csw"], n_levels=2, block=(wl["block"],), n_vec=(wl["nv"],),
              relax_sweeps=wl["relax"], refine_iters=wl["refine"], outer_restart=20, outer_maxit=2000,
              coarse_points=COARSE_POINTS, reserved=(reserved,))
    if mixed:
        kw.update(cycle_prec=w.F32, coarse_store_prec=w.F32, setup_prec=w.F32)
    kw.update(extra)
    return w.Context(**kw)


def coarse_apply_mk(w, torch, nb=24, dims=(16, 16, 16, 32), stores=None, reps=20, nrhs_batch=12):
    """Coarse apply on a coarse lattice far larger than the 256 MB last-level cache."""
    out = {}
    Vc = dims[0] * dims[1] * dims[2] * dims[3]
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    blocks = torch.randn((Vc, 9, nb, nb), dtype=torch.complex64, device="cuda", generator=g)
    for store in stores or (w.F32, w.BF16, w.F64):
        name = {w.F64: "f64", w.F32: "f32", w.BF16: "bf16"}[store]
        op = w.CoarseOperator(dims, nb, store)
        op.set(blocks)
        vdt = torch.complex128 if store == w.F64 else torch.complex64
        x = torch.randn((Vc, nb), dtype=vdt, device="cuda", generator=g)
        y = torch.empty_like(x)
        op.time(x, y, reps=3)
        ms = op.time(x, y, reps=reps)
        sb = {"f64": 16, "f32": 8, "bf16": 4}[name]
        sv = 16 if name == "f64" else 8
        byts = (9.0 * nb * nb * sb + 2.0 * nb * sv) * Vc
        out[name] = {"ms": ms, "GB_s": byts / ms / 1e6, "frac": byts / ms / 1e6 / HBM_PEAK_GBS,
                     "bytes_per_launch": byts}
        del op
        # five-point storage: Mdiag and the forward blocks (the timing does not
        # depend on the values; the backward blocks of `blocks` are ignored)
        op5 = w.CoarseOperator(dims, nb, store)
        op5.set_kernel(3)
        op5.set(blocks)
        op5.time(x, y, reps=3)
        ms5 = op5.time(x, y, reps=reps)
        b5 = (5.0 * nb * nb * sb + 2.0 * nb * sv) * Vc
        out[name]["five_point"] = {"ms": ms5, "GB_s": b5 / ms5 / 1e6, "frac": b5 / ms5 / 1e6 / HBM_PEAK_GBS,
                                   "bytes_per_launch": b5, "speedup_vs_nine": ms / ms5}
        del op5, x, y
        torch.cuda.synchronize()
    # twelve right-hand sides in one launch: matrix-core kernel against the per-row kernel
    batched = {}
    if nrhs_batch:
        for store in (w.F32, w.BF16):
            name = {w.F32: "f32", w.BF16: "bf16"}[store]
            op = w.CoarseOperator(dims, nb, store)
            op.set(blocks)
            x = torch.randn((nrhs_batch, Vc, nb), dtype=torch.complex64, device="cuda", generator=g)
            y = torch.empty_like(x)
            sb = {"f32": 8, "bf16": 4}[name]
            byts = (9.0 * nb * nb * sb + 2.0 * nb * nrhs_batch * 8) * Vc
            flops = 8.0 * 9 * nb * nb * nrhs_batch * Vc
            rec = {}
            # every matrix-core tile forced, then the tuned choice (the default)
            op.set_kernel(2)
            tiles = {}
            for tile in (0, 4, 8, 16, 5, 9):
                if tile and dims[0] % (tile & ~1):
                    continue
                op.set_tile(tile)
                op.time(x, y, reps=2)
                tms = op.time(x, y, reps=max(3, reps // 2))
                tiles[str(tile)] = {"ms": tms, "frac_hbm": byts / tms / 1e6 / HBM_PEAK_GBS}
            op.set_tile(-1)
            for kern, kname in ((2, "matrix_cores"), (1, "vector")):
                op.set_kernel(kern)
                op.time(x, y, reps=2)
                ms = op.time(x, y, reps=max(3, reps // 2))
                rec[kname] = {"ms": ms, "GB_s": byts / ms / 1e6, "frac_hbm": byts / ms / 1e6 / HBM_PEAK_GBS,
                              "TFLOP_s": flops / ms / 1e9}
            tab = op.tune_table()
            ent = [v for k, v in tab.items() if "coarse_mfma_tile" in k]
            rec["matrix_cores"]["tile"] = (0, 4, 8, 16, 5, 9)[ent[0]["choice"]] if ent else None
            rec["matrix_cores"]["tiles"] = tiles
            rec["matrix_cores"]["tuning_table"] = tab
            rec["bytes_per_launch"] = byts
            rec["flops_per_launch"] = flops
            batched[name] = rec
            del op, x, y
            torch.cuda.synchronize()
    del blocks
    torch.cuda.empty_cache()
    return {"coarse_dims": list(dims), "Vc": Vc, "nb": nb, "per_store": out, "nrhs": nrhs_batch,
            "batched": batched}


def coarse_gmres_latency(w, torch, wl, Ud, startd, reps=20, iters=(4, 16)):
    """The coarsest GMRES as one persistent launch is bound by the latency of
    its grid barriers, not by a byte stream: its time per Arnoldi step is the
    slope of the launch time over the number of steps (fixed iteration
    counts, one restart cycle), the intercept the per-launch cost (blocks into
    LDS, residual, final update)."""
    import numpy as np
    out = {}
    r = torch.randn((int(np.prod(wl["L"])), 4, 3), dtype=torch.complex128, device="cuda")
    for k in iters:
        ctx2 = make_context(w, wl, mixed=True, coarse_fixed_iters=k)
        ctx2.set_gauge(Ud)
        ctx2.set_null_vectors(0, startd)
        ctx2.setup()
        ctx2.cycle(r)
        ctx2.profile("coarse_gmres_persistent", True)
        for _ in range(reps):
            ctx2.cycle(r)
        n, ms = ctx2.profile_stats("coarse_gmres_persistent")
        out[k] = ms * 1e3 / max(n, 1)
        ctx2.close()
    k0, k1 = iters
    slope = (out[k1] - out[k0]) / (k1 - k0)
    return {"bound": "latency", "kernel": "coarse_gmres_persistent", "unit": "us",
            "us_per_launch": {str(k): out[k] for k in iters}, "us_per_arnoldi_step": slope,
            "us_per_launch_fixed": out[k0] - slope * k0,
            "grid_barriers_per_step": "1, plus 1 when the step re-orthogonalises",
            "coarse_sites": int(np.prod(wl["L"])) // int(np.prod(wl["block"])), "nb": 2 * wl["nv"]}


def reference_forms(w, torch, wl, Ud, startd, bd):
    """The same mixed solve with reference forms of solver steps: the
    coarsest GMRES as four kernels per Arnoldi step instead of one
    persistent launch (flag 4), the outer Arnoldi step as classical
    Gram-Schmidt applied twice instead of one reduction per step (flag 8),
    both, and the persistent launch through the cooperative-launch API
    (flag 256)."""
    out = {}
    for name, flags in (("coarse_gmres_four_kernels", 4), ("outer_cgs2", 8), ("both", 12),
                        ("coarse_gmres_cooperative_api", 256)):
        ctx = make_context(w, wl, mixed=True, reserved=flags)
        ctx.set_gauge(Ud)
        ctx.set_null_vectors(0, startd)
        ctx.setup()
        best = None
        for _ in range(3):
            x, info, st = ctx.solve(bd)
            if best is None or info[0]["t_solve_s"] < best["solve_s"]:
                best = {"solve_s": info[0]["t_solve_s"], "outer_iters": info[0]["outer_iters"],
                        "coarse_iters": info[0]["coarse_iters"], "true_rel_res": info[0]["true_rel_res"]}
        out[name] = best
        del ctx
    return out


def sap_smoother(w, torch, wl, Ud, startd, bd, iters=4):
    """The benchmark solve with SAP (1 and 2 cycles, `iters` MR steps per
    domain) as the level-0 post-smoother instead of MR(4), and the SAP
    launches' duration.  Algorithmic bytes of one colour's launch: on its half
    of the sites, links, clover, b and x read and x written once, plus x of the
    other half read once (960 B per active site in FP32); flops: the residual
    (1872 per site) and, per MR step, the domain operator (1872) and the
    updates (96)."""
    import numpy as np
    V = int(np.prod(wl["L"]))
    out = {"domains": "level-0 aggregates %s, red-black" % "x".join(map(str, wl["block"])), "block_iters": iters}
    for cycles in (1, 2):
        kw = dict(dims=wl["L"], m0=wl["m0"], c_sw=wl["csw"], n_levels=2, block=(wl["block"],), n_vec=(wl["nv"],),
                  relax_sweeps=wl["relax"], refine_iters=wl["refine"], outer_restart=20, outer_maxit=2000,
                  cycle_prec=w.F32, coarse_store_prec=w.F32, setup_prec=w.F32, smoother=1, sap_block_iters=iters,
                  post_smooth=cycles)
        ctx = w.Context(**kw)
        ctx.set_gauge(Ud)
        ctx.set_null_vectors(0, startd)
        ctx.setup()
        ctx.solve(bd)
        ctx.profile("sap_f32", True)
        x, info, st = ctx.solve(bd)
        n, ms = ctx.profile_stats("sap_f32")
        ctx.profile("sap_f32", False)
        x, info2, st2 = ctx.solve(bd)
        avg = ms / max(n, 1)
        byts = V / 2 * 960.0
        flops = V / 2 * (1872.0 + iters * (1872.0 + 96.0))
        out["cycles_%d" % cycles] = {
            "solve_s": min(info[0]["t_solve_s"], info2[0]["t_solve_s"]), "outer_iters": info[0]["outer_iters"],
            "true_rel_res": info[0]["true_rel_res"], "converged": st == 0,
            "sap_launch_ms": avg, "sap_launches": n, "sap_GB_s": byts / avg / 1e6, "sap_TFLOP_s": flops / avg / 1e9}
        del ctx
    return out


def even_odd(w, torch, wl, Ud, startd, bd):
    """The benchmark solve with the outer FGMRES on the even-odd Schur
    complement (MR(4) and SAP(2 cycles) post-smoothing), FP64 outer and FP32
    cycle as in the main line."""
    out = {}
    for name, extra in (("mr4", {}), ("sap2", dict(smoother=1, sap_block_iters=4, post_smooth=2))):
        kw = dict(dims=wl["L"], m0=wl["m0"], c_sw=wl["csw"], n_levels=2, block=(wl["block"],), n_vec=(wl["nv"],),
                  relax_sweeps=wl["relax"], refine_iters=wl["refine"], outer_restart=20, outer_maxit=2000,
                  cycle_prec=w.F32, coarse_store_prec=w.F32, setup_prec=w.F32, even_odd=1, **extra)
        ctx = w.Context(**kw)
        ctx.set_gauge(Ud)
        ctx.set_null_vectors(0, startd)
        ctx.setup()
        x, i1, st = ctx.solve(bd)
        x, i2, st2 = ctx.solve(bd)
        out[name] = {"solve_s": min(i1[0]["t_solve_s"], i2[0]["t_solve_s"]), "outer_iters": i1[0]["outer_iters"],
                     "true_rel_res": i1[0]["true_rel_res"], "converged": st == 0 and st2 == 0}
        del ctx
    return out


def batched_point_sources(w, torch, wl, fp64=True):
    """Twelve point sources on the 24^3 x 48 lattice: one batched solve (matrix-core
    coarse apply; with and without the HIP-graph cycle; per-row coarse kernel for
    comparison) against the same twelve solves one after another, mixed and FP64."""
    import numpy as np
    import synthetic as syn
    L = wl["L"]
    V = int(np.prod(L))
    s = syn.config_seeds(wl["seed"])
    Ud = torch.from_numpy(syn.gauge_field(L, wl["eps"], s["gauge"])).cuda()
    startd = torch.from_numpy(syn.start_vectors(wl["nv"], V, 12, s["start"])).cuda()
    bd = torch.from_numpy(syn.point_sources(V, site=0)).cuda()
    out = {"workload": wl["name"], "nrhs": 12}
    ctx = make_context(w, wl, mixed=True)
    ctx.set_gauge(Ud)
    ctx.set_null_vectors(0, startd)
    ctx.setup()
    out["setup_s"] = ctx.timers()["setup"]
    fams = ["dslash_f32", "coarse_mfma_f32", "restrict_f32", "prolong_f32"]

    def run(label, profile=False, **kw):
        ctx.solve_batched(bd, **kw)  # first call allocates the batch's Krylov space
        for f in fams:
            ctx.profile(f, profile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info, st = ctx.solve_batched(bd, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = {"solve_s": dt, "outer_iters": [i["outer_iters"] for i in info],
               "max_true_rel_res": max(i["true_rel_res"] for i in info),
               "converged": all(i["converged"] for i in info) and st == 0,
               "coarse_iters": info[0]["coarse_iters"]}
        if profile:
            rec["kernels"] = {}
            for f in fams:
                n, ms = ctx.profile_stats(f)
                ctx.profile(f, False)
                rec["kernels"][f] = {"launches": n, "total_ms": ms, "avg_ms": ms / max(n, 1)}
        print("[bench] %s: %.3f s, iters %s, max res %.2e" % (label, dt, rec["outer_iters"],
                                                              rec["max_true_rel_res"]), file=sys.stderr, flush=True)
        del x
        return rec

    out["batched_mfma"] = run("batched (autotuned kernels)", profile=True)
    out["tuner"] = ctx.tune_table()
    out["batched_mfma_graph"] = run("batched + HIP graph", graph=True)
    out["batched_vector"] = run("batched (per-row coarse kernel)", kernel="vector")
    ctx.solve(bd[:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info, st = ctx.solve(bd)
    torch.cuda.synchronize()
    out["sequential_mixed"] = {"solve_s": time.perf_counter() - t0, "outer_iters": [i["outer_iters"] for i in info],
                               "max_true_rel_res": max(i["true_rel_res"] for i in info)}
    print("[bench] 12 sequential mixed solves: %.3f s" % out["sequential_mixed"]["solve_s"], file=sys.stderr,
          flush=True)
    del ctx
    torch.cuda.empty_cache()
    if fp64:
        c64 = make_context(w, wl, mixed=False)
        c64.set_gauge(Ud)
        c64.set_null_vectors(0, startd)
        c64.setup()
        c64.solve(bd[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, st = c64.solve(bd)
        torch.cuda.synchronize()
        out["sequential_fp64"] = {"solve_s": time.perf_counter() - t0,
                                  "outer_iters": [i["outer_iters"] for i in info],
                                  "max_true_rel_res": max(i["true_rel_res"] for i in info),
                                  "setup_s": c64.timers()["setup"]}
        print("[bench] 12 sequential FP64 solves: %.3f s" % out["sequential_fp64"]["solve_s"], file=sys.stderr,
              flush=True)
        best = min(out["batched_mfma"]["solve_s"], out["batched_mfma_graph"]["solve_s"])
        out["speedup_batched_vs_fp64"] = out["sequential_fp64"]["solve_s"] / best
        out["speedup_batched_vs_sequential_mixed"] = out["sequential_mixed"]["solve_s"] / best
        del c64
    torch.cuda.empty_cache()
    return out


def ragged_solve(w, torch, wl=WORKLOAD_BATCH):
    """The ragged batch as a whole solve: 8^4, 16^4 and 24^3 x 48 (own gauge
    fields and start vectors, the batched workload's parameters), 12 point
    sources each, solved by one wcmg_solve_ragged call (the coarse solves of
    all three share one matrix-core launch per Arnoldi step) against the three
    problems' own batched solves one after another."""
    import numpy as np
    import synthetic as syn
    lats = [(8, 8, 8, 8), (16, 16, 16, 16), tuple(wl["L"])]
    ctxs, bs = [], []
    base = syn.config_seeds(wl["seed"])
    for k, L in enumerate(lats):
        V = int(np.prod(L))
        wk = dict(wl, L=L)
        c = make_context(w, wk, mixed=True)
        c.set_gauge(torch.from_numpy(syn.gauge_field(L, wl["eps"], base["gauge"] + 10 * k)).cuda())
        c.set_null_vectors(0, torch.from_numpy(syn.start_vectors(wl["nv"], V, 12, base["start"] + 10 * k)).cuda())
        c.setup()
        ctxs.append(c)
        bs.append(torch.from_numpy(syn.point_sources(V, site=0)).cuda())
    for c, b in zip(ctxs, bs):  # first calls allocate every Krylov space
        c.solve_batched(b)
    w.solve_ragged(ctxs, bs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sep = [c.solve_batched(b) for c, b in zip(ctxs, bs)]
    torch.cuda.synchronize()
    t_sep = time.perf_counter() - t0
    fam = "coarse_mfma_ragged_f32"
    ctxs[0].profile(fam, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos, st, launches = w.solve_ragged(ctxs, bs)
    torch.cuda.synchronize()
    t_rag = time.perf_counter() - t0
    n, ms = ctxs[0].profile_stats(fam)
    ctxs[0].profile(fam, False)
    out = {"lattices": [list(l) for l in lats], "nrhs_each": 12, "ragged_solve_s": t_rag, "separate_batched_s": t_sep,
           "speedup": t_sep / t_rag, "status": st, "shared_coarse_launches": launches,
           "shared_launch_avg_us": ms * 1e3 / max(n, 1),
           "per_problem": []}
    for k in range(3):
        out["per_problem"].append({
            "lattice": list(lats[k]), "outer_iters": [i["outer_iters"] for i in infos[k]],
            "separate_outer_iters": [i["outer_iters"] for i in sep[k][1]],
            "max_true_rel_res": max(i["true_rel_res"] for i in infos[k]),
            "coarse_iters_all_rhs": infos[k][0]["coarse_iters"]})
    out["converged"] = st == 0 and all(i["converged"] for inf in infos for i in inf)
    print("[bench] ragged solve %.3f s (separate batched solves %.3f s), %d shared coarse launches" % (
        t_rag, t_sep, launches), file=sys.stderr, flush=True)
    for c in ctxs:
        c.close()
    torch.cuda.empty_cache()
    return out


def ragged_batch(w, torch, nrhs=12, reps=50):
    """One matrix-core launch over the coarse operators of three lattices (8^4,
    16^4 and 24^3 x 48 under 4^4 aggregates: 16 + 256 + 2592 coarse sites,
    Nb = 24, nrhs fields each) against the three operators launched one after
    another (sum of their back-to-back launch times)."""
    import numpy as np
    lats = [(2, 2, 2, 2), (4, 4, 4, 4), (6, 6, 6, 12)]
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    out = {"coarse_lattices": [list(l) for l in lats], "nb": 24, "nrhs": nrhs}
    for store, name in ((w.F32, "f32"), (w.BF16, "bf16")):
        ops, ins = [], []
        for Lc in lats:
            Vc = int(np.prod(Lc))
            op = w.CoarseOperator(Lc, 24, store)
            op.set(torch.randn((Vc, 9, 24, 24), dtype=torch.complex64, device="cuda", generator=g))
            op.set_kernel(2)
            ops.append(op)
            ins.append(torch.randn((nrhs, Vc, 24), dtype=torch.complex64, device="cuda", generator=g))
        w.coarse_time_ragged(ops, ins, reps=3)
        t_rag = w.coarse_time_ragged(ops, ins, reps=reps)
        t_sep = 0.0
        for op, x in zip(ops, ins):
            y = torch.empty_like(x)
            op.time(x, y, reps=3)
            t_sep += op.time(x, y, reps=reps)
        sb = 8 if name == "f32" else 4
        byts = sum((9.0 * 24 * 24 * sb + 2.0 * 24 * nrhs * 8) * int(np.prod(l)) for l in lats)
        out[name] = {"ragged_ms": t_rag, "separate_ms": t_sep, "speedup": t_sep / t_rag,
                     "ragged_GB_s": byts / t_rag / 1e6}
    return out


def learned_setup(w, torch, L=(16, 16, 16, 16), ntrain=6, ntest=4, epochs=8, nv=12, ch=32, lr=5e-3, seed=105):
    """Learned near-null proposal: trained on the plain setup's vectors (20
    sweeps + 2 refinement iterations) of ntrain seeded fields with eps ~
    U[0.2, 0.35], m0 = -0.08; on ntest held-out fields the learned setup
    (network + k MR sweeps, no refinement) is compared with the plain setup at
    the same k and with the plain 2-iteration setup: setup s, outer iterations,
    solve s.  Forward and backward throughput of the network kernels (FP32
    matrix cores) from HIP events.

    One context serves every field: each field's links and plain-setup
    vectors stay on the GPU and are loaded into it per training step (a
    context per field would not fit at 24^3 x 48 with 64 fields).  Links and
    start vectors are drawn on the GPU (gauge_field_device,
    start_vectors_device)."""
    import numpy as np
    import synthetic as syn
    V = int(np.prod(L))
    s = syn.config_seeds(seed)
    eps = np.random.default_rng(s["net"]).uniform(0.2, 0.35, ntrain + ntest)
    kw = dict(dims=L, m0=-0.08, c_sw=1.0, n_levels=2, block=((4, 4, 4, 4),), n_vec=(nv,), cycle_prec=w.F32,
              coarse_store_prec=w.F32, setup_prec=w.F32, outer_restart=20, outer_maxit=2000)

    def gauge(f):
        return syn.gauge_field_device(L, eps[f], s["gauge"] + f, "cuda")

    def start(f):
        return syn.start_vectors_device(nv, V, 12, s["start"] + f, "cuda")

    # targets: the plain 2-iteration setup of every field
    t0 = time.perf_counter()
    ctx = w.Context(relax_sweeps=20, refine_iters=2, **kw)
    links, targets = [], []
    for f in range(ntrain + ntest):
        U = gauge(f)
        ctx.set_gauge(U)
        ctx.set_null_vectors(0, start(f))
        ctx.setup()
        links.append(U)
        targets.append(ctx.null_vectors(0).clone())
        if f % 8 == 7:
            print("[bench] learned setup: %d fields set up" % (f + 1), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t0
    print("[bench] learned setup: %d plain setups %.1f s" % (ntrain + ntest, t_targets), file=sys.stderr, flush=True)

    def load(f):
        ctx.set_gauge(links[f])
        ctx.set_null_vectors(0, start(f))
        ctx.rebuild_from_vectors(0, targets[f])

    net = w.Network(nv, ch, act_prec=w.BF16, seed=s["net"])
    init = []
    for f in range(ntrain, ntrain + ntest):
        load(f)
        init.append(net.loss_grad(ctx, grad=False)[0])
    ctx.profile("nn_forward", True)
    ctx.profile("nn_backward", True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_load = 0.0
    curve = []
    for e in range(epochs):
        losses = []
        for f in range(ntrain):
            tl = time.perf_counter()
            load(f)
            torch.cuda.synchronize()
            t_load += time.perf_counter() - tl
            losses.append(net.train_step(ctx, lr=lr))
        curve.append(float(np.mean(losses)))
        print("[bench] learned setup: epoch %d loss %.4f" % (e, curve[-1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    nf, msf = ctx.profile_stats("nn_forward")
    nb_, msb = ctx.profile_stats("nn_backward")
    # useful complex multiply-adds of the three layers per site: 9 (Cin Cout) 12, 8 flops each
    fl = 8.0 * 9 * 12 * V * (nv * ch + ch * ch + ch * nv)
    held = []
    for f in range(ntrain, ntrain + ntest):
        load(f)
        held.append(net.loss_grad(ctx, grad=False)[0])
    ctx.close()
    del links[:ntrain], targets[:ntrain]
    torch.cuda.empty_cache()
    b = torch.from_numpy(syn.complex_gaussian((V, 4, 3), s["rhs"])).cuda()
    rows = []
    for i, f in enumerate(range(ntrain, ntrain + ntest)):
        r = {}
        U = links[i]
        for name, relax, refine, k in (("plain_20sweeps_2refine", 20, 2, None), ("plain_20sweeps", 20, 0, None),
                                       ("plain_5sweeps", 5, 0, None), ("learned_5sweeps", 20, 0, 5),
                                       ("learned_20sweeps", 20, 0, 20)):
            c = w.Context(relax_sweeps=relax, refine_iters=refine, **kw)
            c.set_gauge(U)
            c.set_null_vectors(0, start(f))
            if k is None:
                c.setup()
            else:
                fb, q = c.setup_learned(net, relax_sweeps=k)
            x, info, st = c.solve(b)
            r[name] = {"setup_s": c.timers()["setup"], "outer_iters": info[0]["outer_iters"],
                       "solve_s": info[0]["t_solve_s"], "converged": bool(info[0]["converged"]) and st == 0}
            if k is not None:
                r[name].update(fell_back=fb, quality=q)
            c.close()
            del x
        r["total_s"] = {n: r[n]["setup_s"] + r[n]["solve_s"] for n in list(r)}
        rows.append(r)
        print("[bench] learned setup: held-out field %d: %s" % (f, {n: (r[n]["outer_iters"], round(t, 4))
                                                                    for n, t in r["total_s"].items()}),
              file=sys.stderr, flush=True)
    del links, targets
    torch.cuda.empty_cache()
    names = list(rows[0]["total_s"])
    summary = {n: {"mean_outer_iters": float(np.mean([r[n]["outer_iters"] for r in rows])),
                   "mean_setup_s": float(np.mean([r[n]["setup_s"] for r in rows])),
                   "mean_solve_s": float(np.mean([r[n]["solve_s"] for r in rows])),
                   "mean_total_s": float(np.mean([r["total_s"][n] for r in rows]))} for n in names}
    return {"lattice": list(L), "n_vec": nv, "channels": ch, "train_fields": ntrain, "held_out_fields": ntest,
            "epochs": epochs, "targets_s": t_targets, "train_s": t_train, "train_load_s": t_load,
            "train_loss_curve": curve, "held_out_loss_untrained": init, "held_out_loss_trained": held,
            "summary": summary, "held_out": rows,
            "nn_forward": {"launches": nf, "avg_ms": msf / max(nf, 1), "TFLOP_s": fl / (msf / max(nf, 1)) / 1e9,
                           "frac_fp32_mfma": fl / (msf / max(nf, 1)) / 1e9 / 157.3},
            "nn_backward": {"launches": nb_, "avg_ms": msb / max(nb_, 1),
                            "TFLOP_s": 2 * fl / (msb / max(nb_, 1)) / 1e9,
                            "frac_fp32_mfma": 2 * fl / (msb / max(nb_, 1)) / 1e9 / 157.3}}


def cpu_baseline(wl, U, start, b, gpu_outer_iters, x_gpu=None):
    """The oracle (plain FP64 C++, OpenMP over sites) on all host cores, the
    whole workload, unsampled: its setup (20 MR sweeps, Gram-Schmidt, Galerkin
    coarsening) and refinement timed apart from its FP64 FGMRES solve on the
    same inputs as the GPU; also its outer iteration count and the distance
    between its solution and the GPU's (x_gpu, the last timed solve)."""
    import numpy as np
    import oracle
    H = oracle.Hierarchy(wl["L"], U, m0=wl["m0"], csw=wl["csw"], blocks=(wl["block"],), nv=(wl["nv"],),
                         relax_sweeps=wl["relax"], outer_restart=20, outer_maxit=2000)
    H.set_start(0, start)
    t0 = time.perf_counter()
    H.setup()
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    H.refine(wl["refine"])
    t_ref = time.perf_counter() - t0
    t0 = time.perf_counter()
    xo, ito, rro, sto = H.solve(b)
    t_sol = time.perf_counter() - t0
    rec = {"value": t_sol, "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
           "setup_s": t_init, "refine_s": t_ref, "outer_iters": ito, "true_rel_res": rro,
           "gpu_outer_iters_minus_oracle": gpu_outer_iters - ito,
           "sample": "the whole workload, unsampled: the oracle's setup (20 MR sweeps per vector, Gram-Schmidt, "
                     "Galerkin) %.1f s and refinement %.1f s, then its FP64 FGMRES(20) solve to 1e-10 (value), "
                     "%d outer iterations against the GPU's %d" % (t_init, t_ref, ito, gpu_outer_iters),
           "host_cpu": platform.processor() or platform.machine()}
    if x_gpu is not None:
        rec["rel_diff_gpu_solution"] = float(np.linalg.norm(x_gpu.reshape(-1) - xo) / np.linalg.norm(xo))
    return rec


def oracle_m2(w, torch, wl=WORKLOAD):
    """The whole workload on the oracle, unsampled -- setup (20 MR sweeps, one
    refinement iteration) and FP64 solve -- timed, next to the GPU's mixed
    and FP64 solves on the same inputs: outer iterations and the distance
    between the solutions."""
    import numpy as np
    import oracle
    U, start, b = make_inputs(wl)
    H = oracle.Hierarchy(wl["L"], U, m0=wl["m0"], csw=wl["csw"], blocks=(wl["block"],), nv=(wl["nv"],),
                         relax_sweeps=wl["relax"], outer_restart=20, outer_maxit=2000)
    H.set_start(0, start)
    t0 = time.perf_counter()
    H.setup()
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    H.refine(wl["refine"])
    t_ref = time.perf_counter() - t0
    print("[bench] oracle setup %.1f s + refinement %.1f s" % (t_init, t_ref), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    xo, ito, rro, sto = H.solve(b)
    t_sol = time.perf_counter() - t0
    print("[bench] oracle solve %.1f s, %d outer iterations, res %.2e" % (t_sol, ito, rro), file=sys.stderr,
          flush=True)
    out = {"workload": wl["name"], "cores": oracle.num_threads(),
           "oracle": {"setup_s": t_init, "refine_s": t_ref, "solve_s": t_sol, "outer_iters": ito,
                      "true_rel_res": rro, "status": sto}}
    Ud, startd, bd = (torch.from_numpy(a).cuda() for a in (U, start, b))
    for label, mixed in (("gpu_mixed", True), ("gpu_fp64", False)):
        ctx = make_context(w, wl, mixed=mixed)
        ctx.set_gauge(Ud)
        ctx.set_null_vectors(0, startd)
        ctx.setup()
        x, info, st = ctx.solve(bd)
        xg = x.cpu().numpy().reshape(-1)
        out[label] = {"outer_iters": info[0]["outer_iters"], "true_rel_res": info[0]["true_rel_res"],
                      "solve_s": info[0]["t_solve_s"], "setup_s": ctx.timers()["setup"],
                      "outer_iters_minus_oracle": info[0]["outer_iters"] - ito,
                      "rel_diff_to_oracle_solution": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))}
        ctx.close()
    return out


def kernel_mode(args):
    """Launch one kernel family back to back (for rocprofv3 counter runs) and
    print its mean launch duration from HIP events."""
    import numpy as np
    import torch
    import paper_1904_08678_amd as w
    torch.cuda.set_device(0)
    fam = args.family
    if fam == "copy":
        n = args.mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(args.reps):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"family": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n, "reps": args.reps}))
        return
    if fam == "three_level":
        print(json.dumps({"family": fam, **three_level(w, torch)}))
        return
    if fam == "ragged_solve":
        print(json.dumps({"family": fam, **ragged_solve(w, torch)}))
        return
    if fam == "oracle_m2":
        print(json.dumps({"family": fam, **oracle_m2(w, torch)}))
        return
    if fam == "learned_setup":
        # the learned-setup study at a chosen size: --lattice, --ntrain, --ntest, --epochs
        L = tuple(int(v) for v in args.lattice.split(","))
        res = learned_setup(w, torch, L=L, ntrain=args.ntrain, ntest=args.ntest, epochs=args.epochs)
        print(json.dumps({"family": fam, **res}))
        return
    if fam == "batched_solve":
        # setup plus one batched solve of the twelve point sources on 24^3 x 48
        import synthetic as syn
        wl = WORKLOAD_BATCH
        L = wl["L"]
        V = int(np.prod(L))
        s = syn.config_seeds(wl["seed"])
        ctx = make_context(w, wl, mixed=True, reserved=args.reserved)
        ctx.set_gauge(torch.from_numpy(syn.gauge_field(L, wl["eps"], s["gauge"])).cuda())
        ctx.set_null_vectors(0, torch.from_numpy(syn.start_vectors(wl["nv"], V, 12, s["start"])).cuda())
        ctx.setup()
        bd = torch.from_numpy(syn.point_sources(V, site=0)).cuda()
        t0 = time.perf_counter()
        x, info, st = ctx.solve_batched(bd, graph=args.graph)
        torch.cuda.synchronize()
        print(json.dumps({"family": fam, "solve_s": time.perf_counter() - t0, "status": st,
                          "outer_iters": [i["outer_iters"] for i in info]}))
        return
    if fam == "coarse_latency":
        # the latency line of the persistent coarsest GMRES on its own
        U, start, _ = make_inputs(WORKLOAD)
        res = coarse_gmres_latency(w, torch, WORKLOAD, torch.from_numpy(U).cuda(), torch.from_numpy(start).cuda(),
                                   reps=args.reps)
        print(json.dumps({"family": fam, **res}))
        return
    if fam.startswith("coarse_mk"):
        store = {"f64": w.F64, "f32": w.F32, "bf16": w.BF16}[fam.split("_")[-1]]
        res = coarse_apply_mk(w, torch, stores=(store,), reps=args.reps, nrhs_batch=args.nrhs)
        print(json.dumps({"family": fam, **res}))
        return
    wl = WORKLOAD
    L = wl["L"]
    V = int(np.prod(L))
    U, start, b = make_inputs(wl)
    ctx = make_context(w, wl, mixed=True, reserved=args.reserved)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    nr = max(1, args.nrhs)
    if fam in ("dslash_f32", "dslash_f64"):
        prec = w.F32 if fam.endswith("f32") else w.F64
        x = torch.from_numpy(b).cuda().to(torch.complex64 if prec == w.F32 else torch.complex128)
        x = x.unsqueeze(0).repeat(nr, 1, 1, 1).contiguous()
        ctx.profile(fam, True)
        for _ in range(args.reps):
            ctx.apply_D(0, x, prec)
        n, ms = ctx.profile_stats(fam)
    else:
        ctx.set_null_vectors(0, torch.from_numpy(start).cuda())
        ctx.setup()
        x = torch.from_numpy(b).cuda().to(torch.complex64).unsqueeze(0).repeat(nr, 1, 1, 1).contiguous()
        xc = torch.zeros((nr, V // 256, 24), dtype=torch.complex64, device="cuda")
        ctx.profile(fam, True)
        for _ in range(args.reps):
            if fam == "restrict_f32":
                ctx.restrict(0, x, w.F32)
            else:
                ctx.prolong(0, xc, w.F32)
        n, ms = ctx.profile_stats(fam)
    bpl = algorithmic_bytes(fam, V, V // 256, 24, 12, nr, link_rows=ctx.timers()["dslash_link_rows"])
    print(json.dumps({"family": fam, "nrhs": nr, "launches": n, "avg_ms": ms / max(n, 1), "bytes_per_launch": bpl,
                      "GB_s": bpl / (ms / max(n, 1)) / 1e6, "tuner": ctx.tune_table()}))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-mk", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-sap", action="store_true")
    ap.add_argument("--no-three", action="store_true", help="skip the three-level workload (32^3x64)")
    ap.add_argument("--no-coarse-compare", action="store_true",
                    help="skip the solves with the reference forms of the coarsest GMRES and the outer Arnoldi step")
    ap.add_argument("--kernel", dest="family", default=None,
                    help="only launch one kernel family: dslash_f32, dslash_f64, restrict_f32, prolong_f32, "
                         "coarse_mk_f32, coarse_mk_bf16, coarse_mk_f64, copy, batched_solve, learned_setup, "
                         "three_level, ragged_solve, oracle_m2, coarse_latency")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--reserved", type=int, default=0, help="kernel mode: reserved[0] flags (reference forms)")
    ap.add_argument("--graph", action="store_true", help="batched_solve kernel mode: HIP-graph cycle")
    ap.add_argument("--coarse-points", type=int, default=9, choices=(5, 9),
                    help="coarse blocks stored per site: 9, or 5 (Mdiag and forward hops)")
    ap.add_argument("--lattice", default="24,24,24,48", help="learned_setup kernel mode: lattice")
    ap.add_argument("--ntrain", type=int, default=48)
    ap.add_argument("--ntest", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--nrhs", type=int, default=0, help="right-hand sides for the batched coarse-apply kernel mode")
    args = ap.parse_args()
    global COARSE_POINTS
    COARSE_POINTS = args.coarse_points
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; N=%d is not supported (a multi-GPU run would shard the "
              "lattice by 4D domain decomposition, which is not implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.family:
        kernel_mode(args)
        return

    import numpy as np
    import torch
    import paper_1904_08678_amd as w

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    wl = WORKLOAD
    L = wl["L"]
    V = int(np.prod(L))
    Vc = V // int(np.prod(wl["block"]))
    nb = 2 * wl["nv"]
    print("[bench] generating inputs", file=sys.stderr, flush=True)
    U, start, b = make_inputs(wl)
    Ud, startd, bd = torch.from_numpy(U).cuda(), torch.from_numpy(start).cuda(), torch.from_numpy(b).cuda()

    ctx = make_context(w, wl, mixed=True)
    ctx.set_gauge(Ud)
    ctx.set_null_vectors(0, startd)
    # HBM-bound families (the roofline candidates), then the persistent
    # coarse GMRES, which is bound by its grid barriers, not by a stream
    roof_families = ["dslash_f64", "dslash_f32", "coarse_apply_f32", "restrict_f32", "prolong_f32"]
    families = roof_families + ["coarse_gmres_persistent"]

    last_x = [None]

    def step(prof):
        ctx.setup()
        setup_s = ctx.timers()["setup"]
        for f in families:
            ctx.profile(f, f in prof)
        x, info, st = ctx.solve(bd)
        for f in families:
            ctx.profile(f, False)
        last_x[0] = x
        return setup_s, info[0], st

    # The warmup steps time every family (the kernel table, and the choice of
    # the dominant HBM-bound kernel); the timed steps time only that kernel,
    # so that the events around the other launches do not slow the solve.
    table = {f: [0, 0.0] for f in families}
    table_iters = 0
    for i in range(args.warmup):
        s, inf, st = step(families)
        for f in families:
            n, ms = ctx.profile_stats(f)
            table[f][0] += n
            table[f][1] += ms
        table_iters += inf["coarse_iters"]
        print("[bench] warmup %d: setup %.3f s solve %.4f s iters %d res %.2e" % (
            i, s, inf["t_solve_s"], inf["outer_iters"], inf["true_rel_res"]), file=sys.stderr, flush=True)
    timed_families = [max(roof_families, key=lambda f: table[f][1])] if args.warmup > 0 else families
    stats = {f: [0, 0.0] for f in families}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    setups, solves, infos = [], [], []
    for i in range(args.steps):
        s, inf, st = step(timed_families)
        for f in families:
            n, ms = ctx.profile_stats(f)
            stats[f][0] += n
            stats[f][1] += ms
        setups.append(s)
        solves.append(inf["t_solve_s"])
        infos.append(inf)
        print("[bench] step %d: setup %.3f s solve %.4f s iters %d res %.2e" % (
            i, s, inf["t_solve_s"], inf["outer_iters"], inf["true_rel_res"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    solve_s = float(np.mean(solves))
    ok = all(i["converged"] and i["true_rel_res"] <= 1e-10 for i in infos)

    # dominant kernel of the solve, by total time, timed inside the timed steps
    dom = timed_families[0] if len(timed_families) == 1 else max(roof_families, key=lambda f: stats[f][1])
    if args.warmup == 0:
        table, table_iters = stats, sum(i["coarse_iters"] for i in infos)
    n, ms = stats[dom]
    avg_ms = ms / max(n, 1)
    link_rows = ctx.timers()["dslash_link_rows"]
    bpl = algorithmic_bytes(dom, V, Vc, nb, wl["nv"], link_rows=link_rows)
    achieved = bpl / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": counter_traffic(dom) if dom in TRAFFIC_SOURCES else None,
                "launches": n, "avg_launch_ms": avg_ms, "bytes_per_launch": bpl,
                "bytes_per_site": bpl / V if dom.startswith("dslash") else None,
                "dslash_link_rows": link_rows}
    # kernel table: from the warmup steps (every family timed there)
    kernel_table = {f: {"launches": table[f][0], "total_ms": table[f][1],
                        "avg_ms": table[f][1] / max(table[f][0], 1),
                        "GB_s": algorithmic_bytes(f, V, Vc, nb, wl["nv"], link_rows=link_rows) /
                        (table[f][1] / max(table[f][0], 1)) / 1e6
                        if table[f][0] else None} for f in roof_families}
    n_cg, ms_cg = table["coarse_gmres_persistent"]
    kernel_table["coarse_gmres_persistent"] = {
        "launches": n_cg, "total_ms": ms_cg, "avg_ms": ms_cg / max(n_cg, 1),
        "us_per_coarse_iter": ms_cg * 1e3 / table_iters if n_cg and table_iters else None}
    kernel_table["source"] = "warmup steps" if args.warmup > 0 else "timed steps"

    extra = {}
    if not args.no_fp64:
        print("[bench] plain FP64 solve", file=sys.stderr, flush=True)
        c64 = make_context(w, wl, mixed=False)
        c64.set_gauge(Ud)
        c64.set_null_vectors(0, startd)
        c64.setup()
        x64, inf64, st64 = c64.solve(bd)
        x64b, inf64b, _ = c64.solve(bd)
        extra["fp64"] = {"solve_s": min(inf64[0]["t_solve_s"], inf64b[0]["t_solve_s"]),
                         "setup_s": c64.timers()["setup"], "outer_iters": inf64[0]["outer_iters"],
                         "true_rel_res": inf64[0]["true_rel_res"]}
        extra["speedup_mixed_vs_fp64"] = extra["fp64"]["solve_s"] / solve_s
        del c64
    # setup checkpoint: export the timed context's hierarchy, load it into a
    # fresh context (rebuild from the vectors, no relaxation or refinement)
    t_e = time.perf_counter()
    blob = ctx.export_setup()
    t_e = time.perf_counter() - t_e
    c2 = make_context(w, wl, mixed=True)
    c2.set_gauge(Ud)
    t_i = time.perf_counter()
    c2.import_setup(blob)
    t_i = time.perf_counter() - t_i
    x2, inf2, _ = c2.solve(bd)
    extra["setup_checkpoint"] = {"bytes": len(blob), "export_s": t_e, "import_s": t_i,
                                 "setup_s": float(np.mean(setups)), "solve_outer_iters": inf2[0]["outer_iters"],
                                 "true_rel_res": inf2[0]["true_rel_res"]}
    del c2, blob
    print("[bench] coarsest GMRES: time per Arnoldi step", file=sys.stderr, flush=True)
    latency = coarse_gmres_latency(w, torch, wl, Ud, startd)
    if not args.no_coarse_compare:
        print("[bench] reference forms of the coarsest GMRES and the outer Arnoldi step", file=sys.stderr, flush=True)
        extra["reference_forms"] = reference_forms(w, torch, wl, Ud, startd, bd)
    if not args.no_sap:
        print("[bench] SAP smoother", file=sys.stderr, flush=True)
        extra["sap_smoother"] = sap_smoother(w, torch, wl, Ud, startd, bd)
        print("[bench] even-odd outer solve", file=sys.stderr, flush=True)
        extra["even_odd"] = even_odd(w, torch, wl, Ud, startd, bd)
    if not args.no_mk:
        print("[bench] coarse apply on the 16^3x32 coarse lattice (Vc=131072, Nb=24)", file=sys.stderr, flush=True)
        extra["coarse_apply_large"] = coarse_apply_mk(w, torch)
        for nbx in (16, 32):
            print("[bench] coarse apply on the 16^3x32 coarse lattice, Nb=%d" % nbx, file=sys.stderr, flush=True)
            extra["coarse_apply_large_nb%d" % nbx] = coarse_apply_mk(w, torch, nb=nbx, reps=10)
        extra["coarse_apply_large"]["per_store"]["f32"]["traffic"] = counter_traffic("coarse_apply_f32_large")
        for st in ("f32", "bf16"):
            rec = extra["coarse_apply_large"]["batched"].get(st)
            if rec:
                rec["matrix_cores"]["traffic"] = counter_traffic("coarse_mfma_%s_12rhs" % st)
    if not args.no_batched:
        print("[bench] batched point sources, 24^3x48", file=sys.stderr, flush=True)
        extra["batched_24x48"] = batched_point_sources(w, torch, WORKLOAD_BATCH, fp64=not args.no_fp64)
        print("[bench] ragged batch of coarse operators", file=sys.stderr, flush=True)
        extra["ragged_coarse_apply"] = ragged_batch(w, torch)
        print("[bench] ragged solve: 8^4 + 16^4 + 24^3x48, 12 point sources each", file=sys.stderr, flush=True)
        extra["ragged_solve"] = ragged_solve(w, torch)
    if not args.no_three:
        print("[bench] three-level workload, 32^3x64", file=sys.stderr, flush=True)
        extra["three_level_32x64"] = three_level(w, torch, fp64=not args.no_fp64)
    if not args.no_learned:
        print("[bench] learned setup (16^4, 6 training / 4 held-out fields)", file=sys.stderr, flush=True)
        extra["learned_setup"] = learned_setup(w, torch)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle: the whole workload", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, U, start, b, infos[-1]["outer_iters"], last_x[0].cpu().numpy())

    line = {
        "metric": METRIC, "value": solve_s, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl["name"], "lattice": list(L), "aggregates": list(wl["block"]), "Nb": nb,
                   "m0": wl["m0"], "c_sw": wl["csw"], "eps": wl["eps"], "tol": 1e-10, "precision":
                   "FP32 cycle and coarse blocks, FP64 outer FGMRES", "coarse_points": COARSE_POINTS},
        "converged": ok, "setup_s": float(np.mean(setups)), "outer_iters": infos[-1]["outer_iters"],
        "coarse_iters": infos[-1]["coarse_iters"], "true_rel_res": infos[-1]["true_rel_res"],
        "roofline": roofline, "latency": latency, "kernels": kernel_table, "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
