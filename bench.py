"""Benchmark of the spectral-element Poisson CG hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: 16^3 = 4096 unit-cube hexahedra, N = 9 (10^3 GLL points per element,
4,096,000 local points), load vector f ~ U[0,1) (PCG64 seed 2), homogeneous
Dirichlet box, solved to a relative residual of 1e-8.  One step = one whole
mixed-precision solve (FP32 operator / FP64 reductions, scalars and
refinement); its FP64 CG counterpart is timed the same way next to it.

Prints ONE JSON line: the mixed solve's CG GDOF*iter/s (local points x CG
iterations / solve time), the FP64 solve's, the roofline of the dominant
kernel (fused add2s1 + operator, HIP events on the solver's stream), the
ax+dssum bandwidth at each precision, the energy per solve of both
precisions (GPU package energy counter), and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NEL, N, TOL, SEED = (16, 16, 16), 9, 1e-8, 2
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the fused FP32 operator kernel measured by the
# FETCH_SIZE and WRITE_SIZE counters (scaled by a 256 MiB copy in the same
# runs) in the FP32 configurations listed; profiles/cg_16x16x16_N9_kernels.md
# holds the runs.  The figure is reported only while the source that the
# operator kernel compiles from still hashes to the SHA-256 digests below:
# nek_kernels.hpp up to its gather-scatter section (the operator kernel and
# every helper it calls), nek_np.hpp up to its CG iteration launchers (the
# operator's launch), and the context header in full.  Later edits to other
# kernels and launchers leave it valid.
COUNTER_TRAFFIC = {
    "sources": {
        ("paper_2405_11065_amd/csrc/nek_kernels.hpp", "// --------------------------------------------------"
         "--------- gather-scatter"):
            "e755ca80903cb8ed92ec86b0932793b3385e1fec0fe52efeea909951b882a7e2",
        ("paper_2405_11065_amd/csrc/nek_np.hpp", "    // CG iteration it (1-based)"):
            "5370dc438f42553ad0db76050ddf7632b23cda5b1e5852145f73621ea40220f6",
        ("paper_2405_11065_amd/csrc/nek_internal.hpp", None):
            "ec60c54ea130004c265a803ff81ae11e50b530fd65d6ae95fb149f14f7b5d5c8",
    },
    "bytes_per_launch": {4: 226_600_000, 5: 226_300_000},   # FP32 configuration -> bytes
}


def operator_source_digest(rel, end_marker):
    """SHA-256 of a source file, or of its text before end_marker (None: the
    whole file); a missing marker hashes the whole file, so it cannot match."""
    import hashlib
    with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
        text = fh.read()
    if end_marker is not None and end_marker in text:
        text = text[:text.index(end_marker)]
    return hashlib.sha256(text.encode("utf-8")).hexdigest()


def counter_traffic(variant):
    for (rel, end_marker), digest in COUNTER_TRAFFIC["sources"].items():
        if operator_source_digest(rel, end_marker) != digest:
            return None
    return COUNTER_TRAFFIC["bytes_per_launch"].get(variant)


def ax_dssum_bytes_per_point(sv, sg, sigma):
    """Algorithmic HBM bytes per local point of nek_ax (operator + segment
    dssum): u read, w write, six g factors, then for the element-surface
    fraction sigma: w read + write and the int32 permutation, plus ~1 B of
    segment offsets."""
    return 2 * sv + 6 * sg + sigma * (2 * sv + 4) + 1


def cg_operator_bytes_per_point(sv, sg, sx):
    """Fused CG operator kernel: r, p read, p, w write, six g factors, and the
    deferred x (or correction) update, read + write of sx-byte entries."""
    return 4 * sv + 6 * sg + 2 * sx


def time_ax_dssum(ctx, torch, dtype, reps=20):
    u = torch.rand(ctx.nl, dtype=dtype, device="cuda")
    w = torch.empty_like(u)
    for _ in range(3):
        ctx.ax(u, w)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        ctx.ax(u, w)
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps / 1e3


def ax_dssum_all(ctx, torch):
    """nek_ax time and algorithmic bandwidth at each precision, in the
    context's tuned kernel configuration for that precision."""
    sigma = 1.0 - ((ctx.N - 1) / (ctx.N + 1)) ** 3
    axd = {}
    for prec, dt, sv, sg in (("fp64", torch.float64, 8, 8), ("fp32", torch.float32, 4, 4),
                             ("bf16g", torch.float32, 4, 2)):
        ctx.set_prec(prec)
        t = time_ax_dssum(ctx, torch, dt)
        b = ax_dssum_bytes_per_point(sv, sg, sigma) * ctx.nl
        axd[prec] = {"us": round(t * 1e6, 2), "GBps": round(b / t / 1e9, 1),
                     "frac_hbm": round(b / t / 1e9 / PEAK_HBM_GBS, 3)}
    return axd


def dssum_seg(ctx, torch, reps=20):
    """The standalone sorted-segment direct-stiffness summation (nek_dssum,
    masked) per vector type: mean time per call and algorithmic bandwidth.
    Algorithmic bytes: every surface copy read and written once, its int32
    permutation entry, and per segment its int32 offset and int8 flag."""
    from paper_2405_11065_amd import nek
    nperm, nseg = ctx.size(nek.NEK_SIZE_NPERM), ctx.size(nek.NEK_SIZE_NSEG)
    out = {}
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        w = torch.rand(ctx.nl, dtype=dt, device="cuda")
        ctx.dssum(w)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            ctx.dssum(w)
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) / reps / 1e3
        b = nperm * (2 * w.element_size() + 4) + nseg * 5
        out[name] = {"us": round(t * 1e6, 2), "GBps": round(b / t / 1e9, 1), "frac_hbm": round(b / t / 1e9 / PEAK_HBM_GBS, 3),
                     "segments": nseg, "surface_copies": nperm}
    return out


def copy_bandwidth(torch, mib=512, reps=10):
    """Device-to-device copy of `mib` MiB (read + write counted), beyond the
    256 MB memory-side cache: the practical streaming ceiling that the
    ax + dssum fraction is read against."""
    a = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    t = s.elapsed_time(e) / reps / 1e3
    gbps = 2 * a.numel() * 4 / t / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"MiB": mib, "GBps": round(gbps, 1), "frac_hbm": round(gbps / PEAK_HBM_GBS, 3)}


def cpu_baseline(f, budget_s=12.0):
    """The FP64 oracle on the same workload, fixed iteration windows: its
    serial build on one core, and its OpenMP build (element loop and
    element-wise updates threaded, fixed-order serial reductions, results
    bit-identical) on the threads OpenMP is given (OMP_NUM_THREADS, else the
    cores in the process's affinity mask)."""
    import oracle
    from paper_2405_11065_amd import synth
    P = oracle.Problem(N, NEL, synth.box_vertices(NEL))
    affinity = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or affinity
    oracle.omp_threads(threads)
    out = {}
    for label, omp in (("serial", False), ("openmp", True)):
        t0 = time.perf_counter()
        P.cg(f, tol=0.0, maxit=2, omp=omp)
        per_it = (time.perf_counter() - t0) / 2
        k = max(2, int(budget_s / max(per_it, 1e-6)))
        t0 = time.perf_counter()
        _, it, _ = P.cg(f, tol=0.0, maxit=k, omp=omp)
        dt = time.perf_counter() - t0
        out[label] = {"value": P.nl * it / dt / 1e9, "iters": it, "seconds": round(dt, 2),
                      "cores": oracle.omp_threads() if omp else 1}
    par = out["openmp"]
    return {"value": par["value"], "unit": "GDOF*iter/s", "cores": par["cores"], "kind": "oracle",
            "sample": f"FP64 oracle CG (Table 1 loop) on the same 16^3 N=9 problem, {par['iters']} fixed "
                      f"iterations ({par['seconds']} s) with OpenMP on {par['cores']} threads "
                      f"({affinity} cores in the affinity mask); setup excluded",
            "serial": {"value": out["serial"]["value"], "cores": 1, "iters": out["serial"]["iters"],
                       "seconds": out["serial"]["seconds"]},
            "affinity_cores": affinity, "build": "gcc -O3 -march=x86-64-v3 -fopenmp -ffp-contract=off "
                                                 "(serial: -O2 -ffp-contract=off)"}


def big_case(torch, nek, synth, steps=2, energy=True, jacobi=True):
    """32^3 elements on [0,1]^3, interior vertices moved up to 10 %, N=9
    (32.8 M local points), f = B (sin pi x sin pi y sin pi z + N(0,1e-3)):
    mixed solve with BF16-stored g against FP64 CG, tol 1e-8; then nek_ax
    bandwidth at each precision on this mesh."""
    nel = (32, 32, 32)
    vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=0.1, seed=synth.SEED_C3_VERTICES)
    ctx = nek.Context(nel, 9, vtx=vtx, prec="bf16g")
    X = ctx.get(nek.NEK_GET_XYZ)
    B = ctx.get(nek.NEK_GET_B).reshape(ctx.E, -1)
    noise = synth.normal_noise(ctx.nl, 1e-3, synth.SEED_C3).reshape(ctx.E, -1)
    f = torch.from_numpy((B * (synth.sine_field(X) + noise)).ravel()).cuda()
    del X, B, noise
    x = ctx.new_vector()
    out = {"local_points": ctx.nl}
    roof = {}
    for prec in ("bf16g", "fp32", "fp64"):
        ctx.set_prec(prec)
        ctx.tune(prec, iters=10)
        ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
        ctx.prof_read(0, reset=True)
        ctx.prof_read(1, reset=True)
        ctx.prof_enable(16)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = 0
        for _ in range(steps):
            _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
            its += st["iters"]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ctx.prof_enable(0)
        out[prec] = {"ms_per_solve": round(dt * 1e3, 2), "iters": its / steps, "outer": st["outer_iters"],
                     "GDOF_iter_per_s": round(ctx.nl * its / steps / dt / 1e9, 3),
                     "true_rel_res": st["true_rel_res"], "last_rec_res": st["last_rec_res"],
                     "tuned_variant": ctx.get_variant(prec)}
        roof[prec] = kernel_roofline(ctx, prec)
    out["cg_kernel_roofline"] = roof
    # FP64 CG with the factors recomputed in the kernels (every element is trilinear)
    ctx.set_geometry("trilinear")
    ctx.set_prec("fp64")
    ctx.tune("fp64", iters=10)
    ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out["fp64_trilinear"] = {"ms_per_solve": round(dt * 1e3, 2), "iters": st["iters"],
                             "true_rel_res": st["true_rel_res"], "tuned_variant": ctx.get_variant("fp64")}
    ctx.set_geometry("stored")
    best64 = min(out["fp64"]["ms_per_solve"], out["fp64_trilinear"]["ms_per_solve"])
    out["fastest_fp64"] = "trilinear" if out["fp64_trilinear"]["ms_per_solve"] < out["fp64"]["ms_per_solve"] else "stored"
    out["speedup_vs_fp64"] = round(best64 / out["bf16g"]["ms_per_solve"], 3)
    out["speedup_vs_fp64_stored"] = round(out["fp64"]["ms_per_solve"] / out["bf16g"]["ms_per_solve"], 3)
    out["fp32_speedup_vs_fp64"] = round(best64 / out["fp32"]["ms_per_solve"], 3)
    if energy:
        out["energy"] = big_energy(torch, ctx, f, x, {"bf16g": out["bf16g"]["ms_per_solve"], "fp64": best64},
                                   out["fastest_fp64"])
    for pc in (("jacobi", "fdm", "schwarz") if jacobi else ()):
        # the same solves with a preconditioner (kernels autotuned for it)
        saved = {p: ctx.get_variant(p) for p in ("bf16g", "fp32", "fp64")}
        ctx.set_precond(pc)
        jac = {}
        # with Schwarz the FP32-g inner loop refines every 1e-2 (4 steps) where BF16 g needs 0.3 (14)
        for prec in ("bf16g", "fp32", "fp64") if pc == "schwarz" else ("bf16g", "fp64"):
            ctx.set_prec(prec)
            ctx.tune(prec, iters=10)
            ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            jac[prec] = {"ms_per_solve": round(dt * 1e3, 2), "iters": st["iters"], "outer": st["outer_iters"],
                         "true_rel_res": st["true_rel_res"], "speedup_vs_unpreconditioned":
                         round(out[prec]["ms_per_solve"] / (dt * 1e3), 3)}
        if pc == "schwarz":
            jac["window_kernels"] = schwarz_kernels(torch, ctx, f, x, ("bf16g", "fp64"), steps)
        ctx.set_precond("none")
        for p, v in saved.items():
            ctx.set_variant(p, v)
        out[pc] = jac
    # ax + dssum at this size: the working set exceeds the 256 MB memory-side cache
    ctx.tune("fp32", iters=10)
    out["ax_dssum"] = ax_dssum_all(ctx, torch)
    out["dssum_seg"] = dssum_seg(ctx, torch)
    ctx.close()
    torch.cuda.empty_cache()
    return out


def big_energy(torch, ctx, f, x, ms_per_solve, fp64_geometry="stored"):
    """Energy per solve of the 32^3 case, BF16-g mixed against FP64 (in its
    fastest factor source)."""
    try:
        meter = EnergyCounter(torch)
    except Exception as ex:
        return {"error": f"energy counter unavailable: {ex!r}"}
    out = {}
    try:
        for prec in ("bf16g", "fp64"):
            ctx.set_prec(prec)
            ctx.set_geometry(fp64_geometry if prec == "fp64" else "stored")
            watts, window, calls = steady_power(
                meter.read, lambda: ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True),
                min_window_s=4.0, max_run_s=30.0)
            out[prec] = {"W": round(watts, 1), "window_s": round(window, 2), "solves_in_run": calls,
                         "J_per_solve": round(watts * ms_per_solve[prec] / 1e3, 2)}
        out["energy_reduction_pct"] = round(100 * (1 - out["bf16g"]["J_per_solve"] / out["fp64"]["J_per_solve"]), 2)
        out["fp64_geometry"] = fp64_geometry
    except Exception as ex:
        out["error"] = repr(ex)
    finally:
        ctx.set_geometry("stored")
        meter.close()
    return out


def kernel_roofline(ctx, prec):
    """Sampled mean durations of the two CG kernels (HIP events on the
    solver's stream, every 16th iteration) against their algorithmic bytes:
    the operator kernel moves 4 s_v + 6 s_g + 2 s_x per point (r, p in; p,
    w out; six factors; the deferred iterate / correction update, FP64),
    the gather/update kernel 3 s_v (w, r in; r out)."""
    sv, sg = {"fp64": (8, 8), "fp32": (4, 4), "bf16g": (4, 2)}[prec]
    ops = {"operator": (0, cg_operator_bytes_per_point(sv, sg, 8)), "update": (1, 3 * sv)}
    res = {}
    for name, (k, bpp) in ops.items():
        ms, n = ctx.prof_read(k)
        if not n:
            res[name] = None
            continue
        t = ms / n / 1e3
        gbs = bpp * ctx.nl / t / 1e9
        res[name] = {"avg_us": round(t * 1e6, 2), "bytes_per_point": bpp, "GBps": round(gbs, 1),
                     "frac_hbm": round(gbs / PEAK_HBM_GBS, 3), "sampled_launches": n}
    return res


def operator_kernels(torch, nek, synth, orders=(7, 9, 11), ne=16, reps=20):
    """The plain operator pass (nek_ax_local) with its D contractions on the
    vector ALUs (the kernel form of every CG iteration) and on the matrix
    cores, on the ne^3 box at N + 1 = 8, 10, 12, FP32, BF16-stored factors and
    FP64: mean time per call and algorithmic bandwidth (u read, w written,
    six factors read)."""
    out = {}
    for N in orders:
        ctx = nek.Context((ne, ne, ne), N, prec="fp64")
        for prec, dt in (("fp32", torch.float32), ("bf16g", torch.float32), ("fp64", torch.float64)):
            ctx.set_prec(prec)
            ctx.tune(prec, iters=5)
            u = torch.rand(ctx.nl, dtype=dt, device="cuda")
            w = torch.empty_like(u)
            res = {}
            for kind in ("valu", "mfma"):
                ctx.set_operator_kernel(kind)
                ctx.ax_local(u, w)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    ctx.ax_local(u, w)
                torch.cuda.synchronize()
                t = (time.perf_counter() - t0) / reps
                gbs = ctx.nl * (2 * u.element_size() + (12 if prec == "bf16g" else 6 * u.element_size())) / t / 1e9
                res[kind] = {"us": round(t * 1e6, 1), "GBps": round(gbs, 1)}
            ctx.set_operator_kernel("valu")
            res["mfma_over_valu_time"] = round(res["mfma"]["us"] / res["valu"]["us"], 3)
            out[f"NP{N + 1}_{prec}"] = res
            log(f"operator kernels N={N} {prec}: {res}")
        ctx.close()
        torch.cuda.empty_cache()
    return out


def schwarz_kernels(torch, ctx, f, x, precs, steps, napply=20):
    """The Schwarz window solves on the matrix cores against the vector-ALU
    form (the default takes the matrix cores for FP64 vectors only), on a context already set up for the Schwarz-preconditioned
    solve: mean time of one preconditioner application z = M^-1 r (window
    solves, coarse solve, gather) per vector type, and of the whole solve per
    precision, with each kernel."""
    out = {}
    r = {dt: torch.rand(ctx.nl, dtype=dt, device="cuda") for dt in (torch.float32, torch.float64)}
    for kind in ("mfma", "valu"):
        ctx.set_schwarz_kernel(kind)
        res = {}
        for name, dt in (("apply_fp32_us", torch.float32), ("apply_fp64_us", torch.float64)):
            z = ctx.precond_apply(r[dt])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(napply):
                ctx.precond_apply(r[dt], z)
            torch.cuda.synchronize()
            res[name] = round((time.perf_counter() - t0) / napply * 1e6, 1)
        for prec in precs:
            ctx.set_prec(prec)
            ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
            torch.cuda.synchronize()
            res[f"{prec}_ms_per_solve"] = round((time.perf_counter() - t0) / steps * 1e3, 2)
            res[f"{prec}_iters"] = st["iters"]
        out[kind] = res
    ctx.set_schwarz_kernel("auto")
    out["mfma_speedup"] = {k: round(out["valu"][k] / out["mfma"][k], 3) for k in out["mfma"] if not k.endswith("iters")}
    return out


def precond_case(torch, ctx, f, steps, base, pc="jacobi"):
    """A preconditioner (pc: 'jacobi' diagonal, 'fdm' element-interior fast
    diagonalization with the diagonal elsewhere, or 'schwarz' two-level
    overlapping Schwarz) on the same solve: iterations, time and per-kernel
    sampled durations (for 'fdm' and 'schwarz' the second figure brackets the
    update and preconditioner kernels together) for FP64 CG
    and the mixed solve, against the unpreconditioned runs in `base`
    (prec -> (ms, iters))."""
    out = {}
    saved = {p: ctx.get_variant(p) for p in ("fp32", "fp64")}
    x = ctx.new_vector()
    ctx.set_precond(pc)
    try:
        for prec in ("fp32", "fp64"):
            ctx.set_prec(prec)
            tuned = ctx.tune(prec, iters=30)   # the configuration of the preconditioned kernel pair
            _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
            ctx.prof_read(0, reset=True)
            ctx.prof_read(1, reset=True)
            ctx.prof_enable(16)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = 0
            for _ in range(steps):
                _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
                its += st["iters"]
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            ctx.prof_enable(0)
            k0, n0 = ctx.prof_read(0)
            k1, n1 = ctx.prof_read(1)
            ms0, it0 = base[prec]
            out[prec] = {"ms_per_solve": round(dt * 1e3, 3), "iters": its / steps, "outer": st["outer_iters"],
                         "true_rel_res": st["true_rel_res"], "tuned_variant": tuned[0],
                         "operator_us": round(k0 / max(n0, 1) * 1e3, 2), "update_us": round(k1 / max(n1, 1) * 1e3, 2),
                         "unpreconditioned_ms": round(ms0, 3), "unpreconditioned_iters": it0,
                         "speedup": round(ms0 / (dt * 1e3), 3)}
        if pc == "schwarz":
            out["window_kernels"] = schwarz_kernels(torch, ctx, f, x, ("fp32", "fp64"), steps)
    finally:
        ctx.set_precond("none")
        for p, v in saved.items():
            ctx.set_variant(p, v)
    return out


def refinement_case(torch, nek, f, steps, base_ms):
    """The same mixed solve under the other refinement layouts, each on its
    own context (the layout is a set-up option) and autotuned: restarted
    refinement (CG restarted after every true-residual update, inner
    reduction 1e-4) and the correction d stored in FP32 instead of FP64."""
    out = {}
    for label, kw in (("restarted", {"refine_mode": 1}), ("corr_fp32", {"corr_fp32": 1})):
        c = nek.Context(NEL, N, prec="fp32", **kw)
        c.tune("fp32", iters=30)
        xr = c.new_vector()
        c.cg_solve(f, tol=TOL, maxit=20000, x=xr, raise_on_noconv=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = 0
        for _ in range(steps):
            _, st, _ = c.cg_solve(f, tol=TOL, maxit=20000, x=xr, raise_on_noconv=True)
            its += st["iters"]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[label] = {"ms_per_solve": round(dt * 1e3, 3), "iters": its / steps, "outer": st["outer_iters"],
                      "true_rel_res": st["true_rel_res"], "GDOF_iter_per_s": round(c.nl * its / steps / dt / 1e9, 3),
                      "default_ms_over_this": round(base_ms / (dt * 1e3), 3)}
        c.close()
    return out


def geometry_case(torch, ctx, f, steps, base):
    """The same solves with the geometric factors recomputed in the kernel
    from each element's trilinear map (nek_set_geometry) instead of read from
    memory: FP64 CG and the mixed solve, against the stored-factor runs in
    `base` (prec -> (ms, iters))."""
    out = {}
    saved = {p: ctx.get_variant(p) for p in ("fp32", "fp64")}
    x = ctx.new_vector()
    ctx.set_geometry("trilinear")
    try:
        for prec in ("fp32", "fp64"):
            ctx.set_prec(prec)
            tuned = ctx.tune(prec, iters=30)
            _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = 0
            for _ in range(steps):
                _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
                its += st["iters"]
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            ms0, _ = base[prec]
            out[prec] = {"ms_per_solve": round(dt * 1e3, 3), "iters": its / steps, "true_rel_res": st["true_rel_res"],
                         "GDOF_iter_per_s": round(ctx.nl * its / steps / dt / 1e9, 3),
                         "tuned_variant": tuned[0], "stored_factors_ms": round(ms0, 3),
                         "speedup": round(ms0 / (dt * 1e3), 3)}
    finally:
        ctx.set_geometry("stored")
        for p, v in saved.items():
            ctx.set_variant(p, v)
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class EnergyCounter:
    """The GPU package's energy accumulator, read through amdsmi.

    read() returns (joules, seconds), both from the counter itself: the
    accumulated energy and the firmware timestamp of its last update.  On
    MI355X the accumulator advances about once per second, so energies are
    taken between two updates, never between two arbitrary host instants.
    """

    def __init__(self, torch):
        import amdsmi
        self._smi = amdsmi
        amdsmi.amdsmi_init(amdsmi.AmdSmiInitFlags.INIT_AMD_GPUS)
        handles = amdsmi.amdsmi_get_processor_handles()
        if len(handles) == 1:
            self.h = handles[0]
        else:   # the handle whose PCI bus is cuda:0's
            bus = torch.cuda.get_device_properties(0).pci_bus_id
            match = [h for h in handles if int(amdsmi.amdsmi_get_gpu_device_bdf(h).split(":")[1], 16) == bus]
            if len(match) != 1:
                raise RuntimeError("cannot match cuda:0 to an amdsmi handle")
            self.h = match[0]

    def read(self):
        e = self._smi.amdsmi_get_energy_count(self.h)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6, e["timestamp"] * 1e-9

    def close(self):
        self._smi.amdsmi_shut_down()


def steady_power(read, work, min_window_s=3.0, max_run_s=20.0, clock=time.perf_counter):
    """Mean power while `work` runs back to back.

    `read()` gives (joules, seconds) of an accumulating counter that updates
    at its own pace.  The interval from the last update before the run to
    the first one inside it is partly idle, so the window starts at the first
    update seen after `work` has begun and ends at the last update seen before
    it stops; `work` repeats until that window spans `min_window_s` seconds of
    the counter's clock.  Returns (watts, window seconds, calls of work).
    """
    prev = read()
    snaps = []
    calls = 0
    t0 = clock()
    while True:
        work()
        calls += 1
        cur = read()
        if cur[1] != prev[1]:
            snaps.append(cur)
            prev = cur
        if len(snaps) >= 2 and snaps[-1][1] - snaps[0][1] >= min_window_s:
            break
        if clock() - t0 > max_run_s:
            break
    if len(snaps) < 2 or snaps[-1][1] <= snaps[0][1]:
        raise RuntimeError("energy counter did not advance twice during the run")
    (e0, s0), (e1, s1) = snaps[0], snaps[-1]
    return (e1 - e0) / (s1 - s0), s1 - s0, calls


def energy_to_solution(torch, ctx, solve, ms_per_solve, fp64_geometry="stored"):
    """Energy per solve at each precision (the paper's energy-to-solution,
    Table 6, here for the GPU package): mean package power while the solve
    repeats back to back, times the solve's time from the timed steps.
    Idle power is measured beside it so the dynamic part can be separated.
    FP64 runs in its fastest factor source (fp64_geometry)."""
    try:
        meter = EnergyCounter(torch)
    except Exception as ex:   # no amdsmi or no permission: report, do not fail the bench
        return {"error": f"energy counter unavailable: {ex!r}"}
    out = {"source": "amdsmi energy accumulator, GPU package (compute dies and HBM), ~1 s updates"}
    try:
        torch.cuda.synchronize()
        out["idle_W"] = round(steady_power(meter.read, lambda: time.sleep(0.05), min_window_s=2.0)[0], 1)
        for prec in ("fp32", "fp64"):
            ctx.set_prec(prec)
            ctx.set_geometry(fp64_geometry if prec == "fp64" else "stored")
            watts, window, calls = steady_power(meter.read, solve, min_window_s=4.0)
            ms = ms_per_solve[prec]
            out[prec] = {"W": round(watts, 1), "window_s": round(window, 2), "solves_in_run": calls,
                         "ms_per_solve": ms, "J_per_solve": round(watts * ms / 1e3, 3),
                         "dynamic_J_per_solve": round((watts - out["idle_W"]) * ms / 1e3, 3)}
        out["energy_reduction_pct"] = round(100 * (1 - out["fp32"]["J_per_solve"] / out["fp64"]["J_per_solve"]), 2)
        out["paper_context"] = ("47.14 % energy-to-solution reduction at 128 MPI ranks on a 2x EPYC 7763 node "
                                "(Table 6); a CPU node, not comparable hardware")
        out["fp64_geometry"] = fp64_geometry
    except Exception as ex:
        out["error"] = repr(ex)
    finally:
        ctx.set_geometry("stored")
        meter.close()
    return out


def batch_case(torch, nek, synth, nprob=64, steps=1):
    """64 independent cubes of n_e^3 unit elements, n_e ~ U{2..24}, N ~
    U{5,7,9,11} (PCG64 seed 4), f ~ U[0,1) per problem; one batched mixed
    solve (FP32 operator / FP64 reductions, tol 1e-8) per step, after the
    per-order autotuner.  Beside it: the same batch with plain launches
    instead of graph replay, and every problem solved alone in turn on its
    context (same kernel configuration), whose x must be bit-identical."""
    draw = synth.batch_draw(synth.SEED_C4, nprob)
    t0 = time.perf_counter()
    b = nek.Batch(draw, prec="fp32")
    t_setup = time.perf_counter() - t0
    log(f"batch setup {t_setup:.1f} s, {sum(b.nl) / 1e6:.1f} M local points")
    fs = [torch.from_numpy(synth.uniform_load(b.nl[i], synth.batch_load_seed(synth.SEED_C4, i))).cuda()
          for i in range(b.n)]
    tuned = b.tune("fp32", iters=10)
    xs = [torch.empty(b.nl[i], dtype=torch.float64, device="cuda") for i in range(b.n)]
    b.solve(fs, tol=TOL, maxit=20000, xs=xs, raise_on_noconv=True)   # warm-up (records the graph)
    res = {}
    for mode, graph in (("graph", True), ("plain", False)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st, _ = b.solve(fs, tol=TOL, maxit=20000, xs=xs, graph=graph, raise_on_noconv=True)
        torch.cuda.synchronize()
        res[mode] = ((time.perf_counter() - t0) / steps, st)
        log(f"batch {mode}: {res[mode][0] * 1e3:.1f} ms")
    dt, st = res["graph"]
    work = sum(b.nl[i] * st[i]["iters"] for i in range(b.n))
    xb = [x.clone() for x in xs]
    # every problem alone, one after the other, on the same contexts
    x1 = torch.empty(max(b.nl), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    same = True
    for i in range(b.n):
        xi = x1[:b.nl[i]]
        _, s1, _ = b.ctx[i].cg_solve(fs[i], tol=TOL, maxit=20000, x=xi, raise_on_noconv=True)
        same &= s1["iters"] == st[i]["iters"] and bool(torch.equal(xi, xb[i]))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    log(f"sequential solo solves: {t_seq * 1e3:.1f} ms, bit-identical {same}")
    chunks, captures = b.counters()
    out = {"problems": b.n, "local_points": sum(b.nl), "orders": b.orders(),
           "GDOF_iter_per_s": round(work / dt / 1e9, 3), "ms_per_solve": round(dt * 1e3, 2),
           "ms_plain_launches": round(res["plain"][0] * 1e3, 2),
           "ms_sequential_solo": round(t_seq * 1e3, 2), "speedup_vs_sequential": round(t_seq / dt, 3),
           "bit_identical_to_solo": same, "max_true_rel_res": max(s["true_rel_res"] for s in st),
           "iters_min_max": [min(s["iters"] for s in st), max(s["iters"] for s in st)],
           "tuned_variant": {str(k): v[0] for k, v in tuned.items()}, "graphs_recorded": captures,
           "setup_s": round(t_setup, 1)}
    for c in b.ctx:
        c.close()
    b.close()
    del fs, xs, xb, x1
    torch.cuda.empty_cache()
    return out


def multi_rhs_case(torch, nek, synth, nrhs=(4, 8), steps=2):
    """Many right-hand sides on the headline mesh (16^3 box, N=9): K problems
    with f ~ U[0,1) seeds 2, 3, ... on one mesh form a batch whose members
    share the set-up data and the persistent grid and run interleaved
    (nek_setup_batch); one batched mixed solve per step, against the K solves
    one after another on a standalone context.  Each member's own solve (on
    its share of the grid) must reproduce its batched x bit for bit."""
    out = {}
    for K in nrhs:
        b = nek.Batch([{"nel": NEL, "N": N}] * K, prec="fp32")
        assert all(b.mesh_of(i) == 0 for i in range(K))
        tuned = b.tune("fp32", iters=10)
        fs = [torch.from_numpy(synth.uniform_load(b.nl[i], SEED + i)).cuda() for i in range(K)]
        xs = [torch.empty(b.nl[i], dtype=torch.float64, device="cuda") for i in range(K)]
        b.solve(fs, tol=TOL, maxit=20000, xs=xs, raise_on_noconv=True)   # warm-up (records the graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st, _ = b.solve(fs, tol=TOL, maxit=20000, xs=xs, raise_on_noconv=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        work = sum(b.nl[i] * st[i]["iters"] for i in range(K))
        x1 = torch.empty(b.nl[0], dtype=torch.float64, device="cuda")
        # bit-identity: each member's own solve (on its share of the grid)
        same = True
        for i in range(K):
            _, s1, _ = b.ctx[i].cg_solve(fs[i], tol=TOL, maxit=20000, x=x1, raise_on_noconv=True)
            same &= s1["iters"] == st[i]["iters"] and bool(torch.equal(x1, xs[i]))
        # baseline: the K solves one after another on a standalone context
        # (full persistent grid, autotuned at its first solve)
        solo = nek.Context(NEL, N, prec="fp32")
        solo.cg_solve(fs[0], tol=TOL, maxit=20000, x=x1, raise_on_noconv=True)   # tunes, warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(K):
            solo.cg_solve(fs[i], tol=TOL, maxit=20000, x=x1, raise_on_noconv=True)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        solo.close()
        out[f"K{K}"] = {"ms_per_batch": round(dt * 1e3, 2), "ms_per_rhs": round(dt * 1e3 / K, 2),
                        "GDOF_iter_per_s": round(work / dt / 1e9, 3), "ms_sequential": round(t_seq * 1e3, 2),
                        "speedup_vs_sequential": round(t_seq / dt, 3), "bit_identical_to_solo": same,
                        "iters": [s["iters"] for s in st], "max_true_rel_res": max(s["true_rel_res"] for s in st),
                        "tuned_variant": tuned[N][0]}
        log(f"multi-rhs K={K}: {out[f'K{K}']}")
        for c in b.ctx:
            c.close()
        b.close()
        del fs, xs, x1
        torch.cuda.empty_cache()
    return out


def learned_case(torch, nsolves=10000, steps=(2500, 10000, 40000), neval=16, data_tol=1e-10, holdout=0.05):
    """Learned initial guess: 10,000 FP64 solves (to 1e-10) on 8^3-element
    N=7 meshes of [0,1]^3 (+-10 % interior vertex moves, 64 distinct meshes)
    forced by Gaussian random fields (length scale 0.2) give 5.12 M element
    rows; the rows of the last 5 % of the solves are held out.  The
    518 -> 256 -> 256 -> 512 network trains on the rest with Adam steps of
    4096 rows on the GPU, continued to each length in `steps`; at each length
    the training loss (mean of the last 50 steps), the held-out loss and the
    evaluation: `neval` fresh 16^3-element N=7 problems solved to 1e-8 by
    FP64 CG from zero and from the network's guess (prediction time
    included)."""
    from paper_2405_11065_amd import learned_x0 as lx
    X, T, info = lx.make_dataset(torch, nsolves, tol=data_tol, log=log)
    rows = X.shape[0]
    per_solve = rows // nsolves
    n_train = (nsolves - int(round(holdout * nsolves))) * per_solve
    Xv, Tv = X[n_train:], T[n_train:]
    from paper_2405_11065_amd import nek, synth
    n3 = T.shape[1]
    net = nek.Mlp(n3 + 6, lx.HIDDEN, n3, synth.mlp_init((n3 + 6, lx.HIDDEN, lx.HIDDEN, n3), synth.SEED_C5))
    sweep, done, t_train, hist_all = [], 0, 0.0, []
    for k, total in enumerate(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = net.train(X, T, n_train, 4096, total - done, lr=1e-3, seed=synth.SEED_C5 + k)
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t0
        done = total
        hist_all.append(hist)
        val, _ = net.loss_grad(Xv, Tv)
        ev = lx.evaluate(torch, net, neval=neval)
        sweep.append({"steps": total, "train_loss": float(hist[-50:].mean()), "heldout_loss": float(val),
                      "train_s": round(t_train, 2),
                      "eval": {kk: v for kk, v in ev.items() if kk != "per_problem"}})
        log(f"learned x0: {total} steps, train loss {sweep[-1]['train_loss']:.4f}, held-out {val:.4f}, "
            f"iters saved {ev['iters_saved_frac']:.3f} / energy {ev['energy_iters_saved_frac']:.3f}")
    net.close()
    del X, T, Xv, Tv
    torch.cuda.empty_cache()
    # GEMM work of one training step: forward 3 products, backward 5 (2 m n k flops each)
    n_in, h, n_out, bsz = 518, lx.HIDDEN, 512, 4096
    fl = 2 * bsz * (n_in * h + h * h + h * n_out) * 3 - 2 * bsz * n_in * h
    first = hist_all[0]
    return {"data": info, "feature_mode": lx.MODE, "train_rows": n_train, "heldout_rows": rows - n_train,
            "batch": bsz, "train_steps": done, "train_s": round(t_train, 2),
            "ms_per_step": round(t_train / done * 1e3, 3), "train_TFLOPs_bf16": round(fl * done / t_train / 1e12, 2),
            "loss_first_last": [float(first[:50].mean()), sweep[-1]["train_loss"]],
            "sweep": sweep, "eval": sweep[-1]["eval"], "eval_per_problem": ev["per_problem"]}


def profile_sequence(torch, nek, synth, variants="", geometry="stored", ne=16, precond="none", schwarz_kernel="auto"):
    """A short sequence for counter collection (few dispatches): 40 mixed and
    40 FP64 CG iterations (BF16-g mixed as well on the deformed mesh), then 5
    nek_ax per precision and a 256 MiB copy for calibration.  ne = 16: the
    16^3 N=9 box; ne = 32: the 32^3 N=9 deformed mesh.  geometry 'trilinear'
    runs it with the factors recomputed in the kernels; precond selects the
    solves' preconditioner (20 iterations each with 'schwarz')."""
    nel = (ne, ne, ne)
    vtx = None
    if ne != 16:
        vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=0.1, seed=synth.SEED_C3_VERTICES)
    ctx = nek.Context(nel, N, vtx=vtx, prec="fp32", precond=precond)
    ctx.set_geometry(geometry)
    ctx.set_schwarz_kernel(schwarz_kernel)
    chosen = dict(kv.split("=") for kv in variants.split(",") if kv)
    for prec in ("fp32", "fp64", "bf16g"):
        if prec in chosen:
            ctx.set_variant(prec, int(chosen[prec]))
        else:
            ctx.tune(prec, iters=10)
    f = torch.from_numpy(synth.uniform_load(ctx.nl, SEED)).cuda()
    x = ctx.new_vector()
    out = {}
    its = 20 if precond == "schwarz" else 40
    for prec in ("fp32", "fp64") + (("bf16g",) if ne != 16 else ()):
        ctx.set_prec(prec)
        _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=its, x=x)
        out[prec] = st["iters"]
    for prec, dt in (("fp64", torch.float64), ("fp32", torch.float32), ("bf16g", torch.float32)):
        ctx.set_prec(prec)
        u = torch.rand(ctx.nl, dtype=dt, device="cuda")
        w = torch.empty_like(u)
        for _ in range(5):
            ctx.ax(u, w)
    # calibration: a plain device copy of 256 MiB (read 256 MiB, write 256 MiB)
    a = torch.empty(1 << 25, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profile_sequence": out, "nel": ne, "local_points": ctx.nl, "geometry": geometry,
                      "precond": precond, "copy_bytes": a.numel() * 8,
                      "variants": {p: ctx.get_variant(p) for p in ("fp32", "fp64", "bf16g")}}), flush=True)
    ctx.close()


def profile_ax(torch, nek, synth, ne, variants=""):
    """nek_ax on the ne^3 deformed mesh of [0,1]^3 (N=9, the 32^3 workload's
    mesh at ne = 32), five calls per precision in the given (else the tuned)
    configuration, then a 256 MiB copy for counter calibration: the sequence
    for hardware-counter runs of the operator and assembly passes."""
    nel = (ne, ne, ne)
    vtx = synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=0.1, seed=synth.SEED_C3_VERTICES)
    ctx = nek.Context(nel, 9, vtx=vtx, prec="fp32")
    chosen = dict(kv.split("=") for kv in variants.split(",") if kv)
    out = {}
    for prec, dt in (("fp32", torch.float32), ("bf16g", torch.float32), ("fp64", torch.float64)):
        ctx.set_prec(prec)
        if prec in chosen:
            ctx.set_variant(prec, int(chosen[prec]))
        else:
            ctx.tune(prec, iters=5)
        u = torch.rand(ctx.nl, dtype=dt, device="cuda")
        w = torch.empty_like(u)
        for _ in range(5):
            ctx.ax(u, w)
        out[prec] = ctx.get_variant(prec)
    a = torch.empty(1 << 25, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profile_ax": {"nel": ne, "local_points": ctx.nl, "variants": out},
                      "copy_bytes": a.numel() * 8}), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-big", action="store_true", help="skip the 32^3 deformed-mesh BF16 measurement")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-problem batched solve and the many-right-hand-side batches")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned initial guess (data, training, eval)")
    ap.add_argument("--no-energy", action="store_true", help="skip the energy-to-solution measurement")
    ap.add_argument("--no-jacobi", action="store_true",
                    help="skip the preconditioner (diagonal, fast diagonalization) and in-kernel geometry measurements")
    ap.add_argument("--geometry", default="stored", choices=("stored", "trilinear"),
                    help="with --profile: stored geometric factors or factors recomputed in the kernels")
    ap.add_argument("--profile", action="store_true",
                    help="short fixed sequence for hardware-counter runs: 40 mixed and 40 FP64 CG iterations, "
                         "5 nek_ax per precision and a 256 MiB copy for calibration")
    ap.add_argument("--profile-ne", type=int, default=16, choices=(16, 32),
                    help="with --profile: the 16^3 box or the 32^3 deformed mesh (N=9)")
    ap.add_argument("--precond", default="none", choices=("none", "jacobi", "fdm", "schwarz"),
                    help="with --profile: preconditioner of the profiled solves")
    ap.add_argument("--schwarz-kernel", default="auto", choices=("auto", "mfma", "valu"),
                    help="with --profile --precond schwarz: kernel of the window solves")
    ap.add_argument("--profile-operators", action="store_true",
                    help="only the plain operator pass with vector-ALU and matrix-core D contractions (16^3 box, "
                         "N + 1 = 8, 10, 12, FP32 and FP64), for kernel traces")
    ap.add_argument("--profile-ax", type=int, default=0, metavar="NE",
                    help="short nek_ax sequence on the NE^3 deformed N=9 mesh (5 calls per precision) and a "
                         "256 MiB copy, for counter runs of the operator and assembly passes")
    ap.add_argument("--variants", default="",
                    help="with --profile or --profile-ax: kernel configurations to use, e.g. fp32=4,fp64=2,bf16g=5 "
                         "(default: run the autotuner)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU (no multi-GPU path); --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2405_11065_amd import nek, synth
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    nek.load()
    torch.cuda.set_device(0)

    if args.profile:
        return profile_sequence(torch, nek, synth, args.variants, args.geometry, args.profile_ne, args.precond,
                                args.schwarz_kernel)
    if args.profile_operators:
        print(json.dumps({"operator_kernels_16x16x16": operator_kernels(torch, nek, synth)}), flush=True)
        return None
    if args.profile_ax:
        return profile_ax(torch, nek, synth, args.profile_ax, args.variants)

    ctx = nek.Context(NEL, N, prec="fp32")
    nl = ctx.nl
    f_host = synth.uniform_load(nl, SEED)
    f = torch.from_numpy(f_host).cuda()
    x = ctx.new_vector()

    def solve():
        _, st, _ = ctx.cg_solve(f, tol=TOL, maxit=20000, x=x, raise_on_noconv=True)
        return st

    # autotuner (part of set-up, untimed): kernel configuration per precision
    log("tuning")
    tuned = {prec: ctx.tune(prec, iters=30) for prec in ("fp32", "fp64", "bf16g")}
    ctx.set_prec("fp32")

    # ---- mixed precision (the timed steps)
    for _ in range(args.warmup):
        solve()
    ctx.prof_read(0, reset=True)
    ctx.prof_read(1, reset=True)
    ctx.prof_enable(16)   # sampled HIP events around both CG kernels, every 16th iteration
    iters = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        st = solve()
        iters += st["iters"]
        stats.append(st)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    ctx.prof_enable(0)
    ax_ms, ax_n = ctx.prof_read(0)
    up_ms, up_n = ctx.prof_read(1)
    value = nl * iters / t_mixed / 1e9
    ms_per_step = t_mixed / args.steps * 1e3

    # ---- FP64 CG on the same input, same protocol
    ctx.set_prec("fp64")
    solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it64 = 0
    for _ in range(args.steps):
        st64 = solve()
        it64 += st64["iters"]
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0

    # ---- the preconditioners on the same solve
    base = {"fp32": (ms_per_step, iters / args.steps), "fp64": (t_fp64 / args.steps * 1e3, it64 / args.steps)}
    jac = None if args.no_jacobi else precond_case(torch, ctx, f, args.steps, base, "jacobi")
    log(f"jacobi: {jac}")
    fdmc = None if args.no_jacobi else precond_case(torch, ctx, f, args.steps, base, "fdm")
    log(f"fdm: {fdmc}")
    asm = None if args.no_jacobi else precond_case(torch, ctx, f, args.steps, base, "schwarz")
    log(f"schwarz: {asm}")
    geo = geometry_case(torch, ctx, f, args.steps, base)
    log(f"trilinear geometry: {geo}")
    # the GPU's fastest FP64 CG: stored or in-kernel factors
    ms64_stored = t_fp64 / args.steps * 1e3
    fast64 = "trilinear" if geo["fp64"]["ms_per_solve"] < ms64_stored else "stored"
    ms64_best = min(ms64_stored, geo["fp64"]["ms_per_solve"])
    refine = refinement_case(torch, nek, f, args.steps, ms_per_step)
    log(f"refinement layouts: {refine}")

    # ---- energy-to-solution, mixed vs FP64 (fastest factor source), same solve
    energy = None if args.no_energy else energy_to_solution(
        torch, ctx, solve, {"fp32": ms_per_step, "fp64": ms64_best}, fast64)
    log(f"energy: {energy}")

    # ---- ax + dssum bandwidth at each precision (nek_ax), and a plain copy beside it
    axd = ax_dssum_all(ctx, torch)
    axd["copy_512MiB"] = copy_bandwidth(torch)
    axd["dssum_seg"] = dssum_seg(ctx, torch)
    log(f"sorted-segment dssum: {axd['dssum_seg']}")

    # ---- secondary: 32^3 deformed mesh, N=9, manufactured forcing, BF16 g vs FP64
    big = None if args.no_big else big_case(torch, nek, synth, energy=not args.no_energy, jacobi=not args.no_jacobi)
    log("32^3 case done")
    batch = None if args.no_batch else batch_case(torch, nek, synth)
    multi = None if args.no_batch else multi_rhs_case(torch, nek, synth)
    opk = None if args.no_jacobi else operator_kernels(torch, nek, synth)
    learned = None if args.no_learned else learned_case(torch)

    bpp = cg_operator_bytes_per_point(4, 4, 8)   # FP32 vectors and g, FP64 inner correction
    ax_avg_s = ax_ms / max(ax_n, 1) / 1e3
    achieved = bpp * nl / ax_avg_s / 1e9 if ax_n else None
    cpu = None if args.no_cpu else cpu_baseline(f_host)

    out = {
        "metric": "CG GDOF*iter/s, mixed FP32/FP64 CG to rel residual 1e-8 (FP64 beside it); ax+dssum HBM GB/s",
        "value": round(value, 3),
        "unit": "GDOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "box 16x16x16 unit-cube hexahedra, N=9, f~U[0,1) seed 2, tol 1e-8 relative",
                   "local_points": nl, "precision": "FP32 operator/dssum/p/r/w, FP64 glsc3/scalars/correction/x/"
                                                    "refinement residual; reliable-update refinement"},
        "mixed": {"iters_per_solve": iters / args.steps, "outer_per_solve": stats[-1]["outer_iters"],
                  "true_rel_res": stats[-1]["true_rel_res"], "last_rec_res": stats[-1]["last_rec_res"],
                  "ms_per_solve": round(ms_per_step, 3), "inner_over_fp64_iters": round(iters / max(it64, 1), 4)},
        "fp64": {"value": round(nl * it64 / t_fp64 / 1e9, 3), "iters_per_solve": it64 / args.steps,
                 "ms_per_solve": round(ms64_stored, 3), "true_rel_res": st64["true_rel_res"],
                 "fastest": fast64, "fastest_ms_per_solve": round(ms64_best, 3)},
        "speedup_vs_fp64": round(ms64_best / ms_per_step, 3),
        "speedup_vs_fp64_stored": round(ms64_stored / ms_per_step, 3),
        "refinement_layouts": refine,
        "tuned_variant": {k: {"best": v[0], "us_per_iter": [round(u, 1) for u in v[1]]} for k, v in tuned.items()},
        "ax_dssum": axd,
        "energy": energy,
        "jacobi": jac,
        "fdm": fdmc,
        "schwarz": asm,
        "geometry_trilinear": geo,
        "roofline": {"bound": "hbm", "kernel": f"k_ax<NP=10,f32,f32,CG,x=f64> variant {tuned['fp32'][0]} "
                                               f"(add2s1 + ax_e + FP64 correction update)",
                     "achieved": round(achieved, 1) if achieved else None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4) if achieved else None,
                     "traffic": counter_traffic(tuned["fp32"][0]), "traffic_unit": "bytes per launch",
                     "algorithmic_bytes_per_launch": bpp * nl,
                     "bytes_per_point": bpp, "avg_us": round(ax_avg_s * 1e6, 2), "sampled_launches": ax_n,
                     "update_kernel_avg_us": round(up_ms / max(up_n, 1) * 1e3, 2)},
        "cpu_baseline": cpu,
        "deformed_32x32x32_N9": big,
        "batch_64": batch,
        "multi_rhs_16x16x16_N9": multi,
        "operator_kernels_16x16x16": opk,
        "learned_x0": learned,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
