"""Precision-sensitivity study of the CG solve with the oracle's emulation harness.

    python -m oracle.precision_study [--samples 20] [--procs 8]

Reproduces, on the 4^3-element N=7 box (f ~ U[0,1), PCG64 seed 1, 100 fixed
CG iterations, the iteration count Nekbone runs by default), the two
experiments of the paper's Sect. 4:
  1. a variable-precision sweep: every FP operation rounded to t mantissa
     bits, t from 3 to 52, either in the whole program (initialisation and CG)
     or in the CG loop only; reported are the recursive residual after the
     last iteration (the quantity the paper plots), the true FP64 residual of
     the returned x and its distance to the FP64 solution;
  2. Monte Carlo arithmetic at t = 23: random rounding of results ('rr') and
     perturbation of operands and results ('mca'), `samples` runs each, whole
     program vs CG only; reported are the spread (min / mean / max) of the
     final recursive residual and the significant bits of x,
     s = -log2(sigma / |mu|) per entry, averaged.
Then, to the 1e-8 stopping tolerance of the solver, it compares the paper's
layout (the whole CG loop in 23-bit precision) with the one the GPU path
uses inside its FP64 refinement (operator, dssum and vectors in 23 bits;
dot products and scalars in FP64), without and with the diagonal (Jacobi)
preconditioner.

TEST INFRASTRUCTURE / ANALYSIS ONLY: it calls the oracle and the seeded input
generators, nothing of the GPU path.  Output: one JSON object on stdout.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

NEL, N, MAXIT = (4, 4, 4), 7, 100
SCOPES = {"whole": (1, 1, 1, 1), "cg_only": (0, 1, 1, 1)}


def _problem():
    import oracle
    from paper_2405_11065_amd import synth
    vtx = synth.box_vertices(NEL)
    P = oracle.Problem(N, NEL, vtx)
    return P, vtx, synth.uniform_load(P.nl, synth.SEED_C1)


def _bits(scope, t):
    return tuple(t if on else 52 for on in SCOPES[scope])


def _run(args):
    scope, t, mode, seed, tol, maxit = args
    import oracle
    P, vtx, f = _problem()
    x, it, h = oracle.vprec_cg(N, NEL, vtx, f, t=_bits(scope, t), mode=mode, seed=seed, tol=tol, maxit=maxit)[:3]
    if it < 0:
        return {"scope": scope, "t": t, "mode": mode, "seed": seed, "status": it}
    return {"scope": scope, "t": t, "mode": mode, "seed": seed, "iters": it, "rec_res": float(h[-1]),
            "true_res": float(P.true_residual(x, f)), "x": x}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=20)
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    P, vtx, f = _problem()
    x64, _, h64 = P.cg(f, tol=0.0, maxit=MAXIT)
    nx = np.linalg.norm(x64)
    out = {"workload": "box 4x4x4 unit cubes, N=7, f~U[0,1) seed 1, 100 fixed CG iterations",
           "fp64": {"rec_res": float(h64[-1]), "true_res": float(P.true_residual(x64, f))}}
    with mp.get_context("fork").Pool(args.procs) as pool:
        ts = [3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 18, 20, 23, 26, 30, 40, 52]
        jobs = [(s, t, "rne", 0, 0.0, MAXIT) for s in SCOPES for t in ts]
        sweep = {s: [] for s in SCOPES}
        for r in pool.map(_run, jobs):
            row = {"t": r["t"]}
            if "status" in r:
                row["status"] = r["status"]
            else:
                row.update(rec_res=r["rec_res"], true_res=r["true_res"],
                           rel_dx=float(np.linalg.norm(r["x"] - x64) / nx))
            sweep[r["scope"]].append(row)
        out["vprec_sweep"] = sweep

        mca = {}
        jobs = [(s, 23, m, 1000 + k, 0.0, MAXIT) for s in SCOPES for m in ("rr", "mca") for k in range(args.samples)]
        res = pool.map(_run, jobs)
        for s in SCOPES:
            for m in ("rr", "mca"):
                rs = [r for r in res if r["scope"] == s and r["mode"] == m and "x" in r]
                rec = np.array([r["rec_res"] for r in rs])
                tru = np.array([r["true_res"] for r in rs])
                X = np.stack([r["x"] for r in rs])
                mu, sd = X.mean(0), X.std(0, ddof=1)
                keep = mu != 0
                sig = np.minimum(52.0, -np.log2(np.maximum(sd[keep], 1e-300) / np.abs(mu[keep])))
                mca[f"{s}/{m}"] = {"samples": len(rs), "rec_res_min_mean_max": [rec.min(), rec.mean(), rec.max()],
                                   "true_res_min_mean_max": [tru.min(), tru.mean(), tru.max()],
                                   "sig_bits_x_mean": float(sig.mean()), "sig_bits_x_min": float(sig.min())}
        out["mca_t23"] = mca

        layouts = {"paper_cg_loop_single": (52, 23, 23, 23), "gpu_inner_layout": (52, 23, 23, 52)}
        lay = {}
        import oracle
        for name, bits in layouts.items():
            x, it, h = oracle.vprec_cg(N, NEL, vtx, f, t=bits, mode="rne", tol=1e-8, maxit=3000)[:3]
            lay[name] = {"t_init_op_vec_dot": bits, "iters": int(it), "rec_res": float(h[-1]) if it >= 0 else None,
                         "true_res": float(P.true_residual(x, f)) if it >= 0 else None}
        x, it, h = P.cg(f, tol=1e-8, maxit=3000)
        lay["fp64"] = {"iters": int(it), "rec_res": float(h[-1]), "true_res": float(P.true_residual(x, f))}
        # the same with the diagonal (Jacobi) preconditioner, solveM z = r / m
        m = P.diag()
        for name, bits in layouts.items():
            x, it, h = oracle.vprec_cg(N, NEL, vtx, f, t=bits, mode="rne", tol=1e-8, maxit=3000, m=m)[:3]
            lay[name + "_jacobi"] = {"t_init_op_vec_dot": bits, "iters": int(it),
                                     "rec_res": float(h[-1]) if it >= 0 else None,
                                     "true_res": float(P.true_residual(x, f)) if it >= 0 else None}
        x, it, h = P.pcg(f, m, tol=1e-8, maxit=3000)
        lay["fp64_jacobi"] = {"iters": int(it), "rec_res": float(h[-1]), "true_res": float(P.true_residual(x, f))}
        out["to_tol_1e-8"] = lay
    print(json.dumps(out, default=float))


if __name__ == "__main__":
    main()
