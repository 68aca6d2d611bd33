"""Learned initial guess for the CG solve: data, training and evaluation.

Every step runs in libnek (include/nek_mlp.h and include/nek.h); this module
only sequences the calls and holds device buffers.

  * Data: `nsolves` Poisson problems on order-N meshes of nel elements on
    [0,1]^3 (interior vertices moved up to +-10 % of an element, `nmesh`
    distinct meshes used in turn), each forced by its own Gaussian random field
    (squared-exponential covariance, length scale 0.2, random Fourier features
    drawn with a per-problem seed, f = B o F), solved in FP64 to a relative
    residual of 1e-8 by batched CG.  Each element of each solve gives one
    training row: inputs from nek_x0_features, targets from nek_x0_targets.
  * Training: Adam on minibatches (nek_mlp_train).
  * Evaluation: problems on a larger mesh solved by CG from zero and from the
    network's guess (nek_x0_predict), both to the same tolerance; the guess's
    cost (prediction) is counted in its time.
"""
from __future__ import annotations

import time

import numpy as np

from . import nek, synth

KAPPA = 1.0 / (3.0 * np.pi ** 2)   # u / F of the lowest Dirichlet mode of the unit cube
HIDDEN = 256
MODE = 2   # feature mode of nek_x0_features


def draw_seed(seed: int, i: int) -> int:
    return int(seed) * 1000003 + int(i)


def mesh_spec(nel, N, k, seed):
    return {"nel": tuple(nel), "N": int(N), "hi": (1.0, 1.0, 1.0),
            "vtx": synth.box_vertices(nel, hi=(1.0, 1.0, 1.0), perturb=0.1, seed=draw_seed(seed, 500000 + k))}


def make_dataset(torch, nsolves, nel=(8, 8, 8), N=7, nmesh=64, seed=synth.SEED_C5, length=0.2, features=256,
                 tol=1e-8, log=None, mode=MODE):
    """(X bfloat16 [rows, ld_in], T float32 [rows, n3], info) from nsolves FP64 solves."""
    nmesh = min(nmesh, nsolves)
    batch = nek.Batch([mesh_spec(nel, N, k, seed) for k in range(nmesh)], prec="fp64")
    E, n3 = batch.ctx[0].E, (N + 1) ** 3
    ld_in = (n3 + 6 + 7) // 8 * 8
    X = torch.zeros((nsolves * E, ld_in), dtype=torch.bfloat16, device="cuda")
    T = torch.zeros((nsolves * E, n3), dtype=torch.float32, device="cuda")
    s = torch.empty(E, dtype=torch.float64, device="cuda")
    fs = [batch.ctx[k].new_vector() for k in range(nmesh)]
    xs = [batch.ctx[k].new_vector() for k in range(nmesh)]
    iters, t_solve = 0, 0.0
    t0 = time.perf_counter()
    for r0 in range(0, nsolves, nmesh):
        m = min(nmesh, nsolves - r0)
        for k in range(m):
            nek.grf(batch.ctx[k], synth.FourierFieldDraw(draw_seed(seed, r0 + k), length, features), out=fs[k])
        if m < nmesh:   # idle members solve a zero load (0 iterations)
            for k in range(m, nmesh):
                fs[k].zero_()
        ts = time.perf_counter()
        _, st, _ = batch.solve(fs, tol=tol, maxit=20000, xs=xs, raise_on_noconv=True)
        t_solve += time.perf_counter() - ts
        iters += sum(st[k]["iters"] for k in range(m))
        for k in range(m):
            row = (r0 + k) * E
            nek.x0_features(batch.ctx[k], fs[k], X=X[row:row + E], s=s, mode=mode)
            nek.x0_targets(batch.ctx[k], xs[k], s, KAPPA, T=T[row:row + E])
        if log and (r0 // nmesh) % 20 == 0:
            log(f"data: {r0 + m}/{nsolves} solves")
    torch.cuda.synchronize()
    info = {"solves": nsolves, "rows": nsolves * E, "mesh": f"{nel[0]}x{nel[1]}x{nel[2]} N={N}",
            "distinct_meshes": nmesh, "mean_iters": iters / nsolves, "t_data_s": round(time.perf_counter() - t0, 2),
            "t_solve_s": round(t_solve, 2)}
    for c in batch.ctx:
        c.close()
    batch.close()
    return X, T, info


def train(torch, X, T, steps, batch=4096, lr=1e-3, seed=synth.SEED_C5, n3=512):
    net = nek.Mlp(n3 + 6, HIDDEN, n3, synth.mlp_init((n3 + 6, HIDDEN, HIDDEN, n3), seed))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = net.train(X, T, X.shape[0], batch, steps, lr=lr, seed=seed)
    dt = time.perf_counter() - t0
    return net, hist, dt


def evaluate(torch, net, neval=4, nel=(16, 16, 16), N=7, seed=synth.SEED_C5, length=0.2, features=256, tol=1e-8,
             prec="fp64", check=None, mode=MODE):
    """CG from zero vs from the learned guess on neval fresh forcings.

    check(ctx, f, x) may verify each solution (e.g. with the oracle)."""
    spec = mesh_spec(nel, N, 999, seed)
    ctx = nek.Context(spec["nel"], N, vtx=spec["vtx"], hi=spec["hi"], prec=prec)
    ctx.tune(prec, iters=10)
    f, x, x0 = ctx.new_vector(), ctx.new_vector(), ctx.new_vector()
    rows = []
    for k in range(neval):
        nek.grf(ctx, synth.FourierFieldDraw(draw_seed(seed + 1, k), length, features), out=f)
        torch.cuda.synchronize()
        ctx.cg_solve(f, tol=tol, maxit=20000, x=x)     # warm-up of this load
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st0, _ = ctx.cg_solve(f, tol=tol, maxit=20000, x=x, raise_on_noconv=True)
        t_zero = time.perf_counter() - t0
        if check:
            check(ctx, f, x)
        row = {"iters_zero": st0["iters"], "ms_zero": round(t_zero * 1e3, 2)}
        for tag, policy in (("", nek.NEK_X0_RESIDUAL), ("energy_", nek.NEK_X0_ENERGY)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, alpha, rho0, used = nek.x0_predict(ctx, net, f, KAPPA, x0=x0, policy=policy, mode=mode)
            t_pred = time.perf_counter() - t0
            _, st1, _ = ctx.cg_solve(f, x0=x0, tol=tol, maxit=20000, x=x, raise_on_noconv=True)
            t_x0 = time.perf_counter() - t0
            if check:
                check(ctx, f, x)
            row.update({f"{tag}iters_x0": st1["iters"], f"{tag}ms_x0_incl_predict": round(t_x0 * 1e3, 2),
                        f"{tag}used": used})
        row.update({"ms_predict": round(t_pred * 1e3, 2), "alpha": alpha, "rho0": rho0})
        rows.append(row)
    ctx.close()
    it0 = sum(r["iters_zero"] for r in rows)
    t0s = sum(r["ms_zero"] for r in rows)
    out = {"mesh": f"{nel[0]}x{nel[1]}x{nel[2]} N={N}", "prec": prec, "problems": neval,
           "mean_rho0": float(np.mean([r["rho0"] for r in rows]))}
    for tag in ("", "energy_"):
        it1 = sum(r[f"{tag}iters_x0"] for r in rows)
        t1s = sum(r[f"{tag}ms_x0_incl_predict"] for r in rows)
        out[f"{tag}iters_saved_frac"] = round(1.0 - it1 / it0, 4)
        out[f"{tag}time_saved_frac"] = round(1.0 - t1s / t0s, 4)
        out[f"{tag}used"] = sum(r[f"{tag}used"] for r in rows)
    out["per_problem"] = rows
    return out
