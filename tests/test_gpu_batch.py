"""Batched solves (nek_batch_*) through the C ABI.

A batch must compute, for every problem, exactly what nek_cg_solve computes
on a context of the same mesh, order, options and kernel configuration:
x and the statistics are compared bit for bit (the batched kernels run the
solo kernel bodies on each problem's own workgroup range, and every
reduction is per problem in a fixed order).  Converged problems are also
judged by the FP64 oracle's true residual on the batched x (<= tol).
"""
import numpy as np
import pytest

import oracle
from paper_2405_11065_amd import nek, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-8


def _case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    nek.load()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# small mixed-order batch: several problems per order, uneven sizes, some
# deformed, one order with a single problem
SMALL = [((2, 2, 2), 5, 0.0), ((3, 2, 4), 7, 0.1), ((4, 4, 4), 9, 0.0), ((2, 3, 2), 11, 0.1),
         ((5, 4, 3), 5, 0.1), ((3, 3, 3), 7, 0.0), ((2, 2, 5), 9, 0.1), ((3, 2, 2), 11, 0.0),
         ((6, 5, 4), 7, 0.0), ((1, 2, 1), 3, 0.0)]


def specs(items, seed0=40):
    out = []
    for k, (nel, N, pert) in enumerate(items):
        out.append({"nel": nel, "N": N, "vtx": synth.box_vertices(nel, perturb=pert, seed=seed0 + k)})
    return out


def loads(batch, seed=4):
    return [dev(synth.uniform_load(batch.nl[i], synth.batch_load_seed(seed, i))) for i in range(batch.n)]


def solo_solve(spec, prec, f, variant, maxit=20000, x0=None):
    ctx = nek.Context(spec["nel"], spec["N"], vtx=spec["vtx"], prec=prec)
    ctx.set_variant(prec, variant)
    x, st, _ = ctx.cg_solve(f, x0=x0, tol=TOL, maxit=maxit)
    out = host(x)
    ctx.close()
    return out, st


def oracle_rho(spec, f, x):
    P = oracle.Problem(spec["N"], spec["nel"], spec["vtx"])
    return P.true_residual(x, host(f))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16g"])
def test_batch_equals_solo_and_oracle(prec):
    sp = specs(SMALL)
    _case(f"batch of {len(sp)} prec={prec}")
    b = nek.Batch(sp, prec=prec)
    fs = loads(b)
    xs, st, rc = b.solve(fs, tol=TOL, maxit=20000)
    assert rc == nek.NEK_OK, st
    chunks, captures = b.counters()
    print(f"  chunks {chunks} graphs {captures}")
    assert captures >= 1
    for i, spec in enumerate(sp):
        x = host(xs[i])
        v = b.get_variant(prec, i)
        xs_solo, st_solo = solo_solve(spec, prec, fs[i], v)
        rho = oracle_rho(spec, fs[i], x)
        print(f"  [{i}] N={spec['N']} nel={spec['nel']} iters {st[i]['iters']} outer {st[i]['outer_iters']} "
              f"rho* {rho:.2e} solo iters {st_solo['iters']}")
        assert st[i]["status"] == nek.NEK_OK
        assert rho <= TOL
        assert st[i]["iters"] == st_solo["iters"] and st[i]["outer_iters"] == st_solo["outer_iters"]
        assert st[i]["true_rel_res"] == st_solo["true_rel_res"]
        assert st[i]["last_rec_res"] == st_solo["last_rec_res"]
        assert st[i]["true_rel_res"] == pytest.approx(rho, rel=1e-3)
        assert np.array_equal(x, xs_solo), f"problem {i}: batched x differs from the solo solve"
    b.close()


def test_batch_graph_replay_matches_plain_launches():
    sp = specs(SMALL)
    b = nek.Batch(sp, prec="fp32")
    fs = loads(b, seed=9)
    ref, st_ref, _ = b.solve(fs, tol=TOL, maxit=20000, graph=False)
    ref = [host(x) for x in ref]
    _, captures0 = b.counters()
    assert captures0 == 0
    for rep in range(3):   # graph replays with eager work and syncs between them
        _case(f"graph solve {rep}")
        xs, st, _ = b.solve(fs, tol=TOL, maxit=20000, graph=True)
        for i in range(b.n):
            assert st[i]["iters"] == st_ref[i]["iters"]
            assert np.array_equal(host(xs[i]), ref[i]), f"replay {rep} problem {i}"
        scratch = torch.ones(1 << 20, device="cuda", dtype=torch.float64)
        assert float(scratch.sum()) == float(1 << 20)
    b.close()


def test_batch_tuned_variants_bit_exact():
    sp = specs(SMALL[:6], seed0=60)
    b = nek.Batch(sp, prec="fp32")
    res = b.tune("fp32", iters=8)
    print(f"  tuned {res}")
    assert set(res) == {s["N"] for s in sp}
    for N, (best, us) in res.items():
        assert 0 <= best < len(us) and all(t > 0 for t in us)
        assert us[best] == min(us)
    fs = loads(b, seed=11)
    xs, st, rc = b.solve(fs, tol=TOL, maxit=20000)
    assert rc == nek.NEK_OK
    for i, spec in enumerate(sp):
        assert b.get_variant("fp32", i) == res[spec["N"]][0]
        assert b.ctx[i].get_variant("fp32") == res[spec["N"]][0]
        xs_solo, st_solo = solo_solve(spec, "fp32", fs[i], res[spec["N"]][0])
        assert st[i]["iters"] == st_solo["iters"]
        assert np.array_equal(host(xs[i]), xs_solo)
    b.close()


def test_batch_set_variant_and_every_variant_bit_exact():
    sp = specs([((3, 2, 2), 9, 0.1), ((2, 2, 2), 9, 0.0), ((4, 3, 2), 9, 0.0)], seed0=80)
    b = nek.Batch(sp, prec="fp64")
    fs = loads(b, seed=13)
    for v in range(b.ctx[0].num_variants()):
        _case(f"N=9 variant {v}")
        b.set_variant("fp64", 9, v)
        xs, st, rc = b.solve(fs, tol=TOL, maxit=5000)
        assert rc == nek.NEK_OK
        for i, spec in enumerate(sp):
            xs_solo, st_solo = solo_solve(spec, "fp64", fs[i], v)
            assert st[i]["iters"] == st_solo["iters"]
            assert np.array_equal(host(xs[i]), xs_solo)
    with pytest.raises(nek.NekError):
        b.set_variant("fp64", 9, 99)
    with pytest.raises(nek.NekError):
        b.set_variant("fp64", 4, 0)   # no problem of order 4
    b.close()


def test_batch_edge_cases():
    """Zero load, a projected x0, a tiny maxit and a single-element problem in one batch."""
    sp = specs([((2, 2, 2), 7, 0.0), ((3, 3, 2), 7, 0.1), ((1, 1, 1), 5, 0.0), ((4, 2, 3), 9, 0.0)], seed0=90)
    b = nek.Batch(sp, prec="fp32")
    fs = loads(b, seed=17)
    fs[0].zero_()
    x0s = [None, dev(np.random.default_rng(5).random(b.nl[1])), None, None]
    xs, st, rc = b.solve(fs, x0s=x0s, tol=TOL, maxit=20000)
    assert rc == nek.NEK_OK
    assert st[0]["iters"] == 0 and np.all(host(xs[0]) == 0)
    for i in (1, 2, 3):
        xs_solo, st_solo = solo_solve(sp[i], "fp32", fs[i], b.get_variant("fp32", i), x0=x0s[i])
        assert st[i]["iters"] == st_solo["iters"]
        assert np.array_equal(host(xs[i]), xs_solo)
        assert oracle_rho(sp[i], fs[i], host(xs[i])) <= TOL
    # a cap below what the problems need: every problem stops at it, NOCONV
    xs, st, rc = b.solve(loads(b, seed=19), tol=TOL, maxit=7)
    assert rc == nek.NEK_NOCONV
    for i in range(b.n):
        assert st[i]["iters"] <= 7
    b.close()


def test_batch_bad_arguments():
    sp = specs([((2, 2, 2), 5, 0.0)])
    with pytest.raises(nek.NekError):
        nek.Batch([{"nel": (2, 2, 2), "N": 0}])
    with pytest.raises(nek.NekError):
        nek.Batch([{"nel": (2, 2, 2), "N": 5}, {"nel": (0, 2, 2), "N": 5}])
    b = nek.Batch(sp, prec="fp32")
    with pytest.raises(ValueError):
        b.solve([])
    with pytest.raises(nek.NekError):
        b.get_variant("fp32", 3)
    b.close()


def test_full_64_problem_draw_judged_by_oracle():
    """The whole 64-problem draw (n_e ~ U{2..24}, N ~ U{5,7,9,11}, 259 M local
    points), solved as one batch of mixed FP32-operator solves after the
    per-order autotuner: every problem's x is judged by the FP64 oracle's true
    residual (<= tol), one problem at a time."""
    draw = synth.batch_draw(synth.SEED_C4, 64)
    _case("batch setup: full 64-problem draw")
    b = nek.Batch(draw, prec="fp32")
    fs = [dev(synth.uniform_load(b.nl[i], synth.batch_load_seed(synth.SEED_C4, i))) for i in range(b.n)]
    b.tune("fp32", iters=10)
    _case("batch solve: full 64-problem draw")
    xs, st, rc = b.solve(fs, tol=TOL, maxit=20000, raise_on_noconv=True)
    xs = [host(x) for x in xs]
    b.close()
    worst = 0.0
    for i, spec in enumerate(draw):
        f = synth.uniform_load(len(xs[i]), synth.batch_load_seed(synth.SEED_C4, i))
        P = oracle.Problem(spec["N"], spec["nel"], spec.get("vtx", synth.box_vertices(spec["nel"])))
        rho = P.true_residual(xs[i], f)
        worst = max(worst, rho)
        print(f"  [{i}] N={spec['N']} nel={spec['nel']} iters {st[i]['iters']} rho* {rho:.2e}", flush=True)
        assert st[i]["status"] == nek.NEK_OK and rho <= TOL
        del P
    print(f"  worst oracle rho* over the draw {worst:.2e}")


def test_many_right_hand_sides_share_the_mesh():
    """Problems that repeat an earlier problem's mesh and order share its
    set-up data (nek_batch_mesh_of names the owner) and run interleaved on the
    owner's XCDs; every x and statistic is still bit-identical to a solo
    solve on a context of its own, and judged by the oracle."""
    nel, N = (4, 3, 3), 7
    vtx = synth.box_vertices(nel, perturb=0.1, seed=71)
    sp = [{"nel": nel, "N": N, "vtx": vtx},                              # 0: owner
          {"nel": nel, "N": N, "vtx": vtx},                              # 1: same array
          {"nel": nel, "N": N, "vtx": vtx.copy()},                       # 2: same values
          {"nel": nel, "N": N, "vtx": synth.box_vertices(nel, perturb=0.1, seed=72)},   # 3: another mesh
          {"nel": nel, "N": 5, "vtx": vtx},                              # 4: another order
          {"nel": (2, 3, 2), "N": N},                                    # 5: uniform lattice
          {"nel": (2, 3, 2), "N": N},                                    # 6: the same uniform lattice
          {"nel": nel, "N": N, "vtx": vtx}]                              # 7: owner's mesh again
    roots = [0, 0, 0, 3, 4, 5, 5, 0]
    for prec in ("fp64", "fp32", "bf16g"):
        _case(f"many right-hand sides prec={prec}")
        b = nek.Batch(sp, prec=prec)
        assert [b.mesh_of(i) for i in range(b.n)] == roots
        fs = loads(b, seed=23)
        xs, st, rc = b.solve(fs, tol=TOL, maxit=20000)
        assert rc == nek.NEK_OK
        for i, spec in enumerate(sp):
            v = b.get_variant(prec, i)
            if "vtx" not in spec:
                spec = dict(spec, vtx=synth.box_vertices(spec["nel"]))
            xs_solo, st_solo = solo_solve(spec, prec, fs[i], v)
            x = host(xs[i])
            rho = oracle_rho(spec, fs[i], x)
            print(f"  [{i}] shares {roots[i]} iters {st[i]['iters']} outer {st[i]['outer_iters']} rho* {rho:.2e}")
            assert st[i]["iters"] == st_solo["iters"] and st[i]["true_rel_res"] == st_solo["true_rel_res"]
            assert np.array_equal(x, xs_solo), f"problem {i}"
            assert rho <= TOL
        # a sharing member's context works on its own as well
        x1, st1, _ = b.ctx[1].cg_solve(fs[1], tol=TOL, maxit=20000)
        assert np.array_equal(host(x1), host(xs[1])) and st1["iters"] == st[1]["iters"]
        b.close()


def test_many_right_hand_sides_divide_the_grid():
    """Four right-hand sides on a mesh with more element groups than a
    quarter of the solo persistent grid: each problem runs on a quarter of it
    (every workgroup walks several element groups); the batched x equals the
    member context's own solve bit for bit and the oracle's true residual is
    within tol, in every precision."""
    nel, N, K = (10, 10, 9), 5, 4
    vtx = synth.box_vertices(nel, perturb=0.1, seed=73)
    sp = [{"nel": nel, "N": N, "vtx": vtx}] * K
    for prec in ("fp64", "fp32", "bf16g"):
        _case(f"{K} right-hand sides on 10x10x9 N=5, prec={prec}")
        b = nek.Batch(sp, prec=prec)
        assert [b.mesh_of(i) for i in range(K)] == [0] * K
        fs = loads(b, seed=29)
        xs, st, rc = b.solve(fs, tol=TOL, maxit=20000)
        assert rc == nek.NEK_OK
        for i in range(K):
            x = host(xs[i])
            xi, sti, _ = b.ctx[i].cg_solve(fs[i], tol=TOL, maxit=20000)
            rho = oracle_rho(sp[i], fs[i], x)
            print(f"  [{i}] iters {st[i]['iters']} outer {st[i]['outer_iters']} rho* {rho:.2e}")
            assert np.array_equal(x, host(xi)) and sti["iters"] == st[i]["iters"]
            assert rho <= TOL
        b.close()
