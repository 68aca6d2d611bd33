"""Pins of the oracle's precision-emulation harness (oracle/nek_vprec.c).

The harness re-runs the oracle's init and Table-1 CG with every FP operation
passed through a rounding / Monte Carlo hook (the paper's accuracy-check
method, Sect. 4).  It is pinned by:
  * the rounding hook against independent definitions: NumPy's binary32 and
    binary16 casts (round to nearest even) and exact rational rounding for a
    7-bit mantissa (bfloat16), ties included;
  * the random-rounding hook against its distribution: zero mean, standard
    deviation 2^(e-t)/sqrt(12), bounded by half a unit in the t-th place;
  * the whole pipeline with the hook off (and at t = 52) against the plain
    oracle, bit for bit: geometric factors, residual history and solution.
"""
import math
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from paper_2405_11065_amd import synth  # noqa: E402


def _values(n, seed, lo=-30, hi=30):
    rng = np.random.default_rng(seed)
    mant = rng.uniform(1.0, 2.0, n) * rng.choice([-1.0, 1.0], n)
    return mant * np.exp2(rng.integers(lo, hi, n).astype(float))


def test_round_23_bits_is_binary32():
    for v in _values(20000, 1):
        assert oracle.vp_round(v, 23) == float(np.float32(v))


def test_round_10_bits_is_binary16():
    for v in _values(20000, 2, lo=-10, hi=14):   # binary16 normal range
        assert oracle.vp_round(v, 10) == float(np.float16(v))


def _rne_exact(v, t):
    """v rounded to t explicit mantissa bits with exact rational arithmetic."""
    q = Fraction(v)
    if q == 0:
        return 0.0
    e = math.floor(math.log2(abs(v))) + 1          # |v| in [2^(e-1), 2^e)
    ulp = Fraction(2) ** (e - 1 - t)
    return float(round(q / ulp) * ulp)             # round(): nearest, ties to even


def test_round_7_bits_is_bfloat16_rne():
    vals = list(_values(3000, 3))
    # exact ties: 1 + 2^-8 -> 1 (even), 1 + 3*2^-8 -> 1 + 2^-6 (even), and a carry into the exponent
    vals += [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 2 - 2.0 ** -8, 3.0 * 2.0 ** -20 * (1 + 2.0 ** -8)]
    for v in vals:
        assert oracle.vp_round(v, 7) == _rne_exact(v, 7), v
    assert oracle.vp_round(1 + 2.0 ** -8, 7) == 1.0
    assert oracle.vp_round(1 + 3 * 2.0 ** -8, 7) == 1 + 2.0 ** -6
    assert oracle.vp_round(2 - 2.0 ** -8, 7) == 2.0


def test_round_passes_full_precision_and_specials():
    for v in _values(100, 4):
        assert oracle.vp_round(v, 52) == v
    assert oracle.vp_round(0.0, 10) == 0.0
    assert math.isinf(oracle.vp_round(math.inf, 10))


def test_random_rounding_distribution():
    # the stream is seeded by the last vp_cg call; a tiny run fixes it
    oracle.vprec_cg(1, (1, 1, 1), synth.box_vertices((1, 1, 1)), np.ones(8), maxit=1, seed=123)
    x, t = 1.0 / 3.0, 10                    # frexp exponent of 1/3 is -1
    scale = 2.0 ** (-1 - t)
    d = np.array([oracle.vp_perturb(x, t) - x for _ in range(40000)])
    assert np.all(np.abs(d) <= scale / 2)
    assert abs(d.mean()) < 4 * scale / math.sqrt(12) / math.sqrt(d.size)
    assert d.std() == pytest.approx(scale / math.sqrt(12), rel=0.02)
    assert oracle.vp_perturb(x, 52) == x and oracle.vp_perturb(0.0, 10) == 0.0


@pytest.mark.parametrize("nel,N,perturb", [((2, 2, 2), 4, 0.1), ((3, 2, 2), 5, 0.1), ((4, 4, 4), 7, 0.0)])
def test_hook_off_is_the_oracle_bit_for_bit(nel, N, perturb):
    vtx = synth.box_vertices(nel, perturb=perturb, seed=11)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 3)
    x0, it0, h0 = P.cg(f, tol=0.0, maxit=40)
    x1, it1, h1, g1 = oracle.vprec_cg(N, nel, vtx, f, mode="ieee", maxit=40, want_g=True)
    assert it1 == it0 and np.array_equal(g1, P.g) and np.array_equal(h1, h0) and np.array_equal(x1, x0)
    for mode in ("rne", "rr", "mca"):   # t = 52 leaves every value alone in every mode
        x2, it2, h2 = oracle.vprec_cg(N, nel, vtx, f, mode=mode, t=(52, 52, 52, 52), maxit=40, seed=5)
        assert np.array_equal(x2, x0) and np.array_equal(h2, h0)


def test_tolerance_stop_matches_oracle():
    nel, N = (2, 2, 2), 5
    vtx = synth.box_vertices(nel, perturb=0.1, seed=2)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 4)
    x0, it0, h0 = P.cg(f, tol=1e-8, maxit=500)
    x1, it1, h1 = oracle.vprec_cg(N, nel, vtx, f, tol=1e-8, maxit=500)
    assert it1 == it0 and np.array_equal(x1, x0)


def test_monte_carlo_samples_reproducible_and_distinct():
    nel, N = (2, 2, 2), 4
    vtx = synth.box_vertices(nel, perturb=0.1, seed=3)
    f = synth.uniform_load(2 * 2 * 2 * 125, 5)
    a = oracle.vprec_cg(N, nel, vtx, f, t=(23, 23, 23, 23), mode="rr", seed=7, maxit=20)[0]
    b = oracle.vprec_cg(N, nel, vtx, f, t=(23, 23, 23, 23), mode="rr", seed=7, maxit=20)[0]
    c = oracle.vprec_cg(N, nel, vtx, f, t=(23, 23, 23, 23), mode="rr", seed=8, maxit=20)[0]
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    # a t-bit perturbation moves x by about 2^-t relative, not more than a few orders above
    assert np.linalg.norm(a - c) / np.linalg.norm(a) < 1e-4


def test_rounding_only_the_cg_regions_keeps_init_exact():
    nel, N = (2, 2, 2), 4
    vtx = synth.box_vertices(nel, perturb=0.1, seed=3)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 5)
    _, _, _, g = oracle.vprec_cg(N, nel, vtx, f, t=(52, 10, 10, 10), mode="rne", maxit=5, want_g=True)
    assert np.array_equal(g, P.g)
    _, _, _, g = oracle.vprec_cg(N, nel, vtx, f, t=(10, 52, 52, 52), mode="rne", maxit=5, want_g=True)
    assert not np.array_equal(g, P.g)
    assert np.max(np.abs(g - P.g)) <= 2.0 ** -8 * np.max(np.abs(P.g))


def test_hook_off_preconditioned_is_or_pcg_bit_for_bit():
    nel, N = (3, 2, 2), 5
    vtx = synth.box_vertices(nel, perturb=0.1, seed=12)
    P = oracle.Problem(N, nel, vtx)
    f = synth.uniform_load(P.nl, 6)
    m = P.diag()
    x0, it0, h0 = P.pcg(f, m, tol=0.0, maxit=40)
    x1, it1, h1 = oracle.vprec_cg(N, nel, vtx, f, mode="ieee", maxit=40, m=m)
    assert it1 == it0 and np.array_equal(x1, x0) and np.array_equal(h1, h0)
    x2, it2, h2 = oracle.vprec_cg(N, nel, vtx, f, mode="rne", t=(52, 52, 52, 52), maxit=40, m=m)
    assert np.array_equal(x2, x0)
