"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact everywhere: sorted subset sums (EXPAND), candidate pattern sets on
identical (w, t_lo, t_hi), and final factorisations (which are unique).
"""
import json
import os
import random
import sys

import numpy as np
import pytest

from oracle import rfr_ref as O
import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
MASK = (1 << 64) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_15880_amd as R
    R.lib()
    return R


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


def planted_weights(rng, n, k_rel=2):
    """Random 64-bit weights with a few exact relations planted (so the window is hit)."""
    w = [rng.getrandbits(64) for _ in range(n)]
    for _ in range(k_rel):
        if n < 4:
            break
        idx = rng.sample(range(n - 1), min(n - 1, rng.randint(2, 6)))
        tot = sum(w[i] for i in idx[:-1])
        w[idx[-1]] = (-tot - rng.randint(0, n)) & MASK
    return w


# ------------------------------------------------------------------ EXPAND


@pytest.mark.parametrize("m", [1, 3, 7, 8, 9, 12, 15, 19, 22, 24])
@pytest.mark.parametrize("negate", [False, True])
def test_expand_matches_sorted_subset_sums(R, m, negate):
    rng = random.Random(100 + m)
    w = [rng.getrandbits(64) for _ in range(m)]
    say("expand m=%d negate=%d" % (m, negate))
    got = R.expand_dev(w, negate=negate)
    want = O.expand(w, negate=negate)
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def test_expand_duplicate_heavy(R):
    # many equal keys (zero and repeated weights) stay within one sub-bucket
    w = [0, 0, 5, 5, 1 << 63, 7, (1 << 64) - 7, 3, 3, 3, 11]
    say("expand duplicates")
    assert np.array_equal(R.expand_dev(w), O.expand(w))


@pytest.mark.parametrize("m", [12, 14, 16])
def test_expand_too_clustered_is_reported(R, m):
    # 2^m equal sums exceed the final in-LDS sort (2048 keys per sub-bucket):
    # an error, never a partly sorted output
    say("expand zeros m=%d" % m)
    with pytest.raises(R.RFRError) as e:
        R.expand_dev([0] * m)
    assert e.value.name == "RFR_EOVERFLOW"


# ------------------------------------------------------------------ search


@pytest.mark.parametrize("n", [2, 3, 4, 6, 9, 12, 17, 18, 23, 26])
def test_search_matches_bruteforce(R, n):
    rng = random.Random(n)
    w = planted_weights(rng, n)
    for t_lo, t_hi in [(0, 0), (n + 5, 3), (1 << 20, 1 << 18)]:
        say("search n=%d window=(%d,%d)" % (n, t_lo, t_hi))
        got = R.recombine_dev(w, t_lo, t_hi, cap=1 << 16)
        want = O.search_brute(w, t_lo, t_hi)
        assert got == want


@pytest.mark.parametrize("n", [30, 33, 38, 49])
def test_search_matches_hs_oracle(R, n):
    rng = random.Random(1000 + n)
    w = planted_weights(rng, n, k_rel=4)
    t_lo, t_hi = n + 7, 5
    say("search-hs n=%d" % n)
    got = R.recombine_dev(w, t_lo, t_hi, cap=1 << 12)
    want = O.search_hs(w, t_lo, t_hi)
    assert got == want


def test_search_closed_forms(R):
    n = 12
    say("closed form: zero weights")
    assert R.recombine_dev([0] * n, 0, 0, cap=4096) == list(range(1, 1 << (n - 1)))
    rng = random.Random(5)
    w = [rng.getrandbits(64) for _ in range(n)]
    w[1] = (-w[0]) & MASK
    say("closed form: w0 = -w1")
    assert R.recombine_dev(w, 0, 0) == [0b11]
    say("closed form: powers of two")
    assert R.recombine_dev([1 << i for i in range(n)], 0, 0) == []


def test_search_window_wraps_and_edges(R):
    # keys straddling 0 / 2^64 and sub-bucket edges
    for n in (10, 25, 31):
        rng = random.Random(77 + n)
        w = [rng.getrandbits(64) for _ in range(n)]
        w[0] = (MASK - 2)           # pattern {0} sums to -3
        w[2] = 4                    # pattern {2} sums to +4
        w[3] = (1 << 63) - 1
        w[4] = (1 << 63) + 3        # {3,4} sums to +2
        say("wrap n=%d" % n)
        for t_lo, t_hi in [(3, 4), (2, 3), (100, 100)]:
            assert R.recombine_dev(w, t_lo, t_hi, cap=1 << 12) == O.search_hs(w, t_lo, t_hi)


def test_search_capacity_overflow_reported(R):
    say("overflow")
    with pytest.raises(R.RFRError) as e:
        R.recombine_dev([0] * 14, 0, 0, cap=100)
    assert e.value.name == "RFR_ECANDIDATES"


# ------------------------------------------------------------------ Algorithm E (query design)


@pytest.mark.parametrize("n", [3, 4, 6, 9, 12, 17, 23, 26])
def test_query_design_matches_bruteforce(R, n):
    # Section 3.5: B' expanded, sorted and laid out as the splat table, every
    # A sum generated and queried -- the same pattern set as Algorithm A
    rng = random.Random(300 + n)
    w = planted_weights(rng, n)
    for t_lo, t_hi in [(0, 0), (n + 5, 3), (1 << 20, 1 << 18)]:
        say("query design n=%d window=(%d,%d)" % (n, t_lo, t_hi))
        got = R.recombine_e_dev(w, t_lo, t_hi, cap=1 << 16)
        assert got == O.search_brute(w, t_lo, t_hi)


@pytest.mark.parametrize("n", [30, 33, 38, 45])
def test_query_design_matches_hs_oracle_and_hs_kernels(R, n):
    rng = random.Random(2000 + n)
    w = planted_weights(rng, n, k_rel=4)
    t_lo, t_hi = n + 7, 5
    say("query design n=%d" % n)
    got = R.recombine_e_dev(w, t_lo, t_hi, cap=1 << 12)
    assert got == R.recombine_dev(w, t_lo, t_hi, cap=1 << 12)
    if n <= 38:
        assert got == O.search_hs(w, t_lo, t_hi)


def test_query_design_wraps_and_closed_forms(R):
    for n in (10, 25, 31):
        rng = random.Random(77 + n)
        w = [rng.getrandbits(64) for _ in range(n)]
        w[0] = (MASK - 2)           # pattern {0} sums to -3
        w[2] = 4                    # pattern {2} sums to +4
        w[3] = (1 << 63) - 1
        w[4] = (1 << 63) + 3        # {3,4} sums to +2
        w[n - 2] = MASK             # a B' value at the top of the table
        say("query design wrap n=%d" % n)
        for t_lo, t_hi in [(3, 4), (2, 3), (100, 100)]:
            assert R.recombine_e_dev(w, t_lo, t_hi, cap=1 << 12) == O.search_hs(w, t_lo, t_hi)
    n = 12
    assert R.recombine_e_dev([0] * n, 0, 0, cap=4096) == list(range(1, 1 << (n - 1)))
    rng = random.Random(5)
    w = [rng.getrandbits(64) for _ in range(n)]
    w[1] = (-w[0]) & MASK
    assert R.recombine_e_dev(w, 0, 0) == [0b11]
    assert R.recombine_e_dev([1 << i for i in range(n)], 0, 0) == []
    # B' sums too clustered for the expansion's sort: reported, not searched
    assert R.recombine_e_dev([0] * 30, 0, 0, cap=1 << 10) is None
    with pytest.raises(R.RFRError) as e:
        R.recombine_e_dev([0] * 14, 0, 0, cap=100)
    assert e.value.name == "RFR_ECANDIDATES"


# ------------------------------------------------------------------ end to end


def test_textbook_and_errors(R, ctx):
    cases = [[6, -5, 1], [-1, 0, 0, 0, 0, 0, 1], [0, -1, 0, 1], [0, 6, 6, -36], [1, 0, -10, 0, 1],
             [-2, 0, 1], [-1, 0, 2], [3, 7], [5, 3, 7]]
    for c in cases:
        say("factor", c)
        assert ctx.factor(c) == O.factor(c)
    p = [1]
    for k in range(1, 9):
        p = O.poly_mul_exact(p, [-k, 1])
    assert ctx.factor(p) == O.factor(p)
    # not square-free: factored through the square-free parts
    assert ctx.factor([1, -2, 1]) == (1, [(-1, 1), (-1, 1)])
    assert ctx.factor([0, 0, 1]) == (1, [(0, 1), (0, 1)])
    for bad, name in [([5], "RFR_EINVAL"), ([1, 2, 0], "RFR_EINVAL")]:
        with pytest.raises(R.RFRError) as e:
            ctx.factor(bad)
        assert e.value.name == name


def test_repeated_factors_match_oracle(ctx):
    # Section 2: a polynomial with repeated factors is split by Yun's
    # algorithm and each square-free part is factored
    for w in W.config_repeated(24):
        say("repeated", w.seed, w.degree)
        assert ctx.factor(w.coeffs) == O.factor_general(w.coeffs), w.seed
    # a repeated part large enough to need the device search: (f g)^2 with
    # f, g of degree 20 (square-free part of degree 40, n about 20)
    f, g = W.rand_poly(W._rng(7001), 20, -100, 100), W.rand_poly(W._rng(7002), 20, -100, 100)
    p = O.poly_mul_exact(O.poly_mul_exact(f, g), O.poly_mul_exact(f, g))
    say("repeated degree", len(p) - 1)
    assert ctx.factor(p) == O.factor_general(p)


def test_config_small_exact(ctx):
    w = W.config_small()
    say("config small")
    assert ctx.factor(w.coeffs) == O.factor(w.coeffs)


def test_config_mid_exact_vs_golden(ctx):
    g = json.load(open(os.path.join(HERE, "golden", "golden_mid.json")))["cases"]
    for w in W.config_mid():
        say("config mid seed", w.seed)
        e = g[str(w.seed)]
        assert w.coeffs == e["coeffs"]
        assert ctx.factor(w.coeffs) == (e["content"], [tuple(f) for f in e["factors"]])


def test_config_large_exact_vs_golden(ctx):
    g = json.load(open(os.path.join(HERE, "golden", "golden_large.json")))["cases"]
    for w in W.config_large():
        say("config large seed", w.seed)
        e = g[str(w.seed)]
        r = ctx.factor_full(w.coeffs)
        assert (r["content"], r["factors"]) == (e["content"], [tuple(f) for f in e["factors"]])
        say("  n=%d candidates=%d confirmed=%d window=(%d,%d) ms roots/search/confirm %.1f/%.1f/%.1f" % (
            r["n"], r["n_candidates"], r["n_confirmed"], r["t_lo"], r["t_hi"], r["ms_roots"],
            r["ms_search"], r["ms_confirm"]))


def test_repeat_runs_identical(R):
    # identical candidate sets across repeated launches (race check)
    rng = random.Random(9)
    w = planted_weights(rng, 34, k_rel=6)
    say("repeat n=34")
    first = R.recombine_dev(w, 40, 6)
    for _ in range(3):
        assert R.recombine_dev(w, 40, 6) == first


# ------------------------------------------------------------------ chunked half A


@pytest.mark.parametrize("n,frac", [(14, 0.6), (26, 0.5), (31, 0.3), (34, 0.0), (38, 0.45)])
def test_chunked_search_matches_oracle(R, n, frac):
    # a workspace between the minimum and the full one: half A is streamed in
    # 2^c chunks against the resident B' half
    rng = random.Random(500 + n)
    w = planted_weights(rng, n, k_rel=5)
    L = R.lib()
    full = L.rfr_recombine_workspace_bytes(n)
    mn = L.rfr_recombine_min_workspace_bytes(n)
    ws = int(mn + frac * (full - mn))
    assert mn <= ws < full
    t_lo, t_hi = n + 9, 6
    say("chunked n=%d ws=%d of %d" % (n, ws, full))
    got = R.recombine_dev(w, t_lo, t_hi, cap=1 << 12, ws_bytes=ws)
    want = O.search_brute(w, t_lo, t_hi) if n <= 26 else O.search_hs(w, t_lo, t_hi)
    assert got == want


def test_chunked_zero_weights_and_overflow(R):
    # n = 27: halves of 13 weights, above the one-workgroup size, so a workspace
    # between the minimum and the full one streams half A in chunks
    L = R.lib()
    n = 27
    full = L.rfr_recombine_workspace_bytes(n)
    mn = L.rfr_recombine_min_workspace_bytes(n)
    ws = (mn + full) // 2
    assert mn <= ws < full
    say("chunked zeros")
    # all-zero weights: every pattern is a candidate, far past a small cap
    with pytest.raises(R.RFRError) as e:
        R.recombine_dev([0] * n, 0, 0, cap=100, ws_bytes=ws)
    assert e.value.name == "RFR_ECANDIDATES"
    # a block of zero and of equal weights among random ones: every pattern
    # duplicated over the zero block, equal sums from the repeated weight
    rng = random.Random(2701)
    w = planted_weights(rng, n, k_rel=3)
    for i in (0, 5, 14, 20):
        w[i] = 0
    x = rng.getrandbits(64)
    for i in (2, 9, 17):
        w[i] = x
    w[24] = (-2 * x) & MASK
    say("chunked zero/equal block")
    got = R.recombine_dev(w, n + 9, 6, cap=1 << 14, ws_bytes=ws)
    assert got == O.search_hs(w, n + 9, 6)


def test_many_patterns_per_candidate_key(R):
    # half A = 13 equal weights x: the subsets of size k share the key k x.
    # With half B holding -5x only, 1287 patterns of A pair with one B pattern:
    # all must be returned.  With -5x, -6x and -7x the patterns of the
    # candidate keys outnumber the 4096 (key, pattern) records a search holds,
    # which must be reported as an overflow, never a partial answer.
    rng = random.Random(4811)
    x = rng.getrandbits(64)
    base = [x] * 13 + [rng.getrandbits(64) for _ in range(13)] + [rng.getrandbits(64)]
    w1 = list(base)
    w1[13] = (-5 * x) & MASK
    say("many patterns per key: one B pattern")
    got = R.recombine_dev(w1, 30, 4, cap=1 << 16)
    want = O.search_hs(w1, 30, 4)
    assert len(want) >= 1287
    assert got == want
    w2 = list(w1)
    w2[14] = (-6 * x) & MASK
    w2[15] = (-7 * x) & MASK
    say("many patterns per key: record overflow")
    with pytest.raises(R.RFRError) as e:
        R.recombine_dev(w2, 30, 4, cap=1 << 16)
    assert e.value.name == "RFR_ECANDIDATES"


@pytest.mark.parametrize("n,expect", [(41, 100), (43, 700)])
def test_recovery_of_many_candidate_keys(R, n, expect):
    # random weights with a window wide enough for about `expect` false
    # candidates (2^(n-1) patterns, each in the window with probability
    # width / 2^64; the window stays below 2^32): about 100 key pairs take the
    # meet-in-the-middle recovery of the few-candidate path, about 700 the
    # re-enumeration against a key bitmap.  Both must return the oracle's
    # Horowitz-Sahni candidates.
    rng = random.Random(7300 + expect)
    w = [rng.getrandbits(64) for _ in range(n)]
    t = (expect << 64) // (1 << (n - 1)) // 2
    say("many candidate keys: about %d" % expect)
    got = R.recombine_dev(w, t, t, cap=1 << 14)
    want = O.search_hs(w, t, t)
    assert expect // 2 < len(want) < expect * 2
    assert got == want


def test_small_budget_context_streams_half_a(R):
    # a budget below the full tables of the degree-60 searches: the plain path
    # streams half A and still returns the oracle's factorisations
    g = json.load(open(os.path.join(HERE, "golden", "golden_mid.json")))["cases"]
    with R.Context(0, mem_budget=800 << 10) as c:
        for w in W.config_mid()[6:10]:
            say("budget seed", w.seed)
            e = g[str(w.seed)]
            assert c.factor(w.coeffs) == (e["content"], [tuple(f) for f in e["factors"]])


# ------------------------------------------------------------------ multi-chunk gather
# A level-1 bucket with more tiles than one gather chunk makes the join stage
# its sub-buckets' segments in several chunks (and read the segment bounds
# from global memory instead of preloading them); a tuning table that forces a
# single level-1 bucket routes mid-size searches there.


def _force_tuning(R, tmp_path, lines):
    p = tmp_path / "tune.txt"
    p.write_text("".join("%d %d %d 0\n" % l for l in lines))
    R.load_tuning(str(p))


def _restore_tuning(R, tmp_path, lgs):
    # back to the fixed rule, then to the shipped table if there is one
    _force_tuning(R, tmp_path, [(lg, -1, -1) for lg in lgs])
    if os.path.exists(R.TUNING_PATH):
        R.load_tuning(R.TUNING_PATH)


def test_autotune_table_keeps_results(R, tmp_path):
    # the tuner times every split of two size classes and writes its table;
    # a table changes speed and workspace only, never a result (a degree-50
    # input searches halves of 2^12..2^13 keys, the tuned classes)
    p = W.rand_poly(W._rng(5050), 50, -1000, 1000)
    e = O.factor(p)
    out = tmp_path / "tuned.txt"
    try:
        with R.Context(0) as c:
            assert c.factor(p) == e
            say("autotune 12..13")
            c.autotune(12, 13, str(out))
            rows = [l.split() for l in out.read_text().splitlines() if l and not l.startswith("#")]
            assert [int(r[0]) for r in rows] == [12, 13]
            for r in rows:
                assert len(r) == 5 and int(r[1]) >= 0 and 9 <= int(r[2]) <= 10 and float(r[3]) > 0
                assert int(r[4]) in (0, 1)
            assert c.factor(p) == e
            with pytest.raises(R.RFRError) as err:
                c.autotune(12, 33)
            assert err.value.name == "RFR_EINVAL"
    finally:
        if os.path.exists(R.TUNING_PATH):
            R.load_tuning(R.TUNING_PATH)


def test_multi_chunk_gather_matches_oracle(R, tmp_path):
    lgs = [20, 21, 22]
    try:
        _force_tuning(R, tmp_path, [(lg, 0, 10) for lg in lgs])
        for n in (41, 43):
            rng = random.Random(700 + n)
            w = planted_weights(rng, n, k_rel=5)
            say("multi-chunk gather n=%d" % n)
            assert R.recombine_dev(w, n + 9, 6, cap=1 << 12) == O.search_hs(w, n + 9, 6)
    finally:
        _restore_tuning(R, tmp_path, lgs)


def test_multi_chunk_gather_batched_matches_golden(R, tmp_path):
    g = json.load(open(os.path.join(HERE, "golden", "golden_batch.json")))["cases"]
    ws = [w for w in W.config_batch() if str(w.seed) in g]
    pick = [w for w in ws if 40 <= len(w.coeffs) - 1 <= 80][:48]
    lgs = list(range(14, 23))
    try:
        _force_tuning(R, tmp_path, [(lg, 0, 10) for lg in lgs])
        with R.Context(0) as c:
            say("multi-chunk gather batch of %d" % len(pick))
            got = c.factor_batch([w.coeffs for w in pick])
        for w, r in zip(pick, got):
            e = g[str(w.seed)]
            assert r == (e["content"], [tuple(f) for f in e["factors"]]), w.seed
    finally:
        _restore_tuning(R, tmp_path, lgs)


def _sympy_factor(coeffs):
    """(content, canonical factors) of the complete factorisation (sympy.factor_list)."""
    import sympy
    X = sympy.Symbol("x")
    c, fl = sympy.factor_list(sympy.Poly(list(reversed([int(v) for v in coeffs])), X))
    c = int(c)
    facs = []
    for f, m in fl:
        cs = [int(v) for v in reversed(f.all_coeffs())]
        if cs[-1] < 0:
            cs = [-v for v in cs]
            c = -c if m % 2 else c
        facs.extend([cs] * m)
    return c, O.canonical(facs)


def test_single_element_factors_split_off(ctx):
    # many rational roots (or integer quadratic pair factors) make every
    # subset of them a factor: 2^k candidates.  Such factors are confirmed one
    # element at a time and split off before the search; the result is the
    # complete factorisation (sympy's factor_list as the definition).
    cases = []
    p = [1]
    for k in range(1, 15):
        p = O.poly_mul_exact(p, [-k, 1])          # (x-1)...(x-14): 2^13 candidate patterns
    cases.append(p)
    q = W.rand_poly(W._rng(7003), 12, -50, 50)
    for k in (1, 2, 4, 5, 7, 8, 10, 11, 13, 14):
        q = O.poly_mul_exact(q, [k, 3])           # (3x + k), non-monic rational roots
    cases.append(q)
    r = [1]
    for k in range(1, 9):
        r = O.poly_mul_exact(r, [k * k, 0, 1])    # x^2 + k^2: integer pair factors
    cases.append(r)
    s = [1, 0, -2]                                # both kinds beside x^2 - 2 and a random factor
    for k in range(1, 7):
        s = O.poly_mul_exact(s, [-k, 1])
    for k in range(1, 4):
        s = O.poly_mul_exact(s, [k * k, 0, 1])
    s = O.poly_mul_exact(s, W.rand_poly(W._rng(7004), 10, -9, 9))
    cases.append(s)
    for c in cases:
        say("single-element factors, degree", len(c) - 1)
        got = ctx.factor(c)
        assert got == _sympy_factor(c)
        cont, facs = got
        prod = [cont]
        for f in facs:
            prod = O.poly_mul_exact(prod, list(f))
        assert prod == c


def test_maximum_size_search_recovers_planted_factors(R):
    # the largest served size: a degree-124 product of random degree-40 and
    # degree-84 factors (coefficients in [-1000, 1000]) has n = 65 elements,
    # so both halves hold 2^32 keys (about 80 GB of tables): level-1 buckets
    # of more than one gather chunk, the many-candidate recovery, and every
    # index past 32 bits.  The result must be the two drawn factors, multiply
    # back to p, and equal sympy's complete factorisation.
    rng = W._rng(9101)
    f = W.rand_poly(rng, 40, -1000, 1000)
    g = W.rand_poly(rng, 84, -1000, 1000)
    p = O.poly_mul_exact(f, g)
    with R.Context(0) as c:
        say("maximum size: degree %d" % (len(p) - 1))
        r = c.factor_full(p)
        say("  n=%d candidates=%d search %.0f ms" % (r["n"], r["n_candidates"], r["ms_search"]))
    assert r["n"] == 65
    assert r["factors"] == O.canonical([O.primitive(f), O.primitive(g)])
    prod = [r["content"]]
    for q in r["factors"]:
        prod = O.poly_mul_exact(prod, list(q))
    assert prod == p
    # the complete factorisation by a method independent of RFR (the oracle's
    # search cannot reach n = 65): the two factors are irreducible
    say("  sympy factor_list of the degree-%d product" % (len(p) - 1))
    assert (r["content"], r["factors"]) == _sympy_factor(p)


def test_seventy_element_search_streams_half_a(R):
    # n = 70: half A holds 35 weights, beyond what one enumeration takes, so
    # it is always streamed in chunks against the resident half B' (2^34 keys,
    # about 220 GB of tables).  Beyond the oracle's reach: properties that hold
    # at any size -- every planted relation is found, and every reported
    # pattern's sum lies in the window (Python integers).  With a zero window
    # the 2^69 patterns leave about 32 random ones beside the planted.
    import torch
    n = 70
    rng = random.Random(7070)
    w = [rng.getrandbits(64) for _ in range(n)]
    planted = []
    for k in range(3):
        idx = sorted(rng.sample(range(n - 1), 5))
        w[idx[-1]] = (-sum(w[i] for i in idx[:-1])) & MASK
        planted.append(sum(1 << i for i in idx))
    free_b = torch.cuda.mem_get_info()[0]
    ws_b = min(R.lib().rfr_recombine_workspace_bytes(n), free_b - (8 << 30))
    ws_b = max(R.lib().rfr_recombine_min_workspace_bytes(n), ws_b)
    say("seventy elements: workspace %.0f GB" % (ws_b / 2 ** 30))
    try:
        got = R.recombine_dev(w, 0, 0, cap=1 << 12, ws_bytes=ws_b)
    finally:
        # hand the workspace back to the device (later tests allocate through HIP)
        torch.cuda.empty_cache()
    say("  %d patterns" % len(got))
    assert all(p in got for p in planted if p < (1 << (n - 1)))
    for p in got:
        assert sum(w[i] for i in range(n - 1) if (p >> i) & 1) & MASK == 0
    assert len(got) < 200


def test_flood_inputs_fold_the_second_trace(R, ctx):
    # Swinnerton-Dyer f_5 (1.57M patterns whose root sum is an integer) and
    # f_5 * (x^32 - x - 1) (3.14M): the first search overflows the candidate
    # capacity, the second folds the second trace into the weights and keeps
    # only the patterns whose sum of squares is an integer as well.  Results
    # against the oracle's stored ones (make_golden.py flood).
    g = json.load(open(os.path.join(HERE, "golden", "golden_flood.json")))["cases"]
    ws = W.config_flood()
    for w in ws:
        e = g[str(w.seed)]
        say("flood input seed %d, degree %d" % (w.seed, w.degree))
        r = ctx.factor_full(w.coeffs)
        assert (r["content"], r["factors"]) == (e["content"], [tuple(f) for f in e["factors"]])
        assert r["n"] == e["n"]
        assert r["trace_folded"] == 1
        assert e["tr2_candidates"] <= r["n_candidates"] < e["tr2_candidates"] + 64
        say("  first-trace candidates %d (oracle), after the second trace %d on the device (oracle %d): "
            "%d rejected inside the search; search %.1f ms" % (
                e["tr1_candidates"], r["n_candidates"], e["tr2_candidates"],
                e["tr1_candidates"] - r["n_candidates"], r["ms_search"]))
    # the same inputs inside a batch (their batch slots overflow, then the
    # plain path folds) and an input that needs no folding
    polys = [w.coeffs for w in ws] + [W.config_small().coeffs]
    got = ctx.factor_batch(polys)
    for w, r in zip(ws, got):
        e = g[str(w.seed)]
        assert r == (e["content"], [tuple(f) for f in e["factors"]])
    assert got[-1] == O.factor(W.config_small().coeffs)
    assert ctx.factor_full(W.config_small().coeffs)["trace_folded"] == 0
