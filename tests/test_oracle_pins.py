"""Pins for the CPU oracle against facts fixed independently of it.

Each test ties one oracle function to something other than itself: a library
routine that does not use RFR (sympy's factorisation, minimal polynomials,
integer square roots), a closed form, brute force on tiny inputs, or the
paper's worked example (Section 2, Eq 5-7).
"""
import json
import math
import os
import random

import numpy as np
import pytest
import sympy

from oracle import rfr_ref as R
import workloads as W

X = sympy.Symbol("x")
HERE = os.path.dirname(os.path.abspath(__file__))


def sympy_factor(coeffs):
    """(content, canonical factors) from sympy.factor_list (Zassenhaus/van Hoeij)."""
    c, fl = sympy.factor_list(sympy.Poly(list(reversed([int(v) for v in coeffs])), X))
    c = int(c)
    facs = []
    for f, m in fl:
        cs = [int(v) for v in reversed(f.all_coeffs())]
        if cs[-1] < 0:
            cs = [-v for v in cs]
            c = -c if m % 2 else c
        facs.extend([cs] * m)
    return c, R.canonical(facs)


def reconstruct(cont, facs):
    p = [cont]
    for f in facs:
        p = R.poly_mul_exact(p, f)
    return p


def sd_poly(k):
    """Swinnerton-Dyer f_k (Eq 5) as the minimal polynomial of sqrt(2)+...+sqrt(p_k)."""
    s = sum(sympy.sqrt(sympy.prime(i)) for i in range(1, k + 1))
    mp = sympy.Poly(sympy.minimal_polynomial(s, X), X)
    return [int(v) for v in reversed(mp.all_coeffs())]


# ---------------------------------------------------------------- textbook


@pytest.mark.parametrize("coeffs,expect", [
    ([6, -5, 1], [(-3, 1), (-2, 1)]),
    ([-1, 0, 0, 0, 0, 0, 1], [(-1, 1), (1, 1), (1, -1, 1), (1, 1, 1)]),
    ([0, -1, 0, 1], [(0, 1), (-1, 1), (1, 1)]),
])
def test_textbook_factorisations(coeffs, expect):
    cont, facs = R.factor(coeffs)
    assert cont == 1
    assert facs == R.canonical([list(e) for e in expect])


def test_linear_product_flood_all_candidates_true():
    # prod (x - k), k = 1..8: every weight is 0 or 2^64-1 (the floor of a value
    # within rounding of an integer), so every pattern is a candidate
    p = [1]
    for k in range(1, 9):
        p = R.poly_mul_exact(p, [-k, 1])
    tr = R.Trace()
    cont, facs = R.factor(p, tr)
    assert all(w in (0, (1 << 64) - 1) for w in tr.w)
    assert len(tr.candidates) == 2 ** 7 - 1
    assert facs == R.canonical([[-k, 1] for k in range(1, 9)])


def test_content_sign_and_x_power():
    # -6 x (2x - 1)(3x + 1) = -36x^3 + 6x^2 + 6x
    p = [0, 6, 6, -36]
    cont, facs = R.factor(p)
    assert cont == -6
    assert facs == R.canonical([[0, 1], [-1, 2], [1, 3]])
    assert reconstruct(cont, facs) == p


def test_not_squarefree_raises():
    with pytest.raises(R.OracleError):
        R.factor(R.poly_mul_exact([-1, 1], [-1, 1]))
    with pytest.raises(R.OracleError):
        R.factor([0, 0, 1, 1])


# ---------------------------------------------------------------- paper example


def test_swinnerton_dyer_f2_matches_eq6_and_eq7():
    ex = json.load(open(os.path.join(HERE, "golden", "paper_examples.json")))["sd_f2"]
    assert sd_poly(2) == ex["coeffs_ascending"]
    tr = R.Trace()
    cont, facs = R.factor(ex["coeffs_ascending"], tr)
    assert facs == [tuple(ex["coeffs_ascending"])]
    # the four real roots are +-sqrt2 +- sqrt3 (Eq 6)
    vals = sorted(float(g[1]) for g in tr.groups)
    want = sorted(float(sympy.sympify(r)) for r in ex["roots"])
    assert np.allclose(vals, want, rtol=0, atol=1e-12)
    # Eq 7: dual pairs sum to an integer, so candidates exist, none confirmed
    assert len(tr.candidates) > 0
    assert tr.confirmed == {}


@pytest.mark.parametrize("k", [3, 4])
def test_swinnerton_dyer_irreducible_with_candidates(k):
    p = sd_poly(k)
    tr = R.Trace()
    cont, facs = R.factor(p, tr)
    assert facs == [tuple(p)]
    assert tr.n == 2 ** k                  # all roots real
    assert len(tr.candidates) >= 2 ** (2 ** (k - 1) - 1) - 1


# ---------------------------------------------------------------- sympy on the configs


def test_config_small_matches_sympy():
    w = W.config_small()
    got = R.factor(w.coeffs)
    assert got == sympy_factor(w.coeffs)
    assert reconstruct(*got) == w.coeffs


def test_config_mid_matches_sympy_and_planted():
    for w in W.config_mid():
        got = R.factor(w.coeffs)
        assert got == sympy_factor(w.coeffs), w.seed
        assert reconstruct(*got) == w.coeffs
        if w.kind == "planted":
            for f in w.planted:
                fp = R.primitive(f)
                # each planted factor is a product of returned factors
                rest = fp
                for q in got[1]:
                    r = R.exact_divide(rest, list(q))
                    if r is not None:
                        rest = r
                assert rest in ([1], [-1])
        else:
            assert len(got[1]) == 1


def test_config_batch_sample_matches_sympy():
    ws = W.config_batch()
    rnd = random.Random(7)
    for i in rnd.sample(range(len(ws)), 24):
        w = ws[i]
        got = R.factor(w.coeffs)
        assert got == sympy_factor(w.coeffs), w.seed
        assert reconstruct(*got) == w.coeffs


# ---------------------------------------------------------------- weights (Eq 18)


def test_weights_closed_form_sqrt2_and_monic_transform():
    # roots +-sqrt(2): floor(frac(sqrt2) 2^64) = isqrt(2^129) - 2^64
    w_pos = math.isqrt(2 << 128) - (1 << 64)
    w_neg = (1 << 64) - 1 - w_pos          # frac(-sqrt2) = 1 - frac(sqrt2)
    tr = R.Trace()
    R.factor([-2, 0, 1], tr)
    assert sorted(tr.w) == sorted([w_pos, w_neg])
    # 2x^2 - 1 has roots +-1/sqrt2; its monic transform y^2 - 2 has +-sqrt2
    tr2 = R.Trace()
    R.factor([-1, 0, 2], tr2)
    assert sorted(tr2.w) == sorted([w_pos, w_neg])


def test_weights_rational_roots_are_zero():
    # (2x - 1)(3x + 1): monic-transform roots a_d * (1/2) = 3, a_d * (-1/3) = -2
    tr = R.Trace()
    R.factor(R.poly_mul_exact([-1, 2], [1, 3]), tr)
    assert all(w in (0, (1 << 64) - 1) for w in tr.w)
    # a quadratic with complex roots: element 2Re z = -b/a, weight frac(-b)=0
    tr = R.Trace()
    R.factor([5, 3, 7], tr)   # 7x^2 + 3x + 5, element 7 * (-3/7) = -3
    assert tr.w in ([0], [(1 << 64) - 1])


def test_planted_factor_residue_inside_window():
    for w in W.config_mid()[8:]:
        tr = R.Trace()
        R.factor(w.coeffs, tr)
        found = [s for s in tr.candidates if s in tr.confirmed]
        assert found
        for s in found:
            tot = sum(tr.w[i] for i in range(tr.n) if (s >> i) & 1)
            assert R.in_window(tot, tr.t_lo, tr.t_hi)


# ---------------------------------------------------------------- searches (Alg A / C)


def _py_sums(ws):
    """Independent subset sums: Python ints, bit i of j selects ws[i]."""
    return [sum(ws[i] for i in range(len(ws)) if (j >> i) & 1) % (1 << 64)
            for j in range(1 << len(ws))]


@pytest.mark.parametrize("seed", range(12))
def test_brute_equals_hs_equals_python_definition(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 15)
    ws = [rng.getrandbits(64) for _ in range(n)]
    # plant a few exact relations so the window is hit
    if n >= 4:
        ws[1] = (-ws[0] - rng.randint(0, 5)) % (1 << 64)
        ws[3] = (-(ws[2] + ws[1]) + rng.randint(0, 3)) % (1 << 64)
    t_lo, t_hi = rng.choice([(0, 0), (n + 3, 2), (7, 9), (1 << 20, 1 << 19)])
    sums = _py_sums(ws[:n - 1])
    want = [s for s in range(1, len(sums)) if R.in_window(sums[s], t_lo, t_hi)]
    assert R.search_brute(ws, t_lo, t_hi) == want
    assert R.search_hs(ws, t_lo, t_hi) == want


def test_search_closed_forms():
    rng = random.Random(3)
    n = 12
    # all weights zero: every nonzero pattern
    assert R.search_hs([0] * n, 0, 0) == list(range(1, 1 << (n - 1)))
    # w0 = -w1, the others random 64-bit: only {0, 1}
    ws = [rng.getrandbits(64) for _ in range(n)]
    ws[1] = (-ws[0]) % (1 << 64)
    assert R.search_hs(ws, 0, 0) == [0b11]
    assert R.search_brute(ws, 0, 0) == [0b11]
    # distinct powers of two, zero window: no pattern
    assert R.search_hs([1 << i for i in range(n)], 0, 0) == []


def test_window_wraps_across_zero():
    # sum of pattern {0} is 2^64 - 3: accepted by T_lo >= 3, rejected by T_lo < 3
    ws = [(1 << 64) - 3, 1 << 40, 1 << 41, 5]
    assert R.search_hs(ws, 3, 0) == [1]
    assert R.search_hs(ws, 2, 0) == []
    assert R.search_brute(ws, 3, 0) == [1]


def test_expand_is_sorted_subset_sums():
    rng = random.Random(11)
    ws = [rng.getrandbits(64) for _ in range(10)]
    got = R.expand(ws).tolist()
    assert got == sorted(_py_sums(ws))
    neg = R.expand(ws, negate=True).tolist()
    assert neg == sorted(((-v) % (1 << 64)) for v in _py_sums(ws))


# ---------------------------------------------------------------- sizing (Eq 10-11)


def test_element_count_near_kac_estimate():
    ns = []
    for w in W.config_mid()[:8]:
        cont, k, prim = R.normalise(w.coeffs)
        ts, groups, deltas = R.elements(prim)
        ns.append(len(ts))
        assert 30 <= len(ts) <= 60        # d/2 <= n <= d (Section 1)
    est = 60 / 2 + math.log(60) / math.pi
    assert abs(np.mean(ns) - est) < 3


# ---- square-free decomposition (Section 2: Yun's algorithm ahead of FACTOR)

def sympy_sqf(coeffs):
    """(content, [(part, mult)]) from sympy.sqf_list, parts primitive with lc > 0."""
    c, fl = sympy.sqf_list(sympy.Poly(list(reversed([int(v) for v in coeffs])), X))
    c = int(c)
    parts = []
    for f, m in fl:
        cs = [int(v) for v in reversed(f.all_coeffs())]
        g = R.content(cs)
        if cs[-1] < 0:
            g = -g
        cs = [v // g for v in cs]
        c *= g ** m
        parts.append((tuple(cs), m))
    # sympy keeps a power of x inside the part of its multiplicity; split it off
    out = []
    for cs, m in parts:
        k = 0
        while cs[k] == 0:
            k += 1
        if k:
            out.append(((0, 1), m))
        if len(cs) - k > 1:
            out.append((tuple(cs[k:]), m))
    merged = {}
    for cs, m in out:
        if cs == (0, 1):
            merged[(cs, "x")] = merged.get((cs, "x"), 0) + m
        else:
            merged[(cs, m)] = m
    res = [(cs, m) for (cs, _), m in merged.items()]
    res.sort(key=lambda pm: (pm[1], len(pm[0]), pm[0]))
    return c, res


def test_squarefree_matches_sympy_sqf_list():
    cases = [w.coeffs for w in W.config_repeated()]
    cases += [[0, 0, 0, 1, 1], [1, 2, 1], [-4, 0, 4], [0, 0, 2], [6, -5, 1]]
    for p in cases:
        assert R.squarefree(p) == sympy_sqf(p), p


def test_squarefree_recovers_planted_multiplicities():
    # the drawn factors of these seeds are square-free and pairwise coprime,
    # so the part of multiplicity m is the product of those drawn m times
    for w in W.config_repeated():
        cont, parts = R.squarefree(w.coeffs)
        counts = {}
        for f in w.planted:
            counts[tuple(f)] = counts.get(tuple(f), 0) + 1
        k = counts.pop((0, 1), 0)
        want = {}
        for f, m in counts.items():
            want[m] = R.poly_mul_exact(want.get(m, [1]), list(f))
        want = {m: R.primitive(prod) for m, prod in want.items()}
        got = {m: list(part) for part, m in parts if part != (0, 1)}
        assert got == want, w.seed
        assert [m for part, m in parts if part == (0, 1)] == ([k] if k else []), w.seed
        # reconstruction: content * prod part**mult == p
        q = [cont]
        for part, m in parts:
            for _ in range(m):
                q = R.poly_mul_exact(q, list(part))
        assert q == [int(c) for c in w.coeffs], w.seed


def test_squarefree_of_squarefree_input_is_itself():
    for w in [W.config_small()] + W.config_mid(4):
        cont, k, prim = R.normalise(w.coeffs)
        cont2, parts = R.squarefree(w.coeffs)
        assert cont2 == cont
        assert parts == ([((0, 1), k)] if k else []) + [(tuple(prim), 1)]


def test_factor_general_matches_sympy_factor_list():
    for w in W.config_repeated()[:12]:
        assert R.factor_general(w.coeffs) == sympy_factor(w.coeffs), w.seed


# ---- real-root count (the r real elements of Eq 1) against exact isolation

def _sympy_real_root_count(coeffs):
    """Number of distinct real roots by sympy's exact real-root isolation
    (continued-fraction bisection on the integer polynomial), a routine that
    shares nothing with the oracle's numerical roots."""
    return len(sympy.Poly(list(reversed([int(v) for v in coeffs])), X).intervals())


def _oracle_real_count(coeffs):
    cont, k, prim = R.normalise(coeffs)
    reals, pairs, rr, rp = R.roots_hp(prim)
    assert len(reals) + 2 * len(pairs) == len(prim) - 1
    return len(reals) + (1 if k else 0)


@pytest.mark.parametrize("which", ["mid", "batch", "large"])
def test_real_root_count_matches_exact_isolation(which):
    if which == "mid":
        ws = W.config_mid()
    elif which == "large":
        ws = W.config_large()
    else:
        rnd = random.Random(17)
        allw = W.config_batch()
        ws = [allw[i] for i in rnd.sample(range(len(allw)), 24)]
    for w in ws:
        assert _oracle_real_count(w.coeffs) == _sympy_real_root_count(w.coeffs), w.seed


# ---- stored expected results against sympy's factorisation

@pytest.mark.parametrize("name", ["large", "batch", "mid", "stream"])
def test_golden_files_match_sympy_factor_list(name):
    g = json.load(open(os.path.join(HERE, "golden", "golden_%s.json" % name)))["cases"]
    for seed, e in g.items():
        want = sympy_factor(e["coeffs"])
        assert (e["content"], [tuple(f) for f in e["factors"]]) == want, seed


# ---------------------------------------------------------------- second trace (Section 2, Eq 5-7)


def _sd_sign_vectors(k, groups):
    """Each element's root written as sum_j s_j sqrt(p_j) (Swinnerton-Dyer f_k):
    the sign vector s in {-1, +1}^k matched by value.  Exact algebra then fixes
    which subsets have integer power sums: sum over the subset of s_j must
    vanish for every j (first trace), and of s_j s_l for every j < l (second
    trace), the square roots of distinct primes and of their distinct products
    being linearly independent over Q."""
    import itertools
    ps = [math.sqrt(sympy.prime(i)) for i in range(1, k + 1)]
    combos = {}
    for signs in itertools.product((-1, 1), repeat=k):
        combos[signs] = sum(s * p for s, p in zip(signs, ps))
    S = []
    for kind, z in groups:
        assert kind == "r"
        v = float(z)
        best = min(combos, key=lambda c: abs(combos[c] - v))
        assert abs(combos[best] - v) < 1e-9
        S.append(best)
    return np.array(S, dtype=np.int64)


def _exact_trace_masks(S, pats, nbits):
    bits = ((pats[:, None] >> np.arange(nbits, dtype=np.int64)[None, :]) & 1).astype(np.int64)
    t1 = bits @ S[:nbits]
    ok1 = np.all(t1 == 0, axis=1)
    k = S.shape[1]
    cross = np.stack([S[:nbits, j] * S[:nbits, l] for j in range(k) for l in range(j + 1, k)], axis=1)
    ok2 = np.all(bits @ cross == 0, axis=1)
    return ok1, ok2


def test_second_trace_exact_on_f4_brute_force():
    # every one of the 2^15 patterns of f_4: the oracle's first-trace candidates
    # are exactly the subsets with an integer root sum, and the ones it keeps
    # after the second trace exactly those with integer sums of squares too
    p = W.swinnerton_dyer(4)
    tr = R.Trace()
    R.factor(p, tr)
    n1 = tr.n - 1
    S = _sd_sign_vectors(4, tr.groups)
    pats = np.arange(1, 1 << n1, dtype=np.int64)
    ok1, ok2 = _exact_trace_masks(S, pats, n1)
    assert sorted(tr.candidates) == [int(x) for x in pats[ok1]]
    assert sorted(tr.tr2_kept) == [int(x) for x in pats[ok1 & ok2]]
    assert 0 < len(tr.tr2_kept) < len(tr.candidates)


def test_second_trace_filter_on_f5_flood():
    # f_5: 1.57M patterns with an integer root sum; the second-trace filter
    # keeps exactly those whose sum of squares is an integer as well
    p = W.swinnerton_dyer(5)
    tr = R.Trace()
    cont, facs = R.factor(p, tr)
    assert facs == [tuple(p)]
    S = _sd_sign_vectors(5, tr.groups)
    pats = np.array(sorted(tr.candidates), dtype=np.int64)
    ok1, ok2 = _exact_trace_masks(S, pats, tr.n - 1)
    assert ok1.all()
    assert sorted(tr.tr2_kept) == [int(x) for x in pats[ok2]]
    assert len(tr.candidates) == 1570030 and len(tr.tr2_kept) == 528


def test_flood_goldens_are_the_known_factorisations():
    # golden_flood.json (oracle only, make_golden.py) against facts fixed by
    # construction: f_5 is a minimal polynomial (irreducible), x^32 - x - 1 is
    # irreducible (Selmer), and the product reconstructs exactly
    g = json.load(open(os.path.join(HERE, "golden", "golden_flood.json")))["cases"]
    f5 = W.swinnerton_dyer(5)
    selmer = [-1, -1] + [0] * 30 + [1]
    assert sympy.Poly(list(reversed(selmer)), X).is_irreducible
    ws = W.config_flood()
    want = {9201: (1, R.canonical([f5])), 9202: (1, R.canonical([f5, selmer]))}
    for w in ws:
        e = g[str(w.seed)]
        assert e["coeffs"] == w.coeffs
        got = (e["content"], [tuple(f) for f in e["factors"]])
        assert got == want[w.seed]
        assert reconstruct(*got) == w.coeffs
        assert e["tr2_candidates"] < e["tr1_candidates"]
