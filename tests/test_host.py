"""CPU tests of the library's host side (no GPU needed).

* every symbol include/rfr.h declares is exported by librfr.so;
* the host-stage weights and window (rfr_weights) agree with the oracle's
  high-precision values: identical, or within the window's own error bound;
* error paths of the host stages;
* the window is conservative: planted factors' residues lie inside it.
"""
import os
import re
import subprocess

import pytest

from oracle import rfr_ref as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MOD = 1 << 64


@pytest.fixture(scope="module")
def R():
    import paper_2410_15880_amd as R
    R.lib()
    return R


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "rfr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(rfr_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol(R):
    decl = declared_symbols()
    assert len(decl) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", R.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [d for d in decl if d not in exported]
    assert not missing, missing
    assert sorted(decl) == sorted(R.EXPORTS)


def _signed(x):
    return ((x + (1 << 63)) % MOD) - (1 << 63)


@pytest.mark.parametrize("coeffs", [[6, -5, 1], [-2, 0, 1], [-1, 0, 2], [5, 3, 7], [1, 0, -10, 0, 1],
                                    [3, 7], [-1, 0, 0, 0, 0, 0, 1]])
def test_weights_match_oracle_small(R, coeffs):
    got = R.weights(coeffs)
    tr = O.Trace()
    O.factor(coeffs, tr)
    assert got["n"] == tr.n
    # same elements in the same canonical order; weights within the window
    for a, b in zip(got["w"], tr.w):
        assert abs(_signed(a - b)) <= got["t_hi"]


def test_weights_match_oracle_configs(R):
    for w in [W.config_small()] + W.config_mid()[::3] + W.config_batch()[:40:5]:
        got = R.weights(w.coeffs)
        cont, k, prim = O.normalise(w.coeffs)
        ts, groups, deltas = O.elements(prim)
        ow = O.weights(prim, ts)
        assert got["n"] == len(ts)
        assert got["r"] == sum(1 for g in groups if g[0] == "r")
        for a, b in zip(got["w"], ow):
            assert abs(_signed(a - b)) <= got["t_hi"], w.seed
        # the window accounts for floor quantisation of n weights
        assert got["t_lo"] >= got["n"] + got["t_hi"]


def test_window_conservative_on_planted(R):
    # each planted factor's subset of the product's weights sums into the window
    for w in W.config_mid()[8:]:
        got = R.weights(w.coeffs)
        tr = O.Trace()
        O.factor(w.coeffs, tr)
        for s in tr.confirmed:
            tot = sum(got["w"][i] for i in range(got["n"]) if (s >> i) & 1)
            assert O.in_window(tot, got["t_lo"], got["t_hi"])


def test_weights_errors(R):
    with pytest.raises(R.RFRError) as e:
        R.weights([1, -2, 1])
    assert e.value.name == "RFR_ENOTSQFREE"
    with pytest.raises(R.RFRError) as e:
        R.weights([0, 0, 3])
    assert e.value.name == "RFR_ENOTSQFREE"
    with pytest.raises(R.RFRError) as e:
        R.weights([4])
    assert e.value.name == "RFR_EINVAL"
    with pytest.raises(R.RFRError) as e:
        R.weights([1, 2, 0])
    assert e.value.name == "RFR_EINVAL"


def test_workspace_sizes(R):
    L = R.lib()
    assert L.rfr_recombine_workspace_bytes(1) == 0
    assert L.rfr_recombine_workspace_bytes(200) == 0
    prev = 0
    for n in range(2, 60):
        b = L.rfr_recombine_workspace_bytes(n)
        na = (n - 1 + 1) // 2
        nb = (n - 1) // 2
        assert b >= 8 * ((1 << na) + (1 << nb))
        assert b >= prev
        prev = b
    assert L.rfr_expand_workspace_bytes(0) == 0
    assert L.rfr_expand_workspace_bytes(20) >= 8 << 20


def test_kernel_entry_rejects_bad_arguments_on_host(R):
    # argument checks happen before anything touches a device
    import ctypes as C
    L = R.lib()
    w = (C.c_uint64 * 4)(1, 2, 3, 4)
    st = L.rfr_recombine_dev(w, 1, 0, 0, None, 0, None, None, 1, None)
    assert st == -1
    st = L.rfr_recombine_dev(w, 4, 1 << 33, 0, C.c_void_p(1), 1 << 20, None, C.c_void_p(1), 1, C.c_void_p(1))
    assert st == -1
    st = L.rfr_expand_dev(w, 0, 0, None, 0, None, None)
    assert st == -1


def test_large_roots_do_not_overflow(R):
    # degree-62 and degree-90 inputs with roots near -340 and +100: the Newton
    # step of the polish must not overflow (|p'|^2 > 1e308 if evaluated directly)
    reqs = W.config_stream(300, rate_per_s=1.0, dcap=110)
    for k in (74, 264):
        c = reqs[k].work.coeffs
        got = R.weights(c)
        cont, kk, prim = O.normalise(c)
        ts, groups, deltas = O.elements(prim)
        assert got["n"] == len(ts)
        ow = O.weights(prim, ts)
        for a, b in zip(got["w"], ow):
            assert abs(_signed(a - b)) <= got["t_hi"]


def test_every_stream_request_prepares(R):
    # host roots succeed on the served workload's degree range (up to 128)
    for r in W.config_stream(400, rate_per_s=1.0):
        R.weights(r.work.coeffs)


def test_weights_rounding_tight_against_oracle(R):
    # the product's double-double weights agree with the oracle's 400-bit
    # weights to within a few units (the window only has to cover root error
    # and the floor); this catches any lost bit in the fractional part
    rng = __import__("random").Random(17)
    sample = [w.coeffs for w in rng.sample(W.config_batch(), 24)]
    sample += [r.work.coeffs for r in W.config_stream(60, rate_per_s=1.0)[::6]]
    worst = 0
    for c in sample:
        got = R.weights(c)
        cont, kk, prim = O.normalise(c)
        ts, groups, deltas = O.elements(prim)
        ow = O.weights(prim, ts)
        for a, b in zip(got["w"], ow):
            worst = max(worst, abs(_signed(a - b)))
    assert worst <= 4, worst


def test_results_pack_flattens_in_order(R):
    # host-only ABI call on results laid out by hand: two results, a null
    # (failed) entry between them, then a size check that writes nothing
    import ctypes as C
    import numpy as np
    made = []

    def result(content, factors):
        degs = (C.c_int32 * max(len(factors), 1))(*[len(f) - 1 for f in factors])
        co = (C.c_int64 * max(sum(len(f) for f in factors), 1))(*[c for f in factors for c in f])
        r = R.Result(content=content, nfactors=len(factors), degrees=C.cast(degs, C.POINTER(C.c_int32)),
                     coeffs=C.cast(co, C.POINTER(C.c_int64)))
        made.extend([degs, co, r])
        return C.pointer(r)

    a = [(1, 1), (-3, 0, 2), (5, 4, 0, 1)]
    b = [(0, 1)]
    outs = (C.POINTER(R.Result) * 3)(result(-6, a), None, result(2, b))
    sts = (C.c_int * 3)(0, -4, 0)
    L = R.lib()
    nd, nc = C.c_size_t(), C.c_size_t()
    assert L.rfr_results_pack(outs, 3, None, None, None, 0, None, 0, C.byref(nd), C.byref(nc)) == 0
    assert (nd.value, nc.value) == (4, 2 + 3 + 4 + 2)
    small = np.zeros(4, dtype=np.int64)
    assert L.rfr_results_pack(outs, 3, small.ctypes.data, small.ctypes.data, small.ctypes.data, 4,
                              small.ctypes.data, 3, C.byref(nd), C.byref(nc)) == -1
    assert not small.any()
    res = R._unpack_many(outs, sts, 3)
    assert res[0] == (-6, [tuple(f) for f in a])
    assert isinstance(res[1], R.RFRError)
    assert res[2] == (2, [tuple(f) for f in b])


def test_flatten_batch_inputs(R):
    degs, flat = R._flatten([[1, 2, 3], [4, 5], [6, 7, 8, 9]])
    assert degs.tolist() == [2, 1, 3]
    assert flat.tolist() == list(range(1, 10))
    with pytest.raises(OverflowError):
        R._flatten([[1, 1 << 63]])


def test_squarefree_matches_oracle(R):
    # the library's Yun decomposition (modular gcds) against the oracle's
    # (sympy gcd as its library step) on seeded repeated-factor inputs
    for w in W.config_repeated(60):
        assert R.squarefree(w.coeffs) == O.squarefree(w.coeffs), w.seed


@pytest.mark.parametrize("coeffs", [
    [0, 0, 0, 1],                      # x^3
    [0, 0, 0, 1, 1],                   # x^3 (x + 1)
    [6, -5, 1],                        # square-free
    [-4, 0, 4],                        # content 4, square-free part x^2 - 1
    [1, -5, 10, -10, 5, -1],           # -(x - 1)^5
    [-1, 0, 5, 0, -10, 0, 10, 0, -5, 0, 1],  # (x^2 - 1)^5
    [4, 12, 13, 6, 1],                 # (x^2 + 3x + 2)^2
])
def test_squarefree_edge_cases(R, coeffs):
    assert R.squarefree(coeffs) == O.squarefree(coeffs)


def test_squarefree_rejects_bad_input(R):
    with pytest.raises(R.RFRError):
        R.squarefree([5])            # degree 0
    with pytest.raises(R.RFRError):
        R.squarefree([1, 2, 0])      # zero leading coefficient


def test_squarefree_large_multiplicity(R):
    # (3x - 2)^9 (x^2 + 1)^4: coefficients near 1e7, multiplicities up to 9
    p = [1]
    for _ in range(9):
        p = O.poly_mul_exact(p, [-2, 3])
    for _ in range(4):
        p = O.poly_mul_exact(p, [1, 0, 1])
    assert R.squarefree(p) == O.squarefree(p) == (1, [((1, 0, 1), 4), ((-2, 3), 9)])


def test_window_too_wide_for_the_search_is_a_precision_error(R):
    # (a x - b)(a x - b - 1): two rational roots 1/a apart whose double-double
    # inclusion radii grow like a, so the window grows like a^3 and crosses
    # the search's limit (t_lo + t_hi < 2^32) between a = 2^19 and 2^20.
    # Every a either gives a window the search accepts or RFR_EPRECISION
    # (never a window that the search would reject as a bad argument).
    seen_ok = seen_prec = 0
    for k in range(400):
        a = (1 << 19) + k * 1311
        b = (a * 7) // 3
        p = [b * (b + 1), -(2 * b + 1) * a, a * a]
        try:
            r = R.weights(p)
        except R.RFRError as e:
            assert e.name == "RFR_EPRECISION", (a, e)
            seen_prec += 1
            continue
        assert r["t_lo"] + r["t_hi"] < (1 << 32), a
        assert r["t_lo"] >= r["n"] + r["t_hi"]
        seen_ok += 1
    assert seen_ok > 0 and seen_prec > 0
