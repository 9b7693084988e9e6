"""GPU tests of the batched and served modes against the oracle and plain mode."""
import json
import os
import random
import sys
import time

import pytest

import workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available()
    import paper_2410_15880_amd as R
    R.lib()
    return R


def test_batch_matches_oracle_golden(R):
    g = json.load(open(os.path.join(HERE, "golden", "golden_batch.json")))["cases"]
    ws = W.config_batch()[::32]
    say("batch of", len(ws))
    with R.Context(0) as ctx:
        got = ctx.factor_batch([w.coeffs for w in ws])
    for w, r in zip(ws, got):
        e = g[str(w.seed)]
        assert r == (e["content"], [tuple(f) for f in e["factors"]]), w.seed


def test_batch_full_config_equals_plain(R):
    ws = W.config_batch()
    say("full batch", len(ws))
    with R.Context(0) as ctx:
        t0 = time.perf_counter()
        got = ctx.factor_batch([w.coeffs for w in ws])
        say("  batch s", time.perf_counter() - t0)
        rnd = random.Random(1)
        for i in rnd.sample(range(len(ws)), 64):
            assert got[i] == ctx.factor(ws[i].coeffs), ws[i].seed


def test_batch_mixed_sizes_and_errors(R):
    polys = [[6, -5, 1], [1, -2, 1], [3, 7], W.config_small().coeffs] + [w.coeffs for w in W.config_mid()[:4]]
    polys += [[0, 0, 1], [1, 0, 0, 0, 0, 2]]
    with R.Context(0) as ctx:
        got = ctx.factor_batch(polys)
        assert got[1] == (1, [(-1, 1), (-1, 1)])  # (x - 1)^2 through its square-free part
        assert got[-2] == (1, [(0, 1), (0, 1)])
        for p, r in zip(polys, got):
            assert r == ctx.factor(p)


def test_batch_repeated_factors_match_oracle(R):
    # inputs that are not square-free, mixed with square-free ones, in one batch
    from oracle import rfr_ref as O
    rep = W.config_repeated(24)
    mix = [w.coeffs for w in W.config_batch(64, base_seed=9000)]
    polys = [c for pair in zip([w.coeffs for w in rep], mix) for c in pair] + mix[len(rep):]
    say("batch with repeated factors", len(polys))
    with R.Context(0) as ctx:
        got = ctx.factor_batch(polys)
        for p, r in zip(polys, got):
            assert r == ctx.factor(p)
    for w in rep:
        assert got[2 * rep.index(w)] == O.factor_general(w.coeffs), w.seed


def _sympy_factor(coeffs):
    """(content, canonical factors) of sympy.factor_list (independent of RFR)."""
    import sympy
    from oracle import rfr_ref as O
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


def test_served_alone_equals_in_mix(R):
    # the served stream's inputs: 48 Poisson requests (degrees log-uniform in
    # [24, 128], coefficients in [-1000, 1000], 30 % planted), 6 inputs with
    # repeated factors, and two of the largest size (degree 128: a random one
    # and a 40 x 88 planted product, n about 65 -- 2^32-key halves that are
    # admitted one at a time)
    g = json.load(open(os.path.join(HERE, "golden", "golden_stream.json")))["cases"]
    reqs = W.config_stream(48, rate_per_s=400.0)
    for i, w in enumerate(W.config_repeated(6)):
        reqs.insert(4 + 7 * i, W.Request(reqs[4 + 7 * i].t_arrive, w))
    big = [W.Workload(W.rand_poly(W._rng(5901), 128, -1000, 1000), 5901, "random")]
    rng = W._rng(5902)
    f, h = W.rand_poly(rng, 40, -1000, 1000), W.rand_poly(rng, 88, -1000, 1000)
    big.append(W.Workload(W.poly_mul(f, h), 5902, "planted", [f, h]))
    reqs.insert(10, W.Request(reqs[10].t_arrive, big[0]))
    reqs.insert(30, W.Request(reqs[30].t_arrive, big[1]))
    say("serving", len(reqs))
    with R.Context(0) as ctx:
        alone = [ctx.factor(r.work.coeffs) for r in reqs]
        ctx.serve_start(max_active=6, host_threads=8)
        t0 = time.perf_counter()
        tickets = []
        for r in reqs:
            while time.perf_counter() - t0 < r.t_arrive:
                time.sleep(0.0005)
            tickets.append(ctx.submit(r.work.coeffs))
        done = {}
        deadline = time.time() + 120
        while len(done) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t in done:
                    continue
                p = ctx.poll(t)
                if p is not None:
                    done[t] = p
            time.sleep(0.001)
        ctx.serve_stop()
    assert len(done) == len(tickets)
    pinned = 0
    for t, a, r in zip(tickets, alone, reqs):
        res, lat = done[t]
        assert not isinstance(res, Exception), res
        got = (res["content"], res["factors"])
        # the same alone and in the mix
        assert got == a, r.work.seed
        assert lat >= 0
        # and the oracle's (stored) or, beyond the oracle's reach, sympy's
        e = g.get(str(r.work.seed))
        if e is not None:
            assert r.work.coeffs == e["coeffs"]
            assert got == (e["content"], [tuple(x) for x in e["factors"]]), r.work.seed
            pinned += 1
        else:
            assert r.work.seed in (5901, 5902)
            say("  sympy factor_list, degree", r.work.degree)
            assert got == _sympy_factor(r.work.coeffs), r.work.seed
    assert pinned == len(reqs) - 2


def test_served_small_requests_pass_queued_big_searches(R):
    # Eight degree-100 requests (searches with halves of 2^25..2^27 keys, which
    # run one at a time on the big-search slot) are submitted, then twelve
    # degree-30 ones, to a server with two host workers.  The workers must hand
    # the big searches over and go on with the small requests, so that those
    # finish while the big searches still queue (workers that waited for the
    # slot would hold the small ones back behind the whole queue).  Every
    # result must equal the same request's standalone result.
    bigs = [w.coeffs for w in W.config_large(count=8)]
    smalls = [W.rand_poly(W._rng(8800 + i), 30, -1000, 1000) for i in range(12)]
    with R.Context(0) as ctx:
        alone = [ctx.factor(p) for p in bigs + smalls]
        ctx.serve_start(max_active=4, host_threads=2)
        t0 = time.perf_counter()
        subs, tickets = [], []
        for p in bigs + smalls:
            subs.append(time.perf_counter() - t0)
            tickets.append(ctx.submit(p))
        done = {}
        deadline = time.time() + 60
        while len(done) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in done:
                    q = ctx.poll(t)
                    if q is not None:
                        done[t] = q
            time.sleep(0.0005)
        ctx.serve_stop()
    assert len(done) == len(tickets)
    fin = []
    for t, s, a in zip(tickets, subs, alone):
        res, lat = done[t]
        assert not isinstance(res, Exception), res
        assert (res["content"], res["factors"]) == a
        fin.append(s + lat / 1000.0)
    big_fin, small_fin = sorted(fin[:8]), sorted(fin[8:])
    say("finish: median small %.2f ms, sixth of eight big %.2f ms" % (1e3 * small_fin[6], 1e3 * big_fin[5]))
    assert small_fin[6] < big_fin[5]
