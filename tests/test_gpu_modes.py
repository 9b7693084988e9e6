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


def test_served_alone_equals_in_mix(R):
    reqs = W.config_stream(48, rate_per_s=400.0, dcap=96)
    # a few requests with repeated factors ride in the same stream
    for i, w in enumerate(W.config_repeated(6)):
        reqs.insert(4 + 7 * i, W.Request(reqs[4 + 7 * i].t_arrive, w))
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
    for t, a in zip(tickets, alone):
        res, lat = done[t]
        assert not isinstance(res, Exception), res
        assert (res["content"], res["factors"]) == a
        assert lat >= 0
