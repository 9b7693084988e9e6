"""Benchmark of the RFR hot path on one MI355X.

One step = the whole path (roots, weights, window, device search, confirmation,
atoms) over one batch of 16 seeded degree-100 polynomials (8 random with
coefficients in [-1000, 1000], 8 planted products of degree-30 and degree-70
factors), through the library's batched entry point; the plain entry point
(one call per polynomial) is timed beside it.  Extra legs: the 16 degree-60
polynomials, the 4096-polynomial uneven batch, and the served request stream.

Prints ONE JSON line.  `value` is subset-sum pairs per second: sum over the
batch of N_A * N_B = 2^(n-1) (the pattern space each search covers) divided by
the step time.  The roofline object reports the dominant search kernel's
algorithmic bytes per launch over its average launch duration, timed with HIP
events recorded on the stream the kernel runs on, inside the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per table key for each stage:
# K1 writes each key once; K2 reads and writes it; K3 reads it; K0/K4 only
# enumerate (no table traffic); the scans touch per-workgroup counters only.
STAGE_BYTES_PER_KEY = {"count": 0, "scan": 0, "enum_partition": 8, "tile_sort": 16, "sort_join": 8,
                       "recover": 0}
STAGE_KERNEL = {"count": "k_enum<true>", "scan": "k_scan_cols+k_scan_buckets",
                "enum_partition": "k_enum<false>", "tile_sort": "k_tile2", "sort_join": "k_join<false>",
                "recover": "k_recover+k_pairs"}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_search_kernels_degree100x16.txt")
# the kernels and the radix-split table the library loads at context creation
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2410_15880_amd", "csrc", f) for f in ("rfr_device.hip", "rfr_device.h")]
KERNEL_SOURCES.append(os.path.join(ROOT, "paper_2410_15880_amd", "tuning", "mi355x.txt"))


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(stage):
    """HBM bytes per launch of a stage's kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by what the same counters read
    for a copy of known size), or None when the kernels changed since."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    kv, kern = {}, {}
    for ln in lines:
        p = ln.split()
        if not p or p[0].startswith("#"):
            continue
        if p[0] == "stage" and len(p) >= 6:
            kern[p[1]] = (float(p[3]), float(p[5]))  # stage <name> fetch_kib <x> write_kib <y>
        elif len(p) == 2:
            kv[p[0]] = p[1]
    if kv.get("source_sha256") != kernel_source_hash() or stage not in kern:
        return None
    fk, wk = kern[stage]
    return int((fk * float(kv["fetch_scale"]) + wk * float(kv["write_scale"])) * 1024)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def _oracle_one(coeffs):
    from oracle import rfr_ref as O
    t0 = time.perf_counter()
    O.factor(coeffs)
    return time.perf_counter() - t0


def cpu_baseline(polys, ns, workers=16):
    """The oracle, as it stands, on the workload: one polynomial on one core,
    then all 16 polynomials over a pool of worker processes (one polynomial
    per process at a time), each timed once."""
    import multiprocessing as mp
    i = 0
    one = _oracle_one(polys[i].coeffs)
    procs = max(1, min(workers, os.cpu_count() or 1, len(polys)))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        per = pool.map(_oracle_one, [w.coeffs for w in polys], chunksize=1)
    wall = time.perf_counter() - t0
    pairs = sum(2 ** (n - 1) for n in ns)
    return {"value": pairs / wall, "unit": "pairs/s", "cores": procs, "kind": "oracle",
            "seconds": round(wall, 2), "factorizations_per_s": len(polys) / wall,
            "sample": "all 16 degree-100 polynomials, oracle.factor end to end (numpy sort/searchsorted, "
                      "mpmath roots), one process per polynomial on %d worker processes, one timed run" % procs,
            "per_poly_s": [round(x, 2) for x in per],
            "single_core": {"value": 2 ** (ns[i] - 1) / one, "unit": "pairs/s", "cores": 1,
                            "seconds": round(one, 2), "factorizations_per_s": 1.0 / one,
                            "sample": "1 of the 16 (seed %d, %s, n=%d), one thread" % (
                                polys[i].seed, polys[i].kind, ns[i])}}


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def batched_leg(R, W, ctx, plain_sample=256, reps=3):
    """4096 uneven polynomials: batched entry point vs plain per-polynomial calls."""
    ws = W.config_batch()
    coeffs = [w.coeffs for w in ws]
    res = ctx.factor_batch(coeffs)          # warm-up + graph capture
    t0 = time.perf_counter()
    for _ in range(reps):
        res = ctx.factor_batch(coeffs)
    dt = (time.perf_counter() - t0) / reps
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "golden_batch.json")))["cases"]
    ok = all(res[i] == (golden[str(ws[i].seed)]["content"], [tuple(f) for f in golden[str(ws[i].seed)]["factors"]])
             for i in range(0, len(ws), 32))
    sample = coeffs[:plain_sample]
    designs = {}
    same = True
    for name, code in (("horowitz_sahni", 1), ("query_e", 2), ("per_size_class", 0)):
        ctx.set_design(code)
        t0 = time.perf_counter()
        plain = [ctx.factor(c) for c in sample]
        dtp = time.perf_counter() - t0
        designs[name] = plain_sample / dtp
        same = same and all(p == r for p, r in zip(plain, res[:plain_sample]))
    ctx.set_design(0)
    return {"workload": "4096 polynomials, degree uniform in [16,80], half planted (seeds 4000-8095)",
            "batched_polys_per_s": len(ws) / dt, "batched_ms": round(dt * 1000, 2),
            "plain_polys_per_s": designs["per_size_class"],
            "plain_polys_per_s_by_design": designs,
            "plain_sample": plain_sample,
            "speedup": (len(ws) / dt) / designs["per_size_class"],
            "results_match_oracle_sample": ok, "batched_equals_plain": same}


def mid_leg(R, W, ctx, reps=5):
    """16 degree-60 polynomials: batched entry point and plain per-polynomial calls."""
    ws = W.config_mid()
    coeffs = [w.coeffs for w in ws]
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "golden_mid.json")))["cases"]
    res = ctx.factor_batch(coeffs)
    t0 = time.perf_counter()
    for _ in range(reps):
        res = ctx.factor_batch(coeffs)
    dt = (time.perf_counter() - t0) / reps
    designs = {}
    for name, code in (("horowitz_sahni", 1), ("query_e", 2), ("per_size_class", 0)):
        ctx.set_design(code)
        plain = [ctx.factor(c) for c in coeffs]
        t0 = time.perf_counter()
        for _ in range(reps):
            plain = [ctx.factor(c) for c in coeffs]
        dtp = (time.perf_counter() - t0) / reps
        designs[name] = {"plain_polys_per_s": len(ws) / dtp, "equals_batched": plain == res}
    ctx.set_design(0)
    ok = all(r == (golden[str(w.seed)]["content"], [tuple(f) for f in golden[str(w.seed)]["factors"]])
             for r, w in zip(res, ws))
    return {"workload": "degree-60 x16: 8 random in [-100,100] + 8 planted 20x40 products (seeds 2000-2015)",
            "batched_polys_per_s": len(ws) / dt,
            "plain_polys_per_s": designs["per_size_class"]["plain_polys_per_s"],
            "plain_by_design": designs, "results_match_oracle": ok,
            "batched_equals_plain": all(v["equals_batched"] for v in designs.values())}


def _serve(ctx, reqs, max_active, host_threads, warm=0):
    """Serve `warm` requests at once and wait for them, then submit the rest at
    their arrival times (measured from the first of them) and collect them as
    they finish: (results, latencies in ms from submission to completion,
    submission times in s from the start of the timed part) of the rest, and
    the warm-up requests' results."""
    ctx.serve_start(max_active=max_active, host_threads=host_threads)

    def drain(pending, done):
        for t in list(pending):
            p = ctx.poll(t)
            if p is not None:
                done[t] = p
                del pending[t]

    pending, done = {}, {}
    wt = []
    for r in reqs[:warm]:
        wt.append(ctx.submit(r.work.coeffs))
        pending[wt[-1]] = None
    while pending:
        drain(pending, done)
        time.sleep(0.0005)
    warm_res = [done[t][0] for t in wt]
    timed = reqs[warm:]
    t_first = timed[0].t_arrive
    t0 = time.perf_counter()
    tickets, done, sub_t = [], {}, []
    for r in timed:
        while time.perf_counter() - t0 < r.t_arrive - t_first:
            drain(pending, done)
            time.sleep(0.0002)
        sub_t.append(time.perf_counter() - t0)
        t = ctx.submit(r.work.coeffs)
        tickets.append(t)
        pending[t] = None
    while pending:
        drain(pending, done)
        time.sleep(0.0005)
    ctx.serve_stop()
    res = [done[t][0] for t in tickets]
    lat = [done[t][1] for t in tickets]
    return res, lat, sub_t, warm_res


def served_leg(R, W, ctx, count=1000, warm=100, rhos=(0.5, 0.8, 2.0), max_active=8, host_threads=16):
    """Poisson stream (degrees log-uniform in [24, 128]) served with continuous
    batching, against plain rfr_factor calls one at a time on the same stream.

    Plain capacity is measured by factoring every request one after another
    (a FIFO server that never idles).  At each rate the plain FIFO server is
    then run: one rfr_factor call after another, each request waiting for its
    arrival time.  Served runs submit at the same arrival times.  At rho above
    1 both systems are saturated, so the served throughput there is its
    capacity."""
    total = warm + count
    probe = W.config_stream(total, rate_per_s=1.0)
    for r in probe[:warm]:
        ctx.factor(r.work.coeffs)
    service, alone = [], []
    for k, r in enumerate(probe[warm:]):
        if k % 250 == 0:
            log("plain pass: request %d of %d" % (k, count))
        t0 = time.perf_counter()
        try:
            alone.append(ctx.factor(r.work.coeffs))
        except R.RFRError as e:
            alone.append(("error", e.status))
        service.append(time.perf_counter() - t0)
    cap_plain = len(service) / sum(service)
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "golden_stream.json")))["cases"]
    points = []
    same_all = True
    pinned = 0
    pinned_ok = True
    for rho in rhos:
        log("served run at rho %.1f" % rho)
        rate = rho * cap_plain
        reqs = W.config_stream(total, rate_per_s=rate)
        # warm-up requests are served in the same run; statistics cover the rest
        # the warm-up requests are served and finished first; the timed
        # requests then arrive at their times, measured from the first
        res, lat, sub_t, warm_res = _serve(ctx, reqs, max_active, host_threads, warm=warm)
        log("served run at rho %.1f done" % rho)
        t_first = reqs[warm].t_arrive
        span = max(sub_t[k] + lat[k] / 1000.0 for k in range(count)) - sub_t[0]
        log("plain FIFO run at rho %.1f" % rho)
        lat_fifo, t0 = [], time.perf_counter()
        for r in reqs[warm:]:
            arrive = r.t_arrive - t_first
            while time.perf_counter() - t0 < arrive:
                time.sleep(0.0002)
            try:
                ctx.factor(r.work.coeffs)
            except R.RFRError:
                pass
            lat_fifo.append((time.perf_counter() - t0 - arrive) * 1000.0)
        fin = time.perf_counter() - t0
        def outcome(x):
            return ("error", getattr(x, "status", None)) if isinstance(x, Exception) else \
                (x["content"], x["factors"])
        same = all(outcome(res[k]) == alone[k] for k in range(count))
        errors = sum(1 for a in alone if a[0] == "error")
        same_all = same_all and same
        if rho == rhos[0]:
            # requests whose oracle results are stored (the test stream's, same seeds)
            for r, x in zip(reqs, warm_res + res):
                e = golden.get(str(r.work.seed))
                if e is None:
                    continue
                pinned += 1
                pinned_ok = pinned_ok and not isinstance(x, Exception) and e["coeffs"] == r.work.coeffs and \
                    (x["content"], x["factors"]) == (e["content"], [tuple(f) for f in e["factors"]])
        points.append({"rho": rho, "offered_per_s": round(rate, 1),
                       "served_p50_ms": pct(lat, 50), "served_p99_ms": pct(lat, 99),
                       "served_throughput_per_s": count / span,
                       "plain_fifo_p50_ms": pct(lat_fifo, 50), "plain_fifo_p99_ms": pct(lat_fifo, 99),
                       "plain_fifo_throughput_per_s": count / fin})
    over = points[-1]
    return {"workload": "%d requests after %d warm-up, Poisson, degree log-uniform in [24,128], coefficients in "
                        "[-1000,1000], 30%% planted (seed 5000); rho x plain capacity" % (count, warm),
            "plain_polys_per_s": cap_plain,
            "served_capacity_polys_per_s": over["served_throughput_per_s"],
            "capacity_ratio": over["served_throughput_per_s"] / cap_plain,
            "points": points, "max_active": max_active,
            "each_result_same_alone_and_in_mix": same_all, "requests_failed": errors,
            "oracle_pinned_requests": pinned, "oracle_pinned_match": pinned_ok}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the degree-60, batched and served legs")
    ap.add_argument("--served-count", type=int, default=1000, help="requests per served run (after 100 warm-up)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.empty(1 << 27, dtype=torch.int64, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 8}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent polynomials would shard with no communication).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2410_15880_amd as R
    import workloads as W

    polys = W.config_large()
    coeffs = [w.coeffs for w in polys]
    ns = [R.weights(c)["n"] for c in coeffs]  # host stages only
    # the oracle runs first, in fresh worker processes, before this process
    # touches the GPU
    cb = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the 16 degree-100 polynomials")
        cb = cpu_baseline(polys, ns)
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    log("degree-100 step: %d warm-up + %d timed" % (args.warmup, args.steps))
    pairs_per_step = sum(2 ** (n - 1) for n in ns)
    keys_per_step = 0
    for n in ns:
        n1 = n - 1
        keys_per_step += 2 ** ((n1 + 1) // 2) + 2 ** (n1 // 2)

    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "golden_large.json")))["cases"]
    ctx = R.Context(0)
    for _ in range(args.warmup):
        res = ctx.factor_batch(coeffs)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = ctx.factor_batch(coeffs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    # the same 16 polynomials through the plain entry point, one call each
    plain = [ctx.factor(c) for c in coeffs]
    t0p = time.perf_counter()
    for _ in range(2):
        plain = [ctx.factor(c) for c in coeffs]
    plain_s = (time.perf_counter() - t0p) / 2
    extras = {}
    if not args.no_extras:
        log("degree-60 leg")
        extras["mid"] = mid_leg(R, W, ctx)
        log("batched leg")
        extras["batched"] = batched_leg(R, W, ctx)
        log("served leg")
        extras["served"] = served_leg(R, W, ctx, count=args.served_count)
    ctx.close()

    ok = all(not isinstance(r, Exception) and r == (golden[str(w.seed)]["content"],
                                                     [tuple(f) for f in golden[str(w.seed)]["factors"]])
             for r, w in zip(res, polys))
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = pairs_per_step / (ms_per_step / 1000.0)

    # one launch of each stage serves the whole batch of 16 searches
    nlaunch = max(prof["launches"], 1)
    stage_avg = {k: v / nlaunch for k, v in prof["stage_ms"].items()}
    dom = max(stage_avg, key=lambda k: stage_avg[k])
    keys_per_launch = prof["keys"] / nlaunch
    alg_bytes = STAGE_BYTES_PER_KEY[dom] * keys_per_launch
    achieved = alg_bytes / (stage_avg[dom] / 1000.0) / 1e9 if stage_avg[dom] > 0 else 0.0
    if STAGE_BYTES_PER_KEY[dom] > 0:
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
                    "kernel": STAGE_KERNEL[dom], "avg_launch_ms": round(stage_avg[dom], 4),
                    "alg_bytes_per_launch": int(alg_bytes)}
    else:
        roofline = {"bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                    "traffic": None, "kernel": STAGE_KERNEL[dom], "avg_launch_ms": round(stage_avg[dom], 4)}
    stage_gbs = {}
    for k, v in stage_avg.items():
        b = STAGE_BYTES_PER_KEY[k] * keys_per_launch
        stage_gbs[k] = round(b / (v / 1000.0) / 1e9, 1) if (b > 0 and v > 0) else None
    # the whole search: every stage's algorithmic bytes over the sum of the
    # stages' launch times (the gaps between launches left out)
    search_ms = sum(stage_avg.values())
    search_bytes = sum(STAGE_BYTES_PER_KEY.values()) * keys_per_launch
    search_gbs = search_bytes / (search_ms / 1000.0) / 1e9 if search_ms > 0 else 0.0
    whole_search = {"alg_bytes_per_search": int(search_bytes), "stage_ms_sum": round(search_ms, 4),
                    "achieved": round(search_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(search_gbs / HBM_PEAK_GBS, 4)}

    out = {
        "metric": "subset-sum pairs/s + degree-100 factorizations/s; p50/p99 latency vs plain",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "degree-100 x16: 8 random in [-1000,1000] + 8 planted 30x70 products "
                               "(seeds 3000-3015), one rfr_factor_batch call per step (device roots for "
                               "the 16 in one launch, the 16 searches one after another on one stream)",
                   "polys": len(polys), "degree": 100, "n_elements": ns,
                   "pairs_per_step": pairs_per_step, "keys_per_step": keys_per_step},
        "factorizations_per_s": len(polys) / (ms_per_step / 1000.0),
        "results_match_oracle": ok,
        "plain_factorizations_per_s": len(polys) / plain_s,
        "plain_equals_batched": plain == res,
        "stage_ms_per_launch": {k: round(v, 4) for k, v in stage_avg.items()},
        "searches_per_launch": prof["searches"] / nlaunch,
        "stage_alg_gbs": stage_gbs,
        "whole_search_roofline": whole_search,
        "roofline": roofline,
        "host": host_info(),
    }
    out.update(extras)
    out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
