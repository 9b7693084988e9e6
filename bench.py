"""Benchmark of the RFR hot path on one MI355X.

One step = the whole path (roots, weights, window, device search, confirmation,
atoms) over one batch of 16 seeded degree-100 polynomials (8 random with
coefficients in [-1000, 1000], 8 planted products of degree-30 and degree-70
factors), through the library's batched entry point.

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


def cpu_baseline(polys, ns):
    """The oracle, as it stands, on one polynomial of the workload (bounded sample)."""
    from oracle import rfr_ref as O
    i = 0
    t0 = time.perf_counter()
    got = O.factor(polys[i].coeffs)
    dt = time.perf_counter() - t0
    pairs = 2 ** (ns[i] - 1)
    return {"value": pairs / dt, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "seconds": round(dt, 2),
            "factorizations_per_s": 1.0 / dt,
            "sample": "1 of the 16 degree-100 polynomials (seed %d, %s, n=%d): oracle.factor end to end, "
                      "single thread (numpy sort/searchsorted, mpmath roots)" % (
                          polys[i].seed, polys[i].kind, ns[i])}, got


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
    t0 = time.perf_counter()
    plain = [ctx.factor(c) for c in sample]
    dtp = time.perf_counter() - t0
    same = all(p == r for p, r in zip(plain, res[:plain_sample]))
    return {"workload": "4096 polynomials, degree uniform in [16,80], half planted (seeds 4000-8095)",
            "batched_polys_per_s": len(ws) / dt, "batched_ms": round(dt * 1000, 2),
            "plain_polys_per_s": plain_sample / dtp,
            "plain_sample": plain_sample,
            "speedup": (len(ws) / dt) / (plain_sample / dtp),
            "results_match_oracle_sample": ok, "batched_equals_plain": same}


def served_leg(R, W, ctx, count=300, rho=0.8, dcap=110, max_active=8, host_threads=16):
    """Poisson stream served with continuous batching vs plain FIFO (same stream)."""
    probe = W.config_stream(count, rate_per_s=1.0, dcap=dcap)
    # plain FIFO: measured service time of every request, one at a time
    service = []
    alone = []
    for r in probe:
        t0 = time.perf_counter()
        alone.append(ctx.factor(r.work.coeffs))
        service.append(time.perf_counter() - t0)
    cap_plain = len(service) / sum(service)       # requests/s one at a time
    rate = rho * cap_plain
    reqs = W.config_stream(count, rate_per_s=rate, dcap=dcap)
    # FIFO queue on the measured service times (exact for one server)
    fin, lat_fifo = 0.0, []
    for r, sv in zip(reqs, service):
        fin = max(fin, r.t_arrive) + sv
        lat_fifo.append((fin - r.t_arrive) * 1000.0)
    fifo_span = fin - reqs[0].t_arrive
    # served: submit at the arrival times, collect as they finish
    ctx.serve_start(max_active=max_active, host_threads=host_threads)
    t0 = time.perf_counter()
    tickets = []
    pending = {}
    lat = {}
    for k, r in enumerate(reqs):
        while time.perf_counter() - t0 < r.t_arrive:
            for t in list(pending):
                p = ctx.poll(t)
                if p is not None:
                    lat[t] = p
                    del pending[t]
            time.sleep(0.0002)
        t = ctx.submit(r.work.coeffs)
        tickets.append(t)
        pending[t] = k
    while pending:
        for t in list(pending):
            p = ctx.poll(t)
            if p is not None:
                lat[t] = p
                del pending[t]
        time.sleep(0.0005)
    span = time.perf_counter() - t0
    ctx.serve_stop()
    same = all((not isinstance(lat[t][0], Exception)) and
               (lat[t][0]["content"], lat[t][0]["factors"]) == alone[k] for k, t in enumerate(tickets))
    lats = [lat[t][1] for t in tickets]
    return {"workload": "%d requests, Poisson at %.1f/s (%.1f x plain capacity), degree log-uniform in "
                        "[24,128] capped at %d, coefficients in [-1000,1000], 30%% planted (seed 5000)" % (
                            count, rate, rho, dcap),
            "served_p50_ms": pct(lats, 50), "served_p99_ms": pct(lats, 99),
            "served_throughput_per_s": count / span,
            "plain_fifo_p50_ms": pct(lat_fifo, 50), "plain_fifo_p99_ms": pct(lat_fifo, 99),
            "plain_fifo_throughput_per_s": count / fifo_span,
            "max_active": max_active, "each_result_same_alone_and_in_mix": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and served legs")
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

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    polys = W.config_large()
    coeffs = [w.coeffs for w in polys]
    ns = [R.weights(c)["n"] for c in coeffs]
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
    extras = {}
    if not args.no_extras:
        extras["batched"] = batched_leg(R, W, ctx)
        extras["served"] = served_leg(R, W, ctx)
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
                               "(seeds 3000-3015), plain RFR per polynomial",
                   "polys": len(polys), "degree": 100, "n_elements": ns,
                   "pairs_per_step": pairs_per_step, "keys_per_step": keys_per_step},
        "factorizations_per_s": len(polys) / (ms_per_step / 1000.0),
        "results_match_oracle": ok,
        "stage_ms_per_launch": {k: round(v, 4) for k, v in stage_avg.items()},
        "searches_per_launch": prof["searches"] / nlaunch,
        "stage_alg_gbs": stage_gbs,
        "roofline": roofline,
        "host": host_info(),
    }
    out.update(extras)
    if not args.no_cpu_baseline:
        cb, got = cpu_baseline(polys, ns)
        out["cpu_baseline"] = cb
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
