"""Write expected factorisations for the seeded workloads using the oracle only.

Usage:  python tests/golden/make_golden.py [large|mid|batch|stream|flood] ...

Each output file maps the workload seed to the oracle's (content, factors) for
that seeded input; nothing here touches the HIP library.
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import rfr_ref as R  # noqa: E402
import workloads as W  # noqa: E402


def _one(args):
    seed, coeffs = args
    t0 = time.time()
    cont, facs = R.factor_general(coeffs)
    return seed, {"coeffs": coeffs, "content": cont, "factors": [list(f) for f in facs],
                  "oracle_s": round(time.time() - t0, 2)}


def _one_traced(args):
    """As _one, for a square-free input, with the oracle's candidate counts:
    patterns whose first trace is in the window, and those whose second is too."""
    seed, coeffs = args
    t0 = time.time()
    tr = R.Trace()
    cont, facs = R.factor(coeffs, tr)
    return seed, {"coeffs": coeffs, "content": cont, "factors": [list(f) for f in facs],
                  "n": tr.n, "tr1_candidates": len(tr.candidates), "tr2_candidates": len(tr.tr2_kept),
                  "oracle_s": round(time.time() - t0, 2)}


def build(name):
    if name == "large":
        ws, procs = W.config_large(), 3
    elif name == "mid":
        ws, procs = W.config_mid(), 6
    elif name == "batch":
        ws, procs = W.config_batch()[::32], 6
    elif name == "stream":
        # the served-mode test's requests (degrees up to 116) and the inputs
        # with repeated factors that ride in the same stream; largest first,
        # few at a time (the oracle's halves reach 2^29 sums)
        ws = [r.work for r in W.config_stream(48, rate_per_s=400.0)] + W.config_repeated(6)
        ws.sort(key=lambda w: -w.degree)
        procs = 3
    elif name == "flood":
        ws, procs = W.config_flood(), 2
    else:
        raise SystemExit("unknown set " + name)
    jobs = [(w.seed, w.coeffs) for w in ws]
    with mp.Pool(procs) as pool:
        res = dict(pool.map(_one_traced if name == "flood" else _one, jobs, chunksize=1))
    out = {"_source": "oracle/rfr_ref.py factor_general() on workloads.config_%s" % name,
           "cases": {str(k): res[k] for k in sorted(res)}}
    path = os.path.join(HERE, "golden_%s.json" % name)
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path, len(res))


if __name__ == "__main__":
    for n in sys.argv[1:] or ["mid", "large", "batch"]:
        build(n)
