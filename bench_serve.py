"""Serving benchmark: a Poisson stream of layered-medium solves of mixed
sizes through the request server (continuous batching, admission by device
footprint), against the same stream served one request at a time in FP64.

    python bench_serve.py [--rates 5,50,200] [--count 30] [--warmup 4]

Each request: n ~ U{255, 511, 1023, 2047}, a seeded layered medium with
omega = 2 pi 40 (n+1)/1024 (max kh fixed), one seeded point source, HYB-V
preconditioner with M on the intermediate scales (--variant hyb: HYB-V as
defined, --variant sl: SL-V), relative residual 1e-6.  The served form runs the V-cycle in
complex float under the FP64 Bi-CGSTAB; the baseline runs plain FP64 with at
most one request in flight.  Latency = completion time - submission time on
the library's clock.  Prints one JSON line per (form, rate); the served FP64
form separates the scheduler's effect from the precision's.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    pos = q / 100.0 * (len(xs) - 1)
    lo = int(pos)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (pos - lo)


def make_requests(rate, count, warmup, seed):
    from paper_1312_2880_amd import inputs
    stream = inputs.request_stream(seed=seed, rate=rate, count=count + warmup)
    cache = {}
    reqs = []
    for r in stream:
        key = (r["seed"], r["n"])
        if key not in cache:
            med = inputs.LayeredMedium(r["seed"])
            cache[key] = (inputs.grid_h(r["n"]), med.k(r["n"], r["omega"]), med.source(r["n"]))
        h, k, f = cache[key]
        reqs.append(dict(t=r["t_arrive"], n=r["n"], h=h, k=k, f=f))
    return reqs


def serve(hmg, reqs, precision, max_active, warmup, maxit, vopts):
    ctx = hmg.Context(0)
    ctx.set_max_active(max_active)
    tickets = [None] * len(reqs)
    results = {}
    t0 = time.perf_counter()

    def submitter():
        for q, r in enumerate(reqs):
            delay = r["t"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets[q] = ctx.submit(n=r["n"], h=r["h"], k=r["k"], f=r["f"], rtol=1e-6,
                                    maxit=maxit, precision=precision, **vopts)

    th = threading.Thread(target=submitter)
    th.start()
    while len(results) < len(reqs):
        for q, t in enumerate(tickets):
            if t is None or q in results:
                continue
            res = ctx.poll(t)
            if res is not None:
                results[q] = res[1]
                if len(results) % 8 == 0:
                    print(f"# {len(results)}/{len(reqs)} requests done", flush=True)
        time.sleep(0.0005)
    th.join()
    ctx.close()
    timed = [results[q] for q in range(warmup, len(reqs))]
    lat = [r["t_done"] - r["t_arrive"] for r in timed]
    span = max(r["t_done"] for r in timed) - min(r["t_arrive"] for r in timed)
    return dict(
        solves=len(timed), value=len(timed) / span, p50_s=percentile(lat, 50),
        p99_s=percentile(lat, 99), mean_iters=sum(r["iters"] for r in timed) / len(timed),
        all_converged=all(r["status"] == hmg.OK and r["rel_res_true"] <= 1e-6 for r in timed),
        max_iters=max(r["iters"] for r in timed),
        mean_queue_s=sum(r["t_admit"] - r["t_arrive"] for r in timed) / len(timed))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="5,50,200")
    ap.add_argument("--count", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--max-active", type=int, default=0)
    ap.add_argument("--maxit", type=int, default=3000)
    ap.add_argument("--variant", choices=["sl", "hyb", "hyb-mid"], default="hyb-mid")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    from paper_1312_2880_amd import hmg
    vopts = {"sl": dict(variant=hmg.SL), "hyb": dict(variant=hmg.HYB),
             "hyb-mid": dict(variant=hmg.HYB, hyb_mid=1)}[args.variant]
    vname = {"sl": "SL-V", "hyb": "HYB-V", "hyb-mid": "HYB-V, M on the intermediate scales"}[args.variant]
    for rate in [float(x) for x in args.rates.split(",")]:
        reqs = make_requests(rate, args.count, args.warmup, args.seed)
        for form, prec, act in (("served-fp64", hmg.FP64, args.max_active),
                                ("served-mixed", hmg.MIXED, args.max_active),
                                ("serial-fp64", hmg.FP64, 1)):
            out = serve(hmg, reqs, prec, act, args.warmup, args.maxit, vopts)
            line = {"metric": "solves/s and p50/p99 latency, Poisson request stream",
                    "form": form, "rate_req_s": rate, "unit": "solves/s",
                    "value": round(out["value"], 3),
                    "p50_ms": round(1e3 * out["p50_s"], 2), "p99_ms": round(1e3 * out["p99_s"], 2),
                    "mean_queue_ms": round(1e3 * out["mean_queue_s"], 2),
                    "mean_iters": round(out["mean_iters"], 2), "max_iters": out["max_iters"],
                    "solves": out["solves"],
                    "all_converged": out["all_converged"], "data": "synthetic",
                    "config": {"sizes": [255, 511, 1023, 2047], "variant": vname,
                               "seed": args.seed, "rtol": 1e-6}}
            print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
