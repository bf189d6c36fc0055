"""Batching benchmark: 64 independent constant-k instances of mixed size
(n ~ U{127, 255, 511, 1023}, kh ~ U[0.3, 0.6]), 4 point-source right-hand
sides each, solved together with hmg_solve_batch, against solving the same
instances one after the other.

    python bench_batch.py [--count 64] [--nrhs 4] [--precision mixed|fp64]

HYB-V preconditioner, relative residual 1e-6, x0 = 0.  Prints one JSON line
per form with right-hand-side solves per second and node-RHS per second.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--nrhs", type=int, default=4)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--repeats", type=int, default=2)
    ap.add_argument("--maxit", type=int, default=2000)
    args = ap.parse_args()
    import numpy as np
    import torch
    torch.cuda.set_device(0)
    from paper_1312_2880_amd import hmg, inputs
    prec = hmg.MIXED if args.precision == "mixed" else hmg.FP64
    insts = inputs.batch_instances(seed=args.seed, count=args.count, nrhs=args.nrhs)
    ctx = hmg.Context(0)
    grids = [hmg.Grid(ctx, it["h"], it["k"], np.stack(it["f"]), precision=prec, variant=hmg.HYB)
             for it in insts]
    nodes = sum((it["n"] + 2) ** 2 for it in insts) * args.nrhs
    # warm-up: graph capture and tuning happen here
    ctx.solve_batch(grids, rtol=1e-6, maxit=args.maxit)
    for g in grids:
        g.solve(rtol=1e-6, maxit=args.maxit)
    torch.cuda.synchronize()
    for form in ("batched", "one-by-one"):
        best = None
        for _ in range(args.repeats):
            t0 = time.perf_counter()
            if form == "batched":
                _, infos = ctx.solve_batch(grids, rtol=1e-6, maxit=args.maxit)
            else:
                infos = [g.solve(rtol=1e-6, maxit=args.maxit)[1] for g in grids]
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        flat = [i for inf in infos for i in inf]
        bad = [i for i in flat if not (i["status"] == hmg.OK and i["rel_res_true"] <= 1e-6)]
        ok = not bad
        line = {"metric": "right-hand-side solves/s at rel. residual 1e-6, mixed-size batch",
                "form": form, "value": round(len(flat) / best, 3), "unit": "solves/s",
                "node_rhs_per_s": round(nodes / best, 1), "seconds": round(best, 4),
                "instances": args.count, "nrhs": args.nrhs,
                "mean_iters": round(sum(i["iters"] for i in flat) / len(flat), 2),
                "max_iters": max(i["iters"] for i in flat),
                "all_converged": ok, "not_converged": len(bad), "dtype": args.precision, "data": "synthetic",
                "config": {"sizes": [127, 255, 511, 1023], "kh": [0.3, 0.6], "variant": "HYB-V",
                           "seed": args.seed}}
        print(json.dumps(line), flush=True)
    for g in grids:
        g.close()
    ctx.close()


if __name__ == "__main__":
    main()
