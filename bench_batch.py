"""Batching benchmark: 64 independent constant-k instances of mixed size
(n ~ U{127, 255, 511, 1023}, kh ~ U[0.3, 0.6]), 4 point-source right-hand
sides each, solved together with hmg_solve_batch, against solving the same
instances one after the other (hmg_solve per instance: its four right-hand
sides in one launch per kernel) and against solving every right-hand side
alone (hmg_solve_dev per right-hand side: no batching at all).

    python bench_batch.py [--count 64] [--nrhs 4] [--precision mixed|fp64|both]

HYB-V preconditioner with M on the intermediate scales by default (HYB-V as
defined, --variant hyb, does not converge on the high-kh constant-k instances
of this mix; --variant sl runs SL-V), relative residual 1e-6, x0 = 0.  Prints a progress
line per phase and one JSON line per form with right-hand-side solves per
second and node-RHS per second.
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
    ap.add_argument("--precision", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--maxit", type=int, default=2000)
    ap.add_argument("--variant", choices=["sl", "hyb", "hyb-mid"], default="hyb-mid")
    args = ap.parse_args()
    import numpy as np
    import torch
    torch.cuda.set_device(0)
    from paper_1312_2880_amd import hmg, inputs
    insts = inputs.batch_instances(seed=args.seed, count=args.count, nrhs=args.nrhs)
    nodes = sum((it["n"] + 2) ** 2 for it in insts) * args.nrhs
    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    ctx = hmg.Context(0)
    vopts = {"sl": dict(variant=hmg.SL), "hyb": dict(variant=hmg.HYB),
             "hyb-mid": dict(variant=hmg.HYB, hyb_mid=1)}[args.variant]
    vname = {"sl": "SL-V", "hyb": "HYB-V", "hyb-mid": "HYB-V, M on the intermediate scales"}[args.variant]
    for pname in precs:
        prec = hmg.MIXED if pname == "mixed" else hmg.FP64
        t0 = time.perf_counter()
        grids = [hmg.Grid(ctx, it["h"], it["k"], np.stack(it["f"]), precision=prec, **vopts)
                 for it in insts]
        print(f"# {pname}: {len(grids)} grids created in {time.perf_counter() - t0:.1f} s", flush=True)
        dev_f = [[torch.from_numpy(np.ascontiguousarray(fr)).to("cuda") for fr in it["f"]] for it in insts]
        for form in ("batched", "one-by-one", "one-rhs-at-a-time"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if form == "batched":
                _, infos = ctx.solve_batch(grids, rtol=1e-6, maxit=args.maxit)
            elif form == "one-by-one":
                infos = []
                for q, g in enumerate(grids):
                    infos.append(g.solve(rtol=1e-6, maxit=args.maxit)[1])
                    if q % 16 == 15:
                        print(f"# {pname} one-by-one: {q + 1} instances", flush=True)
            else:
                infos = []
                for q, g in enumerate(grids):
                    row = []
                    for r, d_b in enumerate(dev_f[q]):
                        d_x = torch.zeros_like(d_b)
                        row.append(g.solve_dev(d_x, d_b=d_b, rhs=r, rtol=1e-6, maxit=args.maxit))
                    infos.append(row)
                    if q % 16 == 15:
                        print(f"# {pname} one rhs at a time: {q + 1} instances", flush=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            flat = [i for inf in infos for i in inf]
            bad = [i for i in flat if not (i["status"] == hmg.OK and i["rel_res_true"] <= 1e-6)]
            for q, inf in enumerate(infos):
                for r, i in enumerate(inf):
                    if not (i["status"] == hmg.OK and i["rel_res_true"] <= 1e-6):
                        print(f"# not converged: instance {q} n={insts[q]['n']} kh={insts[q]['kh']:.3f} "
                              f"rhs {r}: iters {i['iters']} status {i['status']} "
                              f"rel_res_true {i['rel_res_true']:.3e} restarts {i['restarts']}", flush=True)
            line = {"metric": "right-hand-side solves/s at rel. residual 1e-6, mixed-size batch",
                    "form": form, "precision": pname, "value": round(len(flat) / dt, 3), "unit": "solves/s",
                    "node_rhs_per_s": round(nodes / dt, 1), "seconds": round(dt, 3),
                    "instances": args.count, "nrhs": args.nrhs,
                    "mean_iters": round(sum(i["iters"] for i in flat) / len(flat), 2),
                    "max_iters": max(i["iters"] for i in flat),
                    "all_converged": not bad, "not_converged": len(bad), "data": "synthetic",
                    "config": {"sizes": [127, 255, 511, 1023], "kh": [0.3, 0.6], "variant": vname,
                               "seed": args.seed, "maxit": args.maxit}}
            print(json.dumps(line), flush=True)
        for g in grids:
            g.close()
    ctx.close()


if __name__ == "__main__":
    main()
