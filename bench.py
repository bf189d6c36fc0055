"""Benchmark: preconditioned Bi-CGSTAB solves of the 1023^2 layered-medium
Helmholtz problem (HYB-V preconditioner, FP64) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|mixed]

One step is one full solve to relative residual 1e-6 from x0 = 0, with k, f
and the hierarchy already resident in device memory.  Prints one JSON line
with solves/s, the roofline figure of the dominant V-cycle kernel (timed with
HIP events on the stream it runs on) and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1312_2880_amd", "csrc", "hmg_fused.hip")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def algorithmic_bytes(kind: str, nodes: int, coarse_nodes: int, cbytes: int, rbytes: int) -> float:
    """Bytes the method must move per launch, every array touched once
    (c = complex size, r = real size of the level precision; per fine node,
    plus c per coarse node where a coarse field is read or written):
      gs_down     read f, k; write coarse f                N (c + r) + Nc c
      gs_up       read f, k, coarse e; write u              N (2c + r) + Nc c
    (the pre-smoothed iterate is recomputed on chip, never stored)
    """
    c, r = cbytes, rbytes
    if kind == "gs_down":
        return nodes * (c + r) + coarse_nodes * c
    if kind == "gs_up":
        return nodes * (2 * c + r) + coarse_nodes * c
    raise KeyError(kind)


def time_kernels(hmg, torch, g, plan, precision, reps=96, sets=24):
    """Average launch duration of the finest-level V-cycle kernels, timed with
    torch events on torch's current stream (the library launches on the
    stream it is given).  Launches cycle through `sets` independent buffer
    sets (about 1 GB in total) so that each one reads its inputs from HBM, not
    from the Infinity Cache."""
    # a dedicated stream: torch's default stream has the NULL handle, which the
    # library reads as "the grid's own stream", and events on it would not
    # bracket the kernels
    stream = torch.cuda.Stream()
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    cb, rb = (16, 8) if precision == "fp64" else (8, 4)
    n0, nc = plan[0]["n"], plan[1]["n"]
    nodes, cnodes = (n0 + 2) ** 2, (nc + 2) ** 2
    gen = torch.Generator(device="cuda").manual_seed(0)

    def field(n):
        return torch.randn((n + 2, n + 2), dtype=cdt, device="cuda", generator=gen)

    bufs = [dict(f=field(n0), uo=field(n0), ec=field(nc), fc=field(nc))
            for _ in range(sets)]
    torch.cuda.synchronize()
    sa, sb = plan[0]["sigma_relax"], plan[0]["sigma_resid"]
    cases = {
        "gs_down": lambda b: g.op_gs_down(0, sa, sb, b["f"], None, b["fc"], stream),
        "gs_up": lambda b: g.op_gs_up(0, sa, b["f"], b["ec"], b["uo"], stream),
    }
    out = {}
    for name, fn in cases.items():
        for q in range(sets):
            fn(bufs[q])
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for q in range(reps):
            fn(bufs[q % sets])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        b = algorithmic_bytes(name, nodes, cnodes, cb, rb)
        out[name] = dict(ms_per_launch=ms, bytes=b, gbs=b / (ms * 1e-3) / 1e9, nodes=nodes)
    del bufs
    return out


def cpu_baseline(h, k, f, variant, budget_s=30.0):
    """The FP64 oracle on the host cores: one full solve of the same problem
    (bounded: the solve is cut at the iteration count that fits the budget
    and the rate extrapolated per full solve)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    og = oracle.Grid(h, k, variant=variant)
    t0 = time.perf_counter()
    _, info = og.bicgstab(f, rtol=1e-6, maxit=400)
    dt = time.perf_counter() - t0
    return dict(value=1.0 / dt, unit="solves/s", cores=threads, kind="oracle",
                sample=f"one full FP64 solve of the same problem on {threads} threads "
                       f"({info['iters']} iterations, {dt:.1f} s)",
                iters=info["iters"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--maxit", type=int, default=400)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   "multi-GPU sharding is not part of this build",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1312_2880_amd import hmg, inputs

    torch.cuda.set_device(0)
    h, k, f = inputs.workload_layered_1023()
    n = k.shape[0] - 2
    prec = hmg.FP64 if args.precision == "fp64" else hmg.MIXED
    ctx = hmg.Context(0)
    g = hmg.Grid(ctx, h, k, f, variant=hmg.HYB, precision=prec)
    plan = g.plan()
    stream = torch.cuda.current_stream()
    d_b = torch.from_numpy(f).to("cuda")
    d_x = torch.zeros_like(d_b)

    infos = []
    for _ in range(args.warmup):
        infos.append(g.solve_dev(d_x, d_b=d_b, rtol=1e-6, maxit=args.maxit, stream=stream))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(g.solve_dev(d_x, d_b=d_b, rtol=1e-6, maxit=args.maxit, stream=stream))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    last = infos[-1]
    ok = all(i["status"] == hmg.OK and i["rel_res_true"] <= 1e-6 for i in infos)

    kt = time_kernels(hmg, torch, g, plan, args.precision)
    # dominant V-cycle kernel: the finest-level kernel with the longest launch
    dom = max(kt, key=lambda name: kt[name]["ms_per_launch"])
    d = kt[dom]
    achieved = d["gbs"]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            tr = json.load(open(TRAFFIC_FILE))
            ent = tr.get(f"{dom}:{args.precision}")
            if ent and ent.get("kernel_source_hash") == kernel_source_hash():
                traffic = ent.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom, "level_nodes": d["nodes"],
                "ms_per_launch": round(d["ms_per_launch"], 5),
                "bytes_per_launch": d["bytes"]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(h, k, f, 2)
        cpu = {k_: (round(v, 5) if isinstance(v, float) else v) for k_, v in cpu.items()}

    line = {
        "metric": "solves/s at rel. residual 1e-6",
        "value": round(args.steps / dt, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if args.precision == "fp64" else "c64/c128",
        "data": "synthetic",
        "config": {"workload": "layered-medium Helmholtz 1023x1023, omega = 2 pi 40, "
                               "HYB-V preconditioned Bi-CGSTAB to 1e-6, seed 2",
                   "n": n, "precision": args.precision,
                   "iters": last["iters"], "rel_res_true": last["rel_res_true"],
                   "all_converged": ok,
                   "levels": [(p["n"], p["smoother"]) for p in plan]},
        "roofline": roofline,
        "kernels": {name: {"ms_per_launch": round(v["ms_per_launch"], 5),
                           "gbs": round(v["gbs"], 1)} for name, v in kt.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    g.close()
    ctx.close()


if __name__ == "__main__":
    main()
