"""Benchmark: preconditioned Bi-CGSTAB solves of the 2047^2 layered-medium
Helmholtz problem (omega = 2 pi 80, HYB-V preconditioner, FP64) on one
MI355X; the same problem with the complex-float preconditioner is reported
beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 2047|1023]
                    [--precision fp64|mixed] [--variant hyb|sl] [--order colour|lex]

(--order lex runs every relaxation in lexicographic order, the sweeps as
wavefronts; the timed kernels are then one sweep per level.)

One step is one full solve to relative residual 1e-6 from x0 = 0, with k, f
and the hierarchy already resident in device memory.  Prints one JSON line
with solves/s, the roofline figure of the dominant V-cycle kernel (its share
of the solve time is the largest; timed with HIP events on the stream it runs
on, rated against its algorithmic HBM bytes), the mixed-precision solve of the
same problem, and the CPU oracle timed per iteration on the same problem.
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


FP64_PEAK_TFLOPS = 78.6       # MI355X FP64 vector, vendor figure
KACZ_ROW_FLOPS = 50           # one Kaczmarz row update, real flops
GS_NODE_FLOPS = 28            # one Gauss-Seidel node update, real flops


def algorithmic_bytes(kind: str, nodes: int, coarse_nodes: int, cbytes: int, rbytes: int,
                      stored_u0: bool = False, sweeps: int = 1) -> float:
    """Bytes the method must move per launch, every array touched once
    (c = complex size, r = real size of the level precision; per fine node,
    plus c per coarse node where a coarse field is read or written):
      gs_down     read f, k; write coarse f (+ write u0)     N (c + r) + Nc c   (+ N c)
      gs_up       read f, k, coarse e (+ read u0 on the      N (2c + r) + Nc c  (+ N c / 2)
                  black nodes); write u
      gs_up_mv    gs_up without u0 and without storing u,    N (3c + r) + Nc c
                  then read the inner product's other
                  vector, write L u (as the FP64 solve
                  runs it)
      kacz_tb     S sweeps, each reading f, k, u and         S N (3c + r)
                  writing u (the per-sweep minimum)
    (FP64 levels store the pre-smoothed iterate u0 for the up kernel, which
    needs it on the black nodes only: the red half-sweep overwrites red
    values unread; complex-float levels recompute it on chip)
    """
    c, r = cbytes, rbytes
    if kind == "gs_down":
        return nodes * (c + r) + coarse_nodes * c + (nodes * c if stored_u0 else 0)
    if kind == "gs_up":
        return nodes * (2 * c + r) + coarse_nodes * c + (nodes * c // 2 if stored_u0 else 0)
    if kind == "gs_up_mv":
        return nodes * (3 * c + r) + coarse_nodes * c
    if kind == "kacz_tb":
        return sweeps * nodes * (3 * c + r)
    raise KeyError(kind)


def vcycle_model_bytes(plan, cbytes: int, rbytes: int) -> float:
    """Bytes one V-cycle must move by the per-level model (c, r as above;
    N nodes of the level, its coarse nodes N/4): a relaxation sweep from
    zero reads f, k and writes u (2c + r), any other sweep also reads u
    (3c + r); the residual with full weighting reads f, k, u and writes
    the coarse right-hand side (2c + r + c/4); the correction reads the
    coarse error and u and writes u (2c + c/4).  A V(1,1) Gauss-Seidel level
    is then N (9.5c + 3r), a 4+4 Kaczmarz level N (27.5c + 9r); the dense
    coarsest level is not counted."""
    c, r = cbytes, rbytes
    tot = 0.0
    for p in plan:
        sweeps = p["pre"] + p["post"]
        if p["smoother"] not in ("GS", "KACZ") or sweeps == 0:
            continue
        nodes = (p["n"] + 2) ** 2
        tot += nodes * ((2 * c + r) + (sweeps - 1) * (3 * c + r) + (2 * c + r + c / 4) + (2 * c + c / 4))
    return tot


def time_vcycle(torch, g, plan, precision, sets=8, count=16):
    """One V-cycle through the C-ABI (hmg_vcycle_dev) on FP64 fields, as
    graph replays over `sets` input/output pairs (about 1 GB at 2047^2, so
    that the finest level reads from HBM), rated on vcycle_model_bytes."""
    n = plan[0]["n"]
    gen = torch.Generator(device="cuda").manual_seed(1)
    rs = [torch.randn((n + 2, n + 2), dtype=torch.complex128, device="cuda", generator=gen) for _ in range(sets)]
    zs = [torch.empty_like(rs[0]) for _ in range(sets)]
    stream = torch.cuda.Stream()
    ms = graph_time(torch, stream, lambda q: g.vcycle_dev(rs[q % sets], zs[q % sets], stream=stream), count)
    cb, rb = (16, 8) if precision == "fp64" else (8, 4)
    model = vcycle_model_bytes(plan, cb, rb)
    achieved = model / (ms * 1e-3) / 1e9
    return {"ms": round(ms, 5), "bytes_model": round(model), "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}


def copy_bandwidth(torch, nbytes=4 << 30, reps=5):
    """Attained bandwidth of a plain device-to-device copy of nbytes (read
    plus write counted, as STREAM does), best of reps, HIP events."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return {"bytes": 2 * nbytes, "ms": round(best, 4), "achieved": round(2 * nbytes / (best * 1e-3) / 1e9, 1),
            "unit": "GB/s", "frac": round(2 * nbytes / (best * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def graph_time(torch, stream, fn, count, reps=3):
    """Average duration of one launch of fn: `count` launches are captured
    into one HIP graph on `stream` and replayed, bracketed by HIP events on
    that stream (so host launch gaps are not counted)."""
    for q in range(count):
        fn(q)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream, capture_error_mode="relaxed"):
        for q in range(count):
            fn(q)
    with torch.cuda.stream(stream):
        graph.replay()
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        with torch.cuda.stream(stream):
            graph.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / count
        best = ms if best is None else min(best, ms)
    del graph
    return best


def lex_cases(g, plan, field, cb, rb):
    """Lexicographic sweeps (one call = one sweep = one launch per tile
    diagonal) on every relaxation level: (name, level, sweep(q), sweeps per
    V-cycle, roofline model, None)."""
    from paper_1312_2880_amd import hmg
    out = []
    for l, p in enumerate(plan):
        if p["smoother"] == "LU":
            continue
        n, kacz = p["n"], p["smoother"] == "KACZ"
        kb = [dict(f=field(n), u=field(n)) for _ in range(2)]
        sm, sig = (hmg.SM_KACZ if kacz else hmg.SM_GS), p["sigma_relax"]
        flops = (KACZ_ROW_FLOPS if kacz else GS_NODE_FLOPS) * (n + 2) ** 2
        out.append(("lex_kacz" if kacz else "lex_gs", l,
                    lambda q, st, l=l, sm=sm, sig=sig, kb=kb: g.op_smooth_lex(
                        l, sm, sig, 1, 0, kb[q % 2]["f"], kb[q % 2]["u"], st),
                    p["pre"] + p["post"],
                    ("alu", flops, algorithmic_bytes("kacz_tb", (n + 2) ** 2, 0, cb, rb)), None))
    return out


def kernel_cases(torch, g, plan, precision, sets=24, fixed=None, lex=False):
    """The V-cycle kernels timed by the benchmark, as closures over device
    buffers shaped like the solve's: (name, level, launch(q), launches per
    V-cycle, roofline model).  The finest-level Gauss-Seidel kernels cycle
    through `sets` buffer sets (about 1 GB) so that they read from HBM."""
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    cb, rb = (16, 8) if precision == "fp64" else (8, 4)
    gen = torch.Generator(device="cuda").manual_seed(0)

    def field(n):
        return torch.randn((n + 2, n + 2), dtype=cdt, device="cuda", generator=gen)

    if lex:
        return lex_cases(g, plan, field, cb, rb)
    out = []
    n0, nc = plan[0]["n"], plan[1]["n"]
    nodes, cnodes = (n0 + 2) ** 2, (nc + 2) ** 2
    if plan[0]["smoother"] == "GS" and plan[0]["pre"] == 1 and plan[0]["post"] == 1:
        # the kernels as the solve runs them: FP64 levels with n <= 511 store
        # u0 in the down kernel and read it in the up kernel
        st_u0 = precision == "fp64" and n0 <= 511
        # larger FP64 levels: the up kernel also forms the Bi-CGSTAB product
        # (alternately the alpha and the omega form, as a solve does)
        mv = precision == "fp64" and n0 > 511
        bufs = [dict(f=field(n0), u0=field(n0), uo=field(n0), ec=field(nc), fc=field(nc)) for _ in range(sets)]
        if mv:
            for b in bufs:
                b.update(mv=field(n0), dot=field(n0))
        sa, sb = plan[0]["sigma_relax"], plan[0]["sigma_resid"]
        out.append(("gs_down", 0, lambda q, st: g.op_gs_down(0, sa, sb, bufs[q % sets]["f"],
                                                             bufs[q % sets]["u0"] if st_u0 else None,
                                                             bufs[q % sets]["fc"], st), 1,
                    ("hbm", algorithmic_bytes("gs_down", nodes, cnodes, cb, rb, st_u0)), None))
        if mv:
            out.append(("gs_up_mv", 0, lambda q, st: g.op_gs_up_product(
                0, sa, 1 + q % 2, bufs[q % sets]["f"], bufs[q % sets]["ec"], None,
                bufs[q % sets]["mv"], bufs[q % sets]["dot"], None, st), 1,
                ("hbm", algorithmic_bytes("gs_up_mv", nodes, cnodes, cb, rb)), None))
        else:
            out.append(("gs_up", 0, lambda q, st: g.op_gs_up(0, sa, bufs[q % sets]["f"], bufs[q % sets]["ec"],
                                                             bufs[q % sets]["uo"], st,
                                                             d_u0=bufs[q % sets]["u0"] if st_u0 else None), 1,
                        ("hbm", algorithmic_bytes("gs_up", nodes, cnodes, cb, rb, st_u0)), None))
    for l, p in enumerate(plan):
        cfg = g.kacz_config(l)
        if cfg < 0:
            continue
        if fixed:
            cfg = fixed[l]
        n = p["n"]
        kb = [dict(f=field(n), u=field(n), uo=field(n)) for _ in range(4)]
        sig = p["sigma_relax"]
        if cfg >= len(hmg_configs()):
            # the whole level in one workgroup: one launch per leg
            out.append(("kacz_level", l,
                        lambda q, st, l=l, sig=sig, p=p, kb=kb: g.op_kacz_level(
                            l, sig, 0.0, p["pre"], kb[q % 4]["f"], kb[q % 4]["u"], None, kb[q % 4]["uo"], None,
                            st),
                        2, ("hbm", algorithmic_bytes("kacz_tb", (n + 2) ** 2, 0, cb, rb, sweeps=p["pre"]),
                            KACZ_ROW_FLOPS * p["pre"] * (n + 2) ** 2), cfg))
            continue
        tile, sweeps, _ = hmg_configs()[cfg]
        out.append(("kacz_tb", l,
                    lambda q, st, l=l, sig=sig, cfg=cfg, kb=kb: g.op_kacz_tiled(
                        l, sig, cfg, kb[q % 4]["f"], kb[q % 4]["u"], None, kb[q % 4]["uo"], st),
                    (p["pre"] + p["post"]) // sweeps,
                    ("hbm", algorithmic_bytes("kacz_tb", (n + 2) ** 2, 0, cb, rb, sweeps=sweeps),
                     KACZ_ROW_FLOPS * sweeps * (n + 2) ** 2), cfg))
    return out


def hmg_configs():
    from paper_1312_2880_amd import hmg
    return hmg.kacz_tile_configs()


def roofline_of(model, ms):
    if model[0] == "hbm":
        achieved = model[1] / (ms * 1e-3) / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4)}
        if len(model) > 2:   # the Kaczmarz row arithmetic, for reference
            out["fp64_tflops"] = round(model[2] / (ms * 1e-3) / 1e12, 4)
        return out
    achieved = model[1] / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 5),
            "hbm_equiv_gbs": round(model[2] / (ms * 1e-3) / 1e9, 1)}


def time_kernels(torch, g, plan, precision, only=None, fixed=None, lex=False):
    stream = torch.cuda.Stream()
    res = []
    for name, level, fn, per_vc, model, cfg in kernel_cases(torch, g, plan, precision, fixed=fixed, lex=lex):
        key = f"{name}@{plan[level]['n']}"
        if only and key != only:
            continue
        ms = graph_time(torch, stream, lambda q: fn(q, stream), 8 if lex else 48)
        res.append(dict(key=key, name=name, level=level, ms=ms, per_vcycle=per_vc, model=model, cfg=cfg))
    torch.cuda.synchronize()
    return res


COPY_BYTES = 512 << 20


def traffic_probe(torch, g, plan, precision, which, fixed, lex=False):
    """Launches kernel `which` (e.g. "kacz_tb@127") as the timing does, then
    copies COPY_BYTES device to device three times (the counter reference)."""
    kt = time_kernels(torch, g, plan, precision, only=which, fixed=fixed, lex=lex)
    if not kt:
        raise SystemExit(f"no kernel {which}")
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_probe": which, "copy_bytes": COPY_BYTES,
                      "kernel_ms": round(kt[0]["ms"], 5)}), flush=True)


ORACLE_COUNTS = os.path.join(ROOT, "tests", "golden", "oracle_counts.json")


def cpu_baseline(h, k, f, variant, n, lex=False, budget_s=12.0):
    """The FP64 oracle on the host cores, on the same problem.  A full
    oracle solve of the 2047^2 problem takes minutes, so the sample is a
    bounded number of Bi-CGSTAB iterations from x0 = 0 (the first call also
    builds the hierarchy, outside the timing): seconds per iteration, times
    the oracle's own iteration count for the whole solve (stored by
    tests/golden/make_oracle_counts.py, which calls only the oracle), gives
    solves/s.  Timed with all host threads and with one."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    order = 1 if lex else 0
    og = oracle.Grid(h, k, variant=variant, gs_order=order, kacz_order=order)
    count_key = f"layered{n}_{'hyb' if variant == oracle.HYB else 'sl'}"
    counts = json.load(open(ORACLE_COUNTS)) if os.path.exists(ORACLE_COUNTS) else {}
    full = counts.get(count_key, {}).get("iters")

    def per_iteration(nthreads, budget):
        oracle.set_threads(nthreads)
        its = 2
        t0 = time.perf_counter()
        og.bicgstab(f, rtol=1e-30, maxit=its)
        dt = time.perf_counter() - t0
        # grow the sample to about `budget` seconds
        more = max(0, min(200, int(budget / max(dt / its, 1e-6)) - its))
        if more:
            t0 = time.perf_counter()
            og.bicgstab(f, rtol=1e-30, maxit=more)
            dt, its = time.perf_counter() - t0, more
        return dt / its, its

    t_all, it_all = per_iteration(threads, budget_s)
    t_one, it_one = per_iteration(1, budget_s / 2)
    oracle.set_threads(threads)
    out = dict(unit="solves/s", cores=threads, kind="oracle",
               s_per_iter=t_all, s_per_iter_1thread=t_one, oracle_iters=full)
    if full:
        out["value"] = 1.0 / (t_all * full)
        out["value_1thread"] = 1.0 / (t_one * full)
    else:
        out["value"] = None
    out["sample"] = (f"{it_all} FP64 oracle Bi-CGSTAB iterations of the same {n}^2 problem on {threads} threads "
                     f"({t_all:.3f} s each) and {it_one} on 1 thread ({t_one:.3f} s each), times the oracle's "
                     f"full-solve count {full} (tests/golden/oracle_counts.json)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--maxit", type=int, default=3000)
    ap.add_argument("--n", type=int, choices=[1023, 2047], default=2047,
                    help="2047: the layered medium at omega = 2 pi 80 (the largest single-GPU "
                         "configuration, the benchmark); 1023: the same medium at omega = 2 pi 40")
    ap.add_argument("--mixed-fp64-levels", type=int, default=0,
                    help="finest levels kept in complex double in the mixed solve (0: all float)")
    ap.add_argument("--mixed-steps", type=int, default=2,
                    help="timed solves of the same problem with the complex-float preconditioner "
                         "(reported beside the FP64 figure; 0: skip)")
    ap.add_argument("--hyb-mid-steps", type=int, default=2,
                    help="timed solves of the same problem with HYB-V's intermediate-scales reading "
                         "(hmg_opts.hyb_mid = 1), reported beside the headline (0: skip)")
    ap.add_argument("--traffic-probe", default=None, metavar="KERNEL@N",
                    help="only launch this kernel (e.g. kacz_tb@127) as the timing does, then "
                         "a plain copy of known size, for the FETCH_SIZE / WRITE_SIZE runs")
    ap.add_argument("--variant", choices=["hyb", "sl"], default="hyb",
                    help="preconditioner (HYB-V: the benchmark; SL-V)")
    ap.add_argument("--order", choices=["colour", "lex"], default="colour",
                    help="relaxation order: coloured sweeps (the benchmark) or the lexicographic "
                         "sweeps of Section 4 (wavefronts, one-pass schedule)")
    ap.add_argument("--kacz-configs", default=None, metavar="C,C,...",
                    help="tile configuration per level for the tiled Kaczmarz levels (-1 elsewhere) "
                         "instead of tuning; counter runs pass the configurations the timed run "
                         "reported, since counters distort the tuner's timings")
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
    h, k, f = inputs.workload_layered_1023() if args.n == 1023 else inputs.workload_layered_2047()
    n = k.shape[0] - 2
    prec = hmg.FP64 if args.precision == "fp64" else hmg.MIXED
    ctx = hmg.Context(0)
    fixed = None
    if args.kacz_configs:
        fixed = [int(c) for c in args.kacz_configs.split(",")]
    lex = args.order == "lex"
    variant = hmg.HYB if args.variant == "hyb" else hmg.SL
    g = hmg.Grid(ctx, h, k, f, variant=variant, precision=prec, autotune=0 if fixed else 1,
                 relax_order=hmg.ORDER_LEX if lex else hmg.ORDER_COLOUR)
    plan = g.plan()
    if args.traffic_probe:
        traffic_probe(torch, g, plan, args.precision, args.traffic_probe, fixed, lex)
        g.close()
        ctx.close()
        return
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

    # the V-cycle kernels: per-launch time from graph replays, share of the
    # solve from launches per iteration (two V-cycles per Bi-CGSTAB iteration)
    kt = time_kernels(torch, g, plan, args.precision, lex=lex)
    mean_iters = sum(i["iters"] for i in infos[args.warmup:]) / args.steps
    it_ms = 1e3 * dt / args.steps / max(mean_iters, 0.5)
    for k_ in kt:
        k_["per_iter"] = 2 * k_["per_vcycle"]
        k_["share"] = k_["ms"] * k_["per_iter"] / it_ms
        k_["roofline"] = roofline_of(k_["model"], k_["ms"])
    dom = max(kt, key=lambda k_: k_["share"])
    # the whole V-cycle, rated on the per-level byte model
    vcycle = time_vcycle(torch, g, plan, args.precision) if not lex else None
    copy = copy_bandwidth(torch)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            tr = json.load(open(TRAFFIC_FILE))
            tkey = dom["key"] + (f"/cfg{dom['cfg']}" if dom["cfg"] is not None else "")
            ent = tr.get(f"{tkey}:{args.precision}")
            if ent and ent.get("kernel_source_hash") == kernel_source_hash():
                traffic = ent.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    roofline = dict(dom["roofline"])
    roofline.update({"traffic": traffic, "kernel": dom["key"], "config": dom["cfg"],
                     "ms_per_launch": round(dom["ms"], 5),
                     "per_launch": dom["model"][1], "share_of_solve": round(dom["share"], 3)})

    x_fp64 = d_x.cpu().numpy()
    mixed = None
    if args.mixed_steps > 0 and args.precision == "fp64":
        gm = hmg.Grid(ctx, h, k, f, variant=variant, precision=hmg.MIXED,
                      relax_order=hmg.ORDER_LEX if lex else hmg.ORDER_COLOUR,
                      fp64_levels=args.mixed_fp64_levels)
        d_xm = torch.zeros_like(d_b)
        minfo = [gm.solve_dev(d_xm, d_b=d_b, rtol=1e-6, maxit=args.maxit, stream=stream)]   # warm-up
        torch.cuda.synchronize()
        t0m = time.perf_counter()
        for _ in range(args.mixed_steps):
            minfo.append(gm.solve_dev(d_xm, d_b=d_b, rtol=1e-6, maxit=args.maxit, stream=stream))
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0m
        xm = d_xm.cpu().numpy()
        mixed = {"value": round(args.mixed_steps / dtm, 4), "unit": "solves/s",
                 "ms_per_step": round(1e3 * dtm / args.mixed_steps, 3),
                 "iters": minfo[-1]["iters"], "fp64_iters": last["iters"],
                 "rel_res_true": minfo[-1]["rel_res_true"],
                 "all_converged": all(i["status"] == hmg.OK and i["rel_res_true"] <= 1e-6 for i in minfo),
                 "rel_diff_vs_fp64": float(np.linalg.norm(xm - x_fp64) / np.linalg.norm(x_fp64)),
                 "fp64_levels": args.mixed_fp64_levels,
                 "precision": "complex-float V-cycle storage, FP64 arithmetic; FP64 outer Bi-CGSTAB"}
        gm.close()

    hyb_mid = None
    if args.hyb_mid_steps > 0 and args.variant == "hyb" and args.precision == "fp64" and not lex:
        gh = hmg.Grid(ctx, h, k, f, variant=variant, precision=prec, hyb_mid=1)
        d_xh = torch.zeros_like(d_b)
        hinfo = [gh.solve_dev(d_xh, d_b=d_b, rtol=1e-6, maxit=args.maxit, stream=stream)]   # warm-up
        torch.cuda.synchronize()
        t0h = time.perf_counter()
        for _ in range(args.hyb_mid_steps):
            hinfo.append(gh.solve_dev(d_xh, d_b=d_b, rtol=1e-6, maxit=args.maxit, stream=stream))
        torch.cuda.synchronize()
        dth = time.perf_counter() - t0h
        hyb_mid = {"value": round(args.hyb_mid_steps / dth, 4), "unit": "solves/s",
                   "ms_per_step": round(1e3 * dth / args.hyb_mid_steps, 3), "iters": hinfo[-1]["iters"],
                   "rel_res_true": hinfo[-1]["rel_res_true"],
                   "all_converged": all(i["status"] == hmg.OK and i["rel_res_true"] <= 1e-6 for i in hinfo),
                   "reading": "HYB-V with M for relaxation on the intermediate scales up to kH ~ 2.5 "
                              "(hmg_opts.hyb_mid = 1), FP64"}
        gh.close()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cpu = cpu_baseline(h, k, f, oracle.HYB if args.variant == "hyb" else oracle.SL, n, lex=lex)
        cpu = {k_: (round(v, 6) if isinstance(v, float) else v) for k_, v in cpu.items()}

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
        "config": {"workload": (f"layered-medium Helmholtz {n}x{n}, omega = 2 pi {40 * (n + 1) // 1024}, "
                                f"{args.variant.upper()}-V preconditioned Bi-CGSTAB to 1e-6, "
                                f"{'FP64' if args.precision == 'fp64' else 'complex-float V-cycle'}, seed 2"
                                + (", lexicographic sweeps" if lex else "")),
                   "n": n, "precision": args.precision,
                   "iters": last["iters"], "mean_iters": mean_iters, "rel_res_true": last["rel_res_true"],
                   "all_converged": ok,
                   "levels": [(p["n"], p["smoother"]) for p in plan],
                   "kacz_configs": ",".join(str(g.kacz_config(l)) for l in range(len(plan)))},
        "roofline": roofline,
        "kernels": {k_["key"]: {"ms_per_launch": round(k_["ms"], 5), "launches_per_iter": k_["per_iter"],
                                "share_of_solve": round(k_["share"], 3), **k_["roofline"]} for k_ in kt},
        "vcycle": vcycle,
        "copy_4gib": copy,
        "mixed": mixed,
        "hyb_mid": hyb_mid,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    g.close()
    ctx.close()


if __name__ == "__main__":
    main()
