"""Iteration-count study of Section 6.1 (Tables 1, 2 and a Table 3 analogue)
on the GPU.

    python study_tables.py [--variants SL-V,HYB-V,HLM-V] [--orders colour,lex]

Model problem: constant k on the unit square, unit point source at the
centre node, x0 = 0, stop at a 1e7 reduction of the residual, half
iterations counted.  Table 1 keeps kh = 0.625 (k = 40 ... 150 on h = 1/64 ...
1/240); Table 2 keeps k = 40 (h = 1/64 ... 1/512); the coarsest level is the
one with kH = 5.  The Table 3 rows use a wedge-type medium of own geometry
(the paper's is shown only in a missing figure): k_ref h = 15/64, k from
k_ref to 2 k_ref, source at the middle of the upper edge.  Each case runs with
the coloured sweeps of the default schedule and with the lexicographic sweeps
of Section 4.

Prints one JSON line per case and, at the end, a markdown table with the
paper's counts, the FP64 oracle's counts (tests/golden/oracle_table_counts.json,
written by tests/golden/make_table_counts.py) and this library's.  The paper's
boundary treatment and coarse-grid details are not given, so its counts are
context, not targets.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--variants", default="SL-V,HYB-V,HLM-V")
    ap.add_argument("--orders", default="colour,lex")
    ap.add_argument("--maxit", type=int, default=400)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    from paper_1312_2880_amd import hmg, inputs
    ref = json.load(open(os.path.join(GOLDEN, "oracle_table_counts.json")))
    paper = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))
    vcode = {"SL-V": hmg.SL, "HYB-V": hmg.HYB, "HLM-V": hmg.HLM}
    ocode = {"colour": hmg.ORDER_COLOUR, "lex": hmg.ORDER_LEX}
    rtol = ref["rtol"]
    ctx = hmg.Context(0)
    results = []
    for row in ref["rows"]:
        n, nc = row["n"], row["coarsest_n"]
        if row.get("medium") == "wedge":
            h, k, f = inputs.wedge_problem(n)
        else:
            h, k, f = inputs.grid_h(n), inputs.constant_k(n, float(row["k"])), inputs.centre_source(n)
        for vname in args.variants.split(","):
            for oname in args.orders.split(","):
                g = hmg.Grid(ctx, h, k, f, variant=vcode[vname], coarsest_n=nc, relax_order=ocode[oname])
                g.solve(rtol=rtol, maxit=args.maxit)          # warm-up (graph capture)
                t0 = time.perf_counter()
                _, info = g.solve(rtol=rtol, maxit=args.maxit)
                dt = time.perf_counter() - t0
                g.close()
                i0 = info[0]
                key = vname + ("-lex" if oname == "lex" else "")
                line = {"table": row["table"], "k": row["k"], "h": f"1/{row['N']}", "variant": vname,
                        "order": oname, "iters": i0["iters"], "converged": i0["status"] == hmg.OK,
                        "rel_res_true": i0["rel_res_true"], "ms_per_solve": round(1e3 * dt, 2),
                        "oracle_iters": row["counts"][key]["iters"],
                        "oracle_converged": row["counts"][key]["status"] == 0}
                results.append(line)
                print(json.dumps(line), flush=True)
    ctx.close()

    def paper_count(table, N, vname):
        t = paper[table]
        if vname not in t or f"1/{N}" not in t["h"]:
            return None
        return t[vname][t["h"].index(f"1/{N}")]

    print()
    print("| table | k (Table 3: k_ref) | h | variant | order | paper | oracle | GPU | GPU ms/solve |")
    print("|---|---:|---|---|---|---:|---:|---:|---:|")
    for r in results:
        N = int(r["h"].split("/")[1])
        pc = paper_count(r["table"], N, r["variant"])
        oc = f"{r['oracle_iters']}" + ("" if r["oracle_converged"] else " (no conv.)")
        gc = f"{r['iters']}" + ("" if r["converged"] else " (no conv.)")
        print(f"| {r['table'][-1]} | {r['k']} | {r['h']} | {r['variant']} | {r['order']} | "
              f"{'' if pc is None else pc} | {oc} | {gc} | {r['ms_per_solve']} |")


if __name__ == "__main__":
    main()
