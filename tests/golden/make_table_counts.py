"""Writes oracle_table_counts.json: Bi-CGSTAB iteration counts of the FP64
oracle on the model problem of Section 6.1 (Tables 1 and 2): constant k on
the unit square, unit point source at the centre node, x0 = 0, stop at a
1e7 reduction of the residual, half iterations counted.

    python tests/golden/make_table_counts.py        (about two minutes)

Rows: Table 1 (kh = 0.625: k = 40, 50, 80, 100, 150 on h = 1/64, 1/80,
1/128, 1/160, 1/240) and Table 2 (k = 40 on h = 1/128, 1/256, 1/512; 1/64 is
Table 1's first row).  The coarsest level is the one with kH = 5 in every
row (n_c = 7, 9, 15, 19, 29), so each row has the same level sequence in kH
(0.625, 1.25, 2.5, 5 for Table 1).  Columns: SL-V, HYB-V and HLM-V, each with
the coloured sweeps and with the lexicographic sweeps of Section 4.  At most
400 iterations (HLM-V does not converge on these problems).

Only the oracle is called.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1312_2880_amd import inputs  # noqa: E402

ROWS = [  # table, k, intervals N = 1/h, coarsest n
    ("table1", 40, 64, 7), ("table1", 50, 80, 9), ("table1", 80, 128, 15),
    ("table1", 100, 160, 19), ("table1", 150, 240, 29),
    ("table2", 40, 128, 7), ("table2", 40, 256, 7), ("table2", 40, 512, 7),
]
VARIANTS = (("SL-V", oracle.SL), ("HYB-V", oracle.HYB), ("HLM-V", oracle.HLM))
RTOL, MAXIT = 1e-7, 400


def main():
    out = {"rtol": RTOL, "maxit": MAXIT, "source": "oracle (FP64, this repository)", "rows": []}
    for table, k0, N, nc in ROWS:
        n = N - 1
        h, k, f = inputs.grid_h(n), inputs.constant_k(n, float(k0)), inputs.centre_source(n)
        row = {"table": table, "k": k0, "N": N, "n": n, "coarsest_n": nc, "counts": {}}
        for vname, v in VARIANTS:
            for order, tag in ((0, ""), (1, "-lex")):
                t0 = time.time()
                g = oracle.Grid(h, k, variant=v, coarsest_n=nc, gs_order=order, kacz_order=order)
                _, info = g.bicgstab(f, rtol=RTOL, maxit=MAXIT)
                row["counts"][vname + tag] = {"iters": info["iters"], "status": info["status"],
                                              "seconds": round(time.time() - t0, 2)}
            row["levels"] = [p["n"] for p in g.plan()]
        print(table, k0, N, {key: val["iters"] for key, val in row["counts"].items()}, flush=True)
        out["rows"].append(row)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_table_counts.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
