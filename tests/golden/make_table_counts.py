"""Writes oracle_table_counts.json: Bi-CGSTAB iteration counts of the FP64
oracle on the model problems of Section 6.1 (Tables 1 and 2: constant k on
the unit square, unit point source at the centre node) and on a wedge-type
analogue of Table 3's medium; x0 = 0, stop at a 1e7 reduction of the
residual, half iterations counted.

    python tests/golden/make_table_counts.py        (about five minutes)

Rows: Table 1 (kh = 0.625: k = 40, 50, 80, 100, 150 on h = 1/64, 1/80,
1/128, 1/160, 1/240) and Table 2 (k = 40 on h = 1/128, 1/256, 1/512; 1/64 is
Table 1's first row).  The coarsest level is the one with kH = 5 in every
row (n_c = 7, 9, 15, 19, 29), so each row has the same level sequence in kH
(0.625, 1.25, 2.5, 5 for Table 1).  Table 3 analogue: the wedge-type medium
of paper_1312_2880_amd.inputs (k_ref h = 15/64, k_ref = 15, 30, 60, 120 on
h = 1/64 ... 1/512, source at the middle of the upper edge), the coarsest
level the one whose largest kH lies in [3.75, 7.5) (n_c = 7, 7, 15, 31).
Columns: SL-V, HYB-V, HLM-V and HYB-V-mid (HYB-V with M on the intermediate
scales, the hyb_mid option), each with the coloured sweeps and with the
lexicographic sweeps of Section 4.  At most 400 iterations (HLM-V does not
converge on most of these problems).

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

ROWS = [  # table, k (table3: k_ref), intervals N = 1/h, coarsest n
    ("table1", 40, 64, 7), ("table1", 50, 80, 9), ("table1", 80, 128, 15),
    ("table1", 100, 160, 19), ("table1", 150, 240, 29),
    ("table2", 40, 128, 7), ("table2", 40, 256, 7), ("table2", 40, 512, 7),
    ("table3", 15, 64, 7), ("table3", 30, 128, 7), ("table3", 60, 256, 15), ("table3", 120, 512, 31),
]


def problem(table, k0, n):
    """(h, k, f) of a row: constant k with the centre source, or the wedge."""
    if table == "table3":
        return inputs.wedge_problem(n)
    return inputs.grid_h(n), inputs.constant_k(n, float(k0)), inputs.centre_source(n)


# HYB-V-mid: HYB-V with M on the intermediate scales (the hyb_mid option)
VARIANTS = (("SL-V", oracle.SL, 0), ("HYB-V", oracle.HYB, 0), ("HLM-V", oracle.HLM, 0),
            ("HYB-V-mid", oracle.HYB, 1))
RTOL, MAXIT = 1e-7, 400


def main():
    out = {"rtol": RTOL, "maxit": MAXIT, "source": "oracle (FP64, this repository)", "rows": []}
    for table, k0, N, nc in ROWS:
        n = N - 1
        h, k, f = problem(table, k0, n)
        row = {"table": table, "k": k0, "N": N, "n": n, "coarsest_n": nc,
               "medium": "wedge" if table == "table3" else "constant", "counts": {}}
        for vname, v, mid in VARIANTS:
            for order, tag in ((0, ""), (1, "-lex")):
                t0 = time.time()
                g = oracle.Grid(h, k, variant=v, coarsest_n=nc, gs_order=order, kacz_order=order,
                                hyb_mid=mid)
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
