"""Writes oracle_counts.json: Bi-CGSTAB iteration counts of the FP64 oracle
(HYB-V, relative residual 1e-6, x0 = 0) on the layered-medium problems of
1023^2 (omega = 2 pi 40) and 2047^2 (omega = 2 pi 80), seed 2.

    python tests/golden/make_oracle_counts.py        (about 10 minutes on 8 cores)

Only the oracle is called.  The inputs are the same bits on every host
(the generators avoid thread- and instruction-set-dependent rounding), but
the iteration is chaotic in its last digits, so the tests that use the
counts allow a margin; the restart count and a sampled residual history are
stored beside them.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1312_2880_amd import inputs  # noqa: E402


def main():
    out = {}
    for name, fn in (("layered1023_hyb", inputs.workload_layered_1023),
                     ("layered2047_hyb", inputs.workload_layered_2047)):
        h, k, f = fn()
        g = oracle.Grid(h, k, variant=oracle.HYB)
        t0 = time.time()
        _, info = g.bicgstab(f, rtol=1e-6, maxit=3000, history=True)
        hist = [float(v) for v in info["history"]]
        out[name] = {"iters": info["iters"], "status": info["status"], "rtol": 1e-6,
                     "restarts": info["restarts"], "seconds": round(time.time() - t0, 1),
                     # relative residual after every 50th half step (entry 0: the start)
                     "history_every_50": hist[::50]}
        print(name, out[name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_counts.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
