"""Section 6.1 ray-correction study on the GPU (the setting of the paper's
ray-correction table: constant k, kh = 0.3125, a unit point source at the
centre, a 1e-7 residual reduction): the number of stationary cycles x <- x +
B (f - L x) and of Bi-CGSTAB iterations for HLM-V, SL-V and HYB-V without and
with the ray correction on ray grids of 3 and 7 interior nodes per side.
A '*' marks a run that did not reach the reduction.

    python study_table4.py
"""
import sys, time, numpy as np
sys.path.insert(0, '.')
from paper_1312_2880_amd import hmg, inputs
ctx = hmg.Context(0)
print("Table 4 setting: kh = 0.3125, point source at the centre, 1e-7 reduction; cycles (stationary) / Bi-CGSTAB iterations")
for k0, n, nc in ((20, 63, 3), (40, 127, 7), (80, 255, 15), (160, 511, 31)):
    h = 1.0 / (n + 1)
    k = np.full((n + 2, n + 2), float(k0))
    f = inputs.centre_source(n)
    row = []
    for vname, v in (("HLM", hmg.HLM), ("SL", hmg.SL), ("HYB", hmg.HYB)):
        for ray_n in (0, 3, 7):
            if ray_n and (n + 1) // (ray_n + 1) < 8:
                continue
            t = time.time()
            g = hmg.Grid(ctx, h, k, f, variant=v, coarsest_n=nc, ray_n=ray_n)
            ts = time.time() - t
            _, ic = g.solve_cycles(rtol=1e-7, maxit=100)
            _, ib = g.solve(rtol=1e-7, maxit=300)
            row.append(f"{vname} ray{ray_n}: {ic[0]['iters']:.0f}{'' if ic[0]['status']==0 else '*'}/{ib[0]['iters']}{'' if ib[0]['status']==0 else '*'}")
            g.close()
    print(f"k={k0} n={n}: " + "; ".join(row), flush=True)
ctx.close()
