"""The allocation-free solve (hmg_solve_dev_static) against hmg_solve_dev:
the same kernels with the reduction partials and the residual history in the
library's fixed per-GPU array, so the two must agree to the FP64 parity bar
(here: the same iteration count and the same solution to 1e-12 relative), on
two calls in a row of which the second is smaller and finds the first one's
contents in the array."""
import sys

import numpy as np
import pytest

from paper_1312_2880_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_static_solve_matches_solve_dev():
    assert torch.cuda.is_available()
    from paper_1312_2880_amd import hmg
    ctx = hmg.Context(0)
    cases = [("layered1023 HYB", inputs.workload_layered_1023(), dict(variant=hmg.HYB), 400),
             ("point63 SL", inputs.workload_const_point(63), dict(variant=hmg.SL), 300)]
    stream = torch.cuda.current_stream()
    for name, (h, k, f), kw, maxit in cases:
        say(f"case static solve {name}")
        g = hmg.Grid(ctx, h, k, f, **kw)
        d_b = torch.from_numpy(f).to("cuda")
        x_ref = torch.zeros_like(d_b)
        x_st = torch.zeros_like(d_b)
        i_ref = g.solve_dev(x_ref, d_b=d_b, rtol=1e-6, maxit=maxit, stream=stream)
        i_st = g.solve_dev_static(x_st, d_b=d_b, rtol=1e-6, maxit=maxit, stream=stream)
        torch.cuda.synchronize()
        a, b = x_st.cpu().numpy(), x_ref.cpu().numpy()
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        say(f"  iters {i_st['iters']} / {i_ref['iters']}, rel diff {err:.2e}")
        assert i_ref["status"] == hmg.OK and i_st["status"] == hmg.OK
        assert i_st["iters"] == i_ref["iters"] and i_st["restarts"] == i_ref["restarts"]
        assert err <= 1e-12
        assert abs(i_st["rel_res_true"] - i_ref["rel_res_true"]) <= 1e-12
        assert len(g.history(0)) == 0      # the static solve keeps no history record
        # sizes beyond the array are rejected on the host, before any work
        with pytest.raises(hmg.HmgError) as e:
            g.solve_dev_static(x_st, d_b=d_b, rtol=1e-6, maxit=400000, stream=stream)
        assert e.value.status == hmg.ERR_TOO_LARGE
        g.close()
    ctx.close()
