"""Staged batches (mppi_batch_*): results equal mppi_step on the same inputs,
and repeated launches advance the resident warm start and tick on device."""
import numpy as np
import pytest

import oracle
import scenarios as sc
from gpu_common import U0_TOL, require_gpu, say, u0_error

pytestmark = pytest.mark.gpu


def test_batch_matches_step_and_advances_ticks():
    M = require_gpu()
    W, b = sc.xavier_weights((67, 128, 128, 1), seed=0)
    kw = dict(K_max=512, T_max=20, G_max=2, hidden=128, n_hidden=2, budget=256 << 20)
    probs = [sc.make_problem(300 + 50 * i, 20, 1 + i % 2, rot="haar", start="moving", seed=30 + i,
                             d_safe=1.0, instance_id=i, tick=M.TICK_RESIDENT) for i in range(4)]
    with M.Engine((W, b), sc.MODEL, **kw) as eng, M.Engine((W, b), sc.MODEL, **kw) as ref_eng:
        bt = eng.batch(probs)
        with pytest.raises(M.MPPIError):           # instances held by the batch
            eng.batch(probs[:1])
        prev = [None] * 4
        for tick in range(3):
            bt.run()
            bt.wait()
            res = bt.results()
            for i, (p, r) in enumerate(zip(probs, res)):
                assert r["status"] == 0 and r["tick_used"] == tick
                s = ref_eng.step(p)        # same instance chain on another engine via mppi_step
                o = oracle.solve(dict(p, tick=tick), (W, b), sc.MODEL,
                                 U_nom=None if prev[i] is None else oracle.shift_warm_start(prev[i]))
                e = u0_error(r["u0"], o["u0"])
                say(f"batch tick {tick} solve {i}: u0 err {e:.2e}")
                assert e <= U0_TOL
                assert s["tick_used"] == tick
                assert np.array_equal(r["U_star"], s["U_star"])      # same kernels, same inputs
                prev[i] = r["U_star"]
        bt.close()
        bt2 = eng.batch(probs[:1])                  # released again
        bt2.close()
