"""Served path (mppi_submit / mppi_poll): continuous batching of uneven
solves on the fused decoder, through the work ring of the persistent served
kernel (the default; tests/test_gpu_ring.py compares it with batched
launches).

* Alone vs in the mix: a request's result does not depend on what it was
  batched with (fixed tile partition per solve, merge in tile order), so the
  served result equals the same request solved alone, bit for bit.
* Admission by device-memory budget: with a budget that holds only a few
  solves, every request still completes, the peak stays within the budget and
  several batches run.
* Error codes: ENOMEM for a request that can never fit, EAGAIN for a full
  queue or (per ticket) a new instance while the instance table is full,
  ENOTFOUND for an unknown ticket.
* A torch-owned pool with no room beyond the budget: each batch's launch
  block is counted at admission, and blocking solves count too.
* Resident warm start across served ticks, checked against the oracle chain.
"""
import time

import numpy as np
import pytest

import oracle
import scenarios as sc
from gpu_common import U0_TOL, require_gpu, say, u0_error

pytestmark = pytest.mark.gpu

LAYERS = (67, 256, 256, 256, 1)


def _engine(M, **kw):
    W, b = sc.xavier_weights(LAYERS, seed=0)
    cfg = dict(K_max=4096, T_max=60, G_max=4, hidden=256, n_hidden=3, precision="bf16x3",
               path="fused", budget=1 << 30)
    cfg.update(kw)
    return M.Engine((W, b), sc.MODEL, **cfg), (W, b)


def _wait(eng, tickets, probs, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t, p in zip(tickets, probs):
            if t in out:
                continue
            rc, r = eng.poll(t, p["K"], p["T"])
            if rc != 1:
                out[t] = (rc, r)
        assert time.time() - t0 < timeout, "served solves did not complete"
        time.sleep(0.001)
    return [out[t] for t in tickets]


def _mix(n, seed=7):
    reqs = sc.serving_requests(seed=seed, n_req=n, K_set=(256, 1024, 2048, 4096), T_set=(20, 30, 40, 60))
    return [dict(p, instance_id=1000 + i) for i, (_, p) in enumerate(reqs)]


@pytest.mark.parametrize("precision", ["bf16x3", "f16x2"])
def test_alone_equals_mix_bitwise(precision):
    M = require_gpu()
    probs = _mix(24)
    served, w = _engine(M, precision=precision)
    alone, _ = _engine(M, precision=precision)
    tickets = []
    for p in probs:
        rc, t = served.submit(p)
        assert rc == 0
        tickets.append(t)
    res = _wait(served, tickets, probs)
    st = served.stats()
    say(f"served {precision}: 24 uneven requests in {st['waves']} batches")
    for p, (rc, r) in zip(probs, res):
        assert rc == 0
        a = alone.step(p)
        assert a["rc"] == 0
        assert np.array_equal(r["U_star"], a["U_star"]), (p["K"], p["T"])
        assert np.array_equal(r["J"], a["J"])
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]
    for p, (rc, r) in list(zip(probs, res))[:3]:
        ref = oracle.solve(p, w, sc.MODEL, contract="bf16w")
        assert u0_error(r["u0"], ref["u0"]) <= U0_TOL
    served.close()
    alone.close()


def test_budget_admission_and_errors():
    M = require_gpu()
    probe, _ = _engine(M)
    fp = probe.footprint(2048, 40, 1)
    probe.close()
    budget = int(2.5 * fp)
    eng, _ = _engine(M, budget=budget, queue_depth=16)
    big = _mix(1)[0]
    big = dict(big, K=4096, T=60, instance_id=1)
    assert eng.footprint(4096, 60, 1) > budget
    rc, _ = eng.submit(big)
    assert rc == M.MPPI_ENOMEM
    probs = [dict(p, K=2048, T=40, instance_id=10 + i) for i, p in enumerate(_mix(16, seed=9))]
    tickets = []
    for p in probs:
        rc, t = eng.submit(p)
        assert rc == 0
        tickets.append(t)
    rc, _ = eng.submit(dict(probs[0], instance_id=99))     # 17th: queue depth 16 may be full
    assert rc in (0, M.MPPI_EAGAIN)
    if rc == 0:
        tickets.append(_)
        probs.append(dict(probs[0], instance_id=99))
    res = _wait(eng, tickets, probs)
    assert all(rc == 0 for rc, _ in res)
    st = eng.stats()
    say(f"budget {budget} B: {st['waves']} batches, peak {st['bytes_peak']} B")
    # solve blocks and each batch's launch block are both counted at admission
    assert st["bytes_peak"] <= st["budget"] and st["waves"] >= 4
    rc, _ = eng.poll(123456789, 8, 8)
    assert rc == M.MPPI_ENOTFOUND
    eng.close()


def test_served_ticks_keep_the_warm_start_resident():
    M = require_gpu()
    eng, w = _engine(M)
    p = dict(_mix(1, seed=11)[0], K=1024, T=30, instance_id=5, tick=M.TICK_RESIDENT)
    prev = None
    for tick in range(4):
        rc, t = eng.submit(p)
        assert rc == 0
        (rc, r), = _wait(eng, [t], [p])
        assert rc == 0 and r["tick_used"] == tick
        ref = oracle.solve(dict(p, tick=tick), w, sc.MODEL, contract="bf16w",
                           U_nom=None if prev is None else oracle.shift_warm_start(prev))
        e = u0_error(r["u0"], ref["u0"])
        say(f"served tick {tick}: u0 err {e:.2e}")
        assert e <= U0_TOL
        prev = r["U_star"]
    eng.close()


def test_full_instance_table_fails_only_new_instances():
    """With the instance table full, a request for a new instance fails with
    EAGAIN on its own; requests of existing instances admitted with it still
    complete."""
    M = require_gpu()
    eng, _ = _engine(M, max_instances=4)
    base = dict(_mix(1, seed=13)[0], K=512, T=20)
    for iid in (1, 2, 3):
        assert eng.step(dict(base, instance_id=iid))["rc"] == 0
    probs = [dict(base, instance_id=iid) for iid in (1, 2, 10, 3, 11)]
    tickets = []
    for p in probs:
        rc, t = eng.submit(p)
        assert rc == 0
        tickets.append(t)
    res = _wait(eng, tickets, probs)
    codes = [rc for rc, _ in res]
    say(f"instance table of 4, three resident: statuses {codes}")
    # FIFO: instance 10 takes the last free slot, 11 finds the table full
    assert codes == [0, 0, 0, 0, M.MPPI_EAGAIN]
    # the table stays usable for the resident instances
    rc, t = eng.submit(probs[0])
    assert rc == 0 and _wait(eng, [t], [probs[0]])[0][0] == 0
    eng.close()


def test_torch_pool_at_a_tight_budget():
    """Device pool from torch with no room beyond the budget: every admitted
    batch (solve blocks and the batch's launch block) fits what admission
    counted, so all requests complete and the peak stays within the budget;
    blocking solves count against the same budget."""
    M = require_gpu()
    probe, _ = _engine(M)
    fp = probe.footprint(1024, 30, 1)
    probe.close()
    budget = 3 * fp
    eng, _ = _engine(M, budget=budget, use_torch_memory=True)
    assert eng.footprint(1024, 30, 1) == fp
    probs = [dict(p, K=1024, T=30, instance_id=200 + i) for i, p in enumerate(_mix(12, seed=21))]
    tickets = []
    for p in probs:
        rc, t = eng.submit(p)
        assert rc == 0
        tickets.append(t)
    res = _wait(eng, tickets, probs)
    assert all(rc == 0 for rc, _ in res), [rc for rc, _ in res]
    st = eng.stats()
    say(f"torch pool, budget {budget} B (3 solves): {st['waves']} batches, peak {st['bytes_peak']} B")
    assert st["bytes_peak"] <= budget and st["waves"] >= 4
    # a blocking solve larger than the whole budget can never run
    assert eng.footprint(4096, 60, 1) > budget
    big = dict(probs[0], K=4096, T=60, instance_id=300)
    assert eng.step(big)["rc"] == M.MPPI_ENOMEM
    eng.close()
