"""Served path through the work ring: a persistent kernel claims the items
that the scheduler publishes in pinned memory (a prep item per solve, then
one item per tile of 16 rollouts) and the last tile of a solve merges it.

* Ring, batched served launches and the blocking solve give the same results
  bit for bit (the tile partition and the merge order depend on the solve
  alone), over a mix of gate counts, horizons and ragged rollout counts.
* The kernel ends by itself once the ring stays empty, and the next request
  starts a new launch with unchanged results.
* A blocking solve issued while the ring kernel is still resident completes.
* Every result of the mix is checked against the oracle on a few requests.
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
        time.sleep(0.0005)
    return [out[t] for t in tickets]


def _mixed(n, seed=5):
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(n):
        K = int(rng.choice([16, 100, 1000, 2048, 4096]))
        T = int(rng.choice([1, 20, 33, 60]))
        G = int(rng.choice([1, 2, 4]))
        probs.append(sc.make_problem(K, T, G, seed=700 + i, instance_id=3000 + i, d_safe=1.0))
    return probs


def _submit_all(eng, probs):
    tickets = []
    for p in probs:
        rc, t = eng.submit(p)
        assert rc == 0
        tickets.append(t)
    return tickets


@pytest.mark.parametrize("precision", ["bf16", "bf16x3", "f16x2"])
def test_ring_equals_batches_and_step(precision):
    M = require_gpu()
    probs = _mixed(20)
    ring, w = _engine(M, precision=precision)
    batches, _ = _engine(M, precision=precision, serve="batches")
    alone, _ = _engine(M, precision=precision)
    res_ring = _wait(ring, _submit_all(ring, probs), probs)
    res_bat = _wait(batches, _submit_all(batches, probs), probs)
    st = ring.stats()
    say(f"ring {precision}: {len(probs)} requests, {st['waves']} publications, "
        f"{st['ring_launches']} kernel launches; batches: {batches.stats()['waves']} launches")
    assert st["ring_launches"] >= 1 and batches.stats()["ring_launches"] == 0
    for p, (rc, r), (rcb, rb) in zip(probs, res_ring, res_bat):
        assert rc == 0 and rcb == 0, (rc, rcb)
        a = alone.step(p)     # the noise counter holds the instance id: the same id, fresh engine
        assert a["rc"] == 0
        for key in ("U_star", "J", "w"):
            assert np.array_equal(r[key], rb[key]), (key, p["K"], p["T"], p["G"])
            assert np.array_equal(r[key], a[key]), (key, p["K"], p["T"], p["G"])
        assert r["tick_used"] == rb["tick_used"] == 0
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]
    if precision != "bf16":
        for p, (rc, r) in list(zip(probs, res_ring))[:3]:
            ref = oracle.solve(p, w, sc.MODEL, contract="bf16w")
            assert u0_error(r["u0"], ref["u0"]) <= U0_TOL
    ring.close()
    batches.close()
    alone.close()


def test_ring_kernel_ends_when_idle_and_relaunches():
    M = require_gpu()
    eng, _ = _engine(M)
    probs = _mixed(3, seed=9)
    outs = []
    for p in probs:
        (rc, r), = _wait(eng, _submit_all(eng, [p]), [p])
        assert rc == 0
        outs.append(r)
        time.sleep(0.2)    # far past the kernel's idle limit: it has ended
    st = eng.stats()
    say(f"three requests 200 ms apart: {st['ring_launches']} ring kernel launches")
    assert st["ring_launches"] == 3
    alone, _ = _engine(M)
    for p, r in zip(probs, outs):
        assert np.array_equal(r["U_star"], alone.step(p)["U_star"])
    alone.close()
    eng.close()


def test_blocking_step_while_ring_kernel_resident():
    M = require_gpu()
    eng, _ = _engine(M)
    probs = _mixed(6, seed=11)
    tickets = _submit_all(eng, probs)
    # the blocking solve waits for the compute units the ring kernel holds
    extra = [dict(probs[0], instance_id=99), dict(probs[1], instance_id=98)]
    a = eng.step(extra[0])
    assert a["rc"] == 0
    res = _wait(eng, tickets, probs)
    assert all(rc == 0 for rc, _ in res)
    # and again right after the ring finished (kernel still polling)
    b = eng.step(extra[1])
    assert b["rc"] == 0
    alone, _ = _engine(M)
    for p, (rc, r) in zip(probs, res):
        assert np.array_equal(r["U_star"], alone.step(p)["U_star"])
    for p, x in zip(extra, (a, b)):
        assert np.array_equal(x["U_star"], alone.step(p)["U_star"])
    alone.close()
    eng.close()


def test_ring_close_with_work_in_flight():
    M = require_gpu()
    eng, _ = _engine(M)
    probs = _mixed(8, seed=13)
    _submit_all(eng, probs)
    eng.close()      # destroy waits for the published solves, then stops the kernel


@pytest.mark.parametrize("variant", ["pe2-f16x2-h256x2", "pe1-bf16-h128x1", "rotor-bf16x3-h256x2", "rotor-bf16-h128x2"])
def test_ring_positional_encoding_and_rotor_rates(variant):
    """The ring kernel's other instantiations (encoded-point layer 1, the
    rotor-thrust-rate input) against the blocking solve, bit for bit."""
    M = require_gpu()
    kind, precision, shape = variant.split("-")
    H, L = int(shape[1:4]), int(shape[-1])
    if kind.startswith("pe"):
        F = int(kind[2:])
        W, b = sc.xavier_weights((3 + 6 * F + 64,) + (H,) * (L + 1) + (1,), seed=10 + F, bias_scale=0.2)
        model, kw = sc.MODEL, dict(pe_freqs=F)
        probs = [sc.make_problem(K, T, G, seed=60 + i, instance_id=500 + i, d_safe=1.0)
                 for i, (K, T, G) in enumerate(((256, 20, 4), (100, 13, 2), (16, 1, 1)))]
    else:
        W, b = sc.xavier_weights((67,) + (H,) * (L + 1) + (1,), seed=8, bias_scale=0.2)
        model, kw = sc.ROTOR_MODEL, {}
        probs = [sc.rotor_problem(K, T, G, seed=1 + i, rot="haar", start="moving", d_safe=1.0, Q_vis=0.3,
                                  instance_id=600 + i)
                 for i, (K, T, G) in enumerate(((256, 20, 4), (100, 13, 2), (16, 1, 1)))]
    cfg = dict(K_max=256, T_max=20, G_max=4, hidden=H, n_hidden=L + 1, precision=precision, path="fused",
               budget=256 << 20, **kw)
    ring = M.Engine((W, b), model, **cfg)
    alone = M.Engine((W, b), model, **cfg)
    res = _wait(ring, _submit_all(ring, probs), probs)
    assert ring.stats()["ring_launches"] >= 1
    for p, (rc, r) in zip(probs, res):
        a = alone.step(p)
        assert rc == 0 and a["rc"] == 0
        assert np.array_equal(r["U_star"], a["U_star"]) and np.array_equal(r["J"], a["J"]), (variant, p["K"])
    say(f"ring {variant}: {len(probs)} solves equal to the blocking solve")
    ring.close()
    alone.close()


def test_staged_batch_while_ring_kernel_resident():
    """A staged batch created, run and read back while served requests keep
    the ring kernel resident (its uploads and read-backs may need compute
    units): everything completes and equals the blocking solve."""
    M = require_gpu()
    eng, _ = _engine(M)
    alone, _ = _engine(M)
    served = _mixed(10, seed=17)
    tickets = _submit_all(eng, served[:5])
    staged = [dict(p, instance_id=7000 + i) for i, p in enumerate(_mixed(3, seed=19))]
    bt = eng.batch(staged)
    tickets += _submit_all(eng, served[5:])
    bt.run()
    bt.wait()
    res_b = bt.results()
    res_s = _wait(eng, tickets, served)
    for p, r in zip(staged, res_b):
        assert r["status"] == 0 and np.array_equal(r["U_star"], alone.step(p)["U_star"])
    for p, (rc, r) in zip(served, res_s):
        assert rc == 0 and np.array_equal(r["U_star"], alone.step(p)["U_star"])
    bt.close()
    eng.close()
    alone.close()


def test_ring_at_the_largest_accepted_solve():
    """The ring at the engine's largest shapes (K = 16384: 1024 tiles per
    solve and 1024 tile factors in the merge; T = 128: 16 merge groups and
    four-step scan chunks; G = 8), beside a ragged solve, against the
    blocking solve bit for bit."""
    M = require_gpu()
    kw = dict(K_max=16384, T_max=128, G_max=8, precision="bf16", budget=2 << 30)
    eng, _ = _engine(M, **kw)
    alone, _ = _engine(M, **kw)
    probs = [sc.make_problem(16384, 128, 8, seed=81, instance_id=1, d_safe=1.0),
             sc.make_problem(5000, 97, 3, seed=82, instance_id=2, d_safe=1.0)]
    res = _wait(eng, _submit_all(eng, probs), probs)
    assert eng.stats()["ring_launches"] >= 1
    for p, (rc, r) in zip(probs, res):
        a = alone.step(p)
        assert rc == 0 and a["rc"] == 0
        for key in ("U_star", "J", "w"):
            assert np.array_equal(r[key], a[key]), (key, p["K"], p["T"], p["G"])
    say("ring at K=16384 T=128 G=8 and K=5000 T=97 G=3: equal to the blocking solve")
    eng.close()
    alone.close()
