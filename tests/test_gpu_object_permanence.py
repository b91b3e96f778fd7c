"""Object permanence (Section IV-B-3): while a gate is out of view the
controller keeps its latest latent code and frame and scores rollouts with
them.  A request marks gate g unobserved with a NULL latent; the engine then
uses the instance's latest observation of gate g (cached on the device as
the folded first-layer term).  The result must equal, bit for bit, the same
request (same instance, tick and nominal: the same noise) with that
observation given explicitly, and match the oracle run on the explicit
problem."""
import numpy as np
import pytest

import oracle
import scenarios as sc
from gpu_common import U0_TOL, require_gpu, say, u0_error

pytestmark = pytest.mark.gpu

LAYERS = (67, 128, 128, 1)


def _engine(M, path, precision, G=3):
    W, b = sc.xavier_weights(LAYERS, seed=4, bias_scale=0.2)
    eng = M.Engine((W, b), sc.MODEL, K_max=256, T_max=20, G_max=G, hidden=LAYERS[1], n_hidden=len(LAYERS) - 2,
                   precision=precision, path=path, budget=256 << 20, max_instances=64)
    return eng, (W, b)


def _pair(seed_a, seed_b, inst):
    """Tick a observes every gate; tick b sees gate 1 only through the cache."""
    a = sc.make_problem(256, 20, 3, rot="haar", start="moving", seed=seed_a, d_safe=1.0,
                        instance_id=inst, tick=3)
    b = sc.make_problem(256, 20, 3, rot="haar", start="moving", seed=seed_b, d_safe=1.0,
                        instance_id=inst, tick=4)
    U = oracle.hover_sequence(20, sc.MODEL["mass"], sc.MODEL["gravity"])
    b["U_nom"] = U
    explicit = dict(b)
    for key in ("gate_z", "gate_R", "gate_t"):
        v = np.array(b[key], copy=True)
        v[1] = a[key][1]
        explicit[key] = v
    hidden = dict(b, gate_cached=[False, True, False])
    # what the request carries for the unobserved gate is ignored
    for key in ("gate_z", "gate_R", "gate_t"):
        v = np.array(b[key], copy=True)
        v[1] = np.nan
        hidden[key] = v
    return a, hidden, explicit


@pytest.mark.parametrize("path,precision,contract", [("plain", "fp32", "fp32"), ("fused", "bf16x3", "bf16w"),
                                                     ("fused", "f16x2", "bf16w")])
def test_unobserved_gate_uses_latest_observation(path, precision, contract):
    M = require_gpu()
    eng, w = _engine(M, path, precision)
    a, hidden, explicit = _pair(21, 22, inst=7)
    assert eng.step(a)["rc"] == 0
    out_h = eng.step(hidden)
    out_e = eng.step(explicit)
    assert out_h["rc"] == 0 and out_e["rc"] == 0
    assert np.array_equal(out_h["U_star"], out_e["U_star"])
    assert np.array_equal(out_h["J"], out_e["J"])
    ref = oracle.solve(explicit, w, sc.MODEL, contract=contract)
    e = u0_error(out_h["u0"], ref["u0"])
    say(f"object permanence {path}/{precision}: u0 err vs oracle {e:.2e}")
    assert e <= U0_TOL
    # a later observation of gate 1 replaces the cached one
    a2 = dict(a, tick=5, U_nom=hidden["U_nom"])
    a2["gate_z"] = np.array(a["gate_z"], copy=True)
    a2["gate_z"][1] = explicit["gate_z"][2]
    assert eng.step(a2)["rc"] == 0
    out_h2 = eng.step(dict(hidden, tick=6))
    explicit2 = dict(explicit, tick=6)
    explicit2["gate_z"] = np.array(explicit["gate_z"], copy=True)
    explicit2["gate_z"][1] = a2["gate_z"][1]
    out_e2 = eng.step(explicit2)
    assert np.array_equal(out_h2["U_star"], out_e2["U_star"])
    eng.close()


def test_unobserved_gate_without_observation_is_rejected():
    M = require_gpu()
    eng, _ = _engine(M, "fused", "bf16x3")
    _, hidden, _ = _pair(31, 32, inst=11)
    assert eng.step(hidden)["rc"] == M.MPPI_EINVAL
    # served path: the request fails alone, the one beside it completes
    a, hidden2, _ = _pair(33, 34, inst=12)
    rc1, t1 = eng.submit(dict(hidden2, instance_id=13))
    rc2, t2 = eng.submit(a)
    assert rc1 == 0 and rc2 == 0
    eng.drain()
    rc, _ = eng.poll(t1, 256, 20)
    assert rc == M.MPPI_EINVAL
    rc, out = eng.poll(t2, 256, 20)
    assert rc == 0 and out["rc"] == 0
    eng.close()


def test_unobserved_gate_in_staged_batch():
    """A staged fleet tick: the unobserved gate's cached fold is read at every
    launch, the observed gates' folds are refreshed."""
    M = require_gpu()
    eng, w = _engine(M, "fused", "bf16x3")
    a, hidden, explicit = _pair(41, 42, inst=20)
    assert eng.step(a)["rc"] == 0
    bt = eng.batch([hidden])
    for _ in range(2):
        bt.run()
        bt.wait()
    res = bt.results()[0]
    bt.close()
    out_e = eng.step(explicit)
    assert res["status"] == 0
    assert np.array_equal(res["U_star"], out_e["U_star"])
    eng.close()
