"""The paper's rotor-thrust-rate input (Section IV-A, Table I bounds): the
four rotor thrusts and the body rate are state, the controls are the thrust
rates.  Parity of the plain FP32 path, the fused BF16X3 path (H = 256) and
the wide decoder (H = 512) with the FP64 oracle under the same model."""
import numpy as np
import pytest

import oracle
import scenarios as sc
from gpu_common import U0_TOL, require_gpu, say, u0_error

pytestmark = pytest.mark.gpu

RM = sc.ROTOR_MODEL
ROTOR_FLOOR = np.array([4.0, 4.0, 4.0, 4.0])   # noise scale of the rate channels (N/s)


def _u0_error(u, ref):
    return float(np.max(np.abs(np.asarray(u) - ref) / np.maximum(np.abs(ref), ROTOR_FLOOR)))


@pytest.mark.parametrize("path,precision,layers,contract", [
    ("plain", "fp32", (67, 128, 128, 1), "fp32"),
    ("fused", "bf16x3", (67, 256, 256, 256, 1), "bf16w"),
    ("fused", "bf16x3", (67, 512, 512, 512, 1), "bf16w"),
    ("fused", "f16x2", (67, 256, 256, 256, 1), "bf16w"),
])
def test_rotor_rates_parity(path, precision, layers, contract):
    M = require_gpu()
    W, b = sc.xavier_weights(layers, seed=8, bias_scale=0.2)
    eng = M.Engine((W, b), RM, K_max=300, T_max=30, G_max=3, hidden=layers[1], n_hidden=len(layers) - 2,
                   precision=precision, path=path, budget=512 << 20)
    for seed, (K, T, G) in ((1, (300, 30, 3)), (2, (64, 12, 1)), (3, (17, 5, 2))):
        prob = sc.rotor_problem(K, T, G, seed=seed, rot="haar", start="moving", d_safe=1.0, Q_vis=0.3,
                                instance_id=40 + seed)
        ref = oracle.solve(prob, (W, b), RM, contract=contract)
        out = eng.step(prob)
        assert out["rc"] == 0
        e = _u0_error(out["u0"], ref["u0"])
        dJ = np.abs(out["J"] - ref["J"]) / (np.abs(ref["J"]) + prob["Q_sdf"] * T + 1.0)
        say(f"rotor rates {path}/{precision} H={layers[1]} K={K} T={T} G={G}: u0 err {e:.2e}, "
            f"max rel dJ {dJ.max():.1e}")
        assert e <= U0_TOL
        assert dJ.max() <= 2e-5
    eng.close()


def test_rotor_rates_hover_and_warm_start():
    """A new instance's nominal is zero thrust rates; at hover thrusts with no
    noise the solve returns zeros and the vehicle does not move."""
    M = require_gpu()
    W, b = sc.xavier_weights((67, 128, 128, 1), seed=9)
    eng = M.Engine((W, b), RM, K_max=64, T_max=10, G_max=1, hidden=128, n_hidden=2,
                   precision="fp32", path="plain", budget=128 << 20)
    prob = sc.rotor_problem(64, 10, 1, seed=5, start="rest", Sigma=np.zeros((4, 4)), instance_id=3)
    prob["thrust0"] = np.full(4, RM["mass"] * RM["gravity"] / 4.0)
    out = eng.step(prob, exports=True)
    assert out["rc"] == 0
    assert np.max(np.abs(out["U_star"])) == 0.0
    assert np.max(np.abs(out["p_rel"])) <= 1e-5
    bad = dict(prob, thrust0=np.array([1.0, 1.0, 1.0, RM["thrust_max"] + 1.0]))
    assert eng.step(bad)["rc"] == M.MPPI_EINVAL
    eng.close()
