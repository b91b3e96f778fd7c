"""FP64 CPU oracle for one MPPI iteration with a Gate-SDF cost.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the package
``paper_2603_07199_amd``, its HIP kernels or its C ABI) may import, call,
link or execute anything in this package; only the tests, the smoke check
and the CPU-baseline leg of the benchmark use it.

The oracle is a plain, slow, step-by-step reading of the method:

* Section IV-A, update equation (eq:mppi_update): Gaussian perturbations of
  the nominal sequence, rollouts through the quadrotor model, the
  softmax-weighted average with temperature lambda.
* Section IV-B: gate-progress cost (eq. 5), perception-alignment cost
  (eq. 6), SDF stage cost and its horizon sum (eqs. 7-8), total cost (eq. 9).
* Section III-A (eqs. 1-2): the analytic guidance Gate-SDF, used as a
  swap-in for the learned decoder in tests.
* Section III-B: the SDF decoder g_phi evaluated on [PE(p); z].

Where the paper is silent the readings are listed in each module's
docstring.  Every function works in float64 except where a precision
contract (``precision.py``) rounds the SDF decoder's operands on purpose.

Every function is pinned by tests/test_oracle_*.py against something other
than itself (closed forms, hand values, library routines, invariants, brute
force).  Not pinned: the learned-SDF *behaviour* of the paper (no trained
weights exist here; seeded random weights stand in), so results that depend
on a trained decoder are "parity unpinned".

Reduced-precision bookkeeping (``precision.near_tie_mask``,
``sdf.mlp_alternatives``, ``solve(..., near_ties=...)``): under the ``bf16``
and ``fp8`` contracts an activation within a small window of a rounding
boundary may legitimately round either way in a float32 evaluation; the
oracle reports how many there are and the range of the field over every
combination of those roundings.
"""
from .philox import philox4x64_10, uniforms_from_words, box_muller, control_noise
from .dynamics import rollout, rotor_rollout, quat_mul, thrust_axis
from .sdf import softplus, mlp_concat, mlp_fold, gate_sdf_analytic
from .precision import bf16_round, e4m3_round, quantise_weights_fp8
from .mppi import solve, mppi_update, shift_warm_start, hover_sequence

__all__ = [
    "philox4x64_10", "uniforms_from_words", "box_muller", "control_noise",
    "rollout", "rotor_rollout", "quat_mul", "thrust_axis",
    "softplus", "mlp_concat", "mlp_fold", "gate_sdf_analytic",
    "bf16_round", "e4m3_round", "quantise_weights_fp8",
    "solve", "mppi_update", "shift_warm_start", "hover_sequence",
]
