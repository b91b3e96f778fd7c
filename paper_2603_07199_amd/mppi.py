"""Thin ctypes binding of the C ABI in ``include/mppi.h`` (argument marshalling
only: every step of the MPPI iteration runs in the library's HIP kernels).

The functions keep the C names: ``mppi_create``, ``mppi_step``,
``mppi_submit``, ``mppi_poll``, ``mppi_drain``, ``mppi_destroy``; the
``Engine`` class wraps them for convenience.  Problem dictionaries use the
field names of ``mppi_request`` (see ``scenarios``).

The library is loaded from the package directory; if it is missing this
module raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmppi.so")

MPPI_OK, MPPI_PENDING = 0, 1
MPPI_EINVAL, MPPI_ENOMEM, MPPI_EAGAIN = -1, -2, -3
MPPI_ENOTFOUND, MPPI_ENUMERIC, MPPI_EDEVICE = -4, -5, -6

PREC = {"fp32": 0, "bf16": 1, "bf16x2": 2, "fp8": 3, "bf16x3": 4, "f16x2": 5}
PATH = {"plain": 0, "fused": 1}
SDF = {"mlp": 0, "analytic": 1}
CFG_TIMING = 1
CFG_SERVE_BATCHES = 2   # served path in batched launches instead of the work ring
REQ_NO_SHIFT = 1
REQ_SDF_AT_P0 = 2
TICK_RESIDENT = 0xFFFFFFFF


class mppi_config(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("path", C.c_int32), ("sdf_kind", C.c_int32),
        ("hidden", C.c_int32), ("n_hidden", C.c_int32), ("latent_dim", C.c_int32),
        ("K_max", C.c_int32), ("T_max", C.c_int32), ("G_max", C.c_int32),
        ("max_instances", C.c_int32), ("max_inflight", C.c_int32), ("queue_depth", C.c_int32),
        ("device", C.c_int32), ("flags", C.c_uint32),
        ("hbm_budget_bytes", C.c_uint64), ("seed", C.c_uint64),
        ("mass", C.c_double), ("gravity", C.c_double),
        ("u_lo", C.c_double * 4), ("u_hi", C.c_double * 4),
        ("sdf_c", C.c_double), ("sdf_tan_alpha", C.c_double),
        ("stream", C.c_void_p), ("device_pool", C.c_void_p), ("device_pool_bytes", C.c_uint64),
        ("dynamics", C.c_int32), ("pe_freqs", C.c_int32),
        ("inertia", C.c_double * 3), ("arm_length", C.c_double), ("yaw_coeff", C.c_double),
        ("thrust_max", C.c_double), ("rate_max", C.c_double),
        ("wave_queries_max", C.c_uint64), ("wide_region", C.c_int32),
    ]


class mppi_sdf_weights(C.Structure):
    _fields_ = [("W", C.POINTER(C.POINTER(C.c_float))), ("b", C.POINTER(C.POINTER(C.c_float))),
                ("act_scale", C.POINTER(C.c_float))]


class mppi_gate(C.Structure):
    _fields_ = [("z", C.POINTER(C.c_float)), ("R", C.c_double * 9), ("t", C.c_double * 3)]


class mppi_request(C.Structure):
    _fields_ = [
        ("instance_id", C.c_uint64), ("tick", C.c_uint32), ("flags", C.c_uint32),
        ("K", C.c_int32), ("T", C.c_int32), ("G", C.c_int32), ("pad_", C.c_int32),
        ("dt", C.c_double), ("x0", C.c_double * 13), ("U_nom", C.POINTER(C.c_double)),
        ("Sigma", C.c_double * 16), ("lambda_", C.c_double),
        ("Q_gate", C.c_double), ("Q_vis", C.c_double), ("Q_sdf", C.c_double),
        ("d_safe", C.c_double), ("R_u", C.c_double), ("wp", C.c_double * 3),
        ("gates", C.POINTER(mppi_gate)), ("thrust0", C.c_double * 4),
    ]


class mppi_result(C.Structure):
    _fields_ = [
        ("U_star", C.POINTER(C.c_double)), ("weights", C.POINTER(C.c_double)),
        ("costs", C.POINTER(C.c_double)), ("samples", C.POINTER(C.c_float)),
        ("positions", C.POINTER(C.c_float)), ("sdf", C.POINTER(C.c_float)),
        ("u0", C.c_double * 4), ("J_min", C.c_double), ("log_eta", C.c_double),
        ("ess", C.c_double), ("tick_used", C.c_uint32), ("status", C.c_int32),
        ("t_submit_ns", C.c_uint64), ("t_admit_ns", C.c_uint64), ("t_done_ns", C.c_uint64),
    ]


class mppi_stats(C.Structure):
    _fields_ = [
        ("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
        ("failed", C.c_uint64), ("waves", C.c_uint64), ("bytes_in_use", C.c_uint64),
        ("bytes_peak", C.c_uint64), ("budget", C.c_uint64), ("sdf_launches", C.c_uint64),
        ("sdf_ms", C.c_double), ("solve_launches", C.c_uint64), ("solve_ms", C.c_double),
        ("tune_runs", C.c_uint64), ("wide_region", C.c_uint64), ("ring_launches", C.c_uint64),
    ]


EXPORTED = ["mppi_create", "mppi_destroy", "mppi_step", "mppi_submit", "mppi_poll",
            "mppi_drain", "mppi_get_stats", "mppi_reset_stats", "mppi_status_str",
            "mppi_solve_footprint", "mppi_batch_create", "mppi_batch_run", "mppi_batch_wait",
            "mppi_batch_results", "mppi_batch_destroy", "mppi_step_noalloc"]

# MPPI_NOALLOC_SCRATCH_BYTES of include/mppi.h
NOALLOC_SCRATCH_BYTES = 16 << 20

_lib = None


def load_library(path=LIB_PATH):
    """Load libmppi.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2603_07199_amd.build`")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.mppi_create.argtypes = [P(mppi_config), P(mppi_sdf_weights), P(C.c_void_p)]
    lib.mppi_destroy.argtypes = [C.c_void_p]
    lib.mppi_step.argtypes = [C.c_void_p, P(mppi_request), P(mppi_result)]
    lib.mppi_submit.argtypes = [C.c_void_p, P(mppi_request), P(C.c_uint64)]
    lib.mppi_poll.argtypes = [C.c_void_p, C.c_uint64, P(mppi_result)]
    lib.mppi_drain.argtypes = [C.c_void_p]
    lib.mppi_get_stats.argtypes = [C.c_void_p, P(mppi_stats)]
    lib.mppi_reset_stats.argtypes = [C.c_void_p]
    lib.mppi_reset_stats.restype = None
    lib.mppi_status_str.argtypes = [C.c_int]
    lib.mppi_status_str.restype = C.c_char_p
    lib.mppi_solve_footprint.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
    lib.mppi_solve_footprint.restype = C.c_uint64
    lib.mppi_batch_create.argtypes = [C.c_void_p, P(mppi_request), C.c_int32, P(C.c_void_p)]
    lib.mppi_batch_run.argtypes = [C.c_void_p, C.c_void_p]
    lib.mppi_batch_wait.argtypes = [C.c_void_p, C.c_void_p]
    lib.mppi_batch_results.argtypes = [C.c_void_p, C.c_void_p, P(mppi_result)]
    lib.mppi_batch_destroy.argtypes = [C.c_void_p, C.c_void_p]
    lib.mppi_step_noalloc.argtypes = [C.c_void_p, P(mppi_request), P(mppi_result)]
    for name in ("mppi_create", "mppi_destroy", "mppi_step", "mppi_submit", "mppi_poll",
                 "mppi_drain", "mppi_get_stats", "mppi_batch_create", "mppi_batch_run",
                 "mppi_batch_wait", "mppi_batch_results", "mppi_batch_destroy", "mppi_step_noalloc"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def status_str(code):
    return load_library().mppi_status_str(int(code)).decode()


class MPPIError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {status_str(code)} ({code})")
        self.code = code


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class _Request:
    """ctypes request built from a problem dict; keeps its buffers alive."""

    def __init__(self, prob):
        self.keep = []
        r = mppi_request()
        r.instance_id = int(prob.get("instance_id", 0))
        r.tick = int(prob.get("tick", 0)) & 0xFFFFFFFF
        r.flags = int(prob.get("flags", 0))
        r.K, r.T, r.G = int(prob["K"]), int(prob["T"]), int(prob["G"])
        r.dt = float(prob["dt"])
        x0 = np.ascontiguousarray(prob["x0"], dtype=np.float64)
        r.x0[:] = list(x0)
        U = prob.get("U_nom")
        if U is not None:
            U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1)
            self.keep.append(U)
            r.U_nom = _dptr(U)
        r.Sigma[:] = list(np.asarray(prob["Sigma"], dtype=np.float64).reshape(16))
        r.lambda_ = float(prob["lam"])
        r.Q_gate, r.Q_vis, r.Q_sdf = float(prob["Q_gate"]), float(prob["Q_vis"]), float(prob["Q_sdf"])
        r.d_safe, r.R_u = float(prob["d_safe"]), float(prob["R_u"])
        r.wp[:] = list(np.asarray(prob["wp"], dtype=np.float64))
        if prob.get("thrust0") is not None:
            r.thrust0[:] = list(np.asarray(prob["thrust0"], dtype=np.float64))
        G = r.G
        gates = (mppi_gate * G)()
        z = np.ascontiguousarray(prob["gate_z"], dtype=np.float32).reshape(G, -1)
        self.keep.append(z)
        # gate_cached[g] True: gate g not observed, use the instance's cached gate (z = NULL)
        cached = prob.get("gate_cached")
        for g in range(G):
            gates[g].z = None if (cached is not None and cached[g]) else _fptr(z[g])
            gates[g].R[:] = list(np.asarray(prob["gate_R"][g], dtype=np.float64).reshape(9))
            gates[g].t[:] = list(np.asarray(prob["gate_t"][g], dtype=np.float64))
        self.keep.append(gates)
        r.gates = gates
        self.req = r


class _Result:
    def __init__(self, K, T, weights=True, costs=True, exports=False):
        self.U = np.zeros((T, 4))
        self.w = np.zeros(K) if weights else None
        self.J = np.zeros(K) if costs else None
        self.samples = np.zeros((K, T, 4), dtype=np.float32) if exports else None
        self.pos = np.zeros((K, T + 1, 3), dtype=np.float32) if exports else None
        self.sdf = np.zeros((K, T), dtype=np.float32) if exports else None
        r = mppi_result()
        r.U_star = _dptr(self.U)
        if weights:
            r.weights = _dptr(self.w)
        if costs:
            r.costs = _dptr(self.J)
        if exports:
            r.samples = _fptr(self.samples)
            r.positions = _fptr(self.pos)
            r.sdf = _fptr(self.sdf)
        self.res = r

    def as_dict(self):
        r = self.res
        out = {"status": int(r.status), "U_star": self.U.copy(), "u0": np.array(list(r.u0)),
               "J_min": r.J_min, "log_eta": r.log_eta, "ess": r.ess, "tick_used": int(r.tick_used),
               "t_submit_ns": int(r.t_submit_ns), "t_admit_ns": int(r.t_admit_ns),
               "t_done_ns": int(r.t_done_ns)}
        if self.w is not None:
            out["w"] = self.w.copy()
        if self.J is not None:
            out["J"] = self.J.copy()
        if self.samples is not None:
            out["samples"], out["p_rel"], out["sdf"] = self.samples.copy(), self.pos.copy(), self.sdf.copy()
        return out


def mppi_create(config, weights):
    """config: dict of mppi_config fields; weights: (W list, b list[, act_scale])."""
    lib = load_library()
    c = mppi_config()
    for k, v in config.items():
        if k in ("u_lo", "u_hi", "inertia"):
            getattr(c, k)[:] = [float(x) for x in v]
        else:
            setattr(c, k, v)
    keep = []
    wp = None
    if weights is not None:
        W, b = weights[0], weights[1]
        Ws = [np.ascontiguousarray(w, dtype=np.float32) for w in W]
        bs = [np.ascontiguousarray(v, dtype=np.float32) for v in b]
        keep += Ws + bs
        Wp = (C.POINTER(C.c_float) * len(Ws))(*[_fptr(w) for w in Ws])
        bp = (C.POINTER(C.c_float) * len(bs))(*[_fptr(v) for v in bs])
        keep += [Wp, bp]
        wp = mppi_sdf_weights()
        wp.W = C.cast(Wp, C.POINTER(C.POINTER(C.c_float)))
        wp.b = C.cast(bp, C.POINTER(C.POINTER(C.c_float)))
        if len(weights) > 2 and weights[2] is not None:
            a = np.ascontiguousarray(weights[2], dtype=np.float32)
            keep.append(a)
            wp.act_scale = _fptr(a)
    h = C.c_void_p()
    rc = lib.mppi_create(C.byref(c), C.byref(wp) if wp is not None else None, C.byref(h))
    if rc != MPPI_OK:
        raise MPPIError(rc, "mppi_create")
    return h


def mppi_destroy(handle):
    return load_library().mppi_destroy(handle)


def mppi_step(handle, prob, weights=True, costs=True, exports=False):
    rq = _Request(prob)
    rs = _Result(prob["K"], prob["T"], weights, costs, exports)
    rc = load_library().mppi_step(handle, C.byref(rq.req), C.byref(rs.res))
    out = rs.as_dict()
    out["rc"] = rc
    return out


def mppi_step_noalloc(handle, prob, weights=True, costs=True):
    """mppi_step on the library's static device scratch (no allocation)."""
    rq = _Request(prob)
    rs = _Result(prob["K"], prob["T"], weights, costs, False)
    rc = load_library().mppi_step_noalloc(handle, C.byref(rq.req), C.byref(rs.res))
    out = rs.as_dict()
    out["rc"] = rc
    return out


def mppi_submit(handle, prob):
    rq = _Request(prob)
    t = C.c_uint64()
    rc = load_library().mppi_submit(handle, C.byref(rq.req), C.byref(t))
    return rc, int(t.value)


def mppi_poll(handle, ticket, K, T, weights=True, costs=True):
    rs = _Result(K, T, weights, costs, False)
    rc = load_library().mppi_poll(handle, C.c_uint64(ticket), C.byref(rs.res))
    if rc == MPPI_PENDING or rc in (MPPI_ENOTFOUND, MPPI_EINVAL):
        return rc, None
    out = rs.as_dict()
    out["rc"] = rc
    return rc, out


def mppi_drain(handle):
    return load_library().mppi_drain(handle)


class Batch:
    """Requests staged once in device memory (``mppi_batch_*``)."""

    def __init__(self, handle, probs):
        lib = load_library()
        self.h = handle
        self.probs = probs
        self._reqs = [_Request(p) for p in probs]
        arr = (mppi_request * len(probs))(*[r.req for r in self._reqs])
        self._arr = arr
        b = C.c_void_p()
        rc = lib.mppi_batch_create(handle, arr, len(probs), C.byref(b))
        if rc != MPPI_OK:
            raise MPPIError(rc, "mppi_batch_create")
        self.b = b

    def run(self):
        rc = load_library().mppi_batch_run(self.h, self.b)
        if rc != MPPI_OK:
            raise MPPIError(rc, "mppi_batch_run")

    def wait(self):
        rc = load_library().mppi_batch_wait(self.h, self.b)
        if rc != MPPI_OK:
            raise MPPIError(rc, "mppi_batch_wait")

    def results(self):
        rs = [_Result(p["K"], p["T"]) for p in self.probs]
        arr = (mppi_result * len(rs))(*[r.res for r in rs])
        rc = load_library().mppi_batch_results(self.h, self.b, arr)
        if rc != MPPI_OK:
            raise MPPIError(rc, "mppi_batch_results")
        out = []
        for r, raw in zip(rs, arr):
            r.res = raw
            out.append(r.as_dict())
        return out

    def close(self):
        if self.b is not None:
            load_library().mppi_batch_destroy(self.h, self.b)
            self.b = None


def default_config(model, K_max=8192, T_max=64, G_max=8, hidden=256, n_hidden=3,
                   precision="fp32", path="plain", sdf_kind="mlp", max_instances=4096,
                   max_inflight=64, queue_depth=4096, budget=1 << 30, seed=0, timing=False,
                   stream=None, device_pool=None, device_pool_bytes=0, pe_freqs=0, wave_queries_max=0,
                   wide_region=0, serve="ring"):
    if serve not in ("ring", "batches"):
        raise ValueError(f"serve must be 'ring' or 'batches', not {serve!r}")
    return {
        "precision": PREC[precision], "path": PATH[path], "sdf_kind": SDF[sdf_kind],
        "hidden": hidden, "n_hidden": n_hidden, "latent_dim": 64,
        "K_max": K_max, "T_max": T_max, "G_max": G_max,
        "max_instances": max_instances, "max_inflight": max_inflight, "queue_depth": queue_depth,
        "device": 0, "flags": (CFG_TIMING if timing else 0) | (CFG_SERVE_BATCHES if serve == "batches" else 0),
        "hbm_budget_bytes": int(budget), "seed": int(seed),
        "mass": float(model["mass"]), "gravity": float(model["gravity"]),
        "u_lo": list(model["u_lo"]), "u_hi": list(model["u_hi"]),
        "sdf_c": 0.5, "sdf_tan_alpha": 0.5,
        "stream": stream, "device_pool": device_pool, "device_pool_bytes": int(device_pool_bytes),
        # vehicle model: model["kind"] == "rotor" selects the rotor-thrust-rate input
        "dynamics": 1 if model.get("kind") == "rotor" else 0,
        "pe_freqs": int(pe_freqs),
        "inertia": list(model.get("inertia", (0.0, 0.0, 0.0))),
        "arm_length": float(model.get("arm_length", 0.0)), "yaw_coeff": float(model.get("yaw_coeff", 0.0)),
        "thrust_max": float(model.get("thrust_max", 0.0)), "rate_max": float(model.get("rate_max", 0.0)),
        "wave_queries_max": int(wave_queries_max),
        # H = 512 decoder: fragment read-ahead region (2, 4, 8; 0 = tuned per shape)
        "wide_region": int(wide_region),
    }


class Engine:
    """Convenience wrapper owning one ``mppi_engine``.

    When ``torch`` is importable and ``use_torch_memory`` is set, the per-solve
    device pool is a torch CUDA allocation and the blocking path runs on
    torch's current stream (torch supplies device memory and streams only).
    """

    def __init__(self, weights, model, use_torch_memory=False, **cfg):
        self._pool = None
        config = default_config(model, **cfg)
        if use_torch_memory:
            import torch
            nbytes = int(config["hbm_budget_bytes"])
            self._pool = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            config["device_pool"] = self._pool.data_ptr()
            config["device_pool_bytes"] = nbytes
            config["stream"] = torch.cuda.current_stream().cuda_stream
        self.config = config
        self.h = mppi_create(config, weights)

    def step(self, prob, **kw):
        return mppi_step(self.h, prob, **kw)

    def step_noalloc(self, prob, **kw):
        return mppi_step_noalloc(self.h, prob, **kw)

    def submit(self, prob):
        return mppi_submit(self.h, prob)

    def poll(self, ticket, K, T, **kw):
        return mppi_poll(self.h, ticket, K, T, **kw)

    def drain(self):
        return mppi_drain(self.h)

    def stats(self):
        s = mppi_stats()
        rc = load_library().mppi_get_stats(self.h, C.byref(s))
        if rc != MPPI_OK:
            raise MPPIError(rc, "mppi_get_stats")
        return {f: getattr(s, f) for f, _ in mppi_stats._fields_}

    def reset_stats(self):
        load_library().mppi_reset_stats(self.h)

    def batch(self, probs):
        return Batch(self.h, probs)

    def footprint(self, K, T, G):
        return int(load_library().mppi_solve_footprint(self.h, K, T, G))

    def close(self):
        if self.h is not None:
            mppi_destroy(self.h)
            self.h = None
            self._pool = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
