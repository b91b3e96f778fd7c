"""Benchmark: MPPI solves of the paper-scale workload on one MI355X.

Workload (one step = one MPPI iteration of every staged request): K = 4096
rollouts, horizon T = 50 (dt = 0.02 s), 4 gates, Gate-SDF decoder
67 -> 256 -> 256 -> 256 -> 1, seeded synthetic inputs (see scenarios/).
With --workload fleet: the large served fleet instead, 1024 instances of
K = 2048, T = 40, 8 gates, decoder 67 -> 512 -> 512 -> 512 -> 1, one step =
one control tick of every instance; --workload small: one small solve
(K = 256, T = 20, one gate, 67 -> 128 -> 128 -> 1).
The requests are staged into device memory before timing (mppi_batch_*), so
the timed region holds kernel launches only; each instance's warm start and
RNG tick advance on the device from step to step.

Prints one JSON line: rollout-steps/s (value), per-step latency p50/p99, the
roofline of the dominant kernel (HIP-event durations recorded by the library
on its own stream), the FP32 plain one-solve-per-launch path on the same
workload for comparison, the float32-accurate bfloat16-weight kinds of the
fused path (BF16X3, F16X2) beside the BF16 default, a served leg (uneven
requests arriving as a Poisson stream through mppi_submit / mppi_poll, with
latency probes of the workload's shape, and the highest load at which the
probes' p99 stays under 5 ms) and the FP64 oracle timed on the host cores
(all affinity cores, and one thread).

    python bench.py [--steps K] [--warmup W] [--path fused|plain]
                    [--precision bf16|bf16x3|f16x2|bf16x2|fp8|fp32] [--batch B]
                    [--workload paper|fleet|small]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import scenarios as sc  # noqa: E402

HBM_PEAK = 8.0e12
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "bf16x2": 2500.0, "bf16x3": 2500.0, "f16x2": 2500.0, "fp8": 5000.0}
# the workload (set by --workload): configuration name, shape, decoder
WORKLOADS = {"paper": ("P2", 1), "fleet": ("S2", 1024), "small": ("P1", 1)}   # name, default solves per step
CFG = "P2"
LAYERS = (67, 256, 256, 256, 1)
K_, T_, G_ = 4096, 50, 4


PE_FREQS = 0   # --pe-freqs: the decoder reads PE(p) with this many frequencies


def _set_workload(name, pe_freqs=0):
    global CFG, LAYERS, K_, T_, G_, PE_FREQS
    CFG = WORKLOADS[name][0]
    c = sc.CONFIGS[CFG]
    LAYERS, K_, T_, G_ = tuple(c["layers"]), c["K"], c["T"], c["G"]
    PE_FREQS = int(pe_freqs)
    LAYERS = (LAYERS[0] + 6 * PE_FREQS,) + LAYERS[1:]


def _workload_str():
    pe = f", PE with {PE_FREQS} frequencies" if PE_FREQS else ""
    return f"MPPI solve K={K_} T={T_} dt=0.02 G={G_} decoder " + "-".join(str(x) for x in LAYERS) + pe
KERNEL_SOURCES = {"plain": "kernels_plain.hip", "fused": "kernels_fused.hip"}


def _problems(n, M):
    return [sc.config_problem(CFG, 1 + i, instance_id=10_000 + i, tick=M.TICK_RESIDENT)
            for i in range(n)]


def _mfma_flops_per_query(layers):
    H = layers[1]
    n_hh = len(layers) - 3          # H x H layers
    return 2.0 * n_hh * H * H


# Vector-unit work of the decoder: one softplus per hidden neuron and query
# (768 at 67-256-256-256-1) of 8 lane-slots each: four full-rate operations
# (scale, 1 + e, max, fused multiply-add) and two transcendentals (base-2
# exponential and logarithm) that issue at half rate on gfx950 (measured:
# the counters give 8 cycles per wave64 transcendental against 4 for the
# other vector operations).  Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz of
# non-packed float32 issue.
SOFTPLUS_LANE_SLOTS = 8
VALU_PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9


def _softplus_per_query(layers):
    return sum(layers[1:-1])


KERNEL_HEADERS = ("device_common.hpp", "kernels.hpp", "ring.hpp", "solve_desc.hpp", "weights.hpp")


def _source_hash(path):
    """sha256 (first 16 hex digits) over the kernel source and the device
    headers it compiles with, in a fixed order."""
    h = hashlib.sha256()
    for name in (KERNEL_SOURCES[path],) + KERNEL_HEADERS:
        with open(os.path.join(ROOT, "paper_2603_07199_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(path, precision, launches_queries):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, or None when absent or taken on a different kernel."""
    f = os.path.join(ROOT, "profiles", f"traffic_{path}_{precision}_{CFG.lower()}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    if t.get("source_sha256_16") != _source_hash(path):
        return None
    return float(t["bytes_per_launch"])


def run_leg(M, path, precision, batch, steps, warmup):
    W, b = sc.xavier_weights(LAYERS, seed=0)
    probs = _problems(batch, M)
    eng = M.Engine((W, b), sc.MODEL, K_max=K_, T_max=T_, G_max=G_, hidden=LAYERS[1],
                   n_hidden=len(LAYERS) - 2, precision=precision, path=path,
                   budget=8 << 30, timing=True, max_instances=max(64, batch), pe_freqs=PE_FREQS)
    bt = eng.batch(probs)
    for _ in range(warmup):
        bt.run()
        bt.wait()
    eng.reset_stats()
    lat = []
    t_start = time.perf_counter()
    t_note = t_start
    for i in range(steps):
        t0 = time.perf_counter()
        bt.run()
        bt.wait()
        t1 = time.perf_counter()
        lat.append(t1 - t0)
        if t1 - t_note > 10.0:          # progress of long legs (fleet ticks)
            print(f"{path}/{precision}: {i + 1}/{steps} steps", file=sys.stderr, flush=True)
            t_note = t1
    elapsed = time.perf_counter() - t_start
    st = eng.stats()
    res = bt.results()
    bt.close()
    eng.close()
    for r in res:
        if r["status"] != 0:
            raise RuntimeError(f"solve failed with status {r['status']}")
    rs = batch * K_ * T_ * steps
    return {
        "rollout_steps_per_s": rs / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "lat_ms": np.array(lat) * 1e3,
        "sdf_ms": st["sdf_ms"] / max(st["sdf_launches"], 1),
        "sdf_launches": st["sdf_launches"],
        "solve_ms": st["solve_ms"] / max(st["solve_launches"], 1),
        "wide_region": int(st["wide_region"]),
    }


def _serve(M, eng, items, gap_scale, id_offset):
    """Submit items (arrival s, problem, is_probe) with arrival gaps scaled by
    gap_scale; return per-request latency (completion - arrival, host
    monotonic clock, the clock the library stamps completions with), the
    served rate and the offered rate."""
    tickets = []
    t0 = time.monotonic_ns()
    for arr, p, is_probe in items:
        p = dict(p, instance_id=p["instance_id"] + id_offset)
        t_arr = t0 + int(arr * gap_scale * 1e9)
        while time.monotonic_ns() < t_arr:
            pass
        rc, t = eng.submit(p)
        if rc != 0:
            raise RuntimeError(f"submit failed: {rc}")
        tickets.append((t, p, is_probe, t_arr))
    lat, lat_probe, done = [], [], {}
    work = 0
    t_first, t_last = None, None
    while len(done) < len(tickets):
        for t, p, is_probe, t_arr in tickets:
            if t in done:
                continue
            rc, r = eng.poll(t, p["K"], p["T"], weights=False, costs=False)
            if rc == M.MPPI_PENDING:
                continue
            if rc != 0:
                raise RuntimeError(f"served solve failed: {rc}")
            done[t] = True
            ms = (r["t_done_ns"] - t_arr) * 1e-6
            (lat_probe if is_probe else lat).append(ms)
            work += p["K"] * p["T"]
            t_first = t_arr if t_first is None else min(t_first, t_arr)
            t_last = r["t_done_ns"] if t_last is None else max(t_last, r["t_done_ns"])
    span = (t_last - t_first) * 1e-9
    return {"rollout_steps_per_s": work / span, "span_s": span,
            "probe_ms": np.array(lat_probe), "all_ms": np.array(lat + lat_probe),
            "offered_rollout_steps_per_s": work / (items[-1][0] * gap_scale),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "probe_latency_ms": {"p50": float(np.percentile(lat_probe, 50)),
                                 "p99": float(np.percentile(lat_probe, 99)), "n": len(lat_probe)}}


def served_leg(M, precision, n_req, plain_subset=64):
    """Uneven requests (K in {1024..8192}, T in {20..60}, G = 1, own instance
    each) arriving as a Poisson stream (mean gap 50 us), every 16th replaced by
    a probe of the benchmark shape (K=4096, T=50, G=4); served through
    mppi_submit / mppi_poll through the work ring of the persistent served
    kernel.  The stream runs twice: at the specified rate, and with the gaps
    stretched so that the offered work is 80% of the rate the first run
    served (latency under a load the GPU keeps up with); then the highest
    load that keeps the probes' p99 under 5 ms is searched.  The same two
    streams also run through the batched served launches, and the plain
    FP32 path runs the first plain_subset requests one solve per launch,
    back to back, for comparison."""
    reqs = sc.serving_requests(n_req=n_req)
    probe = sc.config_problem("P2", 99)
    items = []
    for i, (arr, p) in enumerate(reqs):
        if i % 16 == 15:
            p = dict(probe, instance_id=p["instance_id"])
        items.append((arr, p, i % 16 == 15))
    W, b = sc.config_weights("P2")
    eng = M.Engine((W, b), sc.MODEL, K_max=8192, T_max=60, G_max=4, hidden=256, n_hidden=3,
                   precision=precision, path="fused", budget=8 << 30, queue_depth=4096,
                   max_inflight=4096, max_instances=24 * n_req + 16)
    warm = dict(items[0][1], instance_id=24 * n_req + 8)
    rc, t = eng.submit(warm)
    while eng.poll(t, warm["K"], warm["T"])[0] == M.MPPI_PENDING:
        time.sleep(1e-4)
    eng.reset_stats()
    out = _serve(M, eng, items, 1.0, 0)
    out.pop("probe_ms"), out.pop("all_ms")
    out["requests"] = len(items)
    out["batches"] = int(eng.stats()["waves"])
    scale = out["offered_rollout_steps_per_s"] / (0.8 * out["rollout_steps_per_s"])
    if scale > 1.0:
        r80 = _serve(M, eng, items, scale, 2 * n_req)
        r80.pop("probe_ms"), r80.pop("all_ms")
        out["at_80pct_load"] = dict(r80, gap_scale=scale)
    # the highest offered load (a fraction of the rate served at the
    # specified one) at which the probes' p99 stays under 5 ms: the stream
    # twice per load (64 probes), loads tried from high to low
    ids = 4 * n_req
    best = None
    for frac in (1.0, 0.95, 0.9, 0.85, 0.8, 0.75, 0.7, 0.6, 0.5):
        sc_f = out["offered_rollout_steps_per_s"] / (frac * out["rollout_steps_per_s"])
        if sc_f <= 1.0:
            continue
        runs = []
        for _ in range(2):
            runs.append(_serve(M, eng, items, sc_f, ids))
            ids += n_req
        probes = np.concatenate([r["probe_ms"] for r in runs])
        every = np.concatenate([r["all_ms"] for r in runs])
        p99 = float(np.percentile(probes, 99))
        if p99 < 5.0:
            best = {"offered_rollout_steps_per_s": float(np.mean([r["offered_rollout_steps_per_s"] for r in runs])),
                    "served_rollout_steps_per_s": float(np.mean([r["rollout_steps_per_s"] for r in runs])),
                    "load_fraction": frac, "probe_latency_ms": {"p50": float(np.percentile(probes, 50)), "p99": p99,
                                                                "n": int(probes.size)},
                    "latency_ms": {"p50": float(np.percentile(every, 50)), "p99": float(np.percentile(every, 99))}}
            break
    out["max_load_probe_p99_under_5ms"] = best
    eng.close()
    # the same two streams through the batched served launches (one launch
    # per admission pass) instead of the work ring
    out["mode"] = "ring"
    engb = M.Engine((W, b), sc.MODEL, K_max=8192, T_max=60, G_max=4, hidden=256, n_hidden=3,
                    precision=precision, path="fused", budget=8 << 30, queue_depth=4096,
                    max_inflight=4096, max_instances=24 * n_req + 16, serve="batches")
    rc, t = engb.submit(warm)
    while engb.poll(t, warm["K"], warm["T"])[0] == M.MPPI_PENDING:
        time.sleep(1e-4)
    bat = {}
    for key, g, off in (("at_specified_rate", 1.0, 0), ("at_the_ring_80pct_stream", scale, 2 * n_req)):
        if key == "at_the_ring_80pct_stream" and scale <= 1.0:
            continue
        r = _serve(M, engb, items, g, off)
        r.pop("probe_ms"), r.pop("all_ms")
        bat[key] = r
    out["batched_launches"] = bat
    engb.close()
    # the same kind of requests through the plain FP32 one-solve-per-launch path
    sub = [p for _, p, _ in items[:plain_subset]]
    pe = M.Engine((W, b), sc.MODEL, K_max=8192, T_max=60, G_max=4, hidden=256, n_hidden=3,
                  precision="fp32", path="plain", budget=2 << 30, max_instances=4096)
    pe.step(dict(sub[0], instance_id=1 << 40))
    tp = time.perf_counter()
    pw = 0
    for p in sub:
        r = pe.step(p, weights=False, costs=False)
        if r["rc"] != 0:
            raise RuntimeError(f"plain solve failed: {r['rc']}")
        pw += p["K"] * p["T"]
    out["fp32_plain_same_requests_rollout_steps_per_s"] = pw / (time.perf_counter() - tp)
    pe.close()
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The FP64 oracle, as it stands, on a bounded sample of the workload,
    timed twice on the host: on every core of this process's affinity set and
    on one thread (torch intra-op threads and BLAS pools limited to 1).  The
    sample is the first K_s rollouts of one solve (rollout k's noise, dynamics
    and costs do not depend on K, so the rate is per rollout-step of the same
    work); for the fleet workload one instance, one tick."""
    import torch
    from threadpoolctl import threadpool_limits

    import oracle
    W, b = sc.xavier_weights(LAYERS, seed=0)
    cores = len(os.sched_getaffinity(0))

    def timed(prob, reps):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.solve(prob, (W, b), sc.MODEL)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    prob = sc.config_problem(CFG, 1)
    t_all = timed(prob, 3)
    k1 = max(64, min(K_, int(K_ * min(1.0, 10.0 / max(t_all * cores, 1e-3)))))
    prev = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        with threadpool_limits(1):
            t_one = timed(dict(prob, K=k1), 1)
    finally:
        torch.set_num_threads(prev)
    shape = f"T={T_}, G={G_}, {'-'.join(str(x) for x in LAYERS)} decoder"
    return {"value": K_ * T_ / t_all, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"one full solve of the workload (K={K_}, {shape}) in float64, median of 3: {t_all:.2f} s",
            "cpu_model": _cpu_model(),
            "single_thread": {"value": k1 * T_ / t_one, "unit": "rollout-steps/s", "cores": 1,
                              "sample": f"the first {k1} rollouts of the same solve, one thread: {t_one:.2f} s"}}


def _plain_copy(nbytes):
    """One device-to-device copy of ``nbytes`` through the HIP runtime's copy
    kernel: the known-size reference for the FETCH_SIZE / WRITE_SIZE counters.
    Called through the HIP runtime that the library itself loaded, so a counter
    run needs no torch in the process."""
    hip = ctypes.CDLL("libamdhip64.so.7")
    src, dst = ctypes.c_void_p(), ctypes.c_void_p()
    for ptr in (src, dst):
        if hip.hipMalloc(ctypes.byref(ptr), ctypes.c_size_t(nbytes)) != 0:
            raise RuntimeError("hipMalloc failed for the calibration copy")
    rc = hip.hipMemset(src, 1, ctypes.c_size_t(nbytes))
    rc = rc or hip.hipMemcpy(dst, src, ctypes.c_size_t(nbytes), 3)      # device to device
    rc = rc or hip.hipDeviceSynchronize()
    hip.hipFree(src)
    hip.hipFree(dst)
    if rc != 0:
        raise RuntimeError(f"calibration copy failed: {rc}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--path", default="fused", choices=["plain", "fused"])
    ap.add_argument("--precision", default="bf16", choices=["fp32", "bf16", "bf16x2", "bf16x3", "f16x2", "fp8"])
    ap.add_argument("--batch", type=int, default=0, help="solves per step (default: 1, fleet: 1024)")
    ap.add_argument("--workload", default="paper", choices=sorted(WORKLOADS))
    ap.add_argument("--pe-freqs", type=int, default=0,
                    help="decoder with the positional encoding of the query point (F frequencies)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=512)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs every solve on one GPU "
              "and shards nothing across GPUs; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    _set_workload(args.workload, args.pe_freqs)
    if args.batch <= 0:
        args.batch = WORKLOADS[args.workload][1]
    if args.precision == "fp8":
        raise SystemExit("bench.py runs the bfloat16 kinds and fp32; FP8 needs activation scales "
                         "calibrated per network (see the tests)")
    from paper_2603_07199_amd import mppi as M
    M.load_library()
    if args.copy_mib:
        _plain_copy(args.copy_mib << 20)

    print(f"bench: {_workload_str()}, {args.precision}, {args.steps} steps", file=sys.stderr, flush=True)
    main_leg = run_leg(M, args.path, args.precision, args.batch, args.steps, args.warmup)
    queries = args.batch * K_ * T_ * G_
    flops = _mfma_flops_per_query(LAYERS) * queries          # per launch of the dominant kernel
    achieved = flops / (main_leg["sdf_ms"] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    traffic = _traffic(args.path, args.precision, queries)
    out = {
        "metric": "rollout-steps/s and p50/p99 solve latency, BF16-served vs FP32-plain MPPI",
        "value": main_leg["rollout_steps_per_s"],
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "bf16x2": "bf16x2", "bf16x3": "bf16x3", "f16x2": "f16x2",
                  "fp8": "fp8"}[args.precision],
        "data": "synthetic",
        "config": {"workload": _workload_str(),
                   "path": args.path, "precision": args.precision, "solves_per_step": args.batch,
                   "parallelism": "single-gpu",
                   # H = 512: the weight-fragment read-ahead region tuned for this shape in warm-up
                   **({"wide_region_tuned": main_leg["wide_region"]}
                      if LAYERS[1] == 512 and args.path == "fused" else {})},
        "latency_ms": {"p50": float(np.percentile(main_leg["lat_ms"], 50)),
                       "p99": float(np.percentile(main_leg["lat_ms"], 99))},
        "roofline_valu": {"bound": "alu",
                          "achieved": _softplus_per_query(LAYERS) * SOFTPLUS_LANE_SLOTS * queries
                          / (main_leg["sdf_ms"] * 1e-3),
                          "peak": VALU_PEAK_LANE_SLOTS, "unit": "lane-slot/s",
                          "frac": _softplus_per_query(LAYERS) * SOFTPLUS_LANE_SLOTS * queries
                          / (main_leg["sdf_ms"] * 1e-3) / VALU_PEAK_LANE_SLOTS},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": "k_sdf_f32" if args.path == "plain" else ("k_wide" if LAYERS[1] == 512 else "k_fused"),
                     "kernel_ms": main_leg["sdf_ms"],
                     "algorithmic_flops_per_launch": flops},
    }
    if not args.no_compare and not (args.path == "plain" and args.precision == "fp32"):
        ref = run_leg(M, "plain", "fp32", 1, max(3, args.steps // 4), 1)
        out["fp32_plain"] = {"rollout_steps_per_s": ref["rollout_steps_per_s"],
                             "ms_per_step": ref["ms_per_step"],
                             "speedup": main_leg["rollout_steps_per_s"] / ref["rollout_steps_per_s"]}
    if not args.no_compare and args.path == "fused" and args.precision == "bf16":
        # the bfloat16-weight network at float32 accuracy (no activation
        # rounding): three bfloat16 products per K-step, or two FP16 ones
        for kind in ("bf16x3", "f16x2"):
            alt = run_leg(M, "fused", kind, args.batch, max(3, args.steps // 2), 1)
            out[kind] = {"rollout_steps_per_s": alt["rollout_steps_per_s"], "ms_per_step": alt["ms_per_step"],
                         "kernel_ms": alt["sdf_ms"],
                         "mfma_frac": flops / (alt["sdf_ms"] * 1e-3) / 1e12 / PEAK_TFLOPS[kind],
                         "speedup_vs_bf16": alt["rollout_steps_per_s"] / main_leg["rollout_steps_per_s"]}
    if not args.no_served and args.path == "fused" and args.workload == "paper" and not args.pe_freqs:
        out["served"] = served_leg(M, args.precision, args.served_requests)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
