"""C ABI checks that need no GPU: the library loads and exports every function
declared in include/mppi.h, the ctypes structures match the C layout, status
strings, create() without a usable device, and the host-only engine logic
(arena, admission queue, solve layout) in a g++-built test driver."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_2603_07199_amd import mppi as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mppi.h")
CSRC = os.path.join(ROOT, "paper_2603_07199_amd", "csrc")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(mppi_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = M.load_library()
    names = _declared_functions()
    assert "mppi_create" in names and "mppi_poll" in names
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(M.EXPORTED) == names


def test_status_strings():
    assert M.status_str(0) == "ok"
    assert "invalid" in M.status_str(-1)
    assert M.status_str(12345) == "unknown status"


@pytest.fixture(scope="module")
def layout_probe(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc missing")
    d = tmp_path_factory.mktemp("abi")
    src = d / "probe.c"
    structs = {
        "mppi_config": M.mppi_config, "mppi_sdf_weights": M.mppi_sdf_weights,
        "mppi_gate": M.mppi_gate, "mppi_request": M.mppi_request,
        "mppi_result": M.mppi_result, "mppi_stats": M.mppi_stats,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            cf = "lambda" if f == "lambda_" else f
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = d / "probe"
    subprocess.run([gcc, "-std=c11", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    table = {}
    for line in out.splitlines():
        s, f, v = line.split()
        table[(s, f)] = int(v)
    return structs, table


def test_ctypes_layout_matches_header(layout_probe):
    structs, table = layout_probe
    for cname, cls in structs.items():
        assert C.sizeof(cls) == table[(cname, "size")], cname
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == table[(cname, f)], (cname, f)


def test_create_rejects_bad_config_or_reports_no_device():
    import scenarios as sc
    cfg = M.default_config(sc.MODEL)
    cfg["latent_dim"] = 32
    with pytest.raises(M.MPPIError) as e:
        M.mppi_create(cfg, None)
    assert e.value.code == M.MPPI_EINVAL
    cfg = M.default_config(sc.MODEL, sdf_kind="analytic")
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if not has_gpu:
        with pytest.raises(M.MPPIError) as e:
            M.mppi_create(cfg, None)
        assert e.value.code == M.MPPI_EDEVICE


HOST_TEST = r"""
#include <cassert>
#include <cstdio>
#include <random>
#include <vector>
#include "host_core.hpp"
using namespace mppi;
int main() {
  // arena: alloc/free/coalesce, alignment, exhaustion
  Arena a(1 << 20);
  uint64_t o1, o2, o3;
  assert(a.alloc(1000, &o1) && o1 == 0);
  assert(a.alloc(5000, &o2) && o2 == 1024);
  assert(a.alloc(1, &o3) && o3 == 1024 + 5120);
  assert(a.in_use() == 1024 + 5120 + 256);
  a.release(o2, 5000);
  uint64_t o4;
  assert(a.alloc(4000, &o4) && o4 == 1024);       // first fit reuses the hole
  a.release(o1, 1000); a.release(o4, 4000); a.release(o3, 1);
  assert(a.in_use() == 0 && a.fragments() == 1 && a.largest_free() == (1u << 20));
  uint64_t big;
  assert(!a.alloc((1 << 20) + 1, &big));
  std::mt19937 rng(3);
  std::vector<std::pair<uint64_t, uint64_t>> live;
  for (int i = 0; i < 20000; ++i) {
    if (live.empty() || (rng() % 3)) {
      uint64_t sz = 1 + rng() % 20000, off;
      if (a.alloc(sz, &off)) {
        for (auto& l : live) assert(off + align_up(sz) <= l.first || l.first + align_up(l.second) <= off);
        live.push_back({off, sz});
      }
    } else {
      size_t j = rng() % live.size();
      a.release(live[j].first, live[j].second);
      live.erase(live.begin() + j);
    }
  }
  for (auto& l : live) a.release(l.first, l.second);
  assert(a.in_use() == 0 && a.fragments() == 1);
  // admission: FIFO, budget, in-flight cap, busy instances, never-fits
  Admission q(1000, 2, 4);
  assert(q.push({1, 10, 400}) == 0);
  assert(q.push({2, 11, 700}) == 0);
  assert(q.push({3, 12, 100}) == 0);
  assert(q.push({4, 13, 1001}) == -2);
  assert(q.push({5, 10, 100}) == 0);
  assert(q.push({6, 14, 100}) == -3);             // depth 4 reached
  auto none = [](uint64_t) { return false; };
  auto adm = q.admit(none);
  assert(adm.size() == 1 && adm[0].ticket == 1);  // 2 does not fit, 3 may not overtake it
  q.complete(400);
  adm = q.admit(none);
  assert(adm.size() == 2 && adm[0].ticket == 2 && adm[1].ticket == 3);  // 700 + 100 fit
  adm = q.admit(none);
  assert(adm.empty());                            // in-flight cap of 2
  q.complete(700); q.complete(100);
  adm = q.admit([](uint64_t id) { return id == 10; });
  assert(adm.empty());                            // instance 10 busy
  adm = q.admit(none);
  assert(adm.size() == 1 && adm[0].ticket == 5);
  q.complete(100);
  // same instance twice in one pass: only the first is admitted
  Admission q2(1000, 8, 8);
  q2.push({7, 1, 10}); q2.push({8, 1, 10}); q2.push({9, 2, 10});
  adm = q2.admit(none);
  assert(adm.size() == 2 && adm[0].ticket == 7 && adm[1].ticket == 9);
  // requeue restores order and accounting
  q2.requeue_front(adm);
  assert(q2.in_use() == 0 && q2.inflight() == 0 && q2.queued() == 3);
  adm = q2.admit(none);
  assert(adm.size() == 2 && adm[0].ticket == 7 && adm[1].ticket == 9);
  // work cap per batch: stops before the item that would pass it; the first
  // item is taken whatever its work
  Admission q3(1 << 20, 16, 16);
  q3.push({20, 1, 10, 500}); q3.push({21, 2, 10, 400}); q3.push({22, 3, 10, 300}); q3.push({23, 4, 10, 5000});
  adm = q3.admit(none, 1000);
  assert(adm.size() == 2 && adm[0].ticket == 20 && adm[1].ticket == 21);
  adm = q3.admit(none, 1000);
  assert(adm.size() == 1 && adm[0].ticket == 22);
  adm = q3.admit(none, 1000);
  assert(adm.size() == 1 && adm[0].ticket == 23);
  // memory reserved outside the queue counts against the same budget
  Admission q4(1000, 4, 4);
  assert(q4.reserve(1001) == -2 && q4.reserve(600) == 0 && q4.reserve(500) == -3);
  q4.push({30, 1, 500, 1});
  assert(q4.admit(none).empty());
  q4.unreserve(600);
  adm = q4.admit(none);
  assert(adm.size() == 1 && q4.in_use() == 500);
  // instance id table: sized once, finds what was inserted, refuses past capacity
  IdTable ids;
  ids.reset(100);
  for (int i = 0; i < 100; ++i) assert(ids.insert(1000003ull * i + (1ull << 40), i));
  assert(!ids.insert(7, 100) && ids.size() == 100);
  for (int i = 0; i < 100; ++i) assert(ids.find(1000003ull * i + (1ull << 40)) == i);
  assert(ids.find(7) == -1 && !ids.contains(8));
  assert(ids.insert(1ull << 40, 55) && ids.find(1ull << 40) == 55 && ids.size() == 100);   // existing id
  // layout: regions are disjoint, aligned, and grow with K, T, G
  SolveLayout L = solve_layout(4096, 50, 4, 256, false, 0);
  assert(L.total % kAlign == 0 && L.upload_bytes <= L.result);
  assert(L.samples >= L.result && L.total >= L.samples + 4ull * 4 * 50 * 4096);
  SolveLayout F = solve_layout(4096, 50, 4, 256, true, 256);
  assert(F.total < L.total);
  SolveLayout FS = solve_layout(4096, 50, 4, 256, true, 256, true);   // fused with the field export
  assert(FS.sdf >= F.partials && FS.total >= FS.sdf + 4ull * 50 * 4096 && FS.total > F.total);
  std::printf("HOST OK\n");
  return 0;
}
"""


def test_host_core_logic(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ missing")
    src = tmp_path / "t.cpp"
    src.write_text(HOST_TEST)
    exe = tmp_path / "t"
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "HOST OK" in r.stdout


def test_request_marshals_unobserved_gates_as_null_latent():
    """gate_cached[g] → the request's gate g carries a NULL latent pointer
    (object permanence: the engine uses the instance's cached gate)."""
    import ctypes

    import scenarios as sc
    from paper_2603_07199_amd.mppi import _Request
    prob = sc.make_problem(8, 4, 3, seed=1)
    r = _Request(dict(prob, gate_cached=[False, True, False])).req
    assert bool(r.gates[0].z) and not bool(r.gates[1].z) and bool(r.gates[2].z)
    z0 = ctypes.cast(r.gates[0].z, ctypes.POINTER(ctypes.c_float))
    assert z0[5] == np.float32(prob["gate_z"][0][5])
    r_all = _Request(prob).req
    assert all(bool(r_all.gates[g].z) for g in range(3))


def test_config_flags_match_header():
    """The binding's config flag values are the header's (MPPI_CFG_*)."""
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mppi.h")).read()
    flags = {m.group(1): 1 << int(m.group(2)) for m in re.finditer(r"#define MPPI_CFG_(\w+) \(1u << (\d+)\)", hdr)}
    assert flags == {"TIMING": M.CFG_TIMING, "SERVE_BATCHES": M.CFG_SERVE_BATCHES}
    cfg = M.default_config({"mass": 1.0, "gravity": 9.81, "u_lo": [0] * 4, "u_hi": [1] * 4}, serve="batches")
    assert cfg["flags"] == M.CFG_SERVE_BATCHES
    with pytest.raises(ValueError):
        M.default_config({"mass": 1.0, "gravity": 9.81, "u_lo": [0] * 4, "u_hi": [1] * 4}, serve="waves")
