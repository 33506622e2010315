"""Host-side logic that needs no GPU: the recorded-schedule cache, the gate that ties
stored HBM counter results to the kernel sources, the serving trace generator and the
synthetic input generators."""
import json
import os

import numpy as np

from paper_2211_12265_amd import autotune, serving, workload


def test_schedule_cache_round_trip(tmp_path):
    path = str(tmp_path / "sched.json")
    assert autotune.cached_schedule(2, 10000, "fixed32", path) is None
    autotune.store_schedule(2, 10000, "fixed32", {"waves": 4, "hmax": 16, "grid": 512, "ms": 1.5}, path)
    autotune.store_schedule(5, 10000, "uniform", {"waves": 2, "hmax": 4, "grid": 1024}, path)
    assert autotune.cached_schedule(2, 10000, "fixed32", path) == {"waves": 4, "hmax": 16, "grid": 512}
    assert autotune.cached_schedule(5, 10000, "uniform", path) == {"waves": 2, "hmax": 4, "grid": 1024}
    assert autotune.cached_schedule(3, 10000, "uniform", path) is None
    assert set(json.load(open(path))) == {"L2/10000/fixed32", "L5/10000/uniform"}


def test_recorded_schedules_are_valid():
    for key, sched in autotune.load_cache().items():
        level = int(key.split("/")[0][1:])
        assert sched["waves"] in (1, 2, 4)
        assert 1 <= sched["hmax"] <= autotune.slots_per_batch(level, sched["waves"])
        assert sched["grid"] >= 1


def test_stored_traffic_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    import bench
    src = bench.kernel_source_hash()
    assert src == bench.kernel_source_hash() and len(src) == 64
    rec = {"kernel": "k<2>", "level": 2, "count": 10, "msg_dist": "fixed32", "schedule": "4,16,512",
           "fetch_bytes": 100, "write_bytes": 50, "source_sha256": src, "profile": "p.md"}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "hbm_traffic.json").write_text(json.dumps([rec]))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: src)
    assert bench.stored_traffic("k<2>", 2, 10, "fixed32", "4,16,512")["fetch_bytes"] == 100
    assert bench.stored_traffic("k<2>", 2, 10, "fixed32", "2,4,1024") is None      # other launch configuration
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.stored_traffic("k<2>", 2, 10, "fixed32", "4,16,512") is None      # kernels changed since


def test_serving_trace_mix():
    keys = {2: 512, 3: 307, 5: 205}
    r = serving.build_requests(20000, lam=1e5, keys_per_level=keys, seed=3)
    assert len(r) == 20000
    assert np.all(np.diff(r.t_arrival) >= 0)
    rate = len(r) / r.t_arrival[-1]
    assert 0.95e5 < rate < 1.05e5
    assert abs(float(np.mean(r.op == serving.VERIFY)) - 0.7) < 0.02
    for lv, p in ((2, 0.5), (3, 0.3), (5, 0.2)):
        sel = r.level == lv
        assert abs(float(np.mean(sel)) - p) < 0.02
        assert r.key[sel].min() >= 0 and r.key[sel].max() < keys[lv]
    lens = np.diff(r.msg_off)
    assert lens.min() >= 1 and lens.max() <= 16384
    assert 200 < np.median(lens) < 320          # lognormal, median 256 bytes
    # saturation traces put every request at t = 0
    z = serving.build_requests(100, lam=0.0, keys_per_level=keys, seed=3)
    assert np.all(z.t_arrival == 0)


def test_input_generators_are_seeded():
    a1, o1 = workload.messages(workload.uniform_lengths(50, 0, 300, seed=7), seed=7)
    a2, o2 = workload.messages(workload.uniform_lengths(50, 0, 300, seed=7), seed=7)
    b1, _ = workload.messages(workload.uniform_lengths(50, 0, 300, seed=8), seed=8)
    assert np.array_equal(a1, a2) and np.array_equal(o1, o2)
    assert not (len(a1) == len(b1) and np.array_equal(a1, b1))
    assert o1[0] == 0 and np.all(np.diff(o1.astype(np.int64)) >= 0)
    s = workload.keygen_seeds(4, seed=1)
    assert s.shape == (4, 32) and s.dtype == np.uint8


def test_serving_trace_check_rejects_bad_requests():
    """The Python serving loop refuses, before any device work, a trace whose key rows fall
    outside their level's table (the device would read past the table), an unknown level
    or op, unsorted arrivals and bad message offsets."""
    import pytest
    keys = {2: 12, 3: 7, 5: 5}
    reqs = serving.build_requests(200, lam=1000.0, keys_per_level=keys, seed=3)
    reqs.sig_in = np.zeros(1, np.uint8)
    reqs.sig_off = np.zeros(len(reqs), np.int64)
    serving.check_requests(reqs, keys)
    bad_cases = []
    r = serving.Requests(**vars(reqs)); r.key = reqs.key.copy(); r.key[np.argmax(reqs.level == 3)] = 7
    bad_cases.append((r, keys))
    r = serving.Requests(**vars(reqs)); r.key = reqs.key.copy(); r.key[0] = -1
    bad_cases.append((r, keys))
    bad_cases.append((reqs, {2: 12, 3: 7}))
    r = serving.Requests(**vars(reqs)); r.op = reqs.op.copy(); r.op[5] = 2
    bad_cases.append((r, keys))
    r = serving.Requests(**vars(reqs)); r.t_arrival = reqs.t_arrival[::-1].copy()
    bad_cases.append((r, keys))
    r = serving.Requests(**vars(reqs)); r.msg_off = reqs.msg_off.copy(); r.msg_off[3] = r.msg_off[4] + 1
    bad_cases.append((r, keys))
    for r, k in bad_cases:
        with pytest.raises(ValueError):
            serving.check_requests(r, k)


def test_binding_rejects_undersized_buffers():
    """The ctypes binding checks buffer sizes and element widths on the host before a call
    is launched (the kernels index rows and offsets without bounds checks)."""
    import pytest
    import torch
    from paper_2211_12265_amd.dilithium import _require
    n = 5
    off = torch.zeros(n + 1, dtype=torch.int64)
    sig = torch.zeros((n, 2420), dtype=torch.uint8)
    _require([(off, 8 * (n + 1), 8, "msg_off"), (sig, 2420 * n, 1, "sig"), (None, 4 * n, 4, "key_idx")])
    with pytest.raises(ValueError):
        _require([(off[:n], 8 * (n + 1), 8, "msg_off")])
    with pytest.raises(ValueError):
        _require([(off.to(torch.int32), 8 * (n + 1), 8, "msg_off")])
    with pytest.raises(ValueError):
        _require([(sig[:n - 1], 2420 * n, 1, "sig")])
    with pytest.raises(ValueError):
        _require([(torch.zeros(n, dtype=torch.int64), 4 * n, 4, "key_idx")])


def test_error_word_reporting(tmp_path):
    """The decision of which device-detected condition a context reports (csrc/errwords.h), on
    the host with g++: every condition that is set is named, the code is the most severe one
    (dropped Sign tasks, then an out-of-table key index, then a decreasing msg_off)."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "errwords_check.cpp"
    src.write_text(r'''
#include <stdio.h>
#include "errwords.h"
int main() {
  char t[256];
  for (int m = 0; m < 8; m++) {
    int code = dil::report_error_words(m & 1, (m >> 1) & 1, (m >> 2) & 1, t, sizeof t);
    printf("%d|%d|%s\n", m, code, t);
  }
  char small[8];
  dil::report_error_words(1, 1, 1, small, sizeof small);   // truncated, still terminated
  printf("8|%d|%s\n", (int)strlen(small), small);
  return 0;
}''')
    exe = tmp_path / "errwords_check"
    subprocess.run(["g++", "-std=c++17", "-include", "string.h", "-I",
                    os.path.join(root, "paper_2211_12265_amd", "csrc"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines()
    rows = {int(r.split("|")[0]): r.split("|", 2)[1:] for r in out}
    from paper_2211_12265_amd import dilithium as dl
    for m in range(8):
        dropped, msg, key = m & 1, (m >> 1) & 1, (m >> 2) & 1
        code, text = int(rows[m][0]), rows[m][1]
        want = dl.DIL_EHIP if dropped else dl.DIL_EINVAL if key else dl.DIL_EMSG if msg else dl.DIL_OK
        assert code == want, (m, code)
        assert ("iteration limit" in text) == bool(dropped)
        assert ("msg_off" in text) == bool(msg)
        assert ("key table" in text) == bool(key)
    assert int(rows[8][0]) == 7
