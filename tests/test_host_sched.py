"""The persistent Sign kernels' batch scheduling (paper_2211_12265_amd/csrc/batch_sched.h: claims from
the device work queue, slot assignment, retiring, scratch offsets) replayed on the host under
AddressSanitizer and UndefinedBehaviorSanitizer (tests/sched_replay.cpp), for the launch shapes the
benchmark and the tests use, the 715-workgroup / hmax-14 level-2 shape, and the edge cases (no tasks,
more workgroups than tasks, the attempt limit reached), in both batch layouts (slot by slot over the
held tasks, and task by task with contiguous wavefront ranges as the l = 4 kernels take them).  Every index the kernels derive from their
LDS state is checked, and every task must come out signed once at its smallest passing nonce."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2211_12265_amd", "csrc")

# G, L, K, tasks, workgroups, hmax, pass probability, attempt limit, wavefronts, tail slots per task,
# batch laid out task by task (the l = 4 four-wavefront kernels)
CASES = [
    (64, 4, 4, 10000, 715, 14, 0.235, 16384, 4, 0, 0),   # level 2, four wavefronts, automatic 3-per-CU grid
    (64, 4, 4, 10000, 512, 16, 0.235, 16384, 4, 0, 0),   # level 2 recorded schedule
    (48, 5, 6, 10000, 512, 12, 0.196, 16384, 4, 0, 0),   # level 3 recorded schedule
    (36, 7, 8, 10000, 512, 16, 0.260, 16384, 4, 0, 0),   # level 5 recorded schedule
    (32, 4, 4, 10000, 1024, 6, 0.235, 16384, 2, 0, 0),   # two wavefronts
    (16, 4, 4, 10000, 2048, 3, 0.235, 16384, 1, 0, 0),   # one wavefront
    (9, 7, 8, 100, 20000, 1, 0.260, 16384, 1, 0, 0),     # far more workgroups than tasks
    (64, 4, 4, 0, 512, 16, 0.235, 16384, 4, 0, 0),       # empty batch
    (64, 4, 4, 3000, 64, 64, 0.010, 8, 4, 0, 0),         # tasks dropped at the attempt limit
    (12, 5, 6, 777, 100, 12, 0.500, 16384, 1, 0, 0),     # hmax = G, ragged task count
    (64, 4, 4, 10000, 512, 16, 0.235, 16384, 4, 1, 0),   # short tail batches: one slot per task (rounded to 4)
    (64, 4, 4, 10000, 512, 16, 0.235, 16384, 4, 8, 0),   # level 2, tail of 8 slots per task
    (48, 5, 6, 10000, 512, 12, 0.196, 16384, 4, 12, 0),  # level 3, tail of 12
    (36, 7, 8, 10000, 512, 16, 0.260, 16384, 4, 5, 0),   # level 5, tail of 5 (not a multiple of W)
    (16, 4, 4, 10000, 2048, 3, 0.235, 16384, 1, 3, 0),   # one wavefront, tail of 3
    (64, 4, 4, 3000, 64, 64, 0.010, 8, 4, 2, 0),         # attempt limit reached in tail batches
    (64, 4, 4, 10000, 512, 16, 0.235, 16384, 4, 20, 1),  # level 2 / ML-DSA-44 recorded schedule, tail 20, by task
    (64, 4, 4, 10000, 512, 16, 0.235, 16384, 4, 0, 1),   # full batches, by task
    (64, 4, 4, 10000, 715, 14, 0.235, 16384, 4, 3, 1),   # 715 workgroups, tail 3 (batches of 4-64 slots)
    (64, 4, 4, 3000, 64, 64, 0.010, 8, 4, 1, 1),         # attempt limit, hmax = G, one slot per task
    (64, 4, 4, 777, 300, 5, 0.500, 16384, 4, 7, 1),      # more workgroups than tasks need, tail 7
    (64, 4, 4, 0, 512, 16, 0.235, 16384, 4, 20, 1),      # empty batch
]


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("sched") / "sched_replay")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, "-o", exe, os.path.join(ROOT, "tests", "sched_replay.cpp")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return exe


def test_kernels_use_the_replayed_code():
    src = open(os.path.join(CSRC, "persist.h")).read()
    assert '#include "batch_sched.h"' in src
    # both loop kernels assign and retire through batch_sched.h, and claim through it
    assert len(re.findall(r"sched_assign\(", src)) == 2
    # the four-wavefront kernel's tail batches come from the replayed sched_slots, laid out by
    # the replayed sched_assign / sched_assign_contig, its wavefronts' ranges from sched_wave_range
    assert len(re.findall(r"const int want = TAIL \? sched_slots\(nh, G, W, lds.queue_empty, tail\) : G;", src)) == 1
    assert len(re.findall(r"CONTIG \? sched_assign_contig\(nh, want, .*\n\s*: sched_assign\(nh, want, ", src)) == 1
    assert "sched_wave_range(ns, W, wave, s_lo, s_hi)" in src
    assert len(re.findall(r"sched_assign\(nh, G, ", src)) == 1
    assert len(re.findall(r"sched_retire\(", src)) == 2
    assert "sched_claim(atomicAdd(" in src
    assert src.count("scratch_idx<LV>(G)") == 2


@pytest.mark.parametrize("case", CASES, ids=[f"G{c[0]}-n{c[3]}-grid{c[4]}-h{c[5]}-t{c[9]}-c{c[10]}" for c in CASES])
@pytest.mark.parametrize("seed", [1, 2])
def test_schedule_replay(replay, case, seed):
    args = [str(x) for x in case[:8]] + [str(seed)] + [str(x) for x in case[8:]]
    res = subprocess.run([replay] + args, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    m = re.search(r"evaluated=(\d+) sequential=(\d+) dropped=(\d+)", res.stdout)
    assert m, res.stdout
    evaluated, sequential, dropped = map(int, m.groups())
    tasks = case[3]
    if tasks and case[7] > 1000:
        assert dropped == 0 and sequential >= tasks and evaluated >= sequential
    if case[7] == 8:
        assert dropped > 0
