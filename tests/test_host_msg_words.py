"""The SHAKE256 input blocks of mu = H(prefix || M) as the Sign and Verify kernels build them from
message bytes in memory (paper_2211_12265_amd/csrc/msg_words.h), replayed on the host under
AddressSanitizer and UndefinedBehaviorSanitizer (tests/msg_words_replay.cpp): for the round-3
prefix tr (32 bytes), ML-DSA's tr || 0x00 || 0x00 (66 bytes) and its tr alone before a
formatted message (64 bytes), every byte misalignment of M and
every length up to five blocks, the blocks equal the padded definition and no dword outside the
ones holding M's bytes is read."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2211_12265_amd", "csrc")


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("mw") / "msg_words_replay")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, "-o", exe, os.path.join(ROOT, "tests", "msg_words_replay.cpp")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return exe


def test_kernels_use_the_replayed_code():
    src = open(os.path.join(CSRC, "keccak_pair.h")).read()
    assert '#include "msg_words.h"' in src
    assert "mw_fetch<" in src and "mw_word<" in src and "MwPlan<" in src
    kern = open(os.path.join(CSRC, "kernels.h")).read()
    assert len(re.findall(r"absorb_prefix_msg<mu_prefix_bytes<LV, INTERNAL>\(\)>", kern)) == 2


@pytest.mark.parametrize("prefix", [32, 64, 66])
def test_blocks_match_definition(replay, prefix):
    res = subprocess.run([replay, str(prefix), "700"], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert re.search(r"ok PB=%d cases=2804" % prefix, res.stdout), res.stdout
