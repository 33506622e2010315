"""Benchmark: Dilithium2 batch of 10,000 Sign + 10,000 Verify on one MI355X.

One step = dil_sign_batch over 10,000 tasks (32-byte messages, one key per
task) followed by dil_verify_batch over the 10,000 signatures just produced,
all buffers resident in HBM.  Keys are generated on the GPU before timing.
Prints ONE JSON line (rank 0) with the roofline of the Sign loop kernel
(algorithmic int32 lane-ops per launch over its HIP-event time, against the
chip's 32-bit integer issue rate) and the CPU oracle's rate on the same batch.

  python bench.py [--steps K] [--warmup W] [--mode persistent|staged]
                  [--count N] [--level 2|3|5|44|65|87] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# The serving engine runs every (level, op) group of a batch on its own HIP stream; HIP gives a
# process 4 hardware queues by default, which serialises them.  Must be set before HIP starts.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per operation in int32 lane-ops (a 64-bit logical op or
# rotation counts as two 32-bit ops): Keccak-f[1600] 7440 per permutation,
# one NTT or INTT 7168 (1024 butterflies x (4 mul + 3 add/sub)), one pointwise
# product 1536 (256 x 6).  Per-level counts of permutations / transforms /
# pointwise products per Sign iteration and per fixed part of each operation:
PERM_OPS, XFORM_OPS, PW_OPS = 7440, 7168, 1536
PER_LEVEL = {
    # level: (k, l); ML-DSA-44 / 65 / 87 share the lattice parameters of levels 2 / 3 / 5
    2: (4, 4), 3: (6, 5), 5: (8, 7), 44: (4, 4), 65: (6, 5), 87: (8, 7),
}
MLDSA_BASE = {44: 2, 65: 3, 87: 5}
# SHAKE blocks: rate 136 (SHAKE256), 168 (SHAKE128)
W1_BYTES = {2: 4 * 192, 3: 6 * 128, 5: 8 * 128, 44: 4 * 192, 65: 6 * 128, 87: 8 * 128}
PK_BYTES = {2: 1312, 3: 1952, 5: 2592, 44: 1312, 65: 1952, 87: 2592}
SK_BYTES = {2: 2528, 3: 4000, 5: 4864, 44: 2560, 65: 4032, 87: 4896}
SIG_BYTES = {2: 2420, 3: 3293, 5: 4595, 44: 2420, 65: 3309, 87: 4627}


def level_name(level: int) -> str:
    return f"ML-DSA-{level}" if level in MLDSA_BASE else f"Dilithium{level}"


def mu_prefix(level: int) -> int:
    """bytes hashed before the message for mu: tr (32), or ML-DSA's tr || 0x00 || 0x00 (66)"""
    return 66 if level in MLDSA_BASE else 32
# 256 CUs x 4 SIMDs x 32 lanes of simple 32-bit integer ops per clock x 2.4 GHz
PEAK_INT32_OPS = 256 * 4 * 32 * 2.4e9   # 78.6 T int32 lane-ops/s


def kernel_source_hash() -> str:
    """sha256 over the HIP sources (file names and contents) that define the kernels and their
    launches, to tie stored counter results to the kernels they were taken on (server.hip, the
    host-only serving engine, is left out)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2211_12265_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".h", ".hip")) and name != "server.hip":
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def stored_traffic(kernel: str, level: int, count: int, msg_dist: str, schedule: str):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, copy-calibrated) recorded in
    profiles/hbm_traffic.json for this kernel and launch configuration, or None when there is no
    record or the kernels have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        recs = json.load(f)
    src = kernel_source_hash()
    for r in recs:
        if (r["kernel"], r["level"], r["count"], r["msg_dist"], r["schedule"]) == \
                (kernel, level, count, msg_dist, schedule) and r["source_sha256"] == src:
            return r
    return None


def perms_shake(inlen: int, outlen: int, rate: int) -> int:
    return inlen // rate + 1 + max(0, -(-outlen // rate) - 1)


def sign_iteration_ops(level: int) -> float:
    """Algorithmic int32 ops of one Sign loop iteration (Alg. 2 loop body)."""
    k, l = PER_LEVEL[level]
    gamma1_17 = MLDSA_BASE.get(level, level) == 2
    it_perms = l * perms_shake(66, 576 if gamma1_17 else 640, 136) + perms_shake(64 + W1_BYTES[level], 32, 136) + 1
    it_x = l + k + 1 + l + 2 * k          # NTT(y), INTT(w), NTT(c), INTT(c s1), INTT(c s2), INTT(c t0)
    it_pw = k * l + l + 2 * k             # A y, c s1, c s2, c t0
    return it_perms * PERM_OPS + it_x * XFORM_OPS + it_pw * PW_OPS


def sign_setup_ops(level: int, msg_lens: np.ndarray) -> float:
    """Algorithmic int32 ops of the per-task part before the loop (mu, rho', ExpandA, NTT of s1, s2, t0)."""
    k, l = PER_LEVEL[level]
    perms = sum(perms_shake(mu_prefix(level) + int(m), 64, 136) for m in msg_lens)
    perms += len(msg_lens) * (perms_shake(128 if level in MLDSA_BASE else 96, 64, 136) + k * l * 5)
    return perms * PERM_OPS + len(msg_lens) * (l + 2 * k) * XFORM_OPS


def sign_work(level: int, msg_lens: np.ndarray, iterations: int) -> float:
    """Algorithmic int32 ops for a Sign batch with the given total (sequential) loop iterations."""
    return sign_setup_ops(level, msg_lens) + iterations * sign_iteration_ops(level)


def verify_work(level: int, msg_lens: np.ndarray) -> float:
    k, l = PER_LEVEL[level]
    n = len(msg_lens)
    perms = n * (perms_shake(PK_BYTES[level], 32, 136) + k * l * 5 + 1 + perms_shake(64 + W1_BYTES[level], 32, 136))
    perms += sum(perms_shake(mu_prefix(level) + int(m), 64, 136) for m in msg_lens)
    xf = n * (l + k + 1 + k)
    pw = n * (k * l + k)
    return perms * PERM_OPS + xf * XFORM_OPS + pw * PW_OPS


def cpu_baseline(level: int, seeds, msg, off, msg_desc: str, gpu_sig, min_seconds: float,
                 single: int = 1000) -> dict:
    """The CPU oracle on the host's cores over the benchmark's own batch: the same keys (KeyGen from the
    same seeds, untimed) and the same messages.  Sign and Verify of the whole batch are repeated until
    min_seconds of wall time have passed and the median repetition gives the rate.  The oracle's
    signatures are compared byte for byte with the GPU's signatures of the timed batch.  The only place
    the benchmark runs the oracle."""
    import oracle
    threads = oracle.default_threads()
    n = seeds.shape[0]
    pk, sk = oracle.keygen_batch(level, seeds, nthreads=threads)
    sign_t, ver_t, parity = [], [], None
    start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        sig, _ = oracle.sign_batch(level, sk, msg, off, nthreads=threads)
        t1 = time.perf_counter()
        v = oracle.verify_batch(level, pk, msg, off, sig, nthreads=threads)
        t2 = time.perf_counter()
        assert int(v.sum()) == n
        if parity is None:
            parity = bool(np.array_equal(sig, gpu_sig))
        sign_t.append(t1 - t0)
        ver_t.append(t2 - t1)
        if t2 - start >= min_seconds:
            break
    sign_s, ver_s, wall = float(np.median(sign_t)), float(np.median(ver_t)), time.perf_counter() - start
    # one host thread (the paper's CPU reference column is single-threaded), on the first
    # `single` tasks of the same batch, once
    m = min(single, n)
    t0 = time.perf_counter()
    s1, _ = oracle.sign_batch(level, sk[:m], msg[:int(off[m])], off[:m + 1], nthreads=1)
    t1 = time.perf_counter()
    v1 = oracle.verify_batch(level, pk[:m], msg[:int(off[m])], off[:m + 1], s1, nthreads=1)
    t2 = time.perf_counter()
    assert int(v1.sum()) == m and np.array_equal(s1, sig[:m])
    single_thread = {"value": m / (t2 - t0), "unit": "sign+verify pairs/s", "cores": 1, "kind": "oracle",
                     "sign_per_s": m / (t1 - t0), "verify_per_s": m / (t2 - t1),
                     "sample": f"the first {m} tasks of the same batch, signed and verified once on one thread"}
    return {"value": n / (sign_s + ver_s), "unit": "sign+verify pairs/s", "cores": threads, "kind": "oracle",
            "sign_per_s": n / sign_s, "verify_per_s": n / ver_s, "repetitions": len(sign_t), "wall_s": wall,
            "timed_batch_parity": parity, "single_thread": single_thread,
            "sample": f"the benchmark's whole batch ({n} {level_name(level)} sign + {n} verify, {msg_desc}, the same "
                      f"keys and messages as the GPU run), repeated {len(sign_t)} times ({wall:.1f} s wall, median "
                      f"repetition); plain C oracle on {threads} host threads"}


NTT_FORMS = [(3, "unfused: NTT, pointwise, INTT as three launches through HBM"),
             (2, "fused, one LDS round trip per butterfly level"),
             (1, "fused, levels merged in registers, unpadded LDS transpose"),
             (0, "fused, levels merged in registers, padded LDS transpose (production)")]


def micro_run(steps: int, warmup: int) -> dict:
    """The primitive workloads at 2^20 polynomials: c = INTT(NTT(a) o b) in each form of the
    NTT optimisation ablation, ExpandA from 34-byte inputs, and a plain device copy of the
    same size as the HBM ceiling actually reachable.  Median HIP-event time per call."""
    import torch
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import workload
    n = 1 << 20
    ctx = dl.Context(0)
    ga = torch.from_numpy(workload.uniform_polys(n, seed=0)).cuda()
    gb = torch.from_numpy(workload.uniform_polys(n, seed=0, tag="dil/poly2")).cuda()
    out = torch.empty((n, 256), dtype=torch.int32, device="cuda")
    ref = torch.empty_like(out)

    def timed(fn):
        for _ in range(warmup):
            fn()
        ts = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    res = {"polys": n}
    copy_ms = timed(lambda: out.copy_(ga))
    res["device_copy"] = {"ms": copy_ms, "GB_per_s": 2 * ga.numel() * 4 / copy_ms / 1e6}
    ntt_bytes = 3 * 1024        # a and b read, c written: 1 KiB each per polynomial
    ntt_ops = 2 * XFORM_OPS + PW_OPS
    forms = []
    for variant, name in NTT_FORMS:
        ctx.set_param("ntt.variant", variant)
        ms = timed(lambda: ctx.ntt_mul(ga, gb, out))
        torch.cuda.synchronize()
        if variant == 3:
            ref.copy_(out)
        forms.append({"variant": variant, "form": name, "ms": ms, "polys_per_s": n / ms * 1e3,
                      "GB_per_s": n * ntt_bytes / ms / 1e6, "hbm_frac": n * ntt_bytes / ms / 1e6 / 8000.0,
                      "alu_frac": n * ntt_ops / (ms / 1e3) / PEAK_INT32_OPS,
                      "same_words_as_unfused": bool(torch.equal(out, ref))})
    ctx.set_param("ntt.variant", 0)
    res["ntt_mul"] = {"algorithmic_bytes_per_poly": ntt_bytes, "algorithmic_ops_per_poly": ntt_ops,
                      "forms": forms}
    del ga, gb, ref
    seeds = torch.from_numpy(workload.expand_a_inputs(n, seed=0)).cuda()
    ms = timed(lambda: ctx.expand_a(seeds, out))
    ea_ops, ea_bytes = 5 * PERM_OPS, 34 + 1024
    res["expand_a"] = {"ms": ms, "polys_per_s": n / ms * 1e3, "GB_per_s": n * ea_bytes / ms / 1e6,
                       "hbm_frac": n * ea_bytes / ms / 1e6 / 8000.0,
                       "alu_frac": n * ea_ops / (ms / 1e3) / PEAK_INT32_OPS,
                       "algorithmic_bytes_per_poly": ea_bytes, "algorithmic_ops_per_poly": ea_ops}
    ctx.close()
    return res


T0_FORMS = [(3, "basic: unpack kernel, t0 through HBM, NTT kernel (unpadded transpose)"),
            (2, "fused kernel, same memory access pattern (t0 through HBM inside the kernel)"),
            (1, "unpacking merged into the NTT's registers (unpadded transpose)"),
            (0, "merged + padded transpose (the Sign setup's code path)")]


def t0_ablation_run(steps: int, warmup: int, levels=(2, 5), counts=(10000, 100000)) -> dict:
    """The NTT(t0) stage of signing (dil_t0_ntt_batch) in the four forms of the optimisation
    ablation, on keys generated on the GPU; median HIP-event time per call.  Then the padding
    step inside the Sign loop kernel: the level-2 benchmark batch signed with the recorded
    schedule on padded ("persist.pad" 1) and unpadded (0) transposes, interleaved."""
    import torch
    from paper_2211_12265_amd import autotune
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import workload
    ctx = dl.Context(0)

    def timed(fn):
        for _ in range(warmup):
            fn()
        ts = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    rows = []
    for level in levels:
        k = PER_LEVEL[level][0]
        pkl, skl, _ = dl.sizes(level)
        for n in counts:
            pk = torch.zeros((n, pkl), dtype=torch.uint8, device="cuda")
            sk = torch.zeros((n, skl), dtype=torch.uint8, device="cuda")
            ctx.keygen(level, torch.from_numpy(workload.keygen_seeds(n, seed=level)).cuda(), pk, sk)
            out = torch.empty((n, k, 256), dtype=torch.int32, device="cuda")
            ref = None
            nbytes = n * k * (416 + 1024)   # packed t0 read, NTT(t0) written
            for variant, name in T0_FORMS:
                ctx.set_param("t0.variant", variant)
                ms = timed(lambda: ctx.t0_ntt(level, sk, out))
                torch.cuda.synchronize()
                if ref is None:
                    ref = out.clone()
                rows.append({"level": level, "keys": n, "variant": variant, "form": name, "ms": ms,
                             "polys_per_s": n * k / ms * 1e3, "GB_per_s": nbytes / ms / 1e6,
                             "alu_frac": n * k * XFORM_OPS / (ms / 1e3) / PEAK_INT32_OPS,
                             "same_words_as_basic": bool(torch.equal(out, ref))})
            ctx.set_param("t0.variant", 0)
            del pk, sk, out, ref
    ctx.close()
    # padding inside the Sign loop kernel
    level, n = 2, 10000
    pkl, skl, sgl = dl.sizes(level)
    sched = autotune.cached_schedule(level, n, "fixed32")
    loop = {}
    c0 = dl.Context(0)
    sk = torch.zeros((n, skl), dtype=torch.uint8, device="cuda")
    c0.keygen(level, torch.from_numpy(workload.keygen_seeds(n, seed=0)).cuda(),
              torch.zeros((n, pkl), dtype=torch.uint8, device="cuda"), sk)
    msg, off = workload.messages(workload.fixed_lengths(n, 32), seed=0)
    gm, go = torch.from_numpy(msg).cuda(), torch.from_numpy(off.astype(np.int64)).cuda()
    ctxs, sigs = {}, {}
    for pad in (1, 0):
        c = dl.Context(0, mode=dl.MODE_PERSISTENT)
        autotune.apply_schedule(c, sched)
        c.set_param("persist.pad", pad)
        c.set_param("timing", 1)
        ctxs[pad] = c
        sigs[pad] = torch.zeros((n, sgl), dtype=torch.uint8, device="cuda")
    times = {1: [], 0: []}
    for _ in range(3):
        for pad in (1, 0):
            c = ctxs[pad]
            for _ in range(warmup):
                c.sign(level, sk, gm, go, sigs[pad])
            c.set_param("timing", 1)
            for _ in range(steps):
                c.sign(level, sk, gm, go, sigs[pad])
            torch.cuda.synchronize()
            times[pad] += c.sign_timing(steps)[1]
    for pad in (1, 0):
        loop["padded" if pad else "unpadded"] = {"loop_ms_median": float(np.median(times[pad])),
                                                 "schedule": sched}
        ctxs[pad].close()
    loop["same_signatures"] = bool(torch.equal(sigs[0], sigs[1]))
    c0.close()
    return {"t0_ntt": rows, "sign_loop_kernel_L2_10k": loop}


def serving_run(n_requests: int, seconds: float, streams: int, max_batch: int, short: bool = False) -> dict:
    """Serving loop on 1024 resident key pairs (512 / 307 / 205 at levels 2 / 3 / 5): first a
    saturation probe (all requests at t = 0), then a Poisson stream at half that rate.  `short`
    (the default benchmark line): one saturation pass over n_requests and n_requests Poisson
    arrivals, no load sweep."""
    import torch
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import serving as sv
    from paper_2211_12265_amd import workload
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT)
    keys = {2: 512, 3: 307, 5: 205}
    keysets = {}
    for lv, nk in keys.items():
        pkl, skl, _ = dl.sizes(lv)
        pk = torch.zeros((nk, pkl), dtype=torch.uint8, device="cuda")
        sk = torch.zeros((nk, skl), dtype=torch.uint8, device="cuda")
        ctx.keygen(lv, torch.from_numpy(workload.keygen_seeds(nk, seed=300 + lv)).cuda(), pk, sk)
        keysets[lv] = dl.KeySet(ctx, lv, pk=pk, sk=sk)
    resident = sum(ks.device_bytes() for ks in keysets.values())
    server = sv.NativeServer(keysets, n_streams=streams, max_batch=max_batch, mem_budget=8 << 30)
    # warm-up and saturation probe
    warm = sv.build_requests(4000, lam=0.0, keys_per_level=keys, seed=11)
    sv.attach_signatures(warm, ctx, keysets, seed=11)
    server.serve(warm)
    # saturation: at least 400k requests, all at t = 0, twice; the faster pass counts (a short probe
    # is dominated by its first and last batches)
    sat_reqs = sv.build_requests(n_requests if short else max(n_requests, 400_000), lam=0.0, keys_per_level=keys,
                                 seed=12)
    sv.attach_signatures(sat_reqs, ctx, keysets, seed=12)
    sat_rate = max(len(sat_reqs) / server.serve(sat_reqs).wall for _ in range(1 if short else 2))
    sweep = []
    for frac in (() if short else (0.25, 0.75)):     # latency at a lighter and a heavier load, beside 0.5
        lam_f = frac * sat_rate
        cnt_f = int(min(max(n_requests // 2, lam_f * seconds / 2), 1_000_000))
        r_f = sv.build_requests(cnt_f, lam=lam_f, keys_per_level=keys, seed=14)
        sv.attach_signatures(r_f, ctx, keysets, seed=14)
        s_f = sv.latency_summary(server.serve(r_f), r_f)
        sweep.append({"load": frac, "lambda_per_s": lam_f, "ops_per_s": s_f["ops_per_s"], "p50_ms": s_f["p50_ms"],
                      "p99_ms": s_f["p99_ms"]})
    lam = 0.5 * sat_rate
    count = n_requests if short else int(min(max(n_requests, lam * seconds), 2_000_000))
    reqs = sv.build_requests(count, lam=lam, keys_per_level=keys, seed=13)
    flipped = sv.attach_signatures(reqs, ctx, keysets, seed=13)
    res = server.serve(reqs)
    summ = sv.latency_summary(res, reqs)
    summ["load_sweep"] = sweep
    verify = reqs.op == sv.VERIFY
    summ.update({"engine": "native dil_server", "lambda_per_s": lam, "saturated_ops_per_s": sat_rate,
                 "streams": streams, "max_batch": max_batch, "trace": "short" if short else "full",
                 "resident_key_bytes": resident, "flipped_rejected": bool((res.verdict[verify & flipped] == 0).all()),
                 "valid_accepted": bool((res.verdict[verify & ~flipped] == 1).all()),
                 "mix": "70% verify / 30% sign, levels 2/3/5 at 50/30/20%, lognormal messages (median 256 B, "
                        "cap 16 KiB), 1024 resident key pairs"})
    server.close()
    for ks in keysets.values():
        ks.close()
    ctx.close()
    return summ


def staged_run(level: int, sk, pk, gm, go, ref_sig, steps: int = 5) -> dict:
    """The plain staged form (one launch per stage, host-driven rejection loop) on the same keys,
    messages and batch as the timed persistent run: Sign and Verify timed separately (median of
    `steps`), signatures compared byte for byte with the persistent form's."""
    import torch
    from paper_2211_12265_amd import dilithium as dl
    n = go.shape[0] - 1
    ctx = dl.Context(0, mode=dl.MODE_STAGED)
    sig = torch.zeros_like(ref_sig)
    ver = torch.zeros(n, dtype=torch.int32, device="cuda")
    ctx.sign(level, sk, gm, go, sig)
    ctx.verify(level, pk, gm, go, sig, ver)
    torch.cuda.synchronize()
    ts, tv = [], []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        ctx.sign(level, sk, gm, go, sig)
        e[1].record()
        ctx.verify(level, pk, gm, go, sig, ver)
        e[2].record()
        torch.cuda.synchronize()
        ts.append(e[0].elapsed_time(e[1]))
        tv.append(e[1].elapsed_time(e[2]))
    same = bool(torch.equal(sig, ref_sig))
    ok = bool(int(ver.sum()) == n)
    ctx.close()
    sm, vm = float(np.median(ts)), float(np.median(tv))
    return {"form": "staged (one launch per stage, host-driven rejection loop; Verify on one stream)",
            "sign_per_s": n / (sm * 1e-3), "verify_per_s": n / (vm * 1e-3), "sign_ms_median": sm,
            "verify_ms_median": vm, "value": n / ((sm + vm) * 1e-3), "unit": "sign+verify pairs/s",
            "same_signatures_as_persistent": same, "all_verified": ok, "steps": steps}


PROBE_KINDS = ["v_xor_b32", "v_add_u32", "v_bitop3_b32", "v_alignbit_b32", "v_mul_lo_u32", "v_mad_u64_u32"]


def peak_run(iters: int = 4000, reps: int = 5) -> dict:
    """Vector-ALU issue rates of the integer instructions the kernels use (dil_alu_probe): lane-ops/s
    with eight workgroups of four wavefronts per CU (full occupancy, 8 waves per SIMD) and with one
    workgroup per CU (one wave per SIMD), median of `reps` HIP-event-timed launches, against
    the 256 CU x 4 SIMD x 32 lanes x 2.4 GHz = 78.6 T lane-ops/s the roofline divides by."""
    import torch
    from paper_2211_12265_amd import dilithium as dl
    ctx = dl.Context(0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = torch.zeros(cus * 8 * 256, dtype=torch.int32, device="cuda")
    rows = []
    for kind, name in enumerate(PROBE_KINDS):
        for per_cu, shape in ((8, "8 waves per SIMD"), (1, "1 wave per SIMD")):
            groups = cus * per_cu
            ctx.alu_probe(kind, 16, groups, out)
            ts, n_instr = [], 0
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                n_instr = ctx.alu_probe(kind, iters, groups, out)
                b.record()
                b.synchronize()
                ts.append(a.elapsed_time(b))
            ms = float(np.median(ts))
            rate = n_instr / (ms * 1e-3)
            rows.append({"instruction": name, "occupancy": shape, "groups": groups, "ms": ms,
                         "lane_ops_per_s": rate, "frac_of_78.6T": rate / PEAK_INT32_OPS,
                         "lanes_per_simd_per_clk_at_2.4GHz": rate / (cus * 4 * 2.4e9)})
    ctx.close()
    return {"cus": cus, "iters": iters, "rows": rows, "peak_used": PEAK_INT32_OPS}


# schedules of the one- and two-wavefront shapes the autotuner picked at level 2 (10,000 tasks), used
# by the ablation when it is told not to tune (the four-wavefront shape uses the recorded schedule)
FIXED_SHAPE_SCHEDULES = {1: {"waves": 1, "hmax": 3, "grid": 2048}, 2: {"waves": 2, "hmax": 6, "grid": 1024}}


def ablation_run(level: int, n: int, msg_dist: str, steps: int = 10, tune: bool = True) -> list:
    """Runtime-selectable execution forms timed on the same keys and messages: the staged form
    (one launch per stage, host-driven loop), the persistent kernel in each workgroup shape with
    its autotuned schedule (tune=False: fixed schedules, so that a profiler sees a short, fixed
    launch sequence), and hipGraph replay on / off."""
    import torch
    from paper_2211_12265_amd import autotune
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import workload
    pkl, skl, sgl = dl.sizes(level)
    ctx0 = dl.Context(0)
    pk = torch.zeros((n, pkl), dtype=torch.uint8, device="cuda")
    sk = torch.zeros((n, skl), dtype=torch.uint8, device="cuda")
    ctx0.keygen(level, torch.from_numpy(workload.keygen_seeds(n, seed=0)).cuda(), pk, sk)
    lens = workload.fixed_lengths(n, 32) if msg_dist == "fixed32" else workload.uniform_lengths(n, 32, 4096)
    msg, off = workload.messages(lens, seed=0)
    gm, go = torch.from_numpy(msg).cuda(), torch.from_numpy(off.astype(np.int64)).cuda()
    ref = None
    rows = []
    forms = [("staged", dl.MODE_STAGED, None, 0), ("persistent 1-wave", dl.MODE_PERSISTENT, 1, 1),
             ("persistent 2-wave", dl.MODE_PERSISTENT, 2, 1), ("persistent 4-wave", dl.MODE_PERSISTENT, 4, 1),
             ("persistent 4-wave, no hipGraph", dl.MODE_PERSISTENT, 4, 0)]
    if level in MLDSA_BASE:  # the ML-DSA levels run the four-wavefront loop kernel only
        forms = [f for f in forms if f[2] in (None, 4)]
    for name, mode, waves, graph in forms:
        ctx = dl.Context(0, mode=mode)
        sig = torch.zeros((n, sgl), dtype=torch.uint8, device="cuda")
        ver = torch.zeros(n, dtype=torch.int32, device="cuda")
        sched = None
        if waves and tune:
            t = autotune.tune_sign(ctx, level, lambda: ctx.sign(level, sk, gm, go, sig), count=n, waves=(waves,))
            sched = {k: t["best"][k] for k in ("waves", "hmax", "grid")}
        elif waves:
            sched = FIXED_SHAPE_SCHEDULES.get(waves) or autotune.cached_schedule(level, n, msg_dist)
            autotune.apply_schedule(ctx, sched)
        ctx.set_param("graph", graph)
        for _ in range(2):
            ctx.sign(level, sk, gm, go, sig)
            ctx.verify(level, pk, gm, go, sig, ver)
        torch.cuda.synchronize()
        ts, tv = [], []
        for _ in range(steps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            ctx.sign(level, sk, gm, go, sig)
            e[1].record()
            ctx.verify(level, pk, gm, go, sig, ver)
            e[2].record()
            torch.cuda.synchronize()
            ts.append(e[0].elapsed_time(e[1]))
            tv.append(e[1].elapsed_time(e[2]))
        out = sig.cpu().numpy()
        same = True if ref is None else bool(np.array_equal(out, ref))
        ref = out if ref is None else ref
        ev, seq = ctx.sign_stats()
        rows.append({"form": name, "schedule": sched, "sign_ms": float(np.median(ts)),
                     "verify_ms": float(np.median(tv)), "sign_per_s": n / (float(np.median(ts)) * 1e-3),
                     "verify_per_s": n / (float(np.median(tv)) * 1e-3), "evaluated": ev, "sequential": seq,
                     "all_verified": bool(int(ver.sum()) == n), "same_signatures": same})
        ctx.close()
    ctx0.close()
    return rows


def e2e_run(level: int, n: int, msg_dist: str, stream_counts, chunks_per_stream=(1, 2), reps: int = 5,
            batch_streams=(1, 2, 4)) -> dict:
    """PCIe-inclusive rates: keys, messages, signatures and verdicts live in pinned host memory and
    every call moves them through the multi-stream chunked pipeline.  Reported beside the bench
    line, never as its value."""
    import torch
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import workload
    from paper_2211_12265_amd.pipeline import HostPipeline, pinned
    pkl, skl, sgl = dl.sizes(level)
    ctx = dl.Context(0)
    pk = torch.zeros((n, pkl), dtype=torch.uint8, device="cuda")
    sk = torch.zeros((n, skl), dtype=torch.uint8, device="cuda")
    ctx.keygen(level, torch.from_numpy(workload.keygen_seeds(n, seed=0)).cuda(), pk, sk)
    lens = workload.fixed_lengths(n, 32) if msg_dist == "fixed32" else workload.uniform_lengths(n, 32, 4096)
    msg, off = workload.messages(lens, seed=0)
    h_pk, h_sk = pinned((n, pkl)), pinned((n, skl))
    h_pk.copy_(pk)
    h_sk.copy_(sk)
    h_msg = pinned((len(msg),))
    h_msg.numpy()[:] = msg
    h_sig, h_ver = pinned((n, sgl)), pinned((n,), torch.int32)
    rows = []
    for S, cps, thr in [(S, c, t) for S in stream_counts for c in chunks_per_stream for t in (False, True)
                        if S > 1 or not t]:
        chunk = -(-n // (S * cps))
        p = HostPipeline(level, n_streams=S, chunk=chunk, host_threads=thr)
        p.sign(h_sk, h_msg, off, h_sig)
        p.verify(h_pk, h_msg, off, h_sig, h_ver)
        torch.cuda.synchronize()
        ts, tv = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            p.sign(h_sk, h_msg, off, h_sig)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            p.verify(h_pk, h_msg, off, h_sig, h_ver)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            ts.append(t1 - t0)
            tv.append(t2 - t1)
        p.check()
        rows.append({"streams": S, "chunks_per_stream": cps, "chunk": chunk, "host_threads": thr,
                     "sign_per_s": n / float(np.median(ts)),
                     "verify_per_s": n / float(np.median(tv)), "all_verified": bool(int(h_ver.sum()) == n)})
        p.close()
    # a stream of whole batches: B batches of n tasks back to back in one call, batch b on stream
    # b mod S, so one batch's copies overlap another's kernels (the same keys and messages repeated)
    B = 4
    h_pk_b, h_sk_b = pinned((B * n, pkl)), pinned((B * n, skl))
    h_msg_b = pinned((B * len(msg),))
    for b in range(B):
        h_pk_b[b * n:(b + 1) * n].copy_(h_pk)
        h_sk_b[b * n:(b + 1) * n].copy_(h_sk)
        h_msg_b.numpy()[b * len(msg):(b + 1) * len(msg)] = msg
    off_b = np.concatenate([off[:-1] + b * int(off[-1]) for b in range(B)] + [[B * int(off[-1])]]).astype(np.int64)
    h_sig_b, h_ver_b = pinned((B * n, sgl)), pinned((B * n,), torch.int32)
    for S, thr in [(S, t) for S in batch_streams for t in (False, True) if S > 1 or not t]:
        p = HostPipeline(level, n_streams=S, chunk=n, host_threads=thr)
        p.sign(h_sk_b, h_msg_b, off_b, h_sig_b)
        p.verify(h_pk_b, h_msg_b, off_b, h_sig_b, h_ver_b)
        torch.cuda.synchronize()
        ts, tv = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            p.sign(h_sk_b, h_msg_b, off_b, h_sig_b)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            p.verify(h_pk_b, h_msg_b, off_b, h_sig_b, h_ver_b)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            ts.append(t1 - t0)
            tv.append(t2 - t1)
        p.check()
        rows.append({"streams": S, "batches": B, "chunk": n, "host_threads": thr,
                     "sign_per_s": B * n / float(np.median(ts)),
                     "verify_per_s": B * n / float(np.median(tv)), "all_verified": bool(int(h_ver_b.sum()) == B * n),
                     "same_signatures": bool(np.array_equal(h_sig_b.numpy()[:n], h_sig_b.numpy()[(B - 1) * n:]))})
        p.close()
    ctx.close()
    best = max(rows, key=lambda r: r["sign_per_s"] * r["verify_per_s"] / (r["sign_per_s"] + r["verify_per_s"]))
    return {"what": f"{level_name(level)} batch {n}, host-resident pinned buffers, H2D + kernels + D2H per call, "
                    f"chunked over HIP streams, and {B} whole batches per call over HIP streams "
                    f"(rows with 'batches'; median of {reps})", "rows": rows, "best": best}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--count", type=int, default=10000)
    ap.add_argument("--level", type=int, default=2, choices=[2, 3, 5, 44, 65, 87],
                    help="round-3 level 2 / 3 / 5, or ML-DSA-44 / 65 / 87 (FIPS 204 form)")
    ap.add_argument("--mode", default="persistent", choices=["persistent", "staged"])
    ap.add_argument("--msg-dist", default="fixed32", choices=["fixed32", "uniform"],
                    help="32-byte messages, or lengths uniform on [32, 4096] (the level-3/5 configuration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the schedule autotuner")
    ap.add_argument("--tune", action="store_true",
                    help="re-run the autotuner even if a schedule is recorded for this workload")
    ap.add_argument("--tune-reps", type=int, default=3)
    ap.add_argument("--tune-rounds", type=int, default=1)
    ap.add_argument("--record-schedule", default="",
                    help="after tuning, record the chosen schedule in this JSON file")
    ap.add_argument("--waves", type=int, default=0, choices=[0, 1, 2, 4],
                    help="wavefronts per persistent workgroup (0: let the autotuner choose; the library default 4 without it)")
    ap.add_argument("--schedule", default="",
                    help="fixed persistent schedule 'waves,hmax,grid' (skips the autotuner)")
    ap.add_argument("--graph", type=int, default=1, help="replay Sign/Verify launch sequences as hipGraphs")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time over which the CPU oracle repeats Sign + Verify of the whole batch")
    ap.add_argument("--serving", action="store_true", help="also run the serving loop and report p50/p99")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=100000)
    ap.add_argument("--serving-seconds", type=float, default=5.0)
    ap.add_argument("--serving-streams", type=int, default=4)
    ap.add_argument("--serving-batch", type=int, default=4096)
    ap.add_argument("--ablation", action="store_true",
                    help="only time the execution forms (staged, persistent 1/4-wave, graph on/off) at --level")
    ap.add_argument("--e2e", action="store_true",
                    help="also report PCIe-inclusive rates through the multi-stream host pipeline")
    ap.add_argument("--e2e-streams", default="1,2,4,8,12")
    ap.add_argument("--micro", action="store_true",
                    help="only time the primitive workloads (2^20-polynomial NTT product in each ablation form, "
                         "ExpandA) and print them as one JSON line")
    ap.add_argument("--t0-ablation", action="store_true",
                    help="only run the NTT(t0)-stage ablation (four forms) and the padded / unpadded Sign "
                         "loop kernel, and print one JSON line")
    ap.add_argument("--peak", action="store_true",
                    help="only run the vector-ALU issue-rate probe behind the roofline peak and print one JSON line")
    ap.add_argument("--no-staged", action="store_true", help="skip the staged-form timing in the default line")
    ap.add_argument("--no-serving", action="store_true", help="skip the short serving trace in the default line")
    ap.add_argument("--serving-short-requests", type=int, default=200000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 4, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the batched path runs on a single MI355X "
              f"(--gpus {args.gpus} is not supported: tasks are independent, so a multi-GPU run would split the "
              f"batch into one contiguous task range per GPU)", file=sys.stderr)
        sys.exit(2)

    if args.micro:
        print(json.dumps({"micro": micro_run(args.steps, args.warmup)}), flush=True)
        return
    if args.t0_ablation:
        print(json.dumps({"t0_ablation": t0_ablation_run(steps=max(args.steps, 5), warmup=max(args.warmup, 2))}),
              flush=True)
        return
    if args.peak:
        print(json.dumps({"peak": peak_run()}), flush=True)
        return
    if args.ablation:
        print(json.dumps({"ablation": ablation_run(args.level, args.count, args.msg_dist, steps=max(args.steps, 3),
                                                   tune=not args.no_tune),
                          "level": args.level, "batch": args.count, "msg_dist": args.msg_dist}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_run(args.serving_requests, args.serving_seconds, args.serving_streams,
                                                 args.serving_batch)}), flush=True)
        return

    import torch
    from paper_2211_12265_amd import dilithium as dl
    from paper_2211_12265_amd import workload

    dev = torch.device("cuda:0")
    level, n = args.level, args.count
    pkl, skl, sgl = dl.sizes(level)
    ctx = dl.Context(0, mode=dl.MODE_PERSISTENT if args.mode == "persistent" else dl.MODE_STAGED)
    seeds = workload.keygen_seeds(n, seed=0)
    lens = workload.fixed_lengths(n, 32) if args.msg_dist == "fixed32" else workload.uniform_lengths(n, 32, 4096)
    msg, off = workload.messages(lens, seed=0)
    g_seeds = torch.from_numpy(seeds).to(dev)
    pk = torch.zeros((n, pkl), dtype=torch.uint8, device=dev)
    sk = torch.zeros((n, skl), dtype=torch.uint8, device=dev)
    ctx.keygen(level, g_seeds, pk, sk)
    g_msg = torch.from_numpy(msg).to(dev)
    g_off = torch.from_numpy(off.astype(np.int64)).to(dev)
    sig = torch.zeros((n, sgl), dtype=torch.uint8, device=dev)
    ver = torch.zeros(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        ctx.sign(level, sk, g_msg, g_off, sig)
        if ev is not None:
            ev[1].record(stream)
        ctx.verify(level, pk, g_msg, g_off, sig, ver)
        if ev is not None:
            ev[2].record(stream)

    tuning = None
    schedule_src = None
    from paper_2211_12265_amd import autotune
    cached = autotune.cached_schedule(level, n, args.msg_dist)
    if args.schedule:
        w, h, g = (int(x) for x in args.schedule.split(","))
        autotune.apply_schedule(ctx, {"waves": w, "hmax": h, "grid": g})
        args.waves = w
        schedule_src = "command line"
    elif args.mode == "persistent" and cached and not args.tune and not args.no_tune and not args.waves:
        autotune.apply_schedule(ctx, cached)
        args.waves = cached["waves"]
        args.schedule = f"{cached['waves']},{cached['hmax']},{cached['grid']}"
        schedule_src = "autotuner (recorded)"
    elif args.mode == "persistent" and not args.no_tune:
        # the ML-DSA levels are built in the four-wavefront shape only
        tuning = autotune.tune_sign(ctx, level, lambda: ctx.sign(level, sk, g_msg, g_off, sig), count=n,
                                    reps=args.tune_reps, rounds=args.tune_rounds,
                                    waves=(args.waves,) if args.waves else (4,) if level in MLDSA_BASE else (1, 2, 4))
        schedule_src = "autotuner (this run)"
        if args.record_schedule:
            autotune.store_schedule(level, n, args.msg_dist, tuning["best"], args.record_schedule)
    elif args.mode == "persistent" and args.waves:
        ctx.set_param("persist.waves", args.waves)
    if args.graph:
        ctx.set_param("graph", 1)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.mode == "persistent":
        ctx.set_param("timing", 1)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sign_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    ver_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    evaluated, sequential = ctx.sign_stats()

    # every signature of the timed batch verifies on the GPU; the CPU-baseline leg below also
    # compares all of them byte for byte with the oracle's
    all_verified = bool((ver == 1).all().item())

    ms_per_step = wall * 1e3 / args.steps
    sign_rate = n / (np.median(sign_ms) * 1e-3)
    ver_rate = n / (np.median(ver_ms) * 1e-3)
    if args.mode == "persistent":
        setup_ms, loop_ms = ctx.sign_timing()
        loop_med = float(np.median(loop_ms))
        k_ops = sequential * sign_iteration_ops(level)
        achieved = k_ops / (loop_med * 1e-3)
        kextra = {"kernel_ms_median": loop_med, "setup_ms_median": float(np.median(setup_ms)),
                  "timed_launches": len(loop_ms), "ops_per_launch": k_ops}
        nw = tuning["best"]["waves"] if tuning else (args.waves or 4)
        kbase = f"sg_persistw_k<{level}, {nw}>" if nw > 1 else f"sg_persist_k<{level}>"
        kname = kbase + " (persistent Sign rejection-loop kernel)"
        sched_str = args.schedule if not tuning else \
            f"{tuning['best']['waves']},{tuning['best']['hmax']},{tuning['best']['grid']}"
        rec = stored_traffic(kbase, level, n, args.msg_dist, sched_str)
        if rec:
            kextra["traffic_detail"] = {"fetch_bytes": rec["fetch_bytes"], "write_bytes": rec["write_bytes"],
                                        "profile": rec["profile"]}

    else:
        achieved = sign_work(level, lens, sequential) / (np.median(sign_ms) * 1e-3)
        kname = "dil_sign_batch (whole staged Sign call)"
        kextra = {}
    msg_desc = "32-byte messages" if args.msg_dist == "fixed32" else "uniform 32-4096-byte messages"
    out = {
        "metric": "sign/s and verify/s, Dilithium2 batch 10k on 1 MI355X; p99 latency (serving)",
        "value": n / (ms_per_step * 1e-3),
        "unit": "sign+verify pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{level_name(level)} batch {n} sign + {n} verify, {msg_desc}, "
                               f"one key per task, device-resident buffers", "level": level, "batch": n,
                   "msg_len": 32 if args.msg_dist == "fixed32" else "uniform[32,4096]",
                   "sign_mode": args.mode, "hipgraph": bool(args.graph),
                   "schedule": ({k: tuning["best"][k] for k in ("waves", "hmax", "grid")} if tuning else
                                args.schedule or None), "schedule_source": schedule_src},
        "sign_per_s": sign_rate, "verify_per_s": ver_rate,
        "sign_ms_median": float(np.median(sign_ms)), "verify_ms_median": float(np.median(ver_ms)),
        "sign_iterations": {"sequential": int(sequential), "evaluated": int(evaluated),
                            "per_task": sequential / n},
        "all_verified": all_verified,
        "autotune": None if tuning is None else tuning["table"],
        "roofline": dict({"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT32_OPS / 1e12,
                          "unit": "T int32-ops/s", "frac": achieved / PEAK_INT32_OPS,
                          "traffic": (kextra["traffic_detail"]["fetch_bytes"] + kextra["traffic_detail"]["write_bytes"])
                          if "traffic_detail" in kextra else None,
                          "kernel": kname}, **kextra),
    }
    if args.mode == "persistent" and not args.no_staged:
        out["staged"] = staged_run(level, sk, pk, g_msg, g_off, sig)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(level, seeds, msg, off, msg_desc,
                                           sig.cpu().numpy(), args.cpu_seconds)
    if args.e2e:
        out["e2e_pcie_inclusive"] = e2e_run(level, n, args.msg_dist,
                                            [int(x) for x in args.e2e_streams.split(",") if x])
    if args.serving:
        out["serving"] = serving_run(args.serving_requests, args.serving_seconds, args.serving_streams,
                                     args.serving_batch)
    elif not args.no_serving:
        out["serving"] = serving_run(args.serving_short_requests, args.serving_seconds, args.serving_streams,
                                     args.serving_batch, short=True)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
