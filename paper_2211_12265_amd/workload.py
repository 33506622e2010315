"""Seeded synthetic inputs shared by the tests, the benchmark and the serving demo.

This module holds no arithmetic of the signature scheme: it only draws bytes
and integers from numpy's PCG64 generator, keyed by (seed, tag), so that the
GPU path and the CPU oracle receive identical input buffers.

Recipes (the paper measures on random batched tasks and never states a
message length; these follow the benchmark configurations):
  keygen seeds      32 uniform bytes per task
  messages          uniform bytes; lengths fixed (32 B), uniform on [32, 4096],
                    or lognormal (median 256 B, sigma 1.0, clipped to [1, 16384])
  NTT microbench    coefficients uniform in [0, q) for both operands
  ExpandA microbench 34-byte inputs rho_g || j || i with g = idx // 16,
                    j = idx % 4, i = (idx // 4) % 4 (65,536 level-2 matrices per 2^20)
  serving stream    Poisson arrivals at rate lam; 70% verify / 30% sign;
                    levels 2/3/5 with probability 0.5/0.3/0.2; keys uniform
                    within the level; 1% of verify requests get one flipped bit
"""
from __future__ import annotations

import zlib
from dataclasses import dataclass
from typing import Tuple

import numpy as np

Q = 8380417
N = 256


def _rng(tag: str, seed: int) -> np.random.Generator:
    return np.random.default_rng([int(seed) & 0xFFFFFFFF, zlib.crc32(tag.encode())])


def random_bytes(tag: str, seed: int, shape) -> np.ndarray:
    return _rng(tag, seed).integers(0, 256, size=shape, dtype=np.uint8)


def keygen_seeds(count: int, seed: int = 0) -> np.ndarray:
    """(count, 32) uint8 keygen seeds zeta."""
    return random_bytes("dil/zeta", seed, (count, 32))


def fixed_lengths(count: int, length: int = 32) -> np.ndarray:
    return np.full(count, length, dtype=np.int64)


def uniform_lengths(count: int, lo: int = 32, hi: int = 4096, seed: int = 0) -> np.ndarray:
    return _rng("dil/len", seed).integers(lo, hi + 1, size=count, dtype=np.int64)


def lognormal_lengths(count: int, median: float = 256.0, sigma: float = 1.0, cap: int = 16384,
                      seed: int = 0) -> np.ndarray:
    x = _rng("dil/lognorm", seed).normal(np.log(median), sigma, size=count)
    return np.clip(np.round(np.exp(x)), 1, cap).astype(np.int64)


def messages(lengths: np.ndarray, seed: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Concatenated message bytes and CSR offsets (count + 1 entries, uint64)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    off = np.zeros(lengths.size + 1, dtype=np.uint64)
    np.cumsum(lengths, out=off[1:])
    total = int(off[-1])
    buf = random_bytes("dil/msg", seed, (max(total, 1),))
    return buf, off


def uniform_polys(count: int, seed: int = 0, tag: str = "dil/poly") -> np.ndarray:
    """(count, 256) int32 with coefficients uniform in [0, q)."""
    return _rng(tag, seed).integers(0, Q, size=(count, N), dtype=np.int32)


def expand_a_inputs(count: int, seed: int = 0) -> np.ndarray:
    """(count, 34) uint8 ExpandA stream inputs: rho_g || j || i for g = idx // 16."""
    groups = (count + 15) // 16
    rho = random_bytes("dil/rho", seed, (groups, 32))
    idx = np.arange(count)
    out = np.empty((count, 34), dtype=np.uint8)
    out[:, :32] = rho[idx // 16]
    out[:, 32] = (idx % 4).astype(np.uint8)
    out[:, 33] = ((idx // 4) % 4).astype(np.uint8)
    return out


@dataclass
class Request:
    t_arrival: float   # seconds from stream start (scheduled arrival)
    op: str            # "sign" or "verify"
    level: int
    key: int           # key index within the level's resident key table
    msg: bytes
    flip_bit: int      # -1, or the signature bit to flip (verify only)


def request_stream(count: int, lam: float, keys_per_level: dict, seed: int = 0,
                   p_verify: float = 0.7, level_probs=(0.5, 0.3, 0.2)) -> list:
    """Poisson request stream for the serving loop (see module docstring)."""
    g = _rng("dil/arrive", seed)
    gaps = g.exponential(1.0 / lam, size=count)
    t = np.cumsum(gaps)
    ops = _rng("dil/op", seed).random(count) < p_verify
    lv = _rng("dil/level", seed).choice([2, 3, 5], size=count, p=list(level_probs))
    kr = _rng("dil/key", seed).random(count)
    lens = lognormal_lengths(count, seed=seed)
    msgbuf, off = messages(lens, seed=seed + 1)
    flips = _rng("dil/flip", seed).random(count) < 0.01
    flipbits = _rng("dil/flipbit", seed).integers(0, 1 << 30, size=count)
    out = []
    for i in range(count):
        level = int(lv[i])
        nk = keys_per_level[level]
        out.append(Request(float(t[i]), "verify" if ops[i] else "sign", level, int(kr[i] * nk) % nk,
                           msgbuf[int(off[i]):int(off[i + 1])].tobytes(),
                           int(flipbits[i]) if (ops[i] and flips[i]) else -1))
    return out
