"""Plain CPU oracle for batched Dilithium (round-3 parameter sets 2/3/5).

TEST INFRASTRUCTURE ONLY: the C sources in this folder are the slow,
obviously-correct definition of what the GPU path computes.  Only the test
suite, the package smoke check and the benchmark's CPU-baseline leg may import
this module; the product path never does, and the two share no code.

`build()` compiles the C sources with gcc into ``libdil_oracle.so`` beside
them; `lib()` loads it (building first if it is missing) and declares the
ctypes signatures.  The thin numpy wrappers below only marshal arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["fips202.c", "poly.c", "rounding.c", "sample.c", "scheme.c"]
LIBNAME = os.path.join(HERE, "libdil_oracle.so")

Q = 8380417
N = 256


def build(force: bool = True, out: Optional[str] = None, defines: Optional[list] = None) -> str:
    """Compile the oracle with gcc (plain C11, -O2, pthreads).  `defines` (e.g. ["DIL_PLANT=3"]) and
    `out` are used only by the planted-mistake tests, which build variants elsewhere."""
    target = out or LIBNAME
    if force or not os.path.exists(target):
        srcs = [os.path.join(HERE, s) for s in SOURCES]
        tmp = target + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
               "-Wno-unused-parameter", "-o", tmp] + ["-D" + d for d in (defines or [])] + srcs
        subprocess.run(cmd, check=True)
        os.replace(tmp, target)
    return target


class _Params(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("k", ctypes.c_int), ("l", ctypes.c_int),
                ("eta", ctypes.c_int), ("tau", ctypes.c_int), ("beta", ctypes.c_int),
                ("omega", ctypes.c_int), ("gamma1", ctypes.c_int32), ("gamma2", ctypes.c_int32),
                ("z_bits", ctypes.c_int), ("w1_bits", ctypes.c_int), ("eta_bits", ctypes.c_int),
                ("pk_bytes", ctypes.c_size_t), ("sk_bytes", ctypes.c_size_t),
                ("sig_bytes", ctypes.c_size_t), ("w1_poly_bytes", ctypes.c_size_t),
                ("mldsa", ctypes.c_int), ("tr_bytes", ctypes.c_int), ("ct_bytes", ctypes.c_int)]


_LIB: Optional[ctypes.CDLL] = None
_P = ctypes.c_void_p
_SZ = ctypes.c_size_t


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBNAME):
            build(force=False)
        _LIB = bind(LIBNAME)
    return _LIB


def bind(path: str) -> ctypes.CDLL:
    """Load an oracle shared library and declare its ctypes signatures."""
    if True:
        L = ctypes.CDLL(path)
        sig = {
            "dil_ref_params": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_Params)]),
            "dil_ref_keccak_f1600": (None, [_P]),
            "dil_ref_shake128": (None, [_P, _SZ, _P, _SZ]),
            "dil_ref_shake256": (None, [_P, _SZ, _P, _SZ]),
            "dil_ref_ntt": (None, [_P]),
            "dil_ref_intt": (None, [_P]),
            "dil_ref_ntt_definition": (None, [_P, _P]),
            "dil_ref_poly_mul_schoolbook": (None, [_P, _P, _P]),
            "dil_ref_ntt_mul_batch": (None, [_P, _P, _P, _SZ, ctypes.c_int]),
            "dil_ref_power2round": (None, [_P, _P, _P, _SZ]),
            "dil_ref_decompose": (None, [_P, _P, _P, _SZ, ctypes.c_int32]),
            "dil_ref_make_hint": (None, [_P, _P, _P, _SZ, ctypes.c_int32]),
            "dil_ref_use_hint": (None, [_P, _P, _P, _SZ, ctypes.c_int32]),
            "dil_ref_expand_a": (None, [ctypes.c_int, _P, _P]),
            "dil_ref_expand_a_poly": (None, [_P, _P]),
            "dil_ref_expand_a_polys": (None, [_P, _P, _SZ, ctypes.c_int]),
            "dil_ref_expand_s": (None, [ctypes.c_int, _P, _P]),
            "dil_ref_expand_a_poly_counted": (_SZ, [_P, _P]),
            "dil_ref_expand_s_poly_counted": (_SZ, [ctypes.c_int, _P, ctypes.c_uint16, _P]),
            "dil_ref_expand_mask": (None, [ctypes.c_int, _P, ctypes.c_uint32, _P]),
            "dil_ref_sample_in_ball": (None, [ctypes.c_int, _P, _P]),
            "dil_ref_bitpack": (None, [_P, _SZ, ctypes.c_int, _P]),
            "dil_ref_bitunpack": (None, [_P, _SZ, ctypes.c_int, _P]),
            "dil_ref_keygen": (ctypes.c_int, [ctypes.c_int, _P, _P, _P]),
            "dil_ref_sign": (ctypes.c_int, [ctypes.c_int, _P, _P, _SZ, _P]),
            "dil_ref_set_sign_cap": (None, [ctypes.c_int]),
            "dil_ref_verify": (ctypes.c_int, [ctypes.c_int, _P, _P, _SZ, _P]),
            "dil_ref_keygen_batch": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, ctypes.c_uint32, ctypes.c_int]),
            "dil_ref_sign_batch": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, _P, _P, ctypes.c_uint32,
                                                  ctypes.c_int, _P]),
            "dil_ref_mldsa_mu": (None, [_P, _P, _SZ, _P]),
            "dil_ref_mldsa_sign_internal": (ctypes.c_int, [ctypes.c_int, _P, _P, _SZ, _P, _P]),
            "dil_ref_mldsa_verify_internal": (ctypes.c_int, [ctypes.c_int, _P, _P, _SZ, _P]),
            "dil_ref_sign_batch_ex": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_uint32,
                                                     ctypes.c_int, _P]),
            "dil_ref_verify_batch_ex": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _P, _P, _P, _P, _P,
                                                       ctypes.c_uint32, ctypes.c_int]),
            "dil_ref_sign_batch_rnd": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_uint32,
                                                      ctypes.c_int, _P]),
            "dil_ref_verify_batch": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_uint32,
                                                    ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
    return L


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def params(level: int) -> dict:
    p = _Params()
    if lib().dil_ref_params(level, ctypes.byref(p)) != 0:
        raise ValueError(f"bad level {level}")
    return {f: getattr(p, f) for f, _ in _Params._fields_}


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# ---- primitives -------------------------------------------------------------------------------
def shake128(data: bytes, outlen: int) -> bytes:
    src = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8)
    out = np.zeros(max(outlen, 1), dtype=np.uint8)
    lib().dil_ref_shake128(_ptr(src), len(data), _ptr(out), outlen)
    return out[:outlen].tobytes()


def shake256(data: bytes, outlen: int) -> bytes:
    src = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8)
    out = np.zeros(max(outlen, 1), dtype=np.uint8)
    lib().dil_ref_shake256(_ptr(src), len(data), _ptr(out), outlen)
    return out[:outlen].tobytes()


def keccak_f1600(state: np.ndarray) -> np.ndarray:
    st = np.ascontiguousarray(state, dtype=np.uint64).copy()
    lib().dil_ref_keccak_f1600(_ptr(st))
    return st


def _poly_in(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    assert a.shape == (N,)
    return a.copy()


def ntt(a) -> np.ndarray:
    t = _poly_in(a)
    lib().dil_ref_ntt(_ptr(t))
    return t


def intt(a) -> np.ndarray:
    t = _poly_in(a)
    lib().dil_ref_intt(_ptr(t))
    return t


def ntt_definition(a) -> np.ndarray:
    t = _poly_in(a)
    out = np.zeros(N, dtype=np.int32)
    lib().dil_ref_ntt_definition(_ptr(t), _ptr(out))
    return out


def poly_mul_schoolbook(a, b) -> np.ndarray:
    x, y = _poly_in(a), _poly_in(b)
    out = np.zeros(N, dtype=np.int32)
    lib().dil_ref_poly_mul_schoolbook(_ptr(x), _ptr(y), _ptr(out))
    return out


def ntt_mul_batch(a: np.ndarray, b: np.ndarray, nthreads: Optional[int] = None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    assert a.shape == b.shape and a.shape[-1] == N
    c = np.empty_like(a)
    lib().dil_ref_ntt_mul_batch(_ptr(a), _ptr(b), _ptr(c), a.size // N, nthreads or default_threads())
    return c


def power2round(r: np.ndarray):
    r = np.ascontiguousarray(r, dtype=np.int32)
    r1, r0 = np.empty_like(r), np.empty_like(r)
    lib().dil_ref_power2round(_ptr(r), _ptr(r1), _ptr(r0), r.size)
    return r1, r0


def decompose(r: np.ndarray, gamma2: int):
    r = np.ascontiguousarray(r, dtype=np.int32)
    r1, r0 = np.empty_like(r), np.empty_like(r)
    lib().dil_ref_decompose(_ptr(r), _ptr(r1), _ptr(r0), r.size, gamma2)
    return r1, r0


def make_hint(z: np.ndarray, r: np.ndarray, gamma2: int) -> np.ndarray:
    z = np.ascontiguousarray(z, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.int32)
    h = np.empty_like(r)
    lib().dil_ref_make_hint(_ptr(z), _ptr(r), _ptr(h), r.size, gamma2)
    return h


def use_hint(h: np.ndarray, r: np.ndarray, gamma2: int) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.int32)
    out = np.empty_like(r)
    lib().dil_ref_use_hint(_ptr(h), _ptr(r), _ptr(out), r.size, gamma2)
    return out


def expand_a(level: int, rho: bytes) -> np.ndarray:
    p = params(level)
    out = np.zeros((p["k"], p["l"], N), dtype=np.int32)
    src = np.frombuffer(bytes(rho), dtype=np.uint8).copy()
    lib().dil_ref_expand_a(level, _ptr(src), _ptr(out))
    return out


def expand_a_polys(seeds34: np.ndarray, nthreads: Optional[int] = None) -> np.ndarray:
    seeds34 = np.ascontiguousarray(seeds34, dtype=np.uint8)
    count = seeds34.size // 34
    out = np.zeros((count, N), dtype=np.int32)
    lib().dil_ref_expand_a_polys(_ptr(seeds34), _ptr(out), count, nthreads or default_threads())
    return out


def expand_a_poly_counted(seed34: bytes):
    """One ExpandA polynomial and the number of 3-byte candidates its sampler examined."""
    out = np.zeros(N, dtype=np.int32)
    src = np.frombuffer(bytes(seed34), dtype=np.uint8).copy()
    used = lib().dil_ref_expand_a_poly_counted(_ptr(src), _ptr(out))
    return out, int(used)


def expand_s_poly_counted(eta: int, rhop: bytes, nonce: int):
    """One ExpandS polynomial (centred) and the number of nibbles its sampler examined."""
    out = np.zeros(N, dtype=np.int32)
    src = np.frombuffer(bytes(rhop), dtype=np.uint8).copy()
    used = lib().dil_ref_expand_s_poly_counted(eta, _ptr(src), nonce, _ptr(out))
    return out, int(used)


def expand_s(level: int, rhop: bytes) -> np.ndarray:
    p = params(level)
    out = np.zeros((p["l"] + p["k"], N), dtype=np.int32)
    src = np.frombuffer(bytes(rhop), dtype=np.uint8).copy()
    lib().dil_ref_expand_s(level, _ptr(src), _ptr(out))
    return out


def expand_mask(level: int, rhop: bytes, kappa: int) -> np.ndarray:
    p = params(level)
    out = np.zeros((p["l"], N), dtype=np.int32)
    src = np.frombuffer(bytes(rhop), dtype=np.uint8).copy()
    lib().dil_ref_expand_mask(level, _ptr(src), kappa, _ptr(out))
    return out


def sample_in_ball(level: int, ctilde: bytes) -> np.ndarray:
    out = np.zeros(N, dtype=np.int32)
    src = np.frombuffer(bytes(ctilde), dtype=np.uint8).copy()
    lib().dil_ref_sample_in_ball(level, _ptr(src), _ptr(out))
    return out


def bitpack(v: np.ndarray, b: int) -> bytes:
    v = np.ascontiguousarray(v, dtype=np.uint32)
    out = np.zeros((v.size * b + 7) // 8, dtype=np.uint8)
    lib().dil_ref_bitpack(_ptr(v), v.size, b, _ptr(out))
    return out.tobytes()


def bitunpack(data: bytes, n: int, b: int) -> np.ndarray:
    src = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8).copy()
    out = np.zeros(n, dtype=np.uint32)
    lib().dil_ref_bitunpack(_ptr(src), n, b, _ptr(out))
    return out


# ---- scheme -----------------------------------------------------------------------------------
def keygen(level: int, zeta: bytes):
    p = params(level)
    pk = np.zeros(p["pk_bytes"], dtype=np.uint8)
    sk = np.zeros(p["sk_bytes"], dtype=np.uint8)
    z = np.frombuffer(bytes(zeta), dtype=np.uint8).copy()
    lib().dil_ref_keygen(level, _ptr(z), _ptr(pk), _ptr(sk))
    return pk.tobytes(), sk.tobytes()


def sign(level: int, sk: bytes, msg: bytes):
    """Returns (signature bytes, loop iterations)."""
    p = params(level)
    sig = np.zeros(p["sig_bytes"], dtype=np.uint8)
    s = np.frombuffer(bytes(sk), dtype=np.uint8).copy()
    m = np.frombuffer(bytes(msg) + b"\0", dtype=np.uint8).copy()
    it = lib().dil_ref_sign(level, _ptr(s), _ptr(m), len(msg), _ptr(sig))
    return sig.tobytes(), it


def verify(level: int, pk: bytes, msg: bytes, sig: bytes) -> int:
    k = np.frombuffer(bytes(pk), dtype=np.uint8).copy()
    m = np.frombuffer(bytes(msg) + b"\0", dtype=np.uint8).copy()
    s = np.frombuffer(bytes(sig), dtype=np.uint8).copy()
    return lib().dil_ref_verify(level, _ptr(k), _ptr(m), len(msg), _ptr(s))


def mldsa_mu(tr: bytes, msg: bytes) -> bytes:
    """The ML-DSA message representative H(tr || 0 || 0 || M, 64) (pure signing, empty context)."""
    if len(tr) != 64:
        raise ValueError("tr must be 64 bytes")
    t = np.frombuffer(bytes(tr), dtype=np.uint8).copy()
    m = np.frombuffer(bytes(msg) + b"\0", dtype=np.uint8).copy()
    mu = np.zeros(64, dtype=np.uint8)
    lib().dil_ref_mldsa_mu(_ptr(t), _ptr(m), len(msg), _ptr(mu))
    return mu.tobytes()


def mldsa_format(msg: bytes, ctx: bytes = b"") -> bytes:
    """The formatted message M' = 0x00 || |ctx| || ctx || M of ML-DSA's pure signing."""
    if len(ctx) > 255:
        raise ValueError("context strings hold at most 255 bytes")
    return bytes([0, len(ctx)]) + bytes(ctx) + bytes(msg)


def mldsa_sign_internal(level: int, sk: bytes, mprime: bytes, rnd: Optional[bytes] = None) -> bytes:
    p = params(level)
    sig = np.zeros(p["sig_bytes"], dtype=np.uint8)
    s = np.frombuffer(bytes(sk), dtype=np.uint8).copy()
    m = np.frombuffer(bytes(mprime) + b"\0", dtype=np.uint8).copy()
    r = None if rnd is None else np.frombuffer(bytes(rnd), dtype=np.uint8).copy()
    if lib().dil_ref_mldsa_sign_internal(level, _ptr(s), _ptr(m), len(mprime), None if r is None else _ptr(r),
                                         _ptr(sig)) < 0:
        raise ValueError("internal signing exists at the ML-DSA levels only")
    return sig.tobytes()


def mldsa_verify_internal(level: int, pk: bytes, mprime: bytes, sig: bytes) -> int:
    k = np.frombuffer(bytes(pk), dtype=np.uint8).copy()
    m = np.frombuffer(bytes(mprime) + b"\0", dtype=np.uint8).copy()
    s = np.frombuffer(bytes(sig), dtype=np.uint8).copy()
    return lib().dil_ref_mldsa_verify_internal(level, _ptr(k), _ptr(m), len(mprime), _ptr(s))


def keygen_batch(level: int, seeds: np.ndarray, nthreads: Optional[int] = None):
    p = params(level)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint8).reshape(-1, 32)
    n = seeds.shape[0]
    pk = np.zeros((n, p["pk_bytes"]), dtype=np.uint8)
    sk = np.zeros((n, p["sk_bytes"]), dtype=np.uint8)
    if lib().dil_ref_keygen_batch(level, _ptr(seeds), _ptr(pk), _ptr(sk), n, nthreads or default_threads()):
        raise ValueError("bad arguments")
    return pk, sk


def _msg_arrays(msg: np.ndarray, msg_off: np.ndarray):
    msg = np.ascontiguousarray(msg, dtype=np.uint8)
    if msg.size == 0:
        msg = np.zeros(1, dtype=np.uint8)
    return msg, np.ascontiguousarray(msg_off, dtype=np.uint64)


def sign_batch(level: int, sk: np.ndarray, msg: np.ndarray, msg_off: np.ndarray,
               key_idx: Optional[np.ndarray] = None, nthreads: Optional[int] = None,
               rnd: Optional[np.ndarray] = None, internal: bool = False):
    """Returns (sig [count, SIG] uint8, iterations [count] int32).  rnd: optional per-task bytes for
    the randomized variant, [count, 64] (rho' itself, levels 2/3/5) or [count, 32] (the rnd that
    rho'' hashes, ML-DSA levels 44/65/87); None: deterministic Sign.  internal: the messages are
    ML-DSA formatted messages M' (mu = H(tr || M'))."""
    p = params(level)
    sk = np.ascontiguousarray(sk, dtype=np.uint8)
    msg, msg_off = _msg_arrays(msg, msg_off)
    n = msg_off.size - 1
    sig = np.zeros((n, p["sig_bytes"]), dtype=np.uint8)
    iters = np.zeros(max(n, 1), dtype=np.int32)
    ki = None if key_idx is None else np.ascontiguousarray(key_idx, dtype=np.uint32)
    if rnd is not None:
        rnd = np.ascontiguousarray(rnd, dtype=np.uint8)
        rb = 32 if p["mldsa"] else 64
        if rnd.shape != (n, rb):
            raise ValueError(f"rnd must be [count, {rb}] bytes")
    rc = lib().dil_ref_sign_batch_ex(level, int(internal), _ptr(sk), None if ki is None else _ptr(ki), _ptr(msg),
                                     _ptr(msg_off), None if rnd is None else _ptr(rnd), _ptr(sig), n,
                                     nthreads or default_threads(), _ptr(iters))
    if rc:
        raise ValueError("bad arguments")
    return sig, iters[:n]


def verify_batch(level: int, pk: np.ndarray, msg: np.ndarray, msg_off: np.ndarray, sig: np.ndarray,
                 key_idx: Optional[np.ndarray] = None, nthreads: Optional[int] = None,
                 internal: bool = False) -> np.ndarray:
    pk = np.ascontiguousarray(pk, dtype=np.uint8)
    sig = np.ascontiguousarray(sig, dtype=np.uint8)
    msg, msg_off = _msg_arrays(msg, msg_off)
    n = msg_off.size - 1
    verdict = np.zeros(max(n, 1), dtype=np.int32)
    ki = None if key_idx is None else np.ascontiguousarray(key_idx, dtype=np.uint32)
    rc = lib().dil_ref_verify_batch_ex(level, int(internal), _ptr(pk), None if ki is None else _ptr(ki), _ptr(msg),
                                       _ptr(msg_off), _ptr(sig), _ptr(verdict), n, nthreads or default_threads())
    if rc:
        raise ValueError("bad arguments")
    return verdict[:n]
