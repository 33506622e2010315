"""Thin Python binding of the libdil C-ABI (include/dil.h).

Argument marshalling only: every step of KeyGen / Sign / Verify runs in the
HIP kernels of libdil.so.  Buffers are torch tensors on the GPU; their
device pointers and torch's current HIP stream are passed straight through.
If libdil.so is missing this module raises at import of the library -- there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdil.so")

DIL_OK, DIL_EINVAL, DIL_ENOMEM, DIL_EHIP, DIL_EMSG, DIL_ETIMEDOUT = 0, -1, -2, -3, -4, -5
MODE_STAGED, MODE_PERSISTENT = 0, 1
OP_KEYGEN, OP_SIGN, OP_VERIFY = 0, 1, 2

EXPORTS = [
    "dil_ctx_create", "dil_ctx_destroy", "dil_ctx_set_mode", "dil_ctx_set_param", "dil_ctx_check",
    "dil_last_error", "dil_sizes",
    "dil_keygen_batch", "dil_sign_batch", "dil_sign_batch_rnd", "dil_verify_batch", "dil_sign_stats", "dil_sign_timing",
    "dil_ntt_mul_batch",
    "dil_expand_a_batch", "dil_keyset_create", "dil_keyset_destroy", "dil_keyset_info", "dil_sign_keyset",
    "dil_verify_keyset", "dil_persist_capacity", "dil_ctx_reserve", "dil_server_create", "dil_server_create_tables",
    "dil_server_destroy",
    "dil_server_last_error", "dil_server_stats", "dil_server_run", "dil_ctx_reserve_call", "dil_workspace_bytes",
    "dil_alu_probe", "dil_verify_keyset_noalloc", "dil_t0_ntt_batch",
    "dil_server_start", "dil_server_submit", "dil_server_poll", "dil_server_wait", "dil_server_stop",
]

_LIB: Optional[ctypes.CDLL] = None
_P = ctypes.c_void_p


class DilError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libdil error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load libdil.so (built in-tree by __graft_entry__.build())."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first (python -m "
                           "paper_2211_12265_amd.build); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "dil_ctx_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_size_t]),
        "dil_ctx_destroy": (ctypes.c_int, [_P]),
        "dil_ctx_set_mode": (ctypes.c_int, [_P, ctypes.c_int]),
        "dil_ctx_set_param": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_int64]),
        "dil_ctx_check": (ctypes.c_int, [_P, _P]),
        "dil_last_error": (ctypes.c_char_p, [_P]),
        "dil_sizes": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "dil_keygen_batch": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.c_uint32, _P]),
        "dil_sign_batch": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, _P, ctypes.c_uint32, _P]),
        "dil_sign_batch_rnd": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_uint32, _P]),
        "dil_verify_batch": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_uint32, _P]),
        "dil_sign_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
        "dil_sign_timing": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "dil_ntt_mul_batch": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_uint64, _P]),
        "dil_expand_a_batch": (ctypes.c_int, [_P, _P, _P, ctypes.c_uint64, _P]),
        "dil_t0_ntt_batch": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_uint32, _P]),
        "dil_keyset_create": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_uint32, ctypes.POINTER(_P), _P]),
        "dil_keyset_destroy": (ctypes.c_int, [_P]),
        "dil_keyset_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_uint32),
                                           ctypes.POINTER(ctypes.c_size_t)]),
        "dil_sign_keyset": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, ctypes.c_uint32, _P]),
        "dil_verify_keyset": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, ctypes.c_uint32, _P]),
        "dil_persist_capacity": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_int)]),
        "dil_ctx_reserve": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_uint32]),
        "dil_server_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, _P, _P, ctypes.c_int,
                                             ctypes.c_uint32, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int]),
        "dil_server_create_tables": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, ctypes.c_int, ctypes.c_int,
                                                    ctypes.c_uint32, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_int]),
        "dil_server_destroy": (ctypes.c_int, [_P]),
        "dil_server_last_error": (ctypes.c_char_p, [_P]),
        "dil_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32),
                                            ctypes.POINTER(ctypes.c_size_t)]),
        "dil_verify_keyset_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, ctypes.c_uint32, _P]),
        "dil_alu_probe": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, _P, _P,
                                         ctypes.POINTER(ctypes.c_uint64)]),
        "dil_ctx_reserve_call": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32]),
        "dil_workspace_bytes": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32,
                                               ctypes.POINTER(ctypes.c_size_t)]),
        "dil_server_run": (ctypes.c_int, [_P, ctypes.c_uint32] + [_P] * 12),
        "dil_server_start": (ctypes.c_int, [_P]),
        "dil_server_submit": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_uint32, _P, ctypes.c_uint64,
                                             _P, ctypes.POINTER(ctypes.c_uint64)]),
        "dil_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int32), _P]),
        "dil_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), _P]),
        "dil_server_stop": (ctypes.c_int, [_P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = L
    return L


ROUND3_LEVELS = (2, 3, 5)
MLDSA_LEVELS = (44, 65, 87)  # ML-DSA-44 / 65 / 87 (FIPS 204)


def sizes(level: int) -> Tuple[int, int, int]:
    pk, sk, sg = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    rc = load().dil_sizes(level, ctypes.byref(pk), ctypes.byref(sk), ctypes.byref(sg))
    if rc:
        raise DilError(rc, f"bad level {level}")
    return pk.value, sk.value, sg.value


def _require(checks) -> None:
    """Host-side size checks of a call's buffers, before anything is launched: the kernels
    index rows and offsets without bounds checks, so an undersized tensor would be read or
    written past its end on the device.  checks: (tensor or None, minimum bytes, required
    element size or 0, name); None tensors are skipped."""
    for t, nbytes, esize, name in checks:
        if t is None:
            continue
        if esize and t.element_size() != esize:
            raise ValueError(f"{name}: elements of {esize} bytes expected, got {t.dtype}")
        if t.numel() * t.element_size() < nbytes:
            raise ValueError(f"{name}: {nbytes} bytes needed, tensor holds {t.numel() * t.element_size()}")


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    assert t.is_cuda and t.is_contiguous(), "libdil takes contiguous device tensors"
    return t.data_ptr() if t.numel() > 0 else None


def _stream(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


class Context:
    """One libdil context (workspace pool) on one device."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0, mode: int = MODE_STAGED):
        self.lib = load()
        h = _P()
        rc = self.lib.dil_ctx_create(ctypes.byref(h), device, workspace_bytes)
        if rc:
            raise DilError(rc, "context creation failed")
        self.h = h
        self.device = device
        if mode != MODE_STAGED:
            self.set_mode(mode)

    def close(self):
        if getattr(self, "h", None):
            self.lib.dil_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != DIL_OK:
            raise DilError(rc, self.lib.dil_last_error(self.h).decode(errors="replace"))

    def set_mode(self, mode: int):
        self._check(self.lib.dil_ctx_set_mode(self.h, mode))

    def set_param(self, name: str, value: int):
        self._check(self.lib.dil_ctx_set_param(self.h, name.encode(), int(value)))

    def reserve(self, level: int, count: int):
        self._check(self.lib.dil_ctx_reserve(self.h, level, count))

    def reserve_call(self, level: int, op: int, keyset: bool, count: int):
        """Reserve the workspace of calls of one kind (OP_*) with up to `count` tasks."""
        self._check(self.lib.dil_ctx_reserve_call(self.h, level, op, int(keyset), count))

    def workspace_bytes(self, level: int, op: int, keyset: bool, count: int) -> int:
        """Device workspace bytes of one call of `count` tasks (the library's own layout)."""
        b = ctypes.c_size_t()
        self._check(self.lib.dil_workspace_bytes(self.h, level, op, int(keyset), count, ctypes.byref(b)))
        return b.value

    def check(self, stream=None):
        self._check(self.lib.dil_ctx_check(self.h, _stream(stream)))

    def keygen(self, level: int, seeds, pk, sk, stream=None):
        n = seeds.shape[0]
        pkl, skl, _ = sizes(level)
        _require([(seeds, 32 * n, 1, "seeds"), (pk, pkl * n, 1, "pk"), (sk, skl * n, 1, "sk")])
        self._check(self.lib.dil_keygen_batch(self.h, level, _ptr(seeds), _ptr(pk), _ptr(sk), n, _stream(stream)))

    def sign(self, level: int, sk, msg, msg_off, sig, key_idx=None, stream=None, rnd=None):
        """rnd: optional uint8 device tensor for randomized (hedged) signing: [count, 64], the rho' of each
        task (levels 2 / 3 / 5), or [count, 32], the rnd that rho'' hashes (ML-DSA levels 44 / 65 / 87)."""
        n = msg_off.shape[0] - 1
        _, skl, sgl = sizes(level)
        _require([(msg_off, 8 * (n + 1), 8, "msg_off"), (sig, sgl * n, 1, "sig"),
                  (sk, skl * (n if key_idx is None else 1), 1, "sk"), (key_idx, 4 * n, 4, "key_idx")])
        if rnd is None:
            self._check(self.lib.dil_sign_batch(self.h, level, _ptr(sk), _ptr(key_idx), _ptr(msg) or _ptr(msg_off),
                                                _ptr(msg_off), _ptr(sig), n, _stream(stream)))
        else:
            rb = 32 if level in MLDSA_LEVELS else 64
            if tuple(rnd.shape) != (n, rb):
                raise ValueError(f"rnd must be [count, {rb}] bytes")
            self._check(self.lib.dil_sign_batch_rnd(self.h, level, _ptr(sk), _ptr(key_idx),
                                                    _ptr(msg) or _ptr(msg_off), _ptr(msg_off), _ptr(rnd), _ptr(sig),
                                                    n, _stream(stream)))

    def verify(self, level: int, pk, msg, msg_off, sig, verdict, key_idx=None, stream=None):
        n = msg_off.shape[0] - 1
        pkl, _, sgl = sizes(level)
        _require([(msg_off, 8 * (n + 1), 8, "msg_off"), (sig, sgl * n, 1, "sig"), (verdict, 4 * n, 4, "verdict"),
                  (pk, pkl * (n if key_idx is None else 1), 1, "pk"), (key_idx, 4 * n, 4, "key_idx")])
        self._check(self.lib.dil_verify_batch(self.h, level, _ptr(pk), _ptr(key_idx), _ptr(msg) or _ptr(msg_off),
                                              _ptr(msg_off), _ptr(sig), _ptr(verdict), n, _stream(stream)))

    def sign_stats(self) -> Tuple[int, int]:
        ev, sq = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self.lib.dil_sign_stats(self.h, ctypes.byref(ev), ctypes.byref(sq)))
        return ev.value, sq.value

    def sign_timing(self, max_calls: int = 64):
        """Lists (setup_ms, loop_ms) of the timed persistent Sign calls (set_param("timing", 1) first)."""
        a = (ctypes.c_float * max_calls)()
        b = (ctypes.c_float * max_calls)()
        n = ctypes.c_int()
        self._check(self.lib.dil_sign_timing(self.h, ctypes.cast(a, _P), ctypes.cast(b, _P), max_calls,
                                             ctypes.byref(n)))
        return list(a[:n.value]), list(b[:n.value])

    def persist_capacity(self, level: int) -> Tuple[int, int]:
        """(resident workgroups, candidate slots per batch) of the persistent Sign kernel."""
        r, s = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.dil_persist_capacity(self.h, level, ctypes.byref(r), ctypes.byref(s)))
        return r.value, s.value

    def ntt_mul(self, a, b, c, stream=None):
        self._check(self.lib.dil_ntt_mul_batch(self.h, _ptr(a), _ptr(b), _ptr(c), a.shape[0], _stream(stream)))

    def alu_probe(self, kind: int, iters: int, groups: int, out, stream=None) -> int:
        """Launch the ALU issue-rate probe; returns the lane-instructions it executes."""
        if out.numel() * out.element_size() < groups * 256 * 4:
            raise ValueError("probe output needs groups * 256 words")
        n = ctypes.c_uint64()
        self._check(self.lib.dil_alu_probe(self.h, kind, iters, groups, _ptr(out), _stream(stream), ctypes.byref(n)))
        return n.value

    def t0_ntt(self, level: int, sk, t0_hat, stream=None):
        """t0_hat[n][k][256] = NTT(t0) of each secret key row, reduced to [0, q) (form per "t0.variant")."""
        n = sk.shape[0]
        k = {2: 4, 3: 6, 5: 8}.get(level)
        if k is None:
            raise ValueError("dil_t0_ntt_batch takes the round-3 levels 2, 3 and 5")
        _require([(sk, sizes(level)[1] * n, 1, "sk"), (t0_hat, 4 * k * 256 * n, 4, "t0_hat")])
        self._check(self.lib.dil_t0_ntt_batch(self.h, level, _ptr(sk), _ptr(t0_hat), n, _stream(stream)))

    def expand_a(self, seeds34, out, stream=None):
        self._check(self.lib.dil_expand_a_batch(self.h, _ptr(seeds34), _ptr(out), seeds34.shape[0],
                                                _stream(stream)))


class KeySet:
    """Device-resident key table of one level (A-hat, NTT'd secrets, NTT(t1 2^d), tr kept on the GPU)."""

    def __init__(self, ctx: Context, level: int, pk=None, sk=None, stream=None):
        self.lib = ctx.lib
        rows = (pk if pk is not None else sk).shape[0]
        h = _P()
        ctx._check(self.lib.dil_keyset_create(ctx.h, level, _ptr(pk), _ptr(sk), rows, ctypes.byref(h),
                                              _stream(stream)))
        self.h = h
        self.level = level
        self.n_keys = rows

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        self.lib.dil_keyset_info(self.h, None, None, ctypes.byref(b))
        return b.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.dil_keyset_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sign(self, ctx: Context, key_idx, msg, msg_off, sig, stream=None):
        n = msg_off.shape[0] - 1
        _require([(msg_off, 8 * (n + 1), 8, "msg_off"), (sig, sizes(self.level)[2] * n, 1, "sig"),
                  (key_idx, 4 * n, 4, "key_idx")])
        ctx._check(self.lib.dil_sign_keyset(ctx.h, self.h, _ptr(key_idx), _ptr(msg) or _ptr(msg_off), _ptr(msg_off),
                                            _ptr(sig), n, _stream(stream)))

    def verify(self, ctx: Context, key_idx, msg, msg_off, sig, verdict, stream=None, noalloc: bool = False):
        """noalloc: the entry point that allocates nothing (its workspace in the library's fixed
        per-GPU scratch array; calls overlapping on one GPU race on it)."""
        n = msg_off.shape[0] - 1
        _require([(msg_off, 8 * (n + 1), 8, "msg_off"), (sig, sizes(self.level)[2] * n, 1, "sig"),
                  (verdict, 4 * n, 4, "verdict"), (key_idx, 4 * n, 4, "key_idx")])
        fn = self.lib.dil_verify_keyset_noalloc if noalloc else self.lib.dil_verify_keyset
        ctx._check(fn(ctx.h, self.h, _ptr(key_idx), _ptr(msg) or _ptr(msg_off), _ptr(msg_off), _ptr(sig),
                      _ptr(verdict), n, _stream(stream)))
