"""Continuous-batching request loop over libdil on one GPU.

Requests (mixed-level Sign and Verify, each against one key of a resident
key table; levels 2/3/5 and ML-DSA 44/65/87) arrive
over time, replayed from a trace (`Server.serve`, `NativeServer.serve`) or
submitted one by one from application threads (`Service` over the Python
engine, `NativeService` over the C++ engine's interactive mode).  The loop keeps up to `n_streams`
batches in flight, each on its own HIP stream with its own libdil context
(workspace): whenever a stream is free, the requests that have arrived are
admitted in order as the next batch, split by (level, op) into key-table
calls (dil_sign_keyset / dil_verify_keyset).  Requests that arrive while
earlier batches run are admitted as soon as a stream frees up, so their work
overlaps on the device.

Device memory: every lane reserves up front the workspace of a key-table call
of C requests for each (level, op) (the library's own layout, from
dil_workspace_bytes), C the largest count for which all lanes' workspaces and
device staging buffers fit the memory budget.  A batch holds at most C
requests of each (level, op); the request that would exceed that waits for
the next batch.  Nothing is allocated while serving.

Host <-> device traffic goes through pinned staging buffers per stream
(messages, key indices and input signatures up; signatures and verdicts
down), so a request's latency -- completion time minus its scheduled
arrival -- includes queueing, both copies and the kernels.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import dilithium as dl

SIGN, VERIFY = 0, 1
LEVELS = (2, 3, 5)
DIL_SERVER_MLDSA_INTERNAL = 0x100   # mode flag of the native engine (include/dil.h)


@dataclass
class Requests:
    """A request stream in arrival order (all arrays indexed by request)."""
    t_arrival: np.ndarray      # float64 seconds from stream start
    op: np.ndarray             # int8: 0 sign, 1 verify
    level: np.ndarray          # int8
    key: np.ndarray            # int32 row in the level's key table
    msg: np.ndarray            # uint8, concatenated messages
    msg_off: np.ndarray        # int64, n + 1 CSR offsets
    sig_in: np.ndarray = None  # uint8, concatenated input signatures of verify requests
    sig_off: np.ndarray = None # int64 per request: offset into sig_in (verify) or -1

    def __len__(self):
        return self.t_arrival.size


@dataclass
class Results:
    sig: Dict[int, np.ndarray] = field(default_factory=dict)   # request -> signature bytes (sign)
    verdict: np.ndarray = None                                  # int32 per request (-1 for sign)
    t_done: np.ndarray = None                                   # completion time per request
    sig_buf: np.ndarray = None
    sig_pos: np.ndarray = None                                  # offset of request's signature in sig_buf


def sig_size(level: int) -> int:
    return dl.sizes(level)[2]


def check_requests(reqs: Requests, n_keys: Dict[int, int]) -> None:
    """Reject a malformed trace before any of it runs: the key-table calls read key rows on
    the device without bounds checks, so every request must name a level that has a table
    (n_keys: level -> rows) and a row inside it."""
    n = len(reqs)
    if reqs.msg_off.size != n + 1 or (n and (np.diff(reqs.msg_off) < 0).any()):
        raise ValueError("msg_off must hold n + 1 non-decreasing offsets")
    if n and (np.diff(reqs.t_arrival) < 0).any():
        raise ValueError("arrivals must be sorted")
    if not np.isin(reqs.op, (SIGN, VERIFY)).all():
        raise ValueError("op must be 0 (sign) or 1 (verify)")
    for lv in np.unique(reqs.level):
        lv = int(lv)
        if lv not in n_keys:
            raise ValueError(f"no key table for level {lv}")
        keys = reqs.key[reqs.level == lv]
        if (keys < 0).any() or (keys >= n_keys[lv]).any():
            raise ValueError(f"a level-{lv} request names a key row outside its table ({n_keys[lv]} rows)")
    if (reqs.op == VERIFY).any() and (reqs.sig_in is None or reqs.sig_off is None):
        raise ValueError("verify requests need signatures")


def _gather(buf: np.ndarray, starts: np.ndarray, lens: np.ndarray) -> np.ndarray:
    """Concatenate buf[starts[i] : starts[i] + lens[i]] without a Python loop."""
    total = int(lens.sum())
    if total == 0:
        return np.zeros(0, dtype=buf.dtype)
    first = np.concatenate([[0], np.cumsum(lens)[:-1]])
    idx = np.repeat(starts - first, lens) + np.arange(total)
    return buf[idx]


class _Lane:
    """One stream with its context and pinned staging buffers."""

    def __init__(self, torch, device, max_msg: int, max_tasks: int, max_sig: int, persistent: bool):
        self.torch = torch
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = dl.Context(device.index or 0, mode=dl.MODE_PERSISTENT if persistent else dl.MODE_STAGED)
        if persistent:
            # few tasks per call: four-wavefront workgroups give each task 4 x 64 / l nonces per batch
            self.ctx.set_param("persist.waves", 4)
        pin = dict(pin_memory=True)
        self.h_msg = torch.empty(max_msg, dtype=torch.uint8, **pin)
        self.h_off = torch.empty(max_tasks + 8, dtype=torch.int64, **pin)
        self.h_key = torch.empty(max_tasks, dtype=torch.int32, **pin)
        self.h_sig = torch.empty(max_sig, dtype=torch.uint8, **pin)
        self.h_ver = torch.empty(max_tasks, dtype=torch.int32, **pin)
        self.d_msg = torch.empty(max_msg, dtype=torch.uint8, device=device)
        self.d_off = torch.empty(max_tasks + 8, dtype=torch.int64, device=device)
        self.d_key = torch.empty(max_tasks, dtype=torch.int32, device=device)
        self.d_sig = torch.empty(max_sig, dtype=torch.uint8, device=device)
        self.d_ver = torch.empty(max_tasks, dtype=torch.int32, device=device)
        self.event = None
        self.batch = None
        self.staging_bytes = sum(t.numel() * t.element_size() for t in
                                 (self.d_msg, self.d_off, self.d_key, self.d_sig, self.d_ver))

    def workspace_need(self, cap: int, levels=LEVELS) -> int:
        """Workspace of the largest of this lane's calls with `cap` requests: the lane's calls
        run one after another on its stream and share one context."""
        return max(self.ctx.workspace_bytes(lv, op, True, cap) for lv in levels for op in (dl.OP_SIGN, dl.OP_VERIFY))

    def reserve(self, cap: int, levels=LEVELS):
        for lv in levels:
            for op in (dl.OP_SIGN, dl.OP_VERIFY):
                self.ctx.reserve_call(lv, op, True, cap)

    def close(self):
        self.ctx.close()


class Server:
    def __init__(self, keysets: Dict[int, "dl.KeySet"], n_streams: int = 4, max_batch: int = 4096,
                 mem_budget: int = 2 << 30, max_msg_bytes: int = 64 << 20, persistent: bool = True):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", 0)
        self.keysets = keysets
        self.levels = tuple(sorted(keysets))      # the levels this engine serves
        self.max_batch = max_batch
        self.mem_budget = mem_budget
        max_sig = max_batch * max(sig_size(lv) for lv in self.levels)
        self.lanes = [_Lane(torch, self.device, max_msg_bytes, max_batch, max_sig, persistent)
                      for _ in range(n_streams)]
        self.max_msg_bytes = max_msg_bytes
        # the largest per-(level, op) request count whose reservations fit the budget
        ln0 = self.lanes[0]
        lane_bytes = lambda c: ln0.staging_bytes + ln0.workspace_need(c, self.levels)
        lo, hi = 0, max_batch
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if lane_bytes(mid) * n_streams <= mem_budget:
                lo = mid
            else:
                hi = mid - 1
        if lo == 0:
            raise dl.DilError(dl.DIL_ENOMEM, "the memory budget does not hold one request per (level, op)")
        self.group_cap = lo
        self.reserved_bytes = lane_bytes(lo) * n_streams
        for ln in self.lanes:
            ln.reserve(lo, self.levels)

    def close(self):
        for ln in self.lanes:
            ln.close()

    # ---- batch launch ----
    def _launch(self, lane: _Lane, reqs: Requests, idx: np.ndarray):
        torch = self.torch
        lens = (reqs.msg_off[idx + 1] - reqs.msg_off[idx]).astype(np.int64)
        msg_np = lane.h_msg.numpy()
        off_np = lane.h_off.numpy()
        key_np = lane.h_key.numpy()
        sig_np = lane.h_sig.numpy()
        groups = []
        m_pos = s_pos = t_pos = 0
        for lv in self.levels:
            for op in (SIGN, VERIFY):
                sel = idx[(reqs.level[idx] == lv) & (reqs.op[idx] == op)]
                if sel.size == 0:
                    continue
                gl = (reqs.msg_off[sel + 1] - reqs.msg_off[sel]).astype(np.int64)
                gm = _gather(reqs.msg, reqs.msg_off[sel].astype(np.int64), gl)
                msg_np[m_pos:m_pos + gm.size] = gm
                off_np[t_pos + len(groups):t_pos + len(groups) + sel.size + 1] = np.concatenate(
                    [[0], np.cumsum(gl)])
                key_np[t_pos:t_pos + sel.size] = reqs.key[sel]
                ss = sig_size(lv)
                if op == VERIFY:
                    gs = _gather(reqs.sig_in, reqs.sig_off[sel].astype(np.int64), np.full(sel.size, ss))
                    sig_np[s_pos:s_pos + gs.size] = gs
                groups.append((lv, op, sel, m_pos, gm.size, t_pos, s_pos, ss))
                m_pos += gm.size
                s_pos += sel.size * ss
                t_pos += sel.size
        n_off = t_pos + len(groups)
        with torch.cuda.stream(lane.stream):
            lane.d_msg[:m_pos].copy_(lane.h_msg[:m_pos], non_blocking=True)
            lane.d_off[:n_off].copy_(lane.h_off[:n_off], non_blocking=True)
            lane.d_key[:t_pos].copy_(lane.h_key[:t_pos], non_blocking=True)
            lane.d_sig[:s_pos].copy_(lane.h_sig[:s_pos], non_blocking=True)
            for gi, (lv, op, sel, mp, ml, tp, sp, ss) in enumerate(groups):
                n = sel.size
                d_off = lane.d_off[tp + gi:tp + gi + n + 1]
                d_msg = lane.d_msg[mp:mp + max(ml, 1)]
                d_key = lane.d_key[tp:tp + n]
                d_sig = lane.d_sig[sp:sp + n * ss].view(n, ss)
                ks = self.keysets[lv]
                if op == SIGN:
                    ks.sign(lane.ctx, d_key, d_msg, d_off, d_sig, stream=lane.stream)
                else:
                    ks.verify(lane.ctx, d_key, d_msg, d_off, d_sig, lane.d_ver[tp:tp + n], stream=lane.stream)
            lane.h_sig[:s_pos].copy_(lane.d_sig[:s_pos], non_blocking=True)
            lane.h_ver[:t_pos].copy_(lane.d_ver[:t_pos], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(lane.stream)
        lane.event = ev
        lane.batch = groups

    def _collect(self, lane: _Lane, res: Results, now: float):
        sig_np = lane.h_sig.numpy()
        ver_np = lane.h_ver.numpy()
        for (lv, op, sel, mp, ml, tp, sp, ss) in lane.batch:
            res.t_done[sel] = now
            if op == SIGN:
                rows = sig_np[sp:sp + sel.size * ss].reshape(sel.size, ss)
                for j, r in enumerate(sel):
                    res.sig[int(r)] = rows[j].copy()
            else:
                res.verdict[sel] = ver_np[tp:tp + sel.size]
        lane.event = None
        lane.batch = None

    def _admit(self, reqs: Requests, head: int, end: int) -> int:
        """Requests head.. admitted in arrival order: at most group_cap of each (level, op) and
        at most max_msg_bytes of message data; returns how many."""
        grp = 2 * np.searchsorted(self.levels, reqs.level[head:end]) + reqs.op[head:end]
        nth = np.zeros(end - head, np.int64)       # rank of each request within its group
        for g in np.unique(grp):
            sel = grp == g
            nth[sel] = np.arange(int(sel.sum()))
        over = np.nonzero(nth >= self.group_cap)[0]
        fit = int(over[0]) if over.size else end - head
        m = np.cumsum(np.diff(reqs.msg_off[head:end + 1]))
        return min(fit, int(np.searchsorted(m, self.max_msg_bytes, side="right")))

    # ---- the loop ----
    def serve(self, reqs: Requests, time_scale: float = 1.0) -> Results:
        """Run the request stream; arrivals are honoured in real time (t_arrival * time_scale)."""
        check_requests(reqs, {lv: ks.n_keys for lv, ks in self.keysets.items()})
        n = len(reqs)
        res = Results(verdict=np.full(n, -1, np.int32), t_done=np.full(n, np.nan))
        free = deque(self.lanes)
        busy: List[_Lane] = []
        overlapped = 0
        head = 0
        done = 0
        launch_s: List[float] = []
        sizes: List[int] = []
        arrivals = reqs.t_arrival * time_scale
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            # completions
            for lane in list(busy):
                if lane.event.query():
                    k = lane.batch
                    cnt = sum(g[2].size for g in k)
                    self._collect(lane, res, time.perf_counter() - t0)
                    busy.remove(lane)
                    free.append(lane)
                    done += cnt
            # admission
            arrived = int(np.searchsorted(arrivals, now, side="right"))
            if free and head < arrived:
                fit = self._admit(reqs, head, min(arrived, head + self.max_batch))
                if fit == 0:
                    raise ValueError(f"request {head}'s message does not fit the staging buffer")
                lane = free.popleft()
                idx = np.arange(head, head + fit)
                tl = time.perf_counter()
                self._launch(lane, reqs, idx)
                launch_s.append(time.perf_counter() - tl)
                sizes.append(fit)
                overlapped += 1 if busy else 0
                busy.append(lane)
                head += fit
                continue
            if not busy and head >= arrived and head < n:
                # idle until the next arrival
                wait = arrivals[head] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        res.wall = time.perf_counter() - t0
        res.latency = res.t_done - arrivals
        res.batches = len(sizes)
        res.mean_batch = float(np.mean(sizes)) if sizes else 0.0
        res.host_launch_s = float(np.sum(launch_s))
        res.overlapped = overlapped
        res.group_cap = self.group_cap
        res.reserved_bytes = self.reserved_bytes
        return res


class Service:
    """Interactive front end of the request loop.  `submit` queues one request and returns a
    ticket at once (from any thread); a dispatcher thread admits the queued requests in order as
    batches on the free streams, under the admission rules of `Server` (at most `group_cap`
    requests of each (level, op) and `max_msg_bytes` of messages per batch), so requests
    submitted while earlier batches run join the next one; `poll` returns a ticket's result once
    it is done (None before) and `wait` blocks for it.  A result is the signature bytes of a Sign
    request or the verdict (True / False) of a Verify request; it is handed out once."""

    def __init__(self, keysets: Dict[int, "dl.KeySet"], n_streams: int = 4, max_batch: int = 4096,
                 mem_budget: int = 2 << 30, max_msg_bytes: int = 64 << 20, persistent: bool = True):
        self.server = Server(keysets, n_streams=n_streams, max_batch=max_batch, mem_budget=mem_budget,
                             max_msg_bytes=max_msg_bytes, persistent=persistent)
        self.n_keys = {lv: ks.n_keys for lv, ks in keysets.items()}
        self._cv = threading.Condition()
        self._pending: deque = deque()     # (ticket, level, op, key, msg, sig)
        self._results: Dict[int, object] = {}
        self._next = 0
        self._stop = False
        self._error: Optional[BaseException] = None
        self.batches = 0
        self._thread = threading.Thread(target=self._run, name="dil-service", daemon=True)
        self._thread.start()

    def submit(self, level: int, op: int, key: int, msg: bytes, sig: Optional[bytes] = None) -> int:
        """Queue Sign (op 0) of `msg` with key row `key` of the level's table, or Verify (op 1) of
        `sig` on it; the request is checked here, before anything runs."""
        msg = bytes(msg)
        if level not in self.n_keys:
            raise ValueError(f"no key table for level {level}")
        if op not in (SIGN, VERIFY):
            raise ValueError("op must be 0 (sign) or 1 (verify)")
        if not 0 <= key < self.n_keys[level]:
            raise ValueError(f"key row {key} outside the level-{level} table ({self.n_keys[level]} rows)")
        if len(msg) > self.server.max_msg_bytes:
            raise ValueError("message larger than a batch's staging buffer")
        if op == VERIFY:
            if sig is None or len(sig) != sig_size(level):
                raise ValueError(f"verify needs a {sig_size(level)}-byte signature")
            sig = bytes(sig)
        with self._cv:
            if self._stop:
                raise RuntimeError("service closed")
            t = self._next
            self._next += 1
            self._pending.append((t, level, op, key, msg, sig))
            self._cv.notify_all()
        return t

    def poll(self, ticket: int):
        with self._cv:
            if self._error is not None:
                raise RuntimeError("the dispatcher failed") from self._error
            return self._results.pop(ticket, None)

    def wait(self, ticket: int, timeout: Optional[float] = None):
        with self._cv:
            ok = self._cv.wait_for(lambda: ticket in self._results or self._error is not None, timeout)
            if self._error is not None:
                raise RuntimeError("the dispatcher failed") from self._error
            if not ok:
                raise TimeoutError(f"ticket {ticket} not done")
            return self._results.pop(ticket)

    def close(self):
        """Finish the queued requests, then stop the dispatcher and free the engine."""
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        self._thread.join()
        self.server.close()

    # ---- dispatcher ----
    def _take(self) -> list:
        """The next batch from the queue (called with the lock held): requests in submission order
        while every (level, op) group stays within group_cap and the messages within
        max_msg_bytes."""
        srv = self.server
        count: Dict[tuple, int] = {}
        nbytes = 0
        out = []
        while self._pending and len(out) < srv.max_batch:
            t, lv, op, key, msg, sig = self._pending[0]
            g = (lv, op)
            if count.get(g, 0) >= srv.group_cap or nbytes + len(msg) > srv.max_msg_bytes:
                break
            count[g] = count.get(g, 0) + 1
            nbytes += len(msg)
            out.append(self._pending.popleft())
        return out

    @staticmethod
    def _as_requests(batch: list) -> Requests:
        n = len(batch)
        lens = np.array([len(b[4]) for b in batch], np.int64)
        msg = np.frombuffer(b"".join(b[4] for b in batch), np.uint8) if lens.sum() else np.zeros(0, np.uint8)
        sigs = [b[5] for b in batch if b[2] == VERIFY]
        sig_off = np.full(n, -1, np.int64)
        pos = 0
        for i, b in enumerate(batch):
            if b[2] == VERIFY:
                sig_off[i] = pos
                pos += len(b[5])
        return Requests(t_arrival=np.zeros(n), op=np.array([b[2] for b in batch], np.int8),
                        level=np.array([b[1] for b in batch], np.int8),
                        key=np.array([b[3] for b in batch], np.int32), msg=msg,
                        msg_off=np.concatenate([[0], np.cumsum(lens)]).astype(np.int64),
                        sig_in=np.frombuffer(b"".join(sigs), np.uint8) if sigs else np.zeros(0, np.uint8),
                        sig_off=sig_off)

    def _run(self):
        srv = self.server
        free = deque(srv.lanes)
        busy: List[tuple] = []       # (lane, tickets, Results of the batch)
        try:
            while True:
                for item in list(busy):
                    lane, tickets, res = item
                    if lane.event.query():
                        srv._collect(lane, res, 0.0)
                        out = {t: (res.sig[i].tobytes() if i in res.sig else bool(res.verdict[i] == 1))
                               for i, t in enumerate(tickets)}
                        with self._cv:
                            self._results.update(out)
                            self._cv.notify_all()
                        busy.remove(item)
                        free.append(lane)
                batch = []
                with self._cv:
                    if free and self._pending:
                        batch = self._take()
                    elif not busy:
                        if self._stop and not self._pending:
                            return
                        self._cv.wait(0.01)
                if batch:
                    reqs = self._as_requests(batch)
                    lane = free.popleft()
                    res = Results(verdict=np.full(len(batch), -1, np.int32), t_done=np.zeros(len(batch)))
                    srv._launch(lane, reqs, np.arange(len(batch)))
                    busy.append((lane, [b[0] for b in batch], res))
                    self.batches += 1
                elif busy:
                    time.sleep(0.0001)
        except BaseException as e:   # surfaced to every waiting caller
            with self._cv:
                self._error = e
                self._cv.notify_all()


class NativeServer:
    """The C++ serving engine of libdil (dil_server_*): same admission policy as `Server`, with batch
    formation, staging and harvesting in native code.  Requests are replayed from a trace with their
    arrival times (`serve`)."""

    def __init__(self, keysets: Dict[int, "dl.KeySet"], n_streams: int = 4, max_batch: int = 4096,
                 mem_budget: int = 2 << 30, max_msg_bytes: int = 64 << 20, persistent: bool = True,
                 mldsa_internal: bool = False):
        """mldsa_internal: requests at the ML-DSA levels carry formatted messages M' (context
        strings, pre-hashed messages); round-3 requests are unaffected."""
        import ctypes
        self.lib = dl.load()
        self.keysets = keysets
        h = ctypes.c_void_p()
        tables = (ctypes.c_void_p * max(len(keysets), 1))(*[keysets[lv].h.value for lv in sorted(keysets)])
        rc = self.lib.dil_server_create_tables(ctypes.byref(h), 0, ctypes.cast(tables, ctypes.c_void_p), len(keysets),
                                               n_streams, max_batch, max_msg_bytes, mem_budget,
                                               (dl.MODE_PERSISTENT if persistent else dl.MODE_STAGED) |
                                               (DIL_SERVER_MLDSA_INTERNAL if mldsa_internal else 0))
        if rc:
            raise dl.DilError(rc, "server creation failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.dil_server_destroy(self.h)
            self.h = None

    def serve(self, reqs: Requests, time_scale: float = 1.0) -> Results:
        import ctypes
        n = len(reqs)
        P = lambda a: a.ctypes.data if a is not None and a.size else None
        op = np.ascontiguousarray(reqs.op, dtype=np.uint8)
        level = np.ascontiguousarray(reqs.level, dtype=np.uint8)
        key = np.ascontiguousarray(reqs.key, dtype=np.uint32)
        msg = np.ascontiguousarray(reqs.msg if reqs.msg.size else np.zeros(1, np.uint8), dtype=np.uint8)
        moff = np.ascontiguousarray(reqs.msg_off, dtype=np.uint64)
        arr = np.ascontiguousarray(np.round(reqs.t_arrival * time_scale * 1e9), dtype=np.uint64)
        sig_in = np.ascontiguousarray(reqs.sig_in if reqs.sig_in is not None and reqs.sig_in.size
                                      else np.zeros(1, np.uint8), dtype=np.uint8)
        sig_in_off = np.ascontiguousarray(np.maximum(reqs.sig_off, 0) if reqs.sig_off is not None
                                          else np.zeros(n, np.int64), dtype=np.uint64)
        levels = tuple(sorted(self.keysets))
        sizes = np.array([sig_size(int(lv)) for lv in levels])
        ss = np.where(reqs.op == SIGN, sizes[np.searchsorted(levels, reqs.level)], 0).astype(np.uint64)
        sig_out_off = np.concatenate([[0], np.cumsum(ss)[:-1]]).astype(np.uint64)
        sig_out = np.zeros(max(int(ss.sum()), 1), np.uint8)
        verdict = np.full(n, -1, np.int32)
        done = np.zeros(n, np.uint64)
        rc = self.lib.dil_server_run(self.h, n, P(op), P(level), P(key), P(msg), P(moff), P(sig_in), P(sig_in_off),
                                     P(arr), P(sig_out), P(sig_out_off), P(verdict), P(done))
        if rc:
            raise dl.DilError(rc, self.lib.dil_server_last_error(self.h).decode(errors="replace"))
        b, hs, ov, cap, rb = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_size_t()
        self.lib.dil_server_stats(self.h, ctypes.byref(b), ctypes.byref(hs), ctypes.byref(ov), ctypes.byref(cap),
                                  ctypes.byref(rb))
        res = Results(verdict=verdict, t_done=done.astype(np.float64) * 1e-9)
        for r in np.nonzero(reqs.op == SIGN)[0]:
            o = int(sig_out_off[r])
            res.sig[int(r)] = sig_out[o:o + int(ss[r])]
        res.wall = float(done.max()) * 1e-9
        res.latency = res.t_done - arr.astype(np.float64) * 1e-9
        res.batches = int(b.value)
        res.mean_batch = n / max(int(b.value), 1)
        res.host_launch_s = hs.value
        res.overlapped = int(ov.value)
        res.group_cap = int(cap.value)
        res.reserved_bytes = int(rb.value)
        return res


class NativeService:
    """The interactive front end of the C++ engine (dil_server_start / submit / poll / wait / stop):
    the same interface as `Service`, with the dispatcher thread, batch formation and result
    bookkeeping in native code.  A result is the signature bytes of a Sign request or the verdict
    (True / False) of a Verify request; it is handed out once."""

    def __init__(self, keysets: Dict[int, "dl.KeySet"], n_streams: int = 4, max_batch: int = 4096,
                 mem_budget: int = 2 << 30, max_msg_bytes: int = 64 << 20, persistent: bool = True,
                 mldsa_internal: bool = False):
        import ctypes
        self.server = NativeServer(keysets, n_streams=n_streams, max_batch=max_batch, mem_budget=mem_budget,
                                   max_msg_bytes=max_msg_bytes, persistent=persistent, mldsa_internal=mldsa_internal)
        self.lib = self.server.lib
        self._c = ctypes
        self.n_keys = {lv: ks.n_keys for lv, ks in keysets.items()}
        self.max_msg_bytes = max_msg_bytes
        self._op = {}                      # ticket -> (op, level), for the result's shape
        self._lock = threading.Lock()
        rc = self.lib.dil_server_start(self.server.h)
        if rc:
            self.server.close()
            raise dl.DilError(rc, "dil_server_start failed")

    def _err(self, rc: int, what: str):
        text = self.lib.dil_server_last_error(self.server.h).decode(errors="replace")
        return dl.DilError(rc, f"{what}: {text}")

    def submit(self, level: int, op: int, key: int, msg: bytes, sig: Optional[bytes] = None) -> int:
        """Queue Sign (op 0) of `msg` with key row `key` of the level's table, or Verify (op 1) of
        `sig` on it; malformed requests are refused here, before anything runs."""
        c = self._c
        if getattr(self, "server", None) is None:
            raise RuntimeError("service closed")
        msg = bytes(msg)
        if level not in self.n_keys:
            raise ValueError(f"no key table for level {level}")
        if op not in (SIGN, VERIFY):
            raise ValueError("op must be 0 (sign) or 1 (verify)")
        if not 0 <= key < self.n_keys[level]:
            raise ValueError(f"key row {key} outside the level-{level} table ({self.n_keys[level]} rows)")
        if len(msg) > self.max_msg_bytes:
            raise ValueError("message larger than a batch's staging buffer")
        sbuf = None
        if op == VERIFY:
            if sig is None or len(sig) != sig_size(level):
                raise ValueError(f"verify needs a {sig_size(level)}-byte signature")
            sbuf = c.create_string_buffer(bytes(sig), len(sig))
        mbuf = c.create_string_buffer(msg, max(len(msg), 1))
        t = c.c_uint64()
        rc = self.lib.dil_server_submit(self.server.h, op, level, key, c.cast(mbuf, c.c_void_p), len(msg),
                                        c.cast(sbuf, c.c_void_p) if sbuf is not None else None, c.byref(t))
        if rc:
            raise self._err(rc, "submit")
        with self._lock:
            self._op[t.value] = (op, level)
        return t.value

    def _result(self, ticket: int, verdict, sbuf):
        with self._lock:
            op, _ = self._op.pop(ticket)
        return sbuf.raw if op == SIGN else bool(verdict.value == 1)

    def _buffers(self, ticket: int):
        with self._lock:
            if ticket not in self._op:
                raise KeyError(f"ticket {ticket} is not outstanding")
            op, level = self._op[ticket]
        return self._c.c_int32(), self._c.create_string_buffer(sig_size(level))

    def poll(self, ticket: int):
        """The result once the request has finished, else None (also for a ticket whose result
        was already handed out)."""
        c = self._c
        with self._lock:
            if ticket not in self._op:
                return None
        verdict, sbuf = self._buffers(ticket)
        done = c.c_int()
        rc = self.lib.dil_server_poll(self.server.h, ticket, c.byref(done), c.byref(verdict), c.cast(sbuf, c.c_void_p))
        if rc:
            raise self._err(rc, "poll")
        return self._result(ticket, verdict, sbuf) if done.value else None

    def wait(self, ticket: int, timeout: Optional[float] = None):
        c = self._c
        verdict, sbuf = self._buffers(ticket)
        ms = -1 if timeout is None else max(int(timeout * 1e3), 0)
        rc = self.lib.dil_server_wait(self.server.h, ticket, ms, c.byref(verdict), c.cast(sbuf, c.c_void_p))
        if rc == dl.DIL_ETIMEDOUT:
            raise TimeoutError(f"ticket {ticket} not done")
        if rc:
            raise self._err(rc, "wait")
        return self._result(ticket, verdict, sbuf)

    @property
    def batches(self) -> int:
        b = self._c.c_uint64()
        self.lib.dil_server_stats(self.server.h, self._c.byref(b), None, None, None, None)
        return int(b.value)

    def close(self):
        """Finish the submitted requests, then stop the dispatcher and free the engine."""
        if getattr(self, "server", None) is None:
            return
        rc = self.lib.dil_server_stop(self.server.h)
        self.server.close()
        self.server = None
        if rc:
            raise dl.DilError(rc, "the dispatcher failed")


def latency_summary(res: Results, reqs: Requests) -> dict:
    lat = res.latency * 1e3
    out = {"requests": int(len(reqs)), "wall_s": res.wall, "ops_per_s": len(reqs) / res.wall,
           "batches": res.batches, "mean_batch": res.mean_batch, "host_launch_s": res.host_launch_s,
           "batches_overlapped": getattr(res, "overlapped", None), "group_cap": getattr(res, "group_cap", None),
           "reserved_bytes": getattr(res, "reserved_bytes", None),
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "max_ms": float(lat.max())}
    for op, name in ((SIGN, "sign"), (VERIFY, "verify")):
        m = reqs.op == op
        if m.any():
            out[f"p99_ms_{name}"] = float(np.percentile(lat[m], 99))
    return out


def build_requests(count: int, lam: float, keys_per_level: Dict[int, int], seed: int = 0) -> Requests:
    """Poisson stream: 70% verify / 30% sign, levels 50/30/20%, lognormal messages (see workload.py).
    Verify signatures are filled in by `attach_signatures`."""
    from . import workload
    rng_t = np.random.default_rng([seed, 1])
    gaps = rng_t.exponential(1.0 / lam, size=count) if lam > 0 else np.zeros(count)
    t = np.cumsum(gaps)
    if lam <= 0:
        t[:] = 0.0
    op = (np.random.default_rng([seed, 2]).random(count) < 0.7).astype(np.int8)
    level = np.random.default_rng([seed, 3]).choice([2, 3, 5], size=count, p=[0.5, 0.3, 0.2]).astype(np.int8)
    kr = np.random.default_rng([seed, 4]).random(count)
    key = np.array([int(kr[i] * keys_per_level[int(level[i])]) % keys_per_level[int(level[i])]
                    for i in range(count)], dtype=np.int32)
    lens = workload.lognormal_lengths(count, seed=seed)
    msg, off = workload.messages(lens, seed=seed + 1)
    return Requests(t, op, level, key, msg, off.astype(np.int64))


def attach_signatures(reqs: Requests, ctx: "dl.Context", keysets: Dict[int, "dl.KeySet"], flip_rate: float = 0.01,
                      seed: int = 0):
    """Sign every verify request's message on the GPU (untimed set-up), then flip one random bit in a
    fraction `flip_rate` of them so those must be rejected."""
    import torch
    dev = torch.device("cuda", 0)
    n = len(reqs)
    sig_off = np.full(n, -1, np.int64)
    parts = []
    pos = 0
    flips = np.random.default_rng([seed, 5]).random(n) < flip_rate
    fbits = np.random.default_rng([seed, 6]).integers(0, 1 << 30, size=n)
    flipped = np.zeros(n, bool)
    for lv in np.unique(reqs.level).tolist():
        sel = np.nonzero((reqs.level == lv) & (reqs.op == VERIFY))[0]
        if sel.size == 0:
            continue
        ss = sig_size(lv)
        lens = (reqs.msg_off[sel + 1] - reqs.msg_off[sel])
        gm = _gather(reqs.msg, reqs.msg_off[sel], lens)
        goff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        d_sig = torch.zeros((sel.size, ss), dtype=torch.uint8, device=dev)
        keysets[lv].sign(ctx, torch.from_numpy(reqs.key[sel]).to(dev), torch.from_numpy(gm).to(dev),
                         torch.from_numpy(goff).to(dev), d_sig)
        sigs = d_sig.cpu().numpy()
        for j, r in enumerate(sel):
            if flips[r]:
                b = int(fbits[r] % (ss * 8))
                sigs[j, b // 8] ^= np.uint8(1 << (b % 8))
                flipped[r] = True
        sig_off[sel] = pos + np.arange(sel.size) * ss
        parts.append(sigs.reshape(-1))
        pos += sigs.size
    reqs.sig_in = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    reqs.sig_off = sig_off
    return flipped
