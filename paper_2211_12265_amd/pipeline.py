"""End-to-end host path: Sign / Verify of host-resident batches.

The paper's throughput figures include the host<->device copies and hide them
behind computation with several CUDA streams, one chunk of tasks per stream
(Sec. 4.4, multi-stream execution).  This module is the same pipeline on HIP:
the caller's pinned host buffers are cut into contiguous chunks of tasks;
chunk c goes to stream c mod S, where its rows are copied to device buffers
owned by that stream, signed or verified by the C-ABI on that stream (each
stream has its own libdil context, so workspaces never alias), and its
results copied back.  Copies and kernels of different streams overlap;
operations of one stream stay in order, so a stream's device buffers are
reused by its next chunk without further synchronisation.

Every step of Sign / Verify runs in libdil's kernels; this module only moves
bytes (torch copies on pinned memory) and rebases each chunk's message
offsets, which is host marshalling done once per batch before the copies
start.
"""
from __future__ import annotations

import threading
from typing import List, Optional

import numpy as np

from . import dilithium as dl


def pinned(shape, dtype=None):
    """A new page-locked host tensor (hipHostMalloc through torch)."""
    import torch
    return torch.empty(shape, dtype=dtype or torch.uint8, pin_memory=True)


class _Chunk:
    __slots__ = ("a", "b", "o0", "o1", "off")

    def __init__(self, a, b, o0, o1, off):
        self.a, self.b, self.o0, self.o1, self.off = a, b, o0, o1, off


class HostPipeline:
    """Chunked, multi-stream Sign / Verify of host-resident batches at one level.

    n_streams: HIP streams (and libdil contexts) used; chunk: tasks per chunk.
    mode: Sign execution form of every context (dl.MODE_*).
    host_threads: issue each stream's chunks from a host thread of its own (the
    paper's one host thread per stream, Sec. 4.4), so that the copies and calls
    of one stream are enqueued without waiting behind another stream's; the
    C-ABI calls release the interpreter lock, and each thread uses only its
    stream's context.  False issues every stream from the calling thread.
    Persistent Sign calls of different streams run at the same time, so each
    context gets an equal share of the GPU's resident four-wavefront
    workgroups (and as many held tasks per workgroup as its chunk needs)
    instead of the single-call automatic schedule, which would size every
    launch for the whole GPU.
    """

    def __init__(self, level: int, n_streams: int = 4, chunk: int = 1250, mode: int = dl.MODE_PERSISTENT,
                 device: int = 0, host_threads: bool = False):
        import torch
        if n_streams < 1 or chunk < 1:
            raise ValueError("n_streams and chunk must be positive")
        self.level, self.S, self.chunk = level, n_streams, chunk
        self.host_threads = host_threads
        self.pkl, self.skl, self.sgl = dl.sizes(level)
        self.dev = torch.device("cuda", device)
        self.ctx = [dl.Context(device, mode=mode) for _ in range(n_streams)]
        for c in self.ctx:
            if mode == dl.MODE_PERSISTENT:
                c.set_param("persist.waves", 4)
                resident, slots = c.persist_capacity(level)
                grid = max(1, min(resident // n_streams, -(-chunk // 16)))
                c.set_param("persist.grid", grid)
                c.set_param("persist.hmax", min(slots, -(-chunk // grid)))
            c.reserve(level, chunk)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_streams)]
        # flat, so that [m, PK] and [m, SK] views of it are both contiguous
        self.d_key = [torch.empty(chunk * max(self.pkl, self.skl), dtype=torch.uint8, device=self.dev)
                      for _ in range(n_streams)]
        self.d_sig = [torch.empty((chunk, self.sgl), dtype=torch.uint8, device=self.dev) for _ in range(n_streams)]
        self.d_ver = [torch.empty(chunk, dtype=torch.int32, device=self.dev) for _ in range(n_streams)]
        self.d_off = [torch.empty(chunk + 1, dtype=torch.int64, device=self.dev) for _ in range(n_streams)]
        self.d_msg: List = [None] * n_streams
        self._plan: Optional[List[_Chunk]] = None
        self._plan_key = None

    def close(self):
        for c in self.ctx:
            c.close()
        self.ctx = []

    def plan(self, off: np.ndarray) -> List[_Chunk]:
        """Cut the batch into chunks and rebase each chunk's CSR offsets (pinned, reused)."""
        import torch
        off = np.asarray(off, dtype=np.int64)
        if np.any(np.diff(off) < 0) or off[0] != 0:
            raise ValueError("msg_off must start at 0 and be non-decreasing")
        key = (off.shape[0], int(off[-1]), hash(off.tobytes()))
        if self._plan_key == key:
            return self._plan
        n = off.shape[0] - 1
        plan = []
        for a in range(0, n, self.chunk):
            b = min(n, a + self.chunk)
            o = pinned((b - a + 1,), torch.int64)
            o.numpy()[:] = off[a:b + 1] - off[a]
            plan.append(_Chunk(a, b, int(off[a]), int(off[b]), o))
        longest = max((c.o1 - c.o0 for c in plan), default=0)
        for s in range(self.S):
            if self.d_msg[s] is None or self.d_msg[s].numel() < max(longest, 1):
                self.d_msg[s] = torch.empty(max(longest, 1), dtype=torch.uint8, device=self.dev)
        self._plan, self._plan_key = plan, key
        return plan

    def _issue(self, op: str, s: int, chunks, keys, msg, sig, out):
        """Enqueue chunks on stream s: copies in, the C-ABI call, copy out."""
        import torch
        st, ctx = self.streams[s], self.ctx[s]
        kl = self.skl if op == "sign" else self.pkl
        with torch.cuda.stream(st):
            for c in chunks:
                m = c.b - c.a
                dk = self.d_key[s][:m * kl].view(m, kl)
                dk.copy_(keys[c.a:c.b], non_blocking=True)
                dm = self.d_msg[s][:c.o1 - c.o0]
                if c.o1 > c.o0:
                    dm.copy_(msg[c.o0:c.o1], non_blocking=True)
                do = self.d_off[s][:m + 1]
                do.copy_(c.off, non_blocking=True)
                if op == "sign":
                    ds = self.d_sig[s][:m]
                    ctx.sign(self.level, dk, dm, do, ds, stream=st)
                    out[c.a:c.b].copy_(ds, non_blocking=True)
                else:
                    ds = self.d_sig[s][:m]
                    ds.copy_(sig[c.a:c.b], non_blocking=True)
                    dv = self.d_ver[s][:m]
                    ctx.verify(self.level, dk, dm, do, ds, dv, stream=st)
                    out[c.a:c.b].copy_(dv, non_blocking=True)

    def _run(self, op: str, keys, msg, off, sig, out):
        import torch
        plan = self.plan(off)
        cur = torch.cuda.current_stream(self.dev)
        for s in self.streams:
            s.wait_stream(cur)
        # chunk i goes to stream i mod S
        groups = [plan[s::self.S] for s in range(self.S)]
        if self.host_threads and self.S > 1:
            errors = []

            def work(s):
                try:
                    torch.cuda.set_device(self.dev)
                    self._issue(op, s, groups[s], keys, msg, sig, out)
                except BaseException as e:  # re-raised on the calling thread
                    errors.append(e)

            threads = [threading.Thread(target=work, args=(s,)) for s in range(self.S)]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
            if errors:
                raise errors[0]
        else:
            for s in range(self.S):
                self._issue(op, s, groups[s], keys, msg, sig, out)
        for s in self.streams:
            cur.wait_stream(s)

    def sign(self, sk, msg, off, sig_out):
        """sk: pinned uint8 [n, SK]; msg: pinned uint8 bytes; off: int64 [n + 1]; sig_out: pinned uint8 [n, SIG].
        Asynchronous with respect to the host; synchronise the current stream before reading sig_out."""
        self._run("sign", sk, msg, off, None, sig_out)

    def verify(self, pk, msg, off, sig, verdict_out):
        """pk: pinned uint8 [n, PK]; sig: pinned uint8 [n, SIG]; verdict_out: pinned int32 [n]."""
        self._run("verify", pk, msg, off, sig, verdict_out)

    def check(self):
        """Synchronise every stream and report a device-detected input error once."""
        for st, ctx in zip(self.streams, self.ctx):
            ctx.check(st)

