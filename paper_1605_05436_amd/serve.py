"""Continuous-batching server for exact-sum requests on one GPU.

Requests (device data of n elements, binary64 / binary32 / bfloat16) are
admitted when the server's HBM arena has room for their payload and an exact
accumulator slot is free; on admission the payload is copied into the arena
on a copy stream.  Every scheduler iteration gathers pieces of all admitted
requests (large requests are cut into pieces so small ones are not stuck
behind them) into one batch: one `xsum_batch_add` launch adds every piece into
its request's device state, one `xsum_batch_finalize` launch rounds the
requests whose last piece was in the batch, and their results are copied to
pinned host memory.  Iterations are not waited for: the host keeps
scheduling while earlier batches run, and retires requests when their
iteration's completion event has fired, freeing arena space and slots.

Exact integer accumulation makes results independent of batching, piece
boundaries and order, so a request's result is bit-identical alone and in any
mix (Section 6 of Goodrich & Eldawy: reducers' superaccumulators are merged
exactly; here the merge target persists on the device across launches).

The host side only orchestrates; all arithmetic runs in libxsum.
"""

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import (F64, F32, BF16, SAME, batch_item_dtype, xsum_batch_add,
               xsum_batch_finalize, xsum_batch_item_tasks, new_states,
               stream_handle)
from .arena import ArenaAllocator

ITEMSIZE = {F64: 8, F32: 4, BF16: 2}
NATURAL_OUT = {F64: F64, F32: F32, BF16: F32}


@dataclass
class Request:
    rid: int
    src: object            # client's payload: a contiguous device tensor
    n: int                 # elements
    dtype: int
    out_dtype: int = SAME
    arrival: float = 0.0   # seconds on the server clock
    # filled by the server
    admitted: float = None
    done: float = None
    bits: int = None
    flags: int = None
    slot: int = None
    arena_off: int = None
    pieces: deque = field(default_factory=deque)
    ready_event: object = None   # the payload is complete once this has fired


class ExactSumServer:
    """Continuous-batching exact-sum server on the current CUDA/HIP device.

    arena_bytes   HBM reserved for admitted payloads
    slots         device accumulator states (concurrent requests)
    piece_elems   requests are cut into pieces of at most this many elements
    batch_bytes   byte budget of one batch (pieces of several requests)
    chunk_vectors 16-byte vectors per GPU work item inside a piece

    Streams: the server works on its own compute and copy streams.  At
    construction they wait for the caller's current stream (where the states
    were zeroed); each request's admission copy waits for the stream it was
    submitted from (see submit), and the payload tensor is recorded on the
    copy stream so the caching allocator does not reuse it early.
    """

    def __init__(self, arena_bytes=4 << 30, slots=4096, piece_elems=1 << 24,
                 batch_bytes=512 << 20, chunk_vectors=1 << 16, max_items=8192,
                 ring=8):
        import torch
        self.torch = torch
        dev = torch.device("cuda")
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
        self.arena_base = self.arena.data_ptr()
        assert self.arena_base % 256 == 0
        self.alloc = ArenaAllocator(arena_bytes)
        self.nslots = slots
        self.states = new_states(slots)
        self.free_slots = list(range(slots - 1, -1, -1))
        self.ctl = torch.zeros(32, dtype=torch.int64, device=dev)
        self.compute = torch.cuda.Stream()
        self.copy = torch.cuda.Stream()
        # the states and the control block were zeroed on the caller's
        # stream; the server's own streams start after that work
        here = torch.cuda.current_stream()
        self.compute.wait_stream(here)
        self.copy.wait_stream(here)
        self.piece_elems = piece_elems - piece_elems % 8   # keep 16-byte pieces
        self.batch_bytes = batch_bytes
        self.chunk_vectors = chunk_vectors
        self.max_items = max_items
        # ring of per-iteration staging buffers (pinned host + device)
        self.ring = []
        idt = batch_item_dtype()
        for _ in range(ring):
            self.ring.append({
                "items_h": torch.empty(max_items * idt.itemsize, dtype=torch.uint8).pin_memory(),
                "items_d": torch.empty(max_items * idt.itemsize, dtype=torch.uint8, device=dev),
                "fin_h": torch.empty(2 * max_items, dtype=torch.int32).pin_memory(),
                "fin_d": torch.empty(2 * max_items, dtype=torch.int32, device=dev),
                "out_d": torch.empty(max_items, dtype=torch.int64, device=dev),
                "flags_d": torch.empty(max_items, dtype=torch.int32, device=dev),
                "out_h": torch.empty(max_items, dtype=torch.int64).pin_memory(),
                "flags_h": torch.empty(max_items, dtype=torch.int32).pin_memory(),
                "event": None, "finished": [], "busy": None,
            })
        self.ring_next = 0
        self.waiting = deque()       # arrived, not admitted
        self.active = deque()        # admitted, pieces left to schedule
        self.inflight = deque()      # ring entries whose batch runs
        self.completed = []
        self.gpu_time_ms = 0.0
        self.batches = 0
        self.elements = 0

    # ------------------------------------------------------------ admission --
    def submit(self, req, stream=None):
        """Queue a request.  Its payload may still be in production on
        `stream` (default: the caller's current stream); the admission copy
        waits for everything enqueued there up to this call, so the caller
        must not write req.src after submitting it."""
        nbytes = req.n * ITEMSIZE[req.dtype]
        if nbytes > self.arena.numel():
            raise ValueError("request %d needs %d bytes, more than the whole arena "
                             "(%d bytes); it could never be admitted"
                             % (req.rid, nbytes, self.arena.numel()))
        ready = self.torch.cuda.Event()
        ready.record(stream if stream is not None else self.torch.cuda.current_stream())
        req.ready_event = ready
        self.waiting.append(req)

    def _admit(self, now):
        torch = self.torch
        while self.waiting and self.free_slots:
            req = self.waiting[0]
            nbytes = req.n * ITEMSIZE[req.dtype]
            off, ln = self.alloc.alloc(nbytes)
            if off is None:
                break                      # arena full: wait for completions
            self.waiting.popleft()
            req.arena_off, req.arena_len = off, ln
            req.slot = self.free_slots.pop()
            req.admitted = now
            if nbytes:
                src = req.src.view(torch.uint8).reshape(-1)[:nbytes]
                self.copy.wait_event(req.ready_event)
                with torch.cuda.stream(self.copy):
                    self.arena[off:off + nbytes].copy_(src, non_blocking=True)
                req.src.record_stream(self.copy)
            ev = torch.cuda.Event()
            ev.record(self.copy)
            req.copy_event = ev
            es = ITEMSIZE[req.dtype]
            base = self.arena_base + off
            start = 0
            while True:
                cnt = min(self.piece_elems, req.n - start)
                req.pieces.append((base + start * es, cnt))
                start += cnt
                if start >= req.n:
                    break
            self.active.append(req)

    # ------------------------------------------------------------- batching --
    def _launch_batch(self):
        torch = self.torch
        if not self.active:
            return False
        entry = self.ring[self.ring_next]
        if entry["event"] is not None:
            return False                   # ring full: retire first
        idt = batch_item_dtype()
        items = np.zeros(self.max_items, dtype=idt)
        fin_slots, fin_fmts, finished = [], [], []
        budget = self.batch_bytes
        nitems = 0
        ntasks = 0
        waits = []
        rotate = len(self.active)
        for _ in range(rotate):
            if nitems >= self.max_items or budget <= 0:
                break
            req = self.active.popleft()
            took = False
            while req.pieces and nitems < self.max_items and budget > 0:
                ptr, cnt = req.pieces.popleft()
                t = xsum_batch_item_tasks(ptr, cnt, req.dtype, self.chunk_vectors)
                items[nitems] = (ptr, cnt, req.dtype, req.slot, ntasks)
                ntasks += t
                nitems += 1
                budget -= cnt * ITEMSIZE[req.dtype]
                took = True
            if took:
                waits.append(req.copy_event)
            if req.pieces:
                self.active.append(req)      # continues in a later batch
            else:
                fin_slots.append(req.slot)
                fin_fmts.append(NATURAL_OUT[req.dtype] if req.out_dtype == SAME
                                else req.out_dtype)
                finished.append(req)
        if nitems == 0:
            return False
        nfin = len(finished)
        ih = entry["items_h"].numpy()
        ih[:nitems * idt.itemsize] = items[:nitems].view(np.uint8)
        fh = entry["fin_h"].numpy()
        fh[:nfin] = fin_slots
        fh[self.max_items:self.max_items + nfin] = fin_fmts
        s = self.compute
        for ev in waits:
            s.wait_event(ev)
        with torch.cuda.stream(s):
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record(s)
            entry["items_d"][:nitems * idt.itemsize].copy_(
                entry["items_h"][:nitems * idt.itemsize], non_blocking=True)
            if nfin:
                mi = self.max_items
                entry["fin_d"][:nfin].copy_(entry["fin_h"][:nfin], non_blocking=True)
                entry["fin_d"][mi:mi + nfin].copy_(entry["fin_h"][mi:mi + nfin],
                                                   non_blocking=True)
            sh = stream_handle(s)
            xsum_batch_add(entry["items_d"].data_ptr(), nitems, ntasks,
                           self.chunk_vectors, self.states.data_ptr(),
                           self.ctl.data_ptr(), sh)
            if nfin:
                xsum_batch_finalize(entry["fin_d"].data_ptr(),
                                    entry["fin_d"].data_ptr() + 4 * self.max_items,
                                    nfin, self.states.data_ptr(),
                                    entry["out_d"].data_ptr(),
                                    entry["flags_d"].data_ptr(), sh)
                entry["out_h"][:nfin].copy_(entry["out_d"][:nfin], non_blocking=True)
                entry["flags_h"][:nfin].copy_(entry["flags_d"][:nfin], non_blocking=True)
            end.record(s)
        entry["event"] = end
        entry["busy"] = (start, end)
        entry["finished"] = finished
        self.inflight.append(entry)
        self.ring_next = (self.ring_next + 1) % len(self.ring)
        self.batches += 1
        return True

    # ------------------------------------------------------------- retiring --
    def _retire(self, now_fn, block=False):
        torch = self.torch
        retired = 0
        while self.inflight:
            entry = self.inflight[0]
            ev = entry["event"]
            if block:
                ev.synchronize()
            elif not ev.query():
                break
            self.inflight.popleft()
            now = now_fn()
            st, en = entry["busy"]
            self.gpu_time_ms += st.elapsed_time(en)
            oh = entry["out_h"].numpy()
            fl = entry["flags_h"].numpy()
            for k, req in enumerate(entry["finished"]):
                req.bits = int(oh[k]) & 0xFFFFFFFFFFFFFFFF
                req.flags = int(fl[k])
                req.done = now
                self.alloc.release(req.arena_off, req.arena_len)
                self.free_slots.append(req.slot)
                self.completed.append(req)
                self.elements += req.n
                retired += 1
            entry["event"] = None
            entry["finished"] = []
        return retired

    def step(self, now_fn):
        """One scheduler pass: retire, admit, launch.  Returns True if it did
        anything."""
        did = self._retire(now_fn) > 0
        self._admit(now_fn())
        while self._launch_batch():
            did = True
        return did

    def drain(self, now_fn):
        while self.waiting or self.active or self.inflight:
            if not self.step(now_fn):
                if self.inflight:
                    self._retire(now_fn, block=True)
                else:
                    time.sleep(0)

    def busy(self):
        return bool(self.waiting or self.active or self.inflight)


def run_trace(server, requests, realtime=True, clock=time.perf_counter):
    """Feed requests (sorted by arrival, seconds from start) to the server in
    real time and run until all are complete.  Returns the completed
    requests."""
    t0 = clock()
    now = lambda: clock() - t0
    i = 0
    reqs = sorted(requests, key=lambda r: r.arrival)
    while i < len(reqs) or server.busy():
        t = now()
        while i < len(reqs) and (reqs[i].arrival <= t or not realtime):
            server.submit(reqs[i])
            i += 1
        did = server.step(now)
        if not did:
            if server.inflight and (i >= len(reqs) or reqs[i].arrival > now()):
                # nothing to admit right now: wait briefly for the GPU
                server._retire(now, block=False)
            if i < len(reqs) and not server.busy():
                gap = reqs[i].arrival - now()
                if gap > 2e-4:
                    time.sleep(gap - 1e-4)
    return server.completed


def latency_stats(done):
    lat = np.array([r.done - r.arrival for r in done]) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "count": len(done)}
