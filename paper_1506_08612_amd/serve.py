"""Continuous-batching query server for (text, pattern set) requests.

A request is one text and 1..k patterns; its answer is the occurrence count
of every pattern in the text.  The server

* admits requests in arrival order as long as their text fits the free space
  of a device text arena (admission by HBM footprint); a request that does not
  fit waits until finished requests free their bytes;
* uploads admitted texts from pinned host memory in chunks over two copy
  streams, the request with the fewest bytes left first, while earlier
  batches run on the compute stream;
* fuses every admitted request whose upload has been issued into ONE batched
  scan launch: each request's text is a segment of the arena (gaps between
  texts are segments nobody asks about), each (request, pattern) is a pair,
  and the patterns of each request are merged into multi-pattern automata;
* keeps at most `max_inflight` fused launches on the device; requests that
  arrive while others run are admitted as slots and memory free up and join
  the next launch as soon as their text is on the device, so their work
  overlaps on the device;
* records, per request: arrival, admission, launch and completion times.

`mode="fifo"` is the one-query-per-launch baseline on the same trace: one
request at a time, upload, plan, launch, wait.

Everything device-side is the library's merged batched scan
(dfa_merged_prepare / dfa_merged_run); this module only schedules.
"""
from __future__ import annotations

import bisect
import dataclasses
import time
from typing import List, Optional

import numpy as np

from . import api

ALIGN = 256  # arena placement granularity (the scan wants 16-byte aligned segments)


class Arena:
    """First-fit allocator over [0, size) with coalescing frees (host bookkeeping only)."""

    def __init__(self, size: int):
        self.size = int(size)
        self.free = [(0, self.size)]  # sorted (offset, length)
        self.used = 0

    @staticmethod
    def _round(n: int) -> int:
        return max(ALIGN, (int(n) + ALIGN - 1) // ALIGN * ALIGN)

    def alloc(self, n: int) -> Optional[int]:
        need = self._round(n)
        for i, (off, ln) in enumerate(self.free):
            if ln >= need:
                if ln == need:
                    del self.free[i]
                else:
                    self.free[i] = (off + need, ln - need)
                self.used += need
                return off
        return None

    def release(self, off: int, n: int) -> None:
        need = self._round(n)
        self.used -= need
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, need))
        # coalesce with neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]


def segments_for(placed, arena_size: int):
    """Segment boundaries covering [0, end of the last text) for texts placed at
    (offset, length): every text is a segment; the gaps between texts are segments
    too (no pair refers to them).  Returns (seg_off, seg_of_text).

    An empty text is placed at offset 0 without taking arena space, so it may share
    its offset with a text that starts there; ordering by (offset, length) puts the
    empty one first and keeps the offsets non-decreasing."""
    order = sorted(range(len(placed)), key=lambda i: (placed[i][0], placed[i][1]))
    seg_off = [0]
    seg_of = [0] * len(placed)
    for i in order:
        off, ln = placed[i]
        if off > seg_off[-1]:
            seg_off.append(off)  # gap segment
        seg_of[i] = len(seg_off) - 1
        seg_off.append(off + ln)
    return np.array(seg_off, dtype=np.int64), seg_of


@dataclasses.dataclass
class Request:
    qid: int
    text: np.ndarray       # uint8 host text
    patterns: list         # list[bytes]
    arrival: float = 0.0   # seconds after the start of the run


@dataclasses.dataclass
class Result:
    qid: int
    counts: np.ndarray
    arrival: float
    admitted: float
    launched: float
    done: float
    text_bytes: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Job:
    __slots__ = ("req", "pinned", "offset", "admitted", "launched", "next_byte", "pending_events")


class Server:
    """Continuous-batching server over one device text arena.

    Streams (all at the default priority): `copy_streams` streams that carry text uploads in
    chunks, one stream for plan uploads (the prepare call synchronises it, so it must not
    carry anything else), and one compute stream for the scans.
    """

    def __init__(self, arena_bytes: int = 4 << 30, max_inflight: int = 2, tune: Optional[api.Tune] = None,
                 device: str = "cuda", chunk_bytes: int = 8 << 20, copy_streams: int = 2,
                 chunks_in_flight: int = 4):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.arena_bytes = int(arena_bytes)
        self.arena_buf = torch.empty(self.arena_bytes, dtype=torch.uint8, device=self.device)
        self.copy_streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, copy_streams))]
        self.plan_stream = torch.cuda.Stream(device=self.device)
        self.compute_stream = torch.cuda.Stream(device=self.device)
        self.max_inflight = max_inflight
        self.tune = tune
        self.chunk_bytes = int(chunk_bytes)
        self.chunks_in_flight = int(chunks_in_flight)
        # pinned host copies of the texts served so far, one per distinct array, kept so
        # that a trace served again (or a text carried by many requests) is pinned once;
        # release_pinned() gives the memory back
        self._pinned = {}

    def release_pinned(self) -> None:
        """Free the pinned host copies of every text served so far."""
        self._pinned.clear()

    # -- helpers --------------------------------------------------------------------------
    def _pin(self, text: np.ndarray):
        """Pinned host copy of a text, shared by every request that carries the same array."""
        key = id(text)
        hit = self._pinned.get(key)
        if hit is not None and hit[0] is text:
            return hit[1]
        t = self.torch.from_numpy(np.ascontiguousarray(text, dtype=np.uint8))
        t = t.pin_memory() if t.numel() else t
        self._pinned[key] = (text, t)
        return t

    def _launch(self, jobs: List[_Job]):
        """One fused merged-automaton scan over the jobs' texts (already in the arena);
        returns (event, counts tensor, spans, buffers to keep alive until the event fires)."""
        torch = self.torch
        placed = [(j.offset, j.req.text.size) for j in jobs]
        seg_off, seg_of = segments_for(placed, self.arena_bytes)
        pats, pair_seg, spans = [], [], []
        for ji, j in enumerate(jobs):
            first = len(pair_seg)
            for p in j.req.patterns:
                pats.append(p)
                pair_seg.append(seg_of[ji])
            spans.append((first, len(pair_seg)))
        _, blob, offs, lens = api._pack_patterns(pats)
        so = np.ascontiguousarray(seg_off)
        ps_a = np.array(pair_seg, np.int32)
        pp_a = np.arange(len(pats), dtype=np.int32)
        plan = api.MergedPlan()

        def prepare(ws, wsb, stream):
            api._check(api.lib.dfa_merged_prepare(so.ctypes.data, so.size - 1, blob.ctypes.data, offs.ctypes.data,
                                                  lens.ctypes.data, len(pats), ps_a.ctypes.data, pp_a.ctypes.data,
                                                  ps_a.size, None, 0, ws, wsb, api._tune_ptr(self.tune),
                                                  api.ctypes.byref(plan), stream))

        prepare(None, 0, None)
        ws = torch.empty(max(256, plan.workspace_bytes), dtype=torch.uint8, device=self.device)
        prepare(ws.data_ptr(), ws.numel(), self.plan_stream.cuda_stream)  # synchronises the plan stream
        counts = torch.empty(max(1, ps_a.size), dtype=torch.int64, device=self.device)
        # the allocations above were made on the current stream: order them before the scan
        self.compute_stream.wait_stream(torch.cuda.current_stream(self.device))
        api._check(api.lib.dfa_merged_run(self.arena_buf.data_ptr(), self.arena_bytes, ws.data_ptr(),
                                          api.ctypes.byref(plan), counts.data_ptr(), self.compute_stream.cuda_stream))
        ev = torch.cuda.Event()
        ev.record(self.compute_stream)
        return ev, counts, spans, (ws, counts)

    def _upload_chunk(self, j: _Job, stream_i: int):
        """Enqueue the job's next chunk of text on one of the copy streams."""
        torch = self.torch
        n = j.req.text.size
        a = j.next_byte
        b = min(n, a + self.chunk_bytes)
        st = self.copy_streams[stream_i % len(self.copy_streams)]
        with torch.cuda.stream(st):
            self.arena_buf[j.offset + a:j.offset + b].copy_(j.pinned[a:b], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        j.next_byte = b
        j.pending_events += 1
        return ev

    # -- the loop -------------------------------------------------------------------------
    def serve(self, trace: List[Request], mode: str = "continuous", time_scale: float = 1.0) -> List[Result]:
        """Replay `trace` (arrival times in seconds, scaled by time_scale) and return one
        Result per request, in qid order.

        continuous: requests are admitted in arrival order while their text fits the arena;
        admitted texts are uploaded in chunks, the request with the fewest bytes left first,
        so that a short request never waits behind a long upload; every request whose text
        has arrived joins the next fused launch (at most `max_inflight` launches on the
        device).  fifo: one request at a time -- upload, plan, launch, wait."""
        assert mode in ("continuous", "fifo")
        torch = self.torch
        reqs = sorted(trace, key=lambda r: r.arrival)
        for r in reqs:
            if r.text.size > self.arena_bytes:
                raise ValueError(f"request {r.qid}: text of {r.text.size} bytes exceeds the arena")
        pinned = {r.qid: self._pin(r.text) for r in reqs}
        torch.cuda.synchronize(self.device)
        arena = Arena(self.arena_bytes)
        pending: List[Request] = []
        uploading: List[_Job] = []   # admitted, text not fully on the device
        ready: List[_Job] = []       # text on the device, waiting for a launch slot
        chunk_events = []            # (event, job) in issue order
        inflight = []                # (event, counts, spans, jobs, keep)
        results = {}
        nxt = 0
        issued = 0
        t0 = time.perf_counter()
        clock = lambda: (time.perf_counter() - t0)  # noqa: E731
        fifo = mode == "fifo"
        while len(results) < len(reqs):
            now = clock()
            while nxt < len(reqs) and reqs[nxt].arrival * time_scale <= now:
                pending.append(reqs[nxt])
                nxt += 1
            progressed = False
            # finished launches: answers to the host, arena space back
            still = []
            for ev, counts, spans, jobs, keep in inflight:
                if ev.query():
                    c = counts.cpu().numpy()
                    tdone = clock()
                    for (a, b), j in zip(spans, jobs):
                        results[j.req.qid] = Result(j.req.qid, c[a:b].copy(), j.req.arrival * time_scale,
                                                    j.admitted, j.launched, tdone, int(j.req.text.size))
                        if j.req.text.size:
                            arena.release(j.offset, j.req.text.size)
                    progressed = True
                else:
                    still.append((ev, counts, spans, jobs, keep))
            inflight = still
            # finished chunks
            done_chunks = 0
            for ev, j in chunk_events:
                if not ev.query():
                    break
                j.pending_events -= 1
                done_chunks += 1
            if done_chunks:
                chunk_events = chunk_events[done_chunks:]
                progressed = True
            moved = [j for j in uploading if j.next_byte == j.req.text.size and j.pending_events == 0]
            if moved:
                uploading = [j for j in uploading if not (j.next_byte == j.req.text.size and j.pending_events == 0)]
                ready.extend(moved)
            # admission by footprint, in arrival order (fifo: one request in the system)
            busy = bool(uploading or ready or inflight)
            while pending and not (fifo and busy):
                r = pending[0]
                off = arena.alloc(r.text.size) if r.text.size else 0
                if off is None:
                    break
                pending.pop(0)
                j = _Job()
                j.req, j.pinned, j.offset = r, pinned[r.qid], off
                j.admitted = clock()
                j.launched = 0.0
                j.next_byte = 0
                j.pending_events = 0
                (ready if r.text.size == 0 else uploading).append(j)
                progressed = True
                busy = True
            # uploads: keep a few chunks in flight, fewest bytes left first
            while len(chunk_events) < self.chunks_in_flight:
                cand = [j for j in uploading if j.next_byte < j.req.text.size]
                if not cand:
                    break
                j = min(cand, key=lambda x: x.req.text.size - x.next_byte)
                chunk_events.append((self._upload_chunk(j, issued), j))
                issued += 1
                progressed = True
            # launch every request whose text is on the device when a slot is free
            if ready and len(inflight) < (1 if fifo else self.max_inflight):
                tl = clock()
                for j in ready:
                    j.launched = tl
                ev, counts, spans, keep = self._launch(ready)
                inflight.append((ev, counts, spans, ready, keep))
                ready = []
                progressed = True
            if not progressed:
                if inflight or chunk_events:
                    time.sleep(20e-6)
                elif nxt < len(reqs):
                    wait = reqs[nxt].arrival * time_scale - clock()
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
        torch.cuda.synchronize(self.device)
        return [results[r.qid] for r in sorted(trace, key=lambda r: r.qid)]


def summarize(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    t_first = min(r.arrival for r in results)
    t_last = max(r.done for r in results)
    total = sum(r.text_bytes for r in results)
    return {
        "queries": len(results),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "mean_ms": round(float(lat.mean()), 3),
        "text_GBps": round(total / max(1e-9, t_last - t_first) / 1e9, 3),
        "makespan_s": round(t_last - t_first, 4),
    }


def make_trace(nq: int, rate_hz: float, seed: int = 5, len_lo: float = 1e4, len_hi: float = 5e8,
               pmax: int = 64, mlo: int = 4, mhi: int = 64, n_frac: float = 0.02,
               pool: Optional[int] = None) -> List[Request]:
    """Poisson arrivals of queries: text length log-uniform in [len_lo, len_hi] (ACGT with 'N' runs),
    1..pmax patterns with lengths uniform in [mlo, mhi], half drawn from the text.

    With `pool`, only the first `pool` queries' texts are materialised and every later query
    carries one of them (chosen by a seeded draw) with its own patterns; this keeps host memory
    bounded for long traces (the server still uploads every query's text)."""
    from . import synth
    out = []
    qs = synth.query_trace(nq, rate_hz, seed, len_lo, len_hi, pmax, mlo, mhi)
    rng = np.random.default_rng([seed, 0x504F])
    texts = []
    for i, q in enumerate(qs):
        if pool is None or i < pool:
            text, pats = synth.query_text(q, n_frac=n_frac)
            texts.append(text)
        else:
            text = texts[int(rng.integers(0, len(texts)))]
            pats = synth.query_patterns(text, q)
        out.append(Request(len(out), text, pats, q.arrival_s))
    return out
