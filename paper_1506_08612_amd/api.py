"""ctypes binding over libdfa.so (include/dfa.h).

Argument marshalling only: every step of the scan runs in the HIP library.
PyTorch provides device memory and streams.  Importing this module loads the
library and raises if it has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
# torch ships its own HIP runtime (loaded under a different file name than the
# system one libdfa names).  Importing torch first makes the library bind to
# that same runtime by its soname: two HIP runtimes in one process do not share
# the device, and the second to start reports that there is none.
import torch  # noqa: F401  (load order)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdfa.so")

DFA_OK = 0
DFA_EINVAL = -1
DFA_EHIP = -2
DFA_ENOSPACE = -3
MAX_M = 255
MERGED_GROUPS = 8  # DFA_MERGED_GROUPS
NOALLOC_SCRATCH_BYTES = 64 << 20  # DFA_NOALLOC_SCRATCH_BYTES
ALPHABET = 256


class DfaError(RuntimeError):
    def __init__(self, rc: int, msg: str):
        super().__init__(f"libdfa error {rc}: {msg}")
        self.rc = rc


class Tune(ctypes.Structure):
    """dfa_tune: launch shape; zero fields mean "library default"."""
    _fields_ = [
        ("chain_bytes", ctypes.c_int64),
        ("waves_per_group", ctypes.c_int32),
        ("chains_per_lane", ctypes.c_int32),
        ("dfas_per_group", ctypes.c_int32),
        ("automaton_bytes", ctypes.c_int32),
        ("line_bytes", ctypes.c_int32),
        ("step_bytes", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


class BatchPlan(ctypes.Structure):
    """dfa_batch_plan: filled by dfa_batch_prepare, read by dfa_batch_run."""
    _fields_ = [
        ("nitems", ctypes.c_int64),
        ("ngroups", ctypes.c_int64),
        ("npairs", ctypes.c_int64),
        ("text_bytes", ctypes.c_int64),
        ("tables_bytes", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("items_offset", ctypes.c_int64),
        ("dfas_per_group", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 4),
    ]


class MergedPlan(ctypes.Structure):
    """dfa_merged_plan: filled by dfa_merged_prepare, read by dfa_merged_run."""
    _fields_ = [
        ("nitems", ctypes.c_int64),
        ("nautomata", ctypes.c_int64),
        ("nstates", ctypes.c_int64),
        ("nfinal", ctypes.c_int64),
        ("npairs", ctypes.c_int64),
        ("ncounts", ctypes.c_int64),
        ("text_bytes", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("items_offset", ctypes.c_int64),
        ("outputs_offset", ctypes.c_int64),
        ("entries_offset", ctypes.c_int64),
        ("visits_offset", ctypes.c_int64),
        ("waves_per_group", ctypes.c_int32),
        ("lds_bytes", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 4),
        ("group_items", ctypes.c_int64 * MERGED_GROUPS),
        ("group_lds", ctypes.c_int32 * MERGED_GROUPS),
        ("group_pair", ctypes.c_int32 * MERGED_GROUPS),
    ]

    @property
    def pair_items(self) -> int:
        """Work items walked two bytes per step (pair automata)."""
        return sum(int(self.group_items[g]) for g in range(MERGED_GROUPS) if self.group_pair[g])


_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_vp = ctypes.c_void_p
_TuneP = ctypes.POINTER(Tune)
_PlanP = ctypes.POINTER(BatchPlan)
_MPlanP = ctypes.POINTER(MergedPlan)

# name -> (restype, argtypes); mirrors include/dfa.h
SIGNATURES = {
    "dfa_last_error": (ctypes.c_char_p, []),
    "dfa_version": (ctypes.c_char_p, []),
    "dfa_table_bytes": (_i64, [_i32]),
    "dfa_build": (ctypes.c_int, [_vp, _i32, _vp]),
    "dfa_count_workspace_bytes": (_i64, [_i64, _i32, _i32, _TuneP]),
    "dfa_count": (ctypes.c_int, [_vp, _i64, _vp, _i32, _vp, _vp, _i64, _vp, _i64, _TuneP, _vp]),
    "dfa_count_timed": (_i64, [_vp, _i64, _vp, _i32, _vp, _vp, _i64, _TuneP, _vp]),
    "dfa_count_noalloc": (ctypes.c_int, [_vp, _i64, _vp, _i32, _vp, _vp, _i64, _TuneP, _vp]),
    "dfa_lds_probe": (_i64, [_i32, _i32, _i32, _i64, _vp, _vp]),
    "dfa_set_scan_events": (ctypes.c_int, [_vp, _vp]),
    "dfa_batch_prepare": (ctypes.c_int, [_vp, _i32, _vp, _vp, _i32, _vp, _vp, _i64, _vp, _i64, _TuneP,
                                         _PlanP, _vp]),
    "dfa_batch_run": (ctypes.c_int, [_vp, _i64, _vp, _i64, _vp, _PlanP, _vp, _vp]),
    "dfa_count_batch": (ctypes.c_int, [_vp, _i64, _vp, _i32, _vp, _i64, _vp, _vp, _i32, _vp, _vp, _i64,
                                       _vp, _vp, _i64, _TuneP, _vp]),
    "dfa_ac_build": (_i64, [_vp, _vp, _vp, _i32, _vp, _i64, _vp, _vp, _vp, _i64, _vp]),
    "dfa_merged_prepare": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _i64, _vp, _i64, _vp, _i64,
                                          _TuneP, _MPlanP, _vp]),
    "dfa_degenerate_expand": (_i64, [_vp, _i32, _i32, _vp, _i64]),
    "dfa_fasta_workspace_bytes": (_i64, [_i64]),
    "dfa_fasta_normalize": (ctypes.c_int, [_vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp]),
    "dfa_merged_run": (ctypes.c_int, [_vp, _i64, _vp, _MPlanP, _vp, _vp]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1506_08612_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return lib.dfa_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise DfaError(rc, last_error())
    return rc


def tune(chain_bytes: int = 0, waves_per_group: int = 0, chains_per_lane: int = 0,
         dfas_per_group: int = 0, automaton_bytes: int = 0, line_bytes: int = 0, step_bytes: int = 0) -> Tune:
    return Tune(chain_bytes, waves_per_group, chains_per_lane, dfas_per_group, automaton_bytes,
                line_bytes, step_bytes)


def _tune_ptr(t: Optional[Tune]):
    return ctypes.byref(t) if t is not None else None


def table_bytes(m: int) -> int:
    return _check(lib.dfa_table_bytes(m))


def build_table(pattern: bytes) -> np.ndarray:
    """Host automaton build: (m+1, 256) uint8 transition table."""
    p = np.frombuffer(bytes(pattern), dtype=np.uint8)
    m = p.size
    if m < 1 or m > MAX_M:
        raise DfaError(DFA_EINVAL, f"pattern length {m} outside [1, {MAX_M}]")
    out = np.empty((m + 1, ALPHABET), dtype=np.uint8)
    _check(lib.dfa_build(p.ctypes.data, m, out.ctypes.data))
    return out


# ---------------------------------------------------------------------------
# device-side helpers (torch is only the allocator and stream provider)
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _ptr(t, dtype: str, name: str, min_numel: int = 0):
    """Device address of tensor `t` for the library, after checking what the
    library cannot: that it is a contiguous device tensor of `dtype` with at
    least `min_numel` elements (the library reads and writes whole ranges from
    the address it is given).  None for an empty tensor."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: expected a device tensor, got one on {t.device}")
    if t.dtype != getattr(torch, dtype):
        raise ValueError(f"{name}: expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if t.numel() < min_numel:
        raise ValueError(f"{name}: needs at least {min_numel} elements, has {t.numel()}")
    return t.data_ptr() if t.numel() else None


def _stream_handle(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def to_device(arr, device="cuda") -> "torch.Tensor":
    """Copy a host byte array into a new device tensor (the text stays resident)."""
    torch = _torch()
    a = np.ascontiguousarray(arr)
    t = torch.from_numpy(a.view(np.uint8).reshape(-1))
    return t.to(device, non_blocking=False)


def device_table(pattern: bytes, device="cuda"):
    """Build on the host, upload once: returns (table tensor, m)."""
    tab = build_table(pattern)
    return to_device(tab, device), tab.shape[0] - 1


def count_workspace_bytes(n: int, m: int, want_positions: bool, t: Optional[Tune] = None) -> int:
    return _check(lib.dfa_count_workspace_bytes(n, m, int(bool(want_positions)), _tune_ptr(t)))


def count_async(text, table, m: int, count_out, positions_out=None, cap: int = 0,
                workspace=None, t: Optional[Tune] = None, stream=None) -> None:
    """Enqueue dfa_count on the stream.  All tensors are device tensors:
    text uint8[n], table uint8[(m+1)*256], count_out int64[1], positions_out int64[cap]."""
    txt = _ptr(text, "uint8", "text")
    n = text.numel()
    tab = _ptr(table, "uint8", "table", (int(m) + 1) * ALPHABET if 1 <= m <= MAX_M else 0)
    cnt = _ptr(count_out, "int64", "count_out", 1)
    pos = _ptr(positions_out, "int64", "positions_out", int(cap)) if positions_out is not None else None
    wsp = _ptr(workspace, "uint8", "workspace") if workspace is not None else None
    wsb = workspace.numel() if workspace is not None else 0
    _check(lib.dfa_count(txt, n, tab, m, cnt, pos, int(cap), wsp, wsb, _tune_ptr(t), _stream_handle(stream)))


def count_noalloc_async(text, table, m: int, count_out, positions_out=None, cap: int = 0,
                        t: Optional[Tune] = None, stream=None) -> None:
    """Enqueue dfa_count_noalloc: dfa_count with the positions workspace taken from the
    library's own device scratch (no allocation by the library; calls that overlap on one
    GPU race)."""
    txt = _ptr(text, "uint8", "text")
    tab = _ptr(table, "uint8", "table", (int(m) + 1) * ALPHABET if 1 <= m <= MAX_M else 0)
    cnt = _ptr(count_out, "int64", "count_out", 1)
    pos = _ptr(positions_out, "int64", "positions_out", int(cap)) if positions_out is not None else None
    _check(lib.dfa_count_noalloc(txt, text.numel(), tab, m, cnt, pos, int(cap), _tune_ptr(t),
                                 _stream_handle(stream)))


def count(text, table, m: int, t: Optional[Tune] = None, stream=None) -> int:
    """Exact overlapping match count (synchronises the stream)."""
    torch = _torch()
    with torch.cuda.stream(stream):
        out = torch.empty(1, dtype=torch.int64, device=text.device)
        count_async(text, table, m, out, t=t, stream=stream)
        return int(out.item())


def positions(text, table, m: int, cap: Optional[int] = None, t: Optional[Tune] = None,
              stream=None):
    """(count, sorted int64 start offsets).  If cap is None the count is taken
    first and the output sized from it; otherwise at most cap positions."""
    torch = _torch()
    n = text.numel()
    dev = text.device
    with torch.cuda.stream(stream):
        out = torch.empty(1, dtype=torch.int64, device=dev)
        if cap is None:
            count_async(text, table, m, out, t=t, stream=stream)
            cap = int(out.item())
        pos = torch.empty(max(int(cap), 1), dtype=torch.int64, device=dev)
        wsb = count_workspace_bytes(n, m, True, t)
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
        count_async(text, table, m, out, pos, cap, ws, t=t, stream=stream)
        c = int(out.item())
        return c, pos[:min(c, int(cap))]


def count_timed(text, table, m: int, t: Optional[Tune] = None, stream=None, wg_cap: int = 1 << 22):
    """Count-only scan that also records every workgroup's start/end (wall clock) and
    cycles: returns (count, int64 array of shape (workgroups, 3)) (synchronises)."""
    torch = _torch()
    with torch.cuda.stream(stream):
        out = torch.empty(1, dtype=torch.int64, device=text.device)
        times = torch.zeros(3 * wg_cap, dtype=torch.int64, device=text.device)
        tab = _ptr(table, "uint8", "table", (int(m) + 1) * ALPHABET if 1 <= m <= MAX_M else 0)
        nb = _check(lib.dfa_count_timed(_ptr(text, "uint8", "text"), text.numel(), tab, m, out.data_ptr(),
                                        times.data_ptr(), wg_cap, _tune_ptr(t), _stream_handle(stream)))
        k = min(nb, wg_cap)
        return int(out.item()), times[:3 * k].view(k, 3).cpu().numpy()


LDS_PROBE_MODES = {"scattered": 0, "dependent": 1, "conflict_free": 2}


def lds_probe(width: int, mode: str, blocks: int, iters: int, sink, stream=None) -> int:
    """Enqueue the LDS read probe (mode: scattered, dependent or conflict_free); returns the
    number of reads it makes."""
    return _check(lib.dfa_lds_probe(int(width), LDS_PROBE_MODES[mode], int(blocks), int(iters),
                                    _ptr(sink, "int64", "sink", 1), _stream_handle(stream)))


class ScanEvents:
    """Context manager: while active, every dfa_count call from this thread records
    `begin` / `end` (torch.cuda.Event with timing) around its walk over the whole text,
    so that begin.elapsed_time(end) is that one kernel's duration."""

    def __init__(self, begin, end, stream=None):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream()
        for e in (begin, end):
            if not e.cuda_event:  # torch creates the handle on the first record
                e.record(s)
        self.handles = (begin.cuda_event, end.cuda_event)

    def __enter__(self):
        _check(lib.dfa_set_scan_events(*self.handles))
        return self

    def __exit__(self, *exc):
        _check(lib.dfa_set_scan_events(None, None))
        return False


# ---------------------------------------------------------------------------
# batched scans
# ---------------------------------------------------------------------------

class PatternSet:
    """Automata for a list of patterns: built on the host, uploaded once as one
    device buffer of back-to-back tables."""

    def __init__(self, patterns, device="cuda"):
        self.patterns = [bytes(p) for p in patterns]
        tabs = [build_table(p) for p in self.patterns]
        self.m = np.array([len(p) for p in self.patterns], dtype=np.int32)
        sizes = np.array([t.size for t in tabs], dtype=np.int64)
        self.table_off = np.zeros(len(tabs), dtype=np.int64)
        if len(tabs) > 1:
            self.table_off[1:] = np.cumsum(sizes)[:-1]
        blob = np.concatenate([t.reshape(-1) for t in tabs]) if tabs else np.zeros(256, np.uint8)
        self.tables = to_device(blob, device)

    def __len__(self):
        return len(self.patterns)


def _np(a, dt):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


class Batch:
    """A prepared batch: (segments, pattern set, pairs) planned once; run() is
    device-only and may be captured in a HIP graph and replayed."""

    def __init__(self, seg_off, pset: PatternSet, pair_seg, pair_pat, t: Optional[Tune] = None,
                 stream=None):
        torch = _torch()
        self.seg_off = _np(seg_off, np.int64)
        self.pair_seg = _np(pair_seg, np.int32)
        self.pair_pat = _np(pair_pat, np.int32)
        self.pset = pset
        self.plan = BatchPlan()
        self._prep(None, 0, t, stream)
        dev = pset.tables.device
        self.workspace = torch.empty(max(1, self.plan.workspace_bytes), dtype=torch.uint8, device=dev)
        self._prep(self.workspace.data_ptr(), self.workspace.numel(), t, stream)
        self.counts = torch.zeros(max(1, self.pair_seg.size), dtype=torch.int64, device=dev)

    def _prep(self, ws, wsb, t, stream):
        p = self.pset
        _check(lib.dfa_batch_prepare(self.seg_off.ctypes.data, self.seg_off.size - 1, p.table_off.ctypes.data,
                                     p.m.ctypes.data, len(p), self.pair_seg.ctypes.data,
                                     self.pair_pat.ctypes.data, self.pair_seg.size, ws, wsb, _tune_ptr(t),
                                     ctypes.byref(self.plan), _stream_handle(stream)))

    def run(self, text, stream=None):
        """Enqueue the scan; counts land in self.counts (device int64)."""
        _check(lib.dfa_batch_run(_ptr(text, "uint8", "text"), text.numel(),
                                 self.pset.tables.data_ptr(), self.pset.tables.numel(),
                                 self.workspace.data_ptr(),
                                 ctypes.byref(self.plan), self.counts.data_ptr(), _stream_handle(stream)))
        return self.counts[:self.pair_seg.size]


def count_batch(text, seg_off, pset: PatternSet, pair_seg, pair_pat, t: Optional[Tune] = None,
                stream=None) -> np.ndarray:
    """Per-pair occurrence counts (synchronises)."""
    with _torch().cuda.stream(stream):
        b = Batch(seg_off, pset, pair_seg, pair_pat, t, stream)
        return b.run(text, stream).cpu().numpy()


# ---------------------------------------------------------------------------
# merged multi-pattern automata
# ---------------------------------------------------------------------------

def _pack_patterns(patterns):
    pats = [bytes(p) for p in patterns]
    lens = np.array([len(p) for p in pats], dtype=np.int32)
    offs = np.zeros(len(pats), dtype=np.int64)
    if len(pats) > 1:
        offs[1:] = np.cumsum(lens[:-1])
    blob = np.frombuffer(b"".join(pats) or b"\0", dtype=np.uint8).copy()
    return pats, blob, offs, lens


class AcTable:
    """Host merged automaton from dfa_ac_build: table (nstates, 256) uint16, reporting
    states from first_final on, and per reporting state the indices of its patterns."""

    def __init__(self, table, first_final, out_off, out_pat):
        self.table = table
        self.first_final = int(first_final)
        self.out_off = out_off
        self.out_pat = out_pat

    @property
    def nstates(self) -> int:
        return self.table.shape[0]

    def outputs(self, q: int):
        f = q - self.first_final
        if f < 0:
            return []
        return self.out_pat[self.out_off[f]:self.out_off[f + 1]].tolist()


def ac_build(patterns) -> AcTable:
    """Host build of the merged automaton of `patterns` (1..255 bytes each)."""
    pats, blob, offs, lens = _pack_patterns(patterns)
    ff = ctypes.c_int32()
    nout = ctypes.c_int64()
    ns = _check(lib.dfa_ac_build(blob.ctypes.data, offs.ctypes.data, lens.ctypes.data, len(pats), None, 0,
                                 ctypes.byref(ff), None, None, 0, ctypes.byref(nout)))
    table = np.empty((ns, ALPHABET), dtype=np.uint16)
    out_off = np.empty(ns - ff.value + 1, dtype=np.int32)
    out_pat = np.empty(max(1, nout.value), dtype=np.int32)
    _check(lib.dfa_ac_build(blob.ctypes.data, offs.ctypes.data, lens.ctypes.data, len(pats), table.ctypes.data, ns,
                            ctypes.byref(ff), out_off.ctypes.data, out_pat.ctypes.data, out_pat.size,
                            ctypes.byref(nout)))
    return AcTable(table, ff.value, out_off, out_pat[:nout.value])


class MergedBatch:
    """Batched counting with merged automata: (segments, patterns, pairs) planned and
    uploaded once; run() is device-only and may be captured in a HIP graph.  With
    `pair_dst`, pair k's count goes to counter pair_dst[k] (counts of pairs sharing a
    counter add up) and there are `ncounts` counters."""

    def __init__(self, seg_off, patterns, pair_seg, pair_pat, t: Optional[Tune] = None, device="cuda",
                 stream=None, pair_dst=None, ncounts: int = 0):
        torch = _torch()
        self.seg_off = _np(seg_off, np.int64)
        self.pair_seg = _np(pair_seg, np.int32)
        self.pair_pat = _np(pair_pat, np.int32)
        self.pair_dst = None if pair_dst is None else _np(pair_dst, np.int32)
        self.ncounts = int(ncounts) if pair_dst is not None else self.pair_seg.size
        self.patterns, self._blob, self._offs, self._lens = _pack_patterns(patterns)
        self.plan = MergedPlan()
        self._prep(None, 0, t, stream)
        self.workspace = torch.empty(max(256, self.plan.workspace_bytes), dtype=torch.uint8, device=device)
        self._prep(self.workspace.data_ptr(), self.workspace.numel(), t, stream)
        self.counts = torch.zeros(max(1, self.ncounts), dtype=torch.int64, device=device)

    def _prep(self, ws, wsb, t, stream):
        dst = self.pair_dst.ctypes.data if self.pair_dst is not None else None
        _check(lib.dfa_merged_prepare(self.seg_off.ctypes.data, self.seg_off.size - 1, self._blob.ctypes.data,
                                      self._offs.ctypes.data, self._lens.ctypes.data, len(self.patterns),
                                      self.pair_seg.ctypes.data, self.pair_pat.ctypes.data, self.pair_seg.size,
                                      dst, self.ncounts if dst is not None else 0,
                                      ws, wsb, _tune_ptr(t), ctypes.byref(self.plan), _stream_handle(stream)))

    def run(self, text, stream=None):
        """Enqueue the scan; counts land in self.counts (device int64)."""
        _check(lib.dfa_merged_run(_ptr(text, "uint8", "text"), text.numel(),
                                  self.workspace.data_ptr(), ctypes.byref(self.plan), self.counts.data_ptr(),
                                  _stream_handle(stream)))
        return self.counts[:self.ncounts]


def count_merged(text, seg_off, patterns, pair_seg, pair_pat, t: Optional[Tune] = None,
                 stream=None) -> np.ndarray:
    """Per-pair occurrence counts with merged automata (synchronises)."""
    with _torch().cuda.stream(stream):
        b = MergedBatch(seg_off, patterns, pair_seg, pair_pat, t, device=text.device, stream=stream)
        return b.run(text, stream).cpu().numpy()


# ---------------------------------------------------------------------------
# degenerate patterns
# ---------------------------------------------------------------------------

def expand_degenerate(code: bytes, both_strands: bool = False):
    """The distinct plain k-mers an IUPAC pattern (and, with both_strands, its reverse
    complement) matches, sorted."""
    c = np.frombuffer(bytes(code), dtype=np.uint8).copy()
    k = _check(lib.dfa_degenerate_expand(c.ctypes.data, c.size, int(both_strands), None, 0))
    out = np.empty(max(1, k * c.size), dtype=np.uint8)
    _check(lib.dfa_degenerate_expand(c.ctypes.data, c.size, int(both_strands), out.ctypes.data, k))
    m = c.size
    return [out[i * m:(i + 1) * m].tobytes() for i in range(k)]


class DegenerateBatch:
    """Counts of degenerate patterns: query q asks for the start positions in segment
    seg[q] where code[q] (IUPAC) -- or, if both[q], its reverse complement -- matches.
    Every query becomes its expansions, each a pair of one merged scan whose count goes
    to the query's counter."""

    def __init__(self, seg_off, queries, t: Optional[Tune] = None, device="cuda", stream=None):
        pats, pseg, ppat, pdst = [], [], [], []
        index = {}
        for q, (seg, code, both) in enumerate(queries):
            for km in expand_degenerate(code, both):
                j = index.setdefault(km, len(pats))
                if j == len(pats):
                    pats.append(km)
                pseg.append(int(seg))
                ppat.append(j)
                pdst.append(q)
        self.nqueries = len(queries)
        self.batch = MergedBatch(seg_off, pats or [b"A"], pseg, ppat, t, device=device, stream=stream,
                                 pair_dst=pdst, ncounts=self.nqueries)
        self.counts = self.batch.counts

    def run(self, text, stream=None):
        return self.batch.run(text, stream)


def count_degenerate(text, seg_off, queries, t: Optional[Tune] = None, stream=None) -> np.ndarray:
    """Per-query counts of degenerate patterns (synchronises)."""
    with _torch().cuda.stream(stream):
        b = DegenerateBatch(seg_off, queries, t, device=text.device, stream=stream)
        return b.run(text, stream).cpu().numpy()


# ---------------------------------------------------------------------------
# FASTA input
# ---------------------------------------------------------------------------

def fasta_normalize(raw, rec_cap: int = 1 << 16, stream=None):
    """Normalise device FASTA text: returns (sequence, record starts) as device tensors
    (uint8 view of the kept bytes, int64 starts of the first min(records, rec_cap)
    records) and the exact (kept bytes, records) on the host (synchronises)."""
    torch = _torch()
    src = _ptr(raw, "uint8", "raw")
    n = raw.numel()
    dev = raw.device
    with torch.cuda.stream(stream):
        out = torch.empty(max(1, n), dtype=torch.uint8, device=dev)
        rec = torch.empty(max(1, rec_cap), dtype=torch.int64, device=dev)
        tot = torch.zeros(2, dtype=torch.int64, device=dev)
        wsb = _check(lib.dfa_fasta_workspace_bytes(n))
        ws = torch.empty(max(256, wsb), dtype=torch.uint8, device=dev)
        _check(lib.dfa_fasta_normalize(src, n, out.data_ptr(), rec.data_ptr(), rec_cap,
                                       tot.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream)))
        kept, nrec = (int(x) for x in tot.cpu().tolist())
        return out[:kept], rec[:min(nrec, rec_cap)], kept, nrec


def exported_symbols() -> Sequence[str]:
    return list(SIGNATURES)
