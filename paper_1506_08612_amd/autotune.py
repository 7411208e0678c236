"""Autotuner for the scan launch shapes, with a JSON cache per device.

The launch shape never changes a result, only its speed (the GPU tests check
every shape against the oracle).  For a workload class the tuner times a small
set of candidate shapes on the device with HIP events, keeps the fastest, and
caches the choice in a JSON file keyed by device name, library version and
workload class.  This plays the part of the paper's manual sweep over thread
counts and affinities (Table 4), done per device and per workload.

Cache location: $DFA_TUNE_CACHE, else ~/.cache/paper_1506_08612_amd/tune.json.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import threading
from typing import Dict, Iterable, List, Optional

from . import api

SCAN_CANDIDATES: List[Dict[str, int]] = [
    dict(),  # library default (64-byte rounds, workgroup size from occupancy)
    dict(waves_per_group=2),
    dict(waves_per_group=4),
    dict(waves_per_group=8),
    dict(chain_bytes=1024),
    dict(chain_bytes=2048),
    dict(line_bytes=128),
]

BATCH_CANDIDATES: List[Dict[str, int]] = [
    dict(),  # library default
    dict(dfas_per_group=2),
    dict(dfas_per_group=8),
    dict(dfas_per_group=4, chain_bytes=1024),
    dict(dfas_per_group=4, waves_per_group=4),
]

MERGED_CANDIDATES: List[Dict[str, int]] = [
    dict(),  # library default (64 KiB automata; the plan's round size and waves per workgroup)
    dict(automaton_bytes=48 * 1024),
    dict(automaton_bytes=80 * 1024),
    dict(automaton_bytes=24 * 1024, line_bytes=64),
    dict(automaton_bytes=64 * 1024, waves_per_group=8),
]

_lock = threading.Lock()


def cache_path() -> str:
    p = os.environ.get("DFA_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1506_08612_amd", "tune.json")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass  # a read-only home only costs re-tuning


_LIB_HASH = None


def _lib_hash() -> str:
    """Short hash of the built library: a rebuilt library (other kernels) tunes anew."""
    global _LIB_HASH
    if _LIB_HASH is None:
        h = hashlib.sha256()
        with open(api.LIB_PATH, "rb") as f:
            for block in iter(lambda: f.read(1 << 20), b""):
                h.update(block)
        _LIB_HASH = h.hexdigest()[:12]
    return _LIB_HASH


def device_key() -> str:
    import torch
    name = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    return f"{name}|{api.lib.dfa_version().decode()}|{_lib_hash()}"


def scan_class(n: int, m: int) -> str:
    """Workload class of a single-pattern scan: log2 of the text size, pattern-length band."""
    band = 0 if m <= 8 else 1 if m <= 24 else 2 if m <= 64 else 3
    return f"scan|n2^{max(0, int(math.log2(max(1, n))))}|mband{band}"


def batch_class(total_bytes: int, npat: int, mean_m: float, nseg: int) -> str:
    return (f"batch|n2^{max(0, int(math.log2(max(1, total_bytes))))}|p2^{int(math.log2(max(1, npat)))}"
            f"|m{int(mean_m // 8) * 8}|s2^{int(math.log2(max(1, nseg)))}")


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _pick(key: str, candidates: Iterable[Dict[str, int]], run_one, reps: int, force: bool):
    with _lock:
        cache = _load()
        dk = device_key()
        hit = cache.get(dk, {}).get(key)
    if hit is not None and not force:
        return api.tune(**hit["tune"]), hit
    results = []
    for c in candidates:
        try:
            ms = _time(lambda: run_one(api.tune(**c)), reps)
        except api.DfaError:
            continue
        results.append((ms, c))
    results.sort(key=lambda x: x[0])
    best_ms, best = results[0]
    entry = {"tune": best, "ms": best_ms, "tried": [{"tune": c, "ms": ms} for ms, c in results]}
    with _lock:
        cache = _load()
        cache.setdefault(dk, {})[key] = entry
        _store(cache)
    return api.tune(**best), entry


def tune_scan(text, table, m: int, reps: int = 3, force: bool = False,
              candidates: Optional[Iterable[Dict[str, int]]] = None):
    """Fastest launch shape for count-only scans of this text size and pattern length."""
    import torch
    out = torch.empty(1, dtype=torch.int64, device=text.device)
    key = scan_class(text.numel(), m)
    return _pick(key, candidates or SCAN_CANDIDATES,
                 lambda t: api.count_async(text, table, m, out, t=t), reps, force)


def tune_batch(text, seg_off, pset: "api.PatternSet", pair_seg, pair_pat, reps: int = 2,
               force: bool = False, candidates: Optional[Iterable[Dict[str, int]]] = None):
    """Fastest launch shape for a batched scan of this workload class."""
    import numpy as np
    so = np.asarray(seg_off, dtype=np.int64)
    key = batch_class(int(so[-1] - so[0]), len(pset), float(np.mean(pset.m)) if len(pset) else 0.0,
                      so.size - 1)
    batches = {}

    def run_one(t):
        k = (t.dfas_per_group, t.waves_per_group, t.chain_bytes)
        if k not in batches:
            batches[k] = api.Batch(so, pset, pair_seg, pair_pat, t)
        batches[k].run(text)

    return _pick(key, candidates or BATCH_CANDIDATES, run_one, reps, force)


def tune_merged(text, seg_off, patterns, pair_seg, pair_pat, reps: int = 2, force: bool = False,
                candidates: Optional[Iterable[Dict[str, int]]] = None):
    """Fastest automaton budget and launch shape for a merged batched scan of this
    workload class."""
    import numpy as np
    so = np.asarray(seg_off, dtype=np.int64)
    lens = [len(p) for p in patterns]
    key = "merged|" + batch_class(int(so[-1] - so[0]), len(patterns), float(np.mean(lens)) if lens else 0.0,
                                  so.size - 1)
    built = {}

    def run_one(t):
        k = (t.automaton_bytes, t.waves_per_group, t.chain_bytes, t.line_bytes)
        if k not in built:
            built[k] = api.MergedBatch(so, patterns, pair_seg, pair_pat, t, device=text.device)
        built[k].run(text)

    return _pick(key, candidates or MERGED_CANDIDATES, run_one, reps, force)
