#!/usr/bin/env python3
"""Benchmark of the single-pattern automaton scan at genome scale.

Workload (one "step"): a 3.2 GB genome-like ASCII text (GC 41 %, 'N' runs of
geometric mean length 50 kb covering 5 %), resident in HBM before timing; five
patterns of length 4, 8, 16, 32 and 64 drawn from the text; the five automata
built on the host and their tables uploaded, then dfa_count with sorted positions
(count + every match start) for each pattern, the five calls issued in turn on
three streams (each call's small placement launches overlap the next calls'
walks).  `value` is text bytes scanned per second over the timed steps (5 x 3.2e9
bytes per step).

Also reported:
* roofline -- the step's dominant kernel, its walk over the whole text (the
  per-walk counting pass of count + positions), bracketed by HIP events on the
  launch stream (dfa_set_scan_events) in every call of a second run of the
  same steps right after the timed one, with the calls one after another on
  one stream (an event between two launches leaves the stream idle for ~10-15
  us, so the timed steps bracket no call or walk); algorithmic
  bytes = the text read once; the count-only scan is timed beside it;
* read_reduce_GBps -- a trivial read-reduce over the same device buffer (torch's
  sum of its 8-byte words), the streaming-read rate reached in the same run, and
  both scans' fractions of it;
* cpu_baseline -- the CPU oracle's plain automaton scan (C, one thread) over the
  whole text for the same five patterns, count + positions, every output checked
  against the GPU's; beside it the definition (window compare) on a prefix; the
  batched and segmented legs carry their own, job-parallel over the host's cores;
* lds -- the LDS read rate of this GPU (dfa_lds_probe), the measured ceiling the
  batched leg's LDS bound is taken against;
* study -- the count-only scan over genome sizes 0.2..3.2 GB and the spread of
  its workgroup durations (dfa_count_timed);
* per-pattern latency p50/p99 of the full call (events around each call, in the
  second run of the steps);
* batched -- 1 GB GC-41% text x 1024 patterns (lengths 4..64, half drawn from
  the text) with merged multi-pattern automata in one launch (autotuned
  automaton budget and shape, replayed from a HIP graph) against the same GPU
  running one count-only launch per pattern, in pattern-bytes/s; the batched
  scan with one automaton per pattern is timed beside it;
* fasta -- the genome written as FASTA (24 records, 60 bases per line, 10 %
  soft-masked) normalised on the device into plain sequence and record starts,
  beside torch's streaming read plus device copy of the same bytes (the two
  passes' floor);
* segmented -- 2000 contig-like segments (log-normal lengths, median 200 kB,
  ~2 GB, 2% 'N' runs), 1..16 patterns each, one merged launch;
* serving -- 1000 Poisson arrivals (after 50 warm-up queries) of (text,
  patterns) queries (text log-uniform in [10 kB, 500 MB] drawn from a pool of
  64 texts, 1..64 patterns of length 4..64) at 80% of the capacity the server
  sustains in a closed loop; p50/p99 latency (arrival to counts on the host,
  upload included) and text GB/s, against the one-query-per-launch FIFO form on
  the same trace.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "text GB/s (and % of HBM peak) single-pattern; pattern-bytes/s batched; p50/p99"
# compute-unit clocks per second: 256 CUs at 2.4 GHz
CU_CLOCKS_PER_S = 256 * 2.4e9
HBM_PEAK_GBS = 8000.0
PATTERN_LENGTHS = (4, 8, 16, 32, 64)
SCAN_SOURCES = [os.path.join(ROOT, "paper_1506_08612_amd", "csrc", f) for f in ("dfa_scan.hip", "walk_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "scan_textwalk_genome3200MB_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_text(src: str) -> str:
    """C/C++ source without its comments and with whitespace collapsed (string and
    character literals kept): two sources with the same code_text compile alike."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash(paths) -> str:
    """Hash of the kernel sources' code (comments and layout do not count)."""
    h = hashlib.sha256()
    for p in paths:
        h.update(code_text(open(p, encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per scan launch from the committed counter summary, or None when the
    kernel source changed since the counters were taken."""
    try:
        kv = {}
        for ln in open(TRAFFIC_FILE):
            if ":" in ln and not ln.startswith("#"):
                k, v = ln.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256_16") != source_hash(SCAN_SOURCES):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _events_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def oracle_mod():
    import oracle
    return oracle


def cpu_automaton_baseline(text, pats, counts, pos_bufs):
    """The oracle's plain automaton scan (its C function) over the whole text for every
    pattern, one thread per pattern, the patterns side by side: count and positions in one
    pass into a buffer sized from the GPU's count.  Returns the baseline and whether every
    count and position equals the GPU's."""
    import ctypes
    from concurrent.futures import ThreadPoolExecutor
    o = oracle_mod()
    lib = o.OracleLib(o.build(force=False)).lib
    u8p, i64p = ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int64)
    n = text.size
    tabs = [np.ascontiguousarray(o.transition_table(p)) for p in pats]
    outs = [np.empty(max(1, c), np.int64) for c in counts]

    def scan(i):
        t0 = time.perf_counter()
        c = lib.oracle_automaton_scan(tabs[i].ctypes.data_as(u8p), len(pats[i]), text.ctypes.data_as(u8p), n,
                                      outs[i].ctypes.data_as(i64p), outs[i].size)
        return c, time.perf_counter() - t0

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=len(pats)) as ex:
        res = list(ex.map(scan, range(len(pats))))
    wall = time.perf_counter() - t0
    ok = True
    for i, (c, _) in enumerate(res):
        g = pos_bufs[i][:counts[i]].cpu().numpy()
        ok &= bool(c == counts[i] and np.array_equal(outs[i][:c], g))
    per_core = [n / s / 1e9 for _, s in res]
    log(f"  cpu automaton scans: {wall:.1f} s, per core {[round(x, 3) for x in per_core]} GB/s")
    return ({"value": round(n * len(pats) / wall / 1e9, 4), "unit": "GB/s", "cores": len(pats), "kind": "oracle",
             "per_core_GBps": round(float(np.mean(per_core)), 4),
             "sample": f"the whole {n}-byte text for each of the same {len(pats)} patterns, one thread per "
                       f"pattern side by side: the oracle's automaton scan (table build excluded), count + "
                       f"positions in one pass, {wall:.1f} s on {cpu_model()}"}, ok)


def cpu_pairs_baseline(text, seg_off, patterns, pair_seg, pair_pat, budget):
    """The oracle's per-(segment, pattern) count, job-parallel over the host's cores (one
    single-thread scan per job, on threads: the C call releases the interpreter lock), on the
    segments that start within the first `budget` bytes.  Returns pattern-bytes/s and what
    was scanned."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    seg_off = np.asarray(seg_off, np.int64)
    pair_seg, pair_pat = np.asarray(pair_seg, np.int64), np.asarray(pair_pat, np.int64)
    if seg_off.size == 2:  # one text: its prefix
        end = int(min(budget, seg_off[1]))
        so, keep = np.array([0, end], np.int64), np.ones(pair_seg.size, bool)
    else:
        nseg = max(1, int(np.searchsorted(seg_off, budget, side="right")) - 1)
        so, keep = seg_off[:nseg + 1], pair_seg < nseg
    sample = np.ascontiguousarray(text[:int(so[-1])])
    ps, pp = pair_seg[keep], pair_pat[keep]
    cores = len(os.sched_getaffinity(0))
    jobs = np.array_split(np.arange(ps.size), cores)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(lambda idx: oracle.pair_counts(sample, so, patterns, ps[idx], pp[idx]), jobs))
    wall = time.perf_counter() - t0
    pb = int(np.diff(so)[ps].sum())
    return {"value": round(pb / wall, 1), "unit": "pattern-bytes/s", "cores": cores, "kind": "oracle",
            "sample": f"{so.size - 1} segment(s), {int(so[-1])} B, {ps.size} (segment, pattern) pairs, "
                      f"job-parallel over {cores} threads, {wall:.1f} s on {cpu_model()}"}


def bench_batched(torch, api, synth, n=1_000_000_000, npat=1024, lds_peak=None):
    from paper_1506_08612_amd import autotune, graph
    log(f"batched: {n} bytes x {npat} patterns")
    if lds_peak is None:
        lds_peak = bench_lds(torch, api)["u16_conflict_free"]["reads_per_s"]
    w = synth.many_patterns(n=n, npat=npat)
    d = api.to_device(w.text)
    ps = api.PatternSet(w.patterns)
    out = torch.empty(npat, dtype=torch.int64, device=d.device)
    tabs = [ps.tables[int(o):int(o) + (int(mm) + 1) * 256] for o, mm in zip(ps.table_off, ps.m)]
    pair_seg, pair_pat = np.zeros(npat, np.int64), np.arange(npat)

    def one_per_launch():
        for j in range(npat):
            api.count_async(d, tabs[j], int(ps.m[j]), out[j:j + 1])

    base_ms = _events_ms(torch, one_per_launch, 1)
    ref = out.cpu().numpy()
    # merged multi-pattern automata: autotuned, captured in a HIP graph
    t, entry = autotune.tune_merged(d, [0, n], w.patterns, pair_seg, pair_pat, reps=2)
    b = api.MergedBatch([0, n], w.patterns, pair_seg, pair_pat, t, device=d.device)
    g = graph.GraphedBatch(d, b)
    ms = _events_ms(torch, g.replay, 5)
    equal = bool(np.array_equal(b.counts.cpu().numpy()[:npat], ref))
    # one automaton per pattern (256-column tables), groups of automata per workgroup
    sb = api.Batch([0, n], ps, pair_seg, pair_pat)
    sep_ms = _events_ms(torch, lambda: sb.run(d), 1)
    sep_equal = bool(np.array_equal(sb.counts.cpu().numpy()[:npat], ref))
    deg = bench_degenerate(torch, api, d, n)
    cpu = cpu_pairs_baseline(w.text, [0, n], w.patterns, pair_seg, pair_pat, 24_000_000)
    pb = n * npat
    return deg, {"workload": f"gc41 text {n} B x {npat} patterns m=U[4,64] (half drawn), per-pattern counts",
            "pattern_bytes_per_s": round(pb / (ms * 1e-3), 1),
            "one_per_launch_pattern_bytes_per_s": round(pb / (base_ms * 1e-3), 1),
            "speedup_vs_one_per_launch": round(base_ms / ms, 2),
            "ms": round(ms, 3), "one_per_launch_ms": round(base_ms, 3),
            "method": "merged multi-pattern automata (class-compressed 16-bit tables), HIP graph replay",
            "tune": entry["tune"], "automata": int(b.plan.nautomata), "states": int(b.plan.nstates),
            # every automaton walks the whole text: two 2-byte LDS reads per step (byte class,
            # then the transition), against the conflict-free 2-byte read rate measured on
            # this GPU (the LDS's peak for such reads)
            "lds_bound": {"steps_per_s": round(n * int(b.plan.nautomata) / (ms * 1e-3), 1),
                          "lookups_per_s": round(2 * n * int(b.plan.nautomata) / (ms * 1e-3), 1),
                          "peak_lookups_per_s": lds_peak,
                          "peak_source": "dfa_lds_probe: conflict-free 2-byte reads, this run",
                          "frac": round(2 * n * int(b.plan.nautomata) / (ms * 1e-3) / lds_peak, 4)},
            "items": int(b.plan.nitems), "counts_equal_one_per_launch": equal,
            "separate_automata": {"ms": round(sep_ms, 3), "pattern_bytes_per_s": round(pb / (sep_ms * 1e-3), 1),
                                  "speedup_vs_one_per_launch": round(base_ms / sep_ms, 2),
                                  "counts_equal_one_per_launch": sep_equal},
            "cpu_baseline": cpu}


def bench_degenerate(torch, api, d, n):
    """18 degenerate queries shaped like the paper's pattern table: 9 random 8-mers with one
    position taking one of three bases (IUPAC B/D/H/V), each counted on both strands, and 9
    plain random 8-mers on both strands."""
    from paper_1506_08612_amd import graph, synth
    rng = np.random.default_rng([6, 0x4447])
    codes = []
    for i in range(9):
        s = list(synth.random_pattern(8, rng).decode())
        s[i % 8] = "BDHV"[int(rng.integers(0, 4))]
        codes.append("".join(s).encode())
    codes += [synth.random_pattern(8, rng) for _ in range(9)]
    queries = [(0, c, True) for c in codes]
    b = api.DegenerateBatch([0, n], queries, device=d.device)
    g = graph.GraphedBatch(d, b)
    ms = _events_ms(torch, g.replay, 5)
    nk = int(b.batch.plan.npairs)
    # the oracle's per-position check of the code sets, one thread per query, on a prefix
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    sn = min(n, 40_000_000)
    sample = d[:sn].cpu().numpy()
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(lambda q: oracle.degenerate_count(sample, q[1], q[2]), queries))
    cpu_s = time.perf_counter() - t0
    return {"workload": f"{len(queries)} degenerate 8-mer queries (9 with a 3-way position), both strands, "
                        f"over the same {n} B text; {nk} plain k-mers after expansion",
            "ms": round(ms, 3), "text_GBps": round(n / ms / 1e6, 1),
            "hbm_frac": round(n / ms / 1e6 / HBM_PEAK_GBS, 4),
            "query_bytes_per_s": round(n * len(queries) / (ms * 1e-3), 1),
            "pair_items": int(b.batch.plan.pair_items),
            "counts": [int(x) for x in b.counts.cpu().numpy()[:len(queries)]],
            "cpu_baseline": {"value": round(sn * len(queries) / cpu_s, 1), "unit": "query-bytes/s", "cores": cores,
                             "kind": "oracle",
                             "sample": f"first {sn} bytes, the {len(queries)} queries job-parallel over {cores} "
                                       f"threads, {cpu_s:.1f} s on {cpu_model()}"}}


def bench_merged_kernels(torch, api, synth, reps=3, step_bytes=0, line_bytes=0, automaton_bytes=0, chain_bytes=0,
                         waves=0):
    """The merged scans alone, for kernel traces and shader counters: the 1 GB x 1024-pattern
    plan, the 18 degenerate queries over the same text and the 2000-segment plan, each run
    `reps` times after one warm-up run, with the library's default plan (step_bytes: 1 or 2
    forces one- or two-byte automaton steps; line_bytes: bytes per round; automaton_bytes: the LDS
    budget of one merged automaton; chain_bytes: bytes per walk; waves: waves per workgroup; 0:
    the library's choice)."""
    t = (api.tune(step_bytes=step_bytes, line_bytes=line_bytes, automaton_bytes=automaton_bytes,
                  chain_bytes=chain_bytes, waves_per_group=waves)
         if step_bytes or line_bytes or automaton_bytes or chain_bytes or waves else None)
    from paper_1506_08612_amd import graph
    out = {}
    w = synth.many_patterns()
    n = w.text.size
    d = api.to_device(w.text)
    npat = len(w.patterns)
    jobs = [("many_patterns", api.MergedBatch([0, n], w.patterns, np.zeros(npat, np.int64), np.arange(npat), t,
                                              device=d.device), d)]
    rng = np.random.default_rng([6, 0x4447])  # the degenerate leg's queries
    codes = []
    for i in range(9):
        c = list(synth.random_pattern(8, rng).decode())
        c[i % 8] = "BDHV"[int(rng.integers(0, 4))]
        codes.append("".join(c).encode())
    codes += [synth.random_pattern(8, rng) for _ in range(9)]
    jobs.append(("degenerate", api.DegenerateBatch([0, n], [(0, c, True) for c in codes], t, device=d.device), d))
    ws = synth.uneven_segments()
    dseg = api.to_device(ws.text)
    jobs.append(("segmented", api.MergedBatch(ws.seg_off, ws.patterns, ws.pair_seg, ws.pair_pat, t,
                                              device=dseg.device), dseg))
    for name, b, text in jobs:
        g = graph.GraphedBatch(text, b)
        ms = _events_ms(torch, g.replay, reps)
        plan = b.batch.plan if hasattr(b, "batch") else b.plan
        out[name] = {"ms": round(ms, 4), "text_GBps": round(int(text.numel()) / ms / 1e6, 1),
                     "automata": int(plan.nautomata), "states": int(plan.nstates), "items": int(plan.nitems),
                     "pair_items": int(plan.pair_items), "groups": [int(x) for x in plan.group_items],
                     "line_bytes": int(plan.reserved[1]), "waves": int(plan.waves_per_group)}
        log(name, out[name])
    return out


def bench_lds(torch, api, blocks=1024, iters=8192):
    """LDS read rate of this GPU (dfa_lds_probe): 1- and 2-byte reads at conflict-free
    addresses (the LDS's peak for such reads), at scattered addresses (lanes meeting in a
    bank, as table lookups of different states do) and in chains where each address is
    computed from the previous value (an automaton step), eight per lane.
    1024 workgroups of 512 threads with 16 KiB of LDS each: 4 per CU, 32 waves per CU."""
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = {"cu_clocks_per_s": CU_CLOCKS_PER_S, "blocks": blocks, "iters": iters}
    for width in (1, 2):
        for mode in ("conflict_free", "scattered", "dependent"):
            reads = api.lds_probe(width, mode, blocks, iters, sink)
            ms = _events_ms(torch, lambda: api.lds_probe(width, mode, blocks, iters, sink), 5)
            rate = reads / (ms * 1e-3)
            out[f"u{8 * width}_{mode}"] = {
                "ms": round(ms, 4), "reads_per_s": round(rate, 1),
                "reads_per_clk_per_cu": round(rate / CU_CLOCKS_PER_S, 2)}
    return out


def bench_study(torch, api, text, dtext, pats):
    """Scalability and load balance of the count-only scan (analogues of the paper's
    Figs. 5 and 7): throughput over genome sizes 0.2..3.2 GB (prefixes of the text), and
    the spread of workgroup durations, the per-XCD busy time and the launch's tail at
    3.2 GB for a sparse (m = 8) and a dense (m = 4) pattern."""
    out = {"sizes": []}
    res = torch.empty(1, dtype=torch.int64, device=dtext.device)
    n = text.size
    for gb in (0.2, 0.4, 0.8, 1.6, 3.2):
        k = min(n, int(gb * 1e9)) // 16 * 16
        row = {"bytes": k}
        for p in pats:
            if len(p) not in (4, 8):
                continue
            tab, m = api.device_table(p)
            sub = dtext[:k]
            ms = _events_ms(torch, lambda: api.count_async(sub, tab, m, res), 10)
            row[f"m{m}_GBps"] = round(k / ms / 1e6, 1)
        out["sizes"].append(row)
    for p in pats:
        if len(p) not in (4, 8):
            continue
        tab, m = api.device_table(p)
        api.count_timed(dtext, tab, m)  # warm
        c, t = api.count_timed(dtext, tab, m)
        start, end, cyc = t[:, 0], t[:, 1], t[:, 2].astype(np.float64)
        dur = (end - start).astype(np.float64)
        span = float(end.max() - start.min())
        q = np.percentile(cyc, [5, 50, 95, 99])
        xcd = np.array([cyc[i::8].sum() for i in range(8)])
        out[f"m{m}_workgroups"] = {
            "count": int(c), "workgroups": int(t.shape[0]),
            "cycles_p5_p50_p95_p99": [int(x) for x in q], "cycles_max_over_median": round(float(cyc.max() / q[1]), 3),
            "xcd_busy_max_over_mean": round(float(xcd.max() / xcd.mean()), 4),
            "tail_after_p95_end_frac": round(float((end.max() - np.percentile(end, 95)) / span), 4),
            "mean_resident_workgroups": round(float(dur.sum() / span), 1),
        }
    return out


def fasta_bytes(text: np.ndarray, nrec: int = 24, width: int = 60, seed: int = 8) -> np.ndarray:
    """`text` written as FASTA: nrec records of near-equal length, `width` bases per line,
    a header line per record, and 10 % of the bases soft-masked (lower case) in runs."""
    rng = np.random.default_rng(seed)
    n = text.size
    cuts = np.linspace(0, n, nrec + 1).astype(np.int64)
    parts = []
    for k in range(nrec):
        seq = text[cuts[k]:cuts[k + 1]].copy()
        nmask = int(0.1 * seq.size / 5000)
        for a in rng.integers(0, max(1, seq.size - 5000), size=nmask):
            seg = seq[a:a + 5000]
            np.add(seg, 32, out=seg, where=(seg >= 65) & (seg <= 90))  # upper -> lower case
        parts.append(np.frombuffer(f">chr{k + 1} synthetic record {k + 1} of {nrec}\n".encode(), np.uint8))
        full = seq.size // width
        rows = np.empty((full, width + 1), np.uint8)
        rows[:, :width] = seq[:full * width].reshape(full, width)
        rows[:, width] = 10
        parts.append(rows.reshape(-1))
        if seq.size > full * width:
            parts.append(np.concatenate((seq[full * width:], np.array([10], np.uint8))))
    return np.concatenate(parts)


def bench_fasta(torch, api, text, dtext, reps=5):
    log("fasta: normalising the genome written as FASTA")
    raw = fasta_bytes(text)
    draw = api.to_device(raw)
    n = raw.size
    out = torch.empty(n, dtype=torch.uint8, device=draw.device)
    rec = torch.empty(64, dtype=torch.int64, device=draw.device)
    tot = torch.zeros(2, dtype=torch.int64, device=draw.device)
    ws = torch.empty(max(256, api.lib.dfa_fasta_workspace_bytes(n)), dtype=torch.uint8, device=draw.device)

    def run():
        api._check(api.lib.dfa_fasta_normalize(draw.data_ptr(), n, out.data_ptr(), rec.data_ptr(), 64,
                                               tot.data_ptr(), ws.data_ptr(), ws.numel(),
                                               api._stream_handle(None)))

    ms = _events_ms(torch, run, reps)
    kept, nrec = (int(x) for x in tot.cpu().tolist())
    same = kept == text.size and bool(torch.equal(out[:kept], dtext))
    # the passes' floor on this device: one streaming read of the FASTA text (the summary
    # pass) plus one device copy of it (the write pass reads it again and writes the kept
    # bytes), each timed with torch on the same buffers
    words = draw[:n // 8 * 8].view(torch.int64)
    read_ms = _events_ms(torch, lambda: words.sum(), reps)
    copy_ms = _events_ms(torch, lambda: out.copy_(draw), reps)
    del draw, out, ws, words
    # the oracle's line-by-line normaliser (plain Python), one thread, on a prefix
    import oracle
    sn = 16_000_000
    t0 = time.perf_counter()
    oracle.fasta.normalize(raw[:sn].tobytes())
    cpu_s = time.perf_counter() - t0
    # HBM bytes of the three passes: the text read twice, the kept bytes written once
    return {"workload": f"the {text.size} B genome as FASTA: {nrec} records, 60 bases per line, "
                        f"10% soft-masked; {n} B of FASTA text",
            "ms": round(ms, 3), "GBps": round(n / ms / 1e6, 1), "records": nrec,
            "hbm_frac": round((2 * n + kept) / ms / 1e6 / HBM_PEAK_GBS, 4),
            "read_plus_copy_ms": round(read_ms + copy_ms, 3),
            "frac_of_read_plus_copy": round((read_ms + copy_ms) / ms, 4),
            "normalised_equals_source": same,
            "cpu_baseline": {"value": round(sn / cpu_s / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                             "sample": f"first {sn} bytes of the FASTA text, {cpu_s:.1f} s on {cpu_model()}"}}


def bench_segmented(torch, api, synth):
    from paper_1506_08612_amd import graph
    log("segmented: 2000 contig-like segments")
    w = synth.uneven_segments()
    d = api.to_device(w.text)
    b = api.MergedBatch(w.seg_off, w.patterns, w.pair_seg, w.pair_pat, device=d.device)
    g = graph.GraphedBatch(d, b)
    ms = _events_ms(torch, g.replay, 5)
    sb = api.Batch(w.seg_off, api.PatternSet(w.patterns), w.pair_seg, w.pair_pat)
    sep_ms = _events_ms(torch, lambda: sb.run(d), 3)
    equal = bool(np.array_equal(b.counts.cpu().numpy(), sb.counts.cpu().numpy()))
    seg_len = np.diff(w.seg_off)
    pb = int(seg_len[w.pair_seg].sum())
    cpu = cpu_pairs_baseline(w.text, w.seg_off, w.patterns, w.pair_seg, w.pair_pat, 600_000_000)
    return {"workload": f"{seg_len.size} segments, {int(w.seg_off[-1])} B, {w.pair_seg.size} (segment, pattern) pairs",
            "ms": round(ms, 3), "text_GBps": round(int(w.seg_off[-1]) / ms / 1e6, 1),
            "hbm_frac": round(int(w.seg_off[-1]) / ms / 1e6 / HBM_PEAK_GBS, 4),
            "pattern_bytes_per_s": round(pb / (ms * 1e-3), 1), "items": int(b.plan.nitems),
            "pair_items": int(b.plan.pair_items),
            "method": "merged automata per segment (one byte per step, class bytes from registers), HIP graph replay",
            "separate_automata_ms": round(sep_ms, 3), "counts_equal_separate_automata": equal,
            "cpu_baseline": cpu}


def bench_serving(torch, nq, warm=50, pool=64):
    from paper_1506_08612_amd import serve
    log(f"serving: {warm} warm-up + {nq} measured queries (texts from a pool of {pool})")
    trace = serve.make_trace(warm + nq, rate_hz=1.0, seed=5, pool=pool)
    srv = serve.Server(arena_bytes=8 << 30)
    srv.serve([serve.Request(r.qid, r.text, r.patterns, 0.0) for r in trace[:warm]], mode="continuous")
    meas = trace[warm:]
    closed = [serve.Request(r.qid, r.text, r.patterns, 0.0) for r in meas]
    cap = srv.serve(closed, mode="continuous")
    capacity = nq / max(r.done for r in cap)
    rate = 0.8 * capacity
    # the seeded Poisson trace has rate 1/s: dividing its arrival times by `rate` rescales it
    t_first = meas[0].arrival
    timed = [serve.Request(r.qid, r.text, r.patterns, (r.arrival - t_first) / rate) for r in meas]
    res = srv.serve(timed, mode="continuous")
    cont = serve.summarize(res)
    fifo_res = srv.serve(timed, mode="fifo")
    fifo = serve.summarize(fifo_res)
    srv.release_pinned()
    same = all(np.array_equal(x.counts, y.counts) for x, y in zip(res, fifo_res))
    total = sum(r.text.size for r in meas)
    return {"workload": f"{nq} queries after {warm} warm-up, text log-uniform [1e4, 5e8] B (2% N runs; "
                        f"{pool} distinct texts, each query uploads its own copy), 1..64 patterns m=U[4,64], "
                        f"Poisson arrivals at 0.8 x closed-loop capacity",
            "text_bytes": int(total),
            "capacity_qps": round(capacity, 2), "rate_qps": round(rate, 2),
            "continuous": cont, "one_query_per_launch": fifo,
            "answers_equal_across_modes": bool(same)}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=3_200_000_000, help="text bytes (default 3.2e9)")
    ap.add_argument("--kernel-reps", type=int, default=20, help="count-only launches timed per pattern")
    ap.add_argument("--cpu-sample", type=int, default=200_000_000,
                    help="text prefix (bytes) the CPU oracle's definition (window compare) scans")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run one device copy of this many bytes (counter calibration)")
    ap.add_argument("--skip-extra", action="store_true",
                    help="skip the batched, segmented and serving measurements")
    ap.add_argument("--serve-queries", type=int, default=1000)
    ap.add_argument("--merged-step", type=int, default=0, choices=(0, 1, 2),
                    help="--only merged: bytes per automaton step (0: the library's choice)")
    ap.add_argument("--merged-line", type=int, default=0, choices=(0, 32, 64),
                    help="--only merged: bytes per round (0: the library's choice)")
    ap.add_argument("--merged-chain-bytes", type=int, default=0,
                    help="--only merged: bytes per walk (a multiple of 128; 0: the library's choice)")
    ap.add_argument("--merged-waves", type=int, default=0,
                    help="--only merged: waves per workgroup (0: the library's choice)")
    ap.add_argument("--merged-automaton-bytes", type=int, default=0,
                    help="--only merged: LDS budget of one merged automaton (0: the library's choice)")
    ap.add_argument("--no-study", action="store_true",
                    help="skip the size sweep and workgroup load-balance study of the scan")
    ap.add_argument("--only", choices=("batched", "segmented", "serving", "fasta", "lds", "merged"),
                    help="run only this leg and print its figures (for profiling)")
    a = ap.parse_args(argv)

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch
    from paper_1506_08612_amd import api, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.only:
        def fasta_leg():
            w = synth.paper_scale(n=a.n, ms=PATTERN_LENGTHS)
            return bench_fasta(torch, api, w.text, api.to_device(w.text))

        legs = {"batched": lambda: bench_batched(torch, api, synth)[1],
                "segmented": lambda: bench_segmented(torch, api, synth),
                "fasta": fasta_leg,
                "serving": lambda: bench_serving(torch, a.serve_queries),
                "lds": lambda: bench_lds(torch, api),
                "merged": lambda: bench_merged_kernels(torch, api, synth, step_bytes=a.merged_step,
                                                        line_bytes=a.merged_line,
                                                        automaton_bytes=a.merged_automaton_bytes,
                                                        chain_bytes=a.merged_chain_bytes, waves=a.merged_waves)}
        print(json.dumps({a.only: legs[a.only]()}), flush=True)
        return 0
    stream = torch.cuda.current_stream()

    log(f"generating genome-like text n={a.n}")
    t0 = time.time()
    w = synth.paper_scale(n=a.n, ms=PATTERN_LENGTHS)
    log(f"  generated in {time.time() - t0:.1f}s")
    n = w.text.size

    # upload once; the text stays resident (timed separately, never inside `value`).  The
    # first copy into the new buffer also maps its pages; the same copy again from the same
    # pinned memory into the same buffer gives the link's rate
    pinned = torch.from_numpy(w.text).pin_memory()
    dtext = torch.empty(n, dtype=torch.uint8, device=dev)
    h2d = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dtext.copy_(pinned, non_blocking=True)
        torch.cuda.synchronize()
        h2d.append(time.perf_counter() - t0)
    del pinned

    pats = w.patterns
    # size the outputs from a count-only pass (outside the timed region)
    counts = []
    for p in pats:
        tab, m = api.device_table(p)
        counts.append(api.count(dtext, tab, m))
    log(f"  counts {dict(zip(PATTERN_LENGTHS, counts))}")
    caps = [max(1, c) for c in counts]
    pos_bufs = [torch.empty(c, dtype=torch.int64, device=dev) for c in caps]
    cnt_bufs = [torch.empty(1, dtype=torch.int64, device=dev) for _ in pats]
    wsb = max(api.count_workspace_bytes(n, len(p), True) for p in pats)
    ws = torch.empty(max(1, wsb), dtype=torch.uint8, device=dev)
    # Every step builds the five automata on the host and uploads their tables in one
    # asynchronous copy from pinned memory, then launches the five scans.  The timed steps
    # issue them on three streams (default priority) in turn, each stream with its own
    # workspace: a call's placement and re-walk launches, which fill few CUs, and its walk's
    # last workgroups then overlap the next calls' walks; the step ends when every stream is
    # done.  The second run of the steps (events around every call and walk) issues the calls
    # one after another on one stream.
    nstreams = 3
    streams = (stream,) + tuple(torch.cuda.Stream(device=dev) for _ in range(nstreams - 1))
    wss = (ws,) + tuple(torch.empty(max(1, wsb), dtype=torch.uint8, device=dev) for _ in range(nstreams - 1))
    tab_sizes = [api.table_bytes(len(p)) for p in pats]
    tab_offs = np.concatenate(([0], np.cumsum(tab_sizes)[:-1])).astype(np.int64)
    tab_pinned = torch.empty(int(sum(tab_sizes)), dtype=torch.uint8).pin_memory()
    tab_dev = torch.empty(int(sum(tab_sizes)), dtype=torch.uint8, device=dev)
    tab_np = tab_pinned.numpy()
    copied = torch.cuda.Event()
    copied.record(stream)

    def one_step(events=None):
        copied.synchronize()  # the previous step's upload has left the pinned buffer
        for i, p in enumerate(pats):
            tab_np[tab_offs[i]:tab_offs[i] + tab_sizes[i]] = api.build_table(p).reshape(-1)
        tab_dev.copy_(tab_pinned, non_blocking=True)  # after the previous step's calls on every stream
        copied.record(stream)
        tabs = [tab_dev[tab_offs[i]:tab_offs[i] + tab_sizes[i]] for i in range(len(pats))]
        if events is None:
            for st in streams[1:]:
                st.wait_event(copied)
            for i, p in enumerate(pats):
                api.count_async(dtext, tabs[i], len(p), cnt_bufs[i], pos_bufs[i], caps[i], wss[i % nstreams],
                                stream=streams[i % nstreams])
            for st in streams[1:]:
                stream.wait_stream(st)
            return
        for i, p in enumerate(pats):
            e0, e1, w0, w1 = events[i]
            e0.record(stream)
            with api.ScanEvents(w0, w1, stream):
                api.count_async(dtext, tabs[i], len(p), cnt_bufs[i], pos_bufs[i], caps[i], ws, stream=stream)
            e1.record(stream)

    for _ in range(a.warmup):
        one_step()
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    for _ in range(a.steps):
        one_step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the timed steps' outputs (three streams), kept to be compared with the second run's
    timed_out = [(int(c.item()), int(pb[:min(c0, pb.numel())].sum().item()))
                 for c, pb, c0 in zip(cnt_bufs, pos_bufs, counts)]

    # the same steps again, each call and each text walk bracketed by events
    lat = [[] for _ in pats]
    walk_ms = [[] for _ in pats]
    ev_all = [[tuple(torch.cuda.Event(enable_timing=True) for _ in range(4)) for _ in pats]
              for _ in range(a.steps)]
    for evs in ev_all:  # create the event handles first
        for ev in evs:
            for e in ev:
                e.record(stream)
    torch.cuda.synchronize()
    for evs in ev_all:
        one_step(evs)
    torch.cuda.synchronize()
    for evs in ev_all:
        for i, (e0, e1, w0, w1) in enumerate(evs):
            lat[i].append(e0.elapsed_time(e1))
            walk_ms[i].append(w0.elapsed_time(w1))
    got = [int(c.item()) for c in cnt_bufs]
    assert got == counts, (got, counts)
    second_out = [(int(c.item()), int(pb[:min(c0, pb.numel())].sum().item()))
                  for c, pb, c0 in zip(cnt_bufs, pos_bufs, counts)]
    assert timed_out == second_out, (timed_out, second_out)

    ms_per_step = wall * 1e3 / a.steps
    text_bytes_per_step = n * len(pats)
    value = text_bytes_per_step / (wall / a.steps) / 1e9

    # scan kernel alone (count-only launches), timed with events on the launch stream
    kern = {}
    for i, p in enumerate(pats):
        tab, m = api.device_table(p)
        api.count_async(dtext, tab, m, cnt_bufs[i], stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.kernel_reps):
            api.count_async(dtext, tab, m, cnt_bufs[i], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        kern[len(p)] = e0.elapsed_time(e1) / a.kernel_reps
    count_only_gbs = n / (float(np.mean(list(kern.values()))) * 1e-3) / 1e9
    # a trivial read-reduce over the same buffer (torch's sum of its 8-byte words): the
    # streaming-read rate this device reaches in the same run
    words = dtext[:n // 8 * 8].view(torch.int64)
    red_ms = _events_ms(torch, lambda: words.sum(), 5)
    read_gbs = (n // 8 * 8) / (red_ms * 1e-3) / 1e9
    del words
    walk_avg_ms = float(np.mean([x for w in walk_ms for x in w]))
    achieved = n / (walk_avg_ms * 1e-3) / 1e9
    traffic = read_traffic()

    if a.copy_calibration > 0:
        src = torch.empty(a.copy_calibration, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        dst.copy_(src)                 # runtime blit copy: reads and writes n bytes
        torch.add(src, 1, out=dst)     # elementwise kernel: reads and writes n bytes
        torch.cuda.synchronize()
        del src, dst

    # CPU baselines, one thread: the oracle's plain automaton scan (Alg. 1 with one worker
    # and one lane) over the WHOLE text for each of the five patterns, count + positions in
    # one pass; and the definition (window compare) on a prefix.  Both outputs are checked
    # against the GPU's positions.
    cpu = cpu_def = None
    parity_full = parity_prefix = None
    if not a.no_cpu_baseline:
        cpu, parity_full = cpu_automaton_baseline(w.text, pats, counts, pos_bufs)
        sn = min(a.cpu_sample, n)
        sample = w.text[:sn]
        t0 = time.perf_counter()
        oracle_pos = [oracle_mod().occurrences(sample, p) for p in pats]
        cpu_s = time.perf_counter() - t0
        cpu_def = {"value": round(sn * len(pats) / cpu_s / 1e9, 4), "unit": "GB/s", "cores": 1,
                   "kind": "oracle",
                   "sample": f"first {sn} bytes of the text, the same {len(pats)} patterns, "
                             f"count + positions by the definition (window compare), "
                             f"{cpu_s:.1f} s on {cpu_model()}"}
        ok = True
        for i, p in enumerate(pats):
            g = pos_bufs[i][:min(counts[i], caps[i])].cpu().numpy()
            g = g[g <= sn - len(p)]
            ok &= bool(np.array_equal(g, oracle_pos[i]))
        parity_prefix = ok

    extra = {}
    if not a.no_study:
        extra["study"] = bench_study(torch, api, w.text, dtext, pats)
    if not a.skip_extra:
        extra["fasta"] = bench_fasta(torch, api, w.text, dtext)
        del dtext
        torch.cuda.empty_cache()
        extra["lds"] = bench_lds(torch, api)
        extra["degenerate"], extra["batched"] = bench_batched(
            torch, api, synth, lds_peak=extra["lds"]["u16_conflict_free"]["reads_per_s"])
        torch.cuda.empty_cache()
        extra["segmented"] = bench_segmented(torch, api, synth)
        torch.cuda.empty_cache()
        extra["serving"] = bench_serving(torch, a.serve_queries)
        torch.cuda.empty_cache()

    lat_all = np.array([x for L in lat for x in L])
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": "plain method, paper scale: genome-like ASCII text over ACGTN "
                        "(GC 41%, 5% N-runs of geometric mean 50 kb), one pattern per launch, "
                        "m in {4,8,16,32,64} drawn from the text, count + sorted positions",
            "text_bytes": n,
            "patterns": list(PATTERN_LENGTHS),
            "matches": dict(zip([str(x) for x in PATTERN_LENGTHS], counts)),
        },
        "hbm_frac": round(value / HBM_PEAK_GBS, 4),
        "latency_ms": {"p50": round(float(np.percentile(lat_all, 50)), 4),
                       "p99": round(float(np.percentile(lat_all, 99)), 4),
                       "min": round(float(np.min(lat_all)), 4),
                       "per_pattern_p50": {str(len(p)): round(float(np.percentile(lat[i], 50)), 4)
                                           for i, p in enumerate(pats)}},
        "walk_kernel_ms": {str(len(p)): round(float(np.mean(walk_ms[i])), 4) for i, p in enumerate(pats)},
        "count_only_kernel_ms": {str(k): round(v, 4) for k, v in kern.items()},
        "count_only_frac": round(count_only_gbs / HBM_PEAK_GBS, 4),
        "read_reduce_GBps": round(read_gbs, 1),
        "frac_of_read_reduce": {"text_walk": round(achieved / read_gbs, 4),
                                "count_only": round(count_only_gbs / read_gbs, 4)},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_scan text walk of count + positions (per-walk counts for m < 12, per-wave counts from 12)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
        "cpu_baseline": cpu,
        "cpu_definition_baseline": cpu_def,
        "parity_vs_oracle_full_text": parity_full,
        "parity_vs_oracle_definition_prefix": parity_prefix,
        "h2d_GBps": round(n / min(h2d[1:]) / 1e9, 2),
        "h2d_first_copy_GBps": round(n / h2d[0] / 1e9, 2),
        "h2d_link": "PCIe, host pinned memory to HBM, one copy of the whole text (best of 2 after the first)",
    }
    out.update(extra)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
