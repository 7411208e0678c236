"""Seeded synthetic nucleotide texts and pattern sets.

This module only draws random inputs; it holds none of the matching
arithmetic, so both the CPU oracle tests and the GPU path may use it.

The paper measures on GenBank genomes of 193 MB - 3.25 GB (Table 1) with
8-mer patterns (Table 3).  Neither is available here, so every workload is
synthetic ASCII text with the same sizes and structure:

* bases i.i.d. with GC content 41 % (p_A = p_T = 0.295, p_C = p_G = 0.205),
  drawn as one byte in [0, 200) mapped through a 200-entry lookup;
* assembly gaps: runs of 'N' whose lengths are geometric with a given mean,
  placed at sorted uniform cut points until they cover a given fraction;
* patterns either copied from a pure-ACGT window of the text ("drawn") or
  drawn i.i.d. at the same base composition ("random").

Generation is chunked (64 MiB) with one PCG64 child stream per chunk, so it is
reproducible and parallel.
"""
from __future__ import annotations

import concurrent.futures as _cf
import dataclasses
import math
import os

import numpy as np

CHUNK = 64 << 20
ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)

# one byte in [0, 200) -> base; 59/200 = 0.295 for A and T, 41/200 = 0.205 for C and G
_GC41_LUT = np.empty(256, dtype=np.uint8)
_GC41_LUT[:] = ord("N")
_GC41_LUT[0:59] = ord("A")
_GC41_LUT[59:100] = ord("C")
_GC41_LUT[100:141] = ord("G")
_GC41_LUT[141:200] = ord("T")


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def iid_gc41(n: int, seed: int, out: np.ndarray | None = None) -> np.ndarray:
    """n bytes over {A,C,G,T} with GC content 41 %, reproducible for a given seed."""
    n = int(n)
    if out is None:
        out = np.empty(n, dtype=np.uint8)
    nchunks = max(1, -(-n // CHUNK))
    children = np.random.SeedSequence(seed).spawn(nchunks)

    def fill(c: int) -> None:
        lo = c * CHUNK
        hi = min(n, lo + CHUNK)
        if hi <= lo:
            return
        rng = np.random.Generator(np.random.PCG64(children[c]))
        raw = rng.integers(0, 200, size=hi - lo, dtype=np.uint8)
        np.take(_GC41_LUT, raw, out=out[lo:hi])

    if nchunks == 1:
        fill(0)
    else:
        with _cf.ThreadPoolExecutor(_workers()) as ex:
            list(ex.map(fill, range(nchunks)))
    return out


def n_runs(n: int, frac: float, mean_len: float, rng: np.random.Generator):
    """(starts, lengths) of 'N' runs: geometric lengths (mean mean_len) covering frac*n bytes,
    placed at sorted uniform cut points of the remaining bases."""
    target = int(round(frac * n))
    if target <= 0 or n <= 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    lens = []
    total = 0
    p = 1.0 / max(1.0, float(mean_len))
    while total < target:
        k = rng.geometric(p, size=max(16, int(1.5 * (target - total) / mean_len) + 1)).astype(np.int64)
        for L in k:
            L = int(min(L, target - total))
            lens.append(L)
            total += L
            if total >= target:
                break
    lens = np.array(lens, dtype=np.int64)
    rest = n - total
    cuts = np.sort(rng.integers(0, rest + 1, size=lens.size, dtype=np.int64))
    starts = cuts + np.concatenate(([0], np.cumsum(lens)[:-1]))
    return starts, lens


def apply_n_runs(text: np.ndarray, starts: np.ndarray, lens: np.ndarray) -> None:
    for s, L in zip(starts.tolist(), lens.tolist()):
        text[s:s + L] = ord("N")


def genome_like(n: int, seed: int, n_frac: float = 0.0, n_run_mean: float = 50_000) -> np.ndarray:
    """GC-41 % i.i.d. text of n bytes with optional 'N' runs covering n_frac of it."""
    text = iid_gc41(n, seed)
    if n_frac > 0:
        rng = np.random.default_rng([seed, 0x4E52])
        s, L = n_runs(n, n_frac, n_run_mean, rng)
        apply_n_runs(text, s, L)
    return text


def random_pattern(m: int, rng: np.random.Generator) -> bytes:
    """m bases i.i.d. at GC 41 %."""
    return _GC41_LUT[rng.integers(0, 200, size=m, dtype=np.uint8)].tobytes()


def drawn_pattern(text: np.ndarray, m: int, rng: np.random.Generator, lo: int = 0,
                  hi: int | None = None, tries: int = 10_000):
    """Copy an m-byte pure-ACGT window of text[lo:hi] at a uniform offset.
    Returns (pattern, absolute offset), or (None, -1) if no such window was found."""
    hi = text.size if hi is None else hi
    if hi - lo < m:
        return None, -1
    acgt = np.zeros(256, dtype=bool)
    acgt[ACGT] = True
    for _ in range(tries):
        off = int(rng.integers(lo, hi - m + 1))
        w = text[off:off + m]
        if acgt[w].all():
            return w.tobytes(), off
    return None, -1


# ----------------------------------------------------------------------------------------
# Workload recipes
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class SinglePattern:
    text: np.ndarray
    patterns: list          # list[bytes]
    offsets: list           # planted offset per pattern (-1 for random ones)
    name: str


def tiny_uniform(n: int = 1 << 20, m: int = 8, seed: int = 0) -> SinglePattern:
    """1 MiB uniform ACGT text from default_rng(seed); one m-mer copied from a seeded offset."""
    rng = np.random.default_rng(seed)
    text = ACGT[rng.integers(0, 4, n)]
    off = int(rng.integers(0, n - m + 1))
    return SinglePattern(text, [text[off:off + m].tobytes()], [off], f"uniform-acgt n={n} m={m}")


def paper_scale(n: int = 3_200_000_000, ms=(4, 8, 16, 32, 64), seed: int = 2,
                n_frac: float = 0.05, n_run_mean: float = 50_000) -> SinglePattern:
    """Genome-sized text (GC 41 %, 'N' runs of geometric mean 50 kb covering 5 %) and one
    pattern drawn from the text for each length in ms."""
    text = genome_like(n, seed, n_frac, n_run_mean)
    rng = np.random.default_rng([seed, 0x5041])
    pats, offs = [], []
    for m in ms:
        p, o = drawn_pattern(text, m, rng)
        pats.append(p)
        offs.append(o)
    return SinglePattern(text, pats, offs, f"genome-like n={n} gc=0.41 N={n_frac}")


@dataclasses.dataclass
class PatternBatch:
    text: np.ndarray
    patterns: list          # list[bytes], uneven lengths
    offsets: list           # drawn offset or -1
    name: str


def many_patterns(n: int = 1_000_000_000, npat: int = 1024, mlo: int = 4, mhi: int = 64,
                  seed: int = 3) -> PatternBatch:
    """GC-41 % ACGT text; npat patterns with lengths uniform in [mlo, mhi]; the first half
    drawn from the text, the second half random."""
    text = iid_gc41(n, seed)
    rng = np.random.default_rng([seed, 0x4D50])
    lens = rng.integers(mlo, mhi + 1, size=npat)
    pats, offs = [], []
    for i, m in enumerate(lens.tolist()):
        if i < npat // 2:
            p, o = drawn_pattern(text, m, rng)
            if p is None:
                p, o = random_pattern(m, rng), -1
        else:
            p, o = random_pattern(m, rng), -1
        pats.append(p)
        offs.append(o)
    return PatternBatch(text, pats, offs, f"gc41 n={n} patterns={npat} m=U[{mlo},{mhi}]")


@dataclasses.dataclass
class SegmentBatch:
    text: np.ndarray        # all segments back to back
    seg_off: np.ndarray     # int64[nseg+1]
    patterns: list          # list[bytes]
    pair_seg: np.ndarray    # int64[npairs]
    pair_pat: np.ndarray    # int64[npairs]
    name: str


def uneven_segments(nseg: int = 2000, median: float = 2e5, sigma: float = 1.794,
                    lo: int = 1000, hi: int = 250_000_000, n_frac: float = 0.02,
                    n_run_mean: float = 5000, kmax: int = 16, mlo: int = 6, mhi: int = 48,
                    seed: int = 4, total_cap: int | None = None) -> SegmentBatch:
    """Contig-like segments with log-normal lengths (median 200 kB, clipped to [1 kB, 250 MB]),
    2 % 'N' runs each; every segment gets 1..kmax patterns with lengths uniform in
    [mlo, mhi], half drawn from that segment and half random."""
    rng = np.random.default_rng([seed, 0x5345])
    lens = np.exp(rng.normal(math.log(median), sigma, size=nseg))
    lens = np.clip(np.round(lens), lo, hi).astype(np.int64)
    if total_cap is not None and lens.sum() > total_cap:
        lens = np.maximum(lo, (lens * (total_cap / lens.sum())).astype(np.int64))
    seg_off = np.zeros(nseg + 1, dtype=np.int64)
    seg_off[1:] = np.cumsum(lens)
    text = iid_gc41(int(seg_off[-1]), seed)
    for s in range(nseg):
        a, b = int(seg_off[s]), int(seg_off[s + 1])
        st, L = n_runs(b - a, n_frac, n_run_mean, rng)
        apply_n_runs(text[a:b], st, L)
    pats, pseg, ppat = [], [], []
    for s in range(nseg):
        a, b = int(seg_off[s]), int(seg_off[s + 1])
        k = int(rng.integers(1, kmax + 1))
        for i in range(k):
            m = int(rng.integers(mlo, mhi + 1))
            p = None
            if i % 2 == 0:
                p, _ = drawn_pattern(text, m, rng, a, b, tries=64)
            if p is None:
                p = random_pattern(m, rng)
            pats.append(p)
            pseg.append(s)
            ppat.append(len(pats) - 1)
    return SegmentBatch(text, seg_off, pats, np.array(pseg, np.int64), np.array(ppat, np.int64),
                        f"segments={nseg} total={int(seg_off[-1])}")


@dataclasses.dataclass
class Query:
    arrival_s: float
    text_len: int
    seed: int
    pattern_lens: list


def query_trace(nq: int, rate_hz: float, seed: int = 5, len_lo: float = 1e4, len_hi: float = 5e8,
                pmax: int = 64, mlo: int = 4, mhi: int = 64) -> list:
    """Poisson arrivals at rate_hz; text length log-uniform in [len_lo, len_hi]; 1..pmax patterns
    with lengths uniform in [mlo, mhi] (the query's text is materialised by query_text)."""
    rng = np.random.default_rng([seed, 0x5156])
    t = 0.0
    out = []
    for i in range(nq):
        t += float(rng.exponential(1.0 / rate_hz))
        L = int(round(math.exp(rng.uniform(math.log(len_lo), math.log(len_hi)))))
        k = int(rng.integers(1, pmax + 1))
        ms = rng.integers(mlo, mhi + 1, size=k).tolist()
        qseed = int(rng.integers(0, 2**31))
        out.append(Query(t, L, qseed, ms))
    return out


def query_patterns(text: np.ndarray, q: Query) -> list:
    """The query's patterns over `text`: lengths q.pattern_lens, every other one drawn from the
    text, the rest (and any that finds no pure-ACGT window) random."""
    rng = np.random.default_rng([q.seed, 0x5150])
    pats = []
    for i, m in enumerate(q.pattern_lens):
        p = None
        if i % 2 == 0:
            p, _ = drawn_pattern(text, m, rng, tries=64)
        if p is None:
            p = random_pattern(m, rng)
        pats.append(p)
    return pats


def query_text(q: Query, n_frac: float = 0.02, n_run_mean: float = 5000):
    """Materialise one query: its text and its patterns (half drawn, half random)."""
    text = genome_like(q.text_len, q.seed, n_frac, n_run_mean)
    return text, query_patterns(text, q)
