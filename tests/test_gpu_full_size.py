"""Parity of the batched scans at the benchmark's full sizes, in the launch the benchmark
times (merged automata with the default plan, replayed from a HIP graph): EVERY output is
computed by the C oracle (job-parallel on host threads; the C calls release the interpreter
lock) and must equal the device's bit for bit.

* 1 GB GC-41 % text x 1024 patterns of 4..64 bytes (half drawn from the text): all 1024
  per-pattern counts, checked in eight groups of 128 so that each test stays short;
* 2000 contig-like segments (~1.83 GB): all 17165 (segment, pattern) pair counts;
* 18 degenerate 8-mer queries (9 with a 3-way position), both strands, over the 1 GB text:
  all 18 counts;
* the benchmark's serving trace (1000 queries after 50 warm-up, texts from a pool of 64):
  served closed-loop and paced, every answer equal across the two runs, and a seeded sample
  of 64 answers plus the query with the longest text counted by the oracle.
"""
from __future__ import annotations

import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1506_08612_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1506_08612_amd import api, graph, serve  # noqa: E402

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
GROUPS = 8  # the 1024 per-pattern counts are checked in this many tests


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pool_map(fn, items):
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        return list(ex.map(fn, items))


@pytest.fixture(scope="module")
def gc_text_1gb():
    w = synth.many_patterns()  # the benchmark's many-pattern workload (seed 3)
    return w, api.to_device(w.text)


@pytest.fixture(scope="module")
def many_counts(gc_text_1gb):
    w, d = gc_text_1gb
    n = w.text.size
    npat = len(w.patterns)
    b = api.MergedBatch([0, n], w.patterns, np.zeros(npat, np.int64), np.arange(npat), device=d.device)
    g = graph.GraphedBatch(d, b)
    got = g.replay().cpu().numpy()
    say("automata", int(b.plan.nautomata), "states", int(b.plan.nstates))
    again = g.replay().cpu().numpy()
    assert np.array_equal(got, again)  # a second replay of the graph gives the same counts
    return got


@pytest.mark.parametrize("group", range(GROUPS))
def test_many_patterns_full_size(gc_text_1gb, many_counts, group):
    w, _ = gc_text_1gb
    npat = len(w.patterns)
    idx = list(range(group, npat, GROUPS))  # every pattern lands in exactly one group
    want = _pool_map(lambda j: oracle.count(w.text, w.patterns[j]), idx)
    bad = [(j, len(w.patterns[j]), int(many_counts[j]), c) for j, c in zip(idx, want) if many_counts[j] != c]
    say(f"group {group}: {len(idx)} patterns checked, {len(bad)} differ")
    assert not bad, bad[:8]


def test_many_patterns_groups_cover_every_pattern(gc_text_1gb):
    npat = len(gc_text_1gb[0].patterns)
    seen = sorted(j for g in range(GROUPS) for j in range(g, npat, GROUPS))
    assert seen == list(range(npat))


def test_degenerate_queries_full_size(gc_text_1gb):
    w, d = gc_text_1gb
    n = w.text.size
    rng = np.random.default_rng([6, 0x4447])  # the benchmark's queries
    codes = []
    for i in range(9):
        s = list(synth.random_pattern(8, rng).decode())
        s[i % 8] = "BDHV"[int(rng.integers(0, 4))]
        codes.append("".join(s).encode())
    codes += [synth.random_pattern(8, rng) for _ in range(9)]
    queries = [(0, c, True) for c in codes]
    b = api.DegenerateBatch([0, n], queries, device=d.device)
    g = graph.GraphedBatch(d, b)
    got = g.replay().cpu().numpy()[:len(queries)]
    want = _pool_map(lambda q: oracle.degenerate_count(w.text, codes[q], True), range(len(queries)))
    for q, c in enumerate(want):
        assert got[q] == c, codes[q]


def test_uneven_segments_full_size():
    w = synth.uneven_segments()  # the benchmark's segmented workload
    d = api.to_device(w.text)
    b = api.MergedBatch(w.seg_off, w.patterns, w.pair_seg, w.pair_pat, device=d.device)
    g = graph.GraphedBatch(d, b)
    got = g.replay().cpu().numpy()
    npairs = w.pair_seg.size
    say("pairs", npairs, "bytes", int(w.seg_off[-1]))
    # jobs of whole pairs, the longest segments first so that the pool drains evenly
    seg_len = np.diff(w.seg_off)[w.pair_seg]
    order = np.argsort(-seg_len, kind="stable")
    jobs = [order[i::4 * THREADS] for i in range(4 * THREADS)]

    def one(idx):
        return idx, oracle.pair_counts(w.text, w.seg_off, w.patterns, w.pair_seg[idx], w.pair_pat[idx])

    want = np.full(npairs, -1, np.int64)
    for idx, c in _pool_map(one, jobs):
        want[idx] = c
    assert (want >= 0).all()  # every pair was counted by the oracle
    bad = np.nonzero(got[:npairs] != want)[0]
    assert bad.size == 0, [(int(k), int(w.pair_seg[k]), int(w.pair_pat[k])) for k in bad[:8]]


def test_serving_trace_full_size():
    """The benchmark's serving trace: every answer of the paced run equals the closed-loop
    run's, and a seeded sample (plus the longest text) equals the oracle's counts."""
    warm, nq, pool = 50, 1000, 64
    trace = serve.make_trace(warm + nq, rate_hz=1.0, seed=5, pool=pool)
    meas = trace[warm:]
    srv = serve.Server(arena_bytes=8 << 30)
    closed = srv.serve([serve.Request(r.qid, r.text, r.patterns, 0.0) for r in meas], mode="continuous")
    capacity = nq / max(r.done for r in closed)
    rate = 0.8 * capacity
    t_first = meas[0].arrival
    paced = srv.serve([serve.Request(r.qid, r.text, r.patterns, (r.arrival - t_first) / rate) for r in meas],
                      mode="continuous")
    srv.release_pinned()
    say(f"served {nq} queries, capacity {capacity:.0f}/s, launches closed {len({r.launched for r in closed})}, "
        f"paced {len({r.launched for r in paced})}")
    for a, b in zip(closed, paced):
        assert a.qid == b.qid and np.array_equal(a.counts, b.counts), a.qid
    rng = np.random.default_rng([5, 0x5345])
    sample = sorted(set(int(i) for i in rng.choice(nq, size=64, replace=False))
                    | {int(np.argmax([r.text.size for r in meas]))})
    jobs = [(i, j) for i in sample for j in range(len(meas[i].patterns))]
    want = _pool_map(lambda ij: oracle.count(meas[ij[0]].text, meas[ij[0]].patterns[ij[1]]), jobs)
    for (i, j), c in zip(jobs, want):
        assert closed[i].counts[j] == c, (meas[i].qid, j)
    say(f"{len(sample)} answers ({len(jobs)} counts) equal the oracle's")
