"""Parity of the batched scans at the benchmark's full sizes, in the launch the benchmark
times (merged automata with the default plan, replayed from a HIP graph): a sample of the
outputs is computed one by one by the C oracle (on host threads; the C calls release the
interpreter lock) and must equal the device's bit for bit.

* 1 GB GC-41 % text x 1024 patterns of 4..64 bytes (half drawn from the text);
* 2000 contig-like segments (~1.83 GB, 17165 (segment, pattern) pairs);
* 18 degenerate 8-mer queries (9 with a 3-way position), both strands, over the 1 GB text.
"""
from __future__ import annotations

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

from paper_1506_08612_amd import api, graph  # noqa: E402

THREADS = 16


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gc_text_1gb():
    w = synth.many_patterns()  # the benchmark's many-pattern workload (seed 3)
    return w, api.to_device(w.text)


def test_many_patterns_full_size(gc_text_1gb):
    w, d = gc_text_1gb
    n = w.text.size
    npat = len(w.patterns)
    b = api.MergedBatch([0, n], w.patterns, np.zeros(npat, np.int64), np.arange(npat), device=d.device)
    g = graph.GraphedBatch(d, b)
    got = g.replay().cpu().numpy()
    say("automata", int(b.plan.nautomata), "states", int(b.plan.nstates))
    rng = np.random.default_rng(1)
    sample = [int(j) for j in rng.choice(npat, size=16, replace=False)]
    sample += [int(np.argmin([len(p) for p in w.patterns])), int(np.argmax([len(p) for p in w.patterns]))]
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        want = list(ex.map(lambda j: oracle.count(w.text, w.patterns[j]), sample))
    for j, c in zip(sample, want):
        assert got[j] == c, (j, len(w.patterns[j]))


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
    sample = [0, 4, 9, 17]
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        want = list(ex.map(lambda q: oracle.degenerate_count(w.text, codes[q], True), sample))
    for q, c in zip(sample, want):
        assert got[q] == c, codes[q]


def test_uneven_segments_full_size():
    w = synth.uneven_segments()  # the benchmark's segmented workload
    d = api.to_device(w.text)
    b = api.MergedBatch(w.seg_off, w.patterns, w.pair_seg, w.pair_pat, device=d.device)
    g = graph.GraphedBatch(d, b)
    got = g.replay().cpu().numpy()
    npairs = w.pair_seg.size
    seg_len = np.diff(w.seg_off)
    say("pairs", npairs, "bytes", int(w.seg_off[-1]))
    rng = np.random.default_rng(2)
    sample = list(rng.choice(npairs, size=48, replace=False))
    sample.append(int(np.argmax(seg_len[w.pair_seg])))   # a pair on the longest segment
    sample.append(int(np.argmin(seg_len[w.pair_seg])))   # and on the shortest
    sample = np.array(sample, np.int64)

    def one(k):
        return int(oracle.pair_counts(w.text, w.seg_off, w.patterns, w.pair_seg[k:k + 1], w.pair_pat[k:k + 1])[0])

    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        want = list(ex.map(one, [int(k) for k in sample]))
    for k, c in zip(sample, want):
        assert got[k] == c, (int(k), int(w.pair_seg[k]), int(w.pair_pat[k]))
