"""Texts longer than 2^32 bytes: byte offsets past 4 GiB go through the 64-bit paths
(walk and tile starts, positions, segment offsets).  A 4.6e9-byte genome-like text
(GC 41 %, 'N' runs) with patterns planted across and past the 2^32 boundary:

* the single-pattern scan (count + sorted positions, default launch shape) for patterns
  of 4, 12 and 33 bytes against the oracle's window-compare definition, every position;
* the merged scan over segments that end below, straddle and start past 2^32, every
  (segment, pattern) count against the oracle.

FASTA normalisation keeps its unit and output offsets in 64 bits too; it is checked at
3.25 GB only (the oracle's line-by-line definition is too slow for 4.6 GB here).
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

from paper_1506_08612_amd import api  # noqa: E402

N = 4_600_000_000
B32 = 1 << 32
THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def big():
    say("generating", N, "bytes")
    text = synth.genome_like(N, 41, n_frac=0.02, n_run_mean=5000)
    rng = np.random.default_rng(404)
    pats = [synth.random_pattern(m, rng) for m in (4, 12, 33)]
    # each pattern twice past 2^32 (apart from the others' copies); the longest also across
    # 2^32 and ending right at the text's end
    for k, p in enumerate(pats):
        for at in (B32 + 12_345 + 1000 * k, N - 200 * (k + 1)):
            text[at:at + len(p)] = np.frombuffer(p, np.uint8)
    for at in (B32 - len(pats[-1]) // 2, N - len(pats[-1])):
        text[at:at + len(pats[-1])] = np.frombuffer(pats[-1], np.uint8)
    d = api.to_device(text)
    yield text, pats, d
    del d
    torch.cuda.empty_cache()


def test_single_pattern_past_4gib(big):
    text, pats, d = big
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        wants = list(ex.map(lambda p: oracle.occurrences(text, p), pats))
    for p, want in zip(pats, wants):
        say("m", len(p), "matches", want.size, "past 2^32", int((want >= B32).sum()))
        assert (want >= B32).sum() >= 2 and (want < B32).any()
        tab, m = api.device_table(p)
        assert api.count(d, tab, m) == want.size
        c, pos = api.positions(d, tab, m)
        assert c == want.size
        assert np.array_equal(pos.cpu().numpy(), want)


def test_merged_segments_past_4gib(big):
    text, pats, d = big
    seg_off = np.array([0, 1_000_000_000, B32 - 300, B32 + 100, B32 + 150_000_000, N], np.int64)
    rng = np.random.default_rng(405)
    patterns = list(pats) + [synth.random_pattern(int(m), rng) for m in (5, 6, 8, 16)]
    pair_seg, pair_pat = [], []
    for s in (2, 3, 4):  # the segments at and past 2^32 (the first two are long and carry no pairs)
        for j in range(len(patterns)):
            pair_seg.append(s)
            pair_pat.append(j)
    pair_seg = np.array(pair_seg, np.int32)
    pair_pat = np.array(pair_pat, np.int32)
    got = api.count_merged(d, seg_off, patterns, pair_seg, pair_pat)
    chunks = [np.flatnonzero(pair_seg == s) for s in (2, 3, 4)]
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        parts = list(ex.map(lambda idx: oracle.pair_counts(text, seg_off, patterns, pair_seg[idx], pair_pat[idx]),
                            chunks))
    want = np.zeros(pair_seg.size, np.int64)
    for idx, part in zip(chunks, parts):
        want[idx] = part
    say("pairs", pair_seg.size, "total", int(want.sum()))
    assert want[(pair_seg == 2) & (pair_pat == len(pats) - 1)].sum() >= 1  # the copy across 2^32
    assert np.array_equal(got, want)
