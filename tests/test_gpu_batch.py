"""GPU parity of the batched / segmented scan (dfa_batch_prepare + dfa_batch_run) against
the CPU oracle's per-(segment, pattern) counts: bit-exact on every input."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_1506_08612_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1506_08612_amd import api  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_batch(text, seg_off, pats, pair_seg, pair_pat, t=None):
    d = api.to_device(text)
    ps = api.PatternSet(pats)
    return api.count_batch(d, seg_off, ps, pair_seg, pair_pat, t)


def check_batch(text, seg_off, pats, pair_seg, pair_pat, t=None):
    got = run_batch(text, seg_off, pats, pair_seg, pair_pat, t)
    want = oracle.pair_counts(text, seg_off, pats, pair_seg, pair_pat)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(int(k), int(pair_seg[k]), len(pats[pair_pat[k]]), int(got[k]), int(want[k]))
                           for k in bad[:10]]
    return got


def test_many_patterns_one_text():
    """One text, patterns of every length 1..80 (drawn and random), all in one launch."""
    text = synth.genome_like(2_000_003, 31, 0.02, 3000)
    rng = np.random.default_rng(1)
    pats = []
    for i in range(300):
        m = 1 + i % 80
        p, _ = synth.drawn_pattern(text, m, rng) if i % 2 == 0 else (None, -1)
        pats.append(p if p is not None else synth.random_pattern(m, rng))
    say("one text, 300 patterns")
    check_batch(text, [0, text.size], pats, [0] * len(pats), list(range(len(pats))))


def test_uneven_segments():
    w = synth.uneven_segments(nseg=150, median=20_000, sigma=1.5, lo=1, hi=2_000_000, seed=7)
    say(f"segments {w.seg_off.size - 1} total {w.seg_off[-1]} pairs {w.pair_seg.size}")
    check_batch(w.text, w.seg_off, w.patterns, w.pair_seg, w.pair_pat)


def test_empty_and_tiny_segments():
    rng = np.random.default_rng(3)
    lens = [0, 1, 2, 3, 15, 16, 17, 0, 100, 1000, 5, 0]
    seg_off = np.concatenate(([0], np.cumsum(lens))).astype(np.int64)
    text = np.frombuffer(b"AC", np.uint8)[rng.integers(0, 2, int(seg_off[-1]))].copy()
    pats = [b"A", b"C", b"AC", b"CA", b"ACA", b"AAAA", b"ACACACACACACACACA"]
    ps_, pp_ = [], []
    for s in range(len(lens)):
        for j in range(len(pats)):
            ps_.append(s)
            pp_.append(j)
    say("tiny segments")
    check_batch(text, seg_off, pats, ps_, pp_)


def test_match_across_segment_border_not_counted():
    text = np.frombuffer(b"ACGTAC" + b"GTACGT" * 1000, np.uint8).copy()
    seg_off = [0, 6, text.size]
    got = check_batch(text, seg_off, [b"ACGT"], [0, 1], [0, 0])
    assert got[0] == 1


@pytest.mark.parametrize("tn", [dict(dfas_per_group=4), dict(dfas_per_group=16), dict(waves_per_group=1),
                                dict(waves_per_group=3, dfas_per_group=4), dict(chain_bytes=16),
                                dict(chain_bytes=48, waves_per_group=2), dict(chain_bytes=4096)],
                         ids=lambda d: ",".join(f"{k}={v}" for k, v in d.items()))
def test_result_independent_of_launch_shape(tn):
    w = synth.uneven_segments(nseg=40, median=50_000, sigma=1.0, lo=1, hi=500_000, seed=11)
    say(f"tune {tn}")
    check_batch(w.text, w.seg_off, w.patterns, w.pair_seg, w.pair_pat, api.tune(**tn))


def test_duplicates_and_agreement_with_single_scan():
    text = synth.genome_like(1_000_000, 5, 0.03, 500)
    pats = [text[1000:1008].tobytes(), text[1000:1008].tobytes(), b"ACGT", b"ACGT", text[5:69].tobytes()]
    got = check_batch(text, [0, text.size], pats, [0] * 5, list(range(5)))
    assert got[0] == got[1] and got[2] == got[3]
    d = api.to_device(text)
    for p, c in zip(pats, got):
        tab, m = api.device_table(p)
        assert api.count(d, tab, m) == c


def test_replay_after_prepare():
    """prepare once, run many times (the form a HIP graph replays)."""
    w = synth.uneven_segments(nseg=30, median=30_000, sigma=1.0, lo=100, hi=300_000, seed=13)
    d = api.to_device(w.text)
    ps = api.PatternSet(w.patterns)
    b = api.Batch(w.seg_off, ps, w.pair_seg, w.pair_pat)
    want = oracle.pair_counts(w.text, w.seg_off, w.patterns, w.pair_seg, w.pair_pat)
    for _ in range(3):
        got = b.run(d).cpu().numpy()
        assert np.array_equal(got, want)
