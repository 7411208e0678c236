"""GPU parity of the merged multi-pattern scan (dfa_merged_prepare + dfa_merged_run)
against the CPU oracle's per-(segment, pattern) counts: bit-exact on every input,
for every launch shape and automaton budget."""
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

from paper_1506_08612_amd import api, graph  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check(text, seg_off, pats, pair_seg, pair_pat, t=None):
    d = api.to_device(text)
    got = api.count_merged(d, seg_off, pats, pair_seg, pair_pat, t)
    want = oracle.pair_counts(text, seg_off, pats, np.asarray(pair_seg), np.asarray(pair_pat))
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(int(k), int(pair_seg[k]), len(pats[pair_pat[k]]), int(got[k]), int(want[k]))
                           for k in bad[:10]]
    return got


def _mixed_patterns(text, rng, lens):
    pats = []
    for i, m in enumerate(lens):
        p = None
        if i % 2 == 0:
            p, _ = synth.drawn_pattern(text, m, rng)
        pats.append(p if p is not None else synth.random_pattern(m, rng))
    return pats


LENGTHS = [1, 2, 3, 4, 5, 8, 15, 16, 17, 18, 31, 33, 48, 64, 65, 66, 100, 200, 255]


def test_one_text_all_lengths():
    text = synth.genome_like(3_000_011, 41, 0.02, 3000)
    rng = np.random.default_rng(2)
    pats = _mixed_patterns(text, rng, LENGTHS * 6)
    pats += [pats[3], pats[4][1:], b"N" * 5, b"ACGTN"]  # repeat, suffix, N bytes
    say("one text,", len(pats), "patterns")
    check(text, [0, text.size], pats, [0] * len(pats), list(range(len(pats))))


@pytest.mark.parametrize("tune", [
    dict(automaton_bytes=4096), dict(automaton_bytes=120 * 1024), dict(waves_per_group=1),
    dict(waves_per_group=2), dict(waves_per_group=8), dict(chain_bytes=128), dict(chain_bytes=2048),
    dict(chain_bytes=256, waves_per_group=3, automaton_bytes=8192),
    dict(line_bytes=32), dict(line_bytes=64), dict(line_bytes=32, step_bytes=2),
    dict(waves_per_group=16), dict(waves_per_group=16, line_bytes=64, chain_bytes=128),
    dict(waves_per_group=16, automaton_bytes=8192, line_bytes=32),
    dict(line_bytes=64, step_bytes=2, chain_bytes=128, waves_per_group=1),
])
def test_launch_shapes(tune):
    text = synth.genome_like(1_500_007, 43, 0.02, 2000)
    rng = np.random.default_rng(3)
    pats = _mixed_patterns(text, rng, [4, 6, 8, 12, 16, 17, 20, 32, 40, 64, 70] * 8)
    say("tune", tune)
    check(text, [0, text.size], pats, [0] * len(pats), list(range(len(pats))), api.tune(**tune))


def test_uneven_segments():
    w = synth.uneven_segments(nseg=160, median=20_000, sigma=1.5, lo=1, hi=2_000_000, seed=7)
    say(f"segments {w.seg_off.size - 1} total {w.seg_off[-1]} pairs {w.pair_seg.size}")
    check(w.text, w.seg_off, w.patterns, w.pair_seg, w.pair_pat)


def test_unaligned_tiny_and_empty_segments():
    rng = np.random.default_rng(4)
    lens = [0, 1, 2, 3, 15, 16, 17, 0, 100, 127, 128, 129, 1000, 5, 0, 70_001, 300_017, 33]
    seg_off = np.concatenate(([5], 5 + np.cumsum(lens))).astype(np.int64)  # starts off the 128-byte grid
    text = np.frombuffer(b"AC", np.uint8)[rng.integers(0, 2, int(seg_off[-1]) + 7)].copy()
    pats = [b"A", b"C", b"AC", b"CA", b"ACA", b"AAAA", b"ACACACACACACACACA", b"C" * 20, b"AC" * 40]
    ps_, pp_ = [], []
    for s in range(len(lens)):
        for j in range(len(pats)):
            ps_.append(s)
            pp_.append(j)
    say("tiny segments")
    check(text, seg_off, pats, ps_, pp_)
    check(text, seg_off, pats, ps_, pp_, api.tune(chain_bytes=128, waves_per_group=1))


def test_periodic_text_dense_matches():
    """Every position matches: the visit counters and the overlap rule under load."""
    text = np.full(2_000_000 + 13, ord("A"), np.uint8)
    pats = [b"A", b"AA", b"A" * 7, b"A" * 17, b"A" * 64, b"A" * 65, b"A" * 255, b"C"]
    seg_off = [0, 999_999, 1_000_000, text.size]
    ps_, pp_ = [], []
    for s in range(3):
        for j in range(len(pats)):
            ps_.append(s)
            pp_.append(j)
    got = check(text, seg_off, pats, ps_, pp_)
    assert got[0] == 999_999


def test_bytes_outside_acgt():
    rng = np.random.default_rng(6)
    text = rng.integers(0, 256, 1_000_003, dtype=np.uint8)
    text[::7] = 0
    pats = [text[i:i + m].tobytes() for i, m in ((5, 3), (100, 8), (4000, 20), (77, 2), (123456, 1))]
    pats += [bytes([0, 0]), bytes([255]), bytes(range(200, 216))]
    check(text, [0, 500_000, text.size], pats, [0] * len(pats) + [1] * len(pats),
          list(range(len(pats))) * 2)


def test_matches_separate_automata_batch():
    w = synth.uneven_segments(nseg=60, median=30_000, sigma=1.2, lo=100, hi=1_000_000, seed=9)
    d = api.to_device(w.text)
    a = api.count_merged(d, w.seg_off, w.patterns, w.pair_seg, w.pair_pat)
    b = api.count_batch(d, w.seg_off, api.PatternSet(w.patterns), w.pair_seg, w.pair_pat)
    assert np.array_equal(a, b)


def test_no_pairs_and_no_segments():
    d = api.to_device(np.frombuffer(b"ACGT" * 100, np.uint8).copy())
    assert api.count_merged(d, [0, 400], [b"ACGT"], [], []).size == 0
    assert api.count_merged(d, [0], [b"ACGT"], [], []).size == 0


def test_graph_replay_and_repeat():
    text = synth.genome_like(1_000_000, 47, 0.02, 1000)
    rng = np.random.default_rng(8)
    pats = _mixed_patterns(text, rng, [5, 9, 13, 30, 60] * 10)
    d = api.to_device(text)
    b = api.MergedBatch([0, text.size], pats, [0] * len(pats), list(range(len(pats))))
    want = oracle.pair_counts(text, [0, text.size], pats, np.zeros(len(pats), np.int64), np.arange(len(pats)))
    g = graph.GraphedBatch(d, b)
    for rep in range(3):
        assert np.array_equal(g.replay().cpu().numpy(), want), rep
        assert np.array_equal(b.run(d).cpu().numpy(), want), rep  # eager run between replays
        torch.cuda.synchronize()


@pytest.mark.slow
def test_many_patterns_scale():
    """1024 patterns of lengths 4..64 over 64 MB: the many-pattern workload at a size the
    oracle finishes in seconds on the host's threads; every pattern is checked."""
    from concurrent.futures import ThreadPoolExecutor
    w = synth.many_patterns(n=64_000_000, npat=1024)
    d = api.to_device(w.text)
    n = w.text.size
    got = api.count_merged(d, [0, n], w.patterns, [0] * 1024, list(range(1024)))
    with ThreadPoolExecutor(max_workers=16) as ex:
        want = list(ex.map(lambda p: oracle.count(w.text, p), w.patterns))
    for j, c in enumerate(want):
        assert got[j] == c, j


def _plan_pair_items(b):
    return b.plan.pair_items  # items walked two bytes per step


@pytest.mark.parametrize("step", [1, 2, 0])
def test_pair_and_one_step_automata(step):
    """Two bytes per step (pair automata) and one byte per step give the oracle's counts:
    segments of uneven length, all pattern lengths, a dense periodic text (every pair has a
    reporting state after its first byte) and degenerate queries on both strands."""
    t = api.tune(step_bytes=step, automaton_bytes=64 * 1024) if step else None
    w = synth.uneven_segments(nseg=120, median=30_000, sigma=1.5, lo=1, hi=1_500_000, seed=17)
    say("step", step, "segments", w.seg_off.size - 1, "pairs", w.pair_seg.size)
    check(w.text, w.seg_off, w.patterns, w.pair_seg, w.pair_pat, t)
    b = api.MergedBatch(w.seg_off, w.patterns, w.pair_seg, w.pair_pat, t)
    npi = _plan_pair_items(b)
    assert (npi > 0) if step == 2 else (npi == 0), (step, npi, b.plan.nitems)
    text = synth.genome_like(2_000_003, 47, 0.02, 3000)
    rng = np.random.default_rng(12)
    pats = _mixed_patterns(text, rng, LENGTHS * 3)
    check(text, [0, text.size], pats, [0] * len(pats), list(range(len(pats))), t)
    dense = np.full(700_001, ord("A"), np.uint8)
    dense[::97] = ord("C")
    dp = [b"A", b"AA", b"AAA", b"A" * 8, b"A" * 33, b"CA", b"AC", b"ACA", b"CAAAAAAAAAAAAAAAAAAAAAAAAAAAAAAAAAAC"]
    seg = [0, 1, 2, 3, 100_000, 100_001, 400_000, dense.size]
    ps_ = [s for s in range(len(seg) - 1) for _ in dp]
    pp_ = [j for _ in range(len(seg) - 1) for j in range(len(dp))]
    check(dense, seg, dp, ps_, pp_, t)
    # degenerate queries (one automaton of k-mers and their reverse complements)
    qrng = np.random.default_rng(13)
    codes = []
    for i in range(6):
        c = list(synth.random_pattern(8, qrng).decode())
        c[i % 8] = "BDHV"[i % 4]
        codes.append("".join(c).encode())
    d = api.to_device(text)
    got = api.count_degenerate(d, [0, 1_000_000, text.size], [(i % 2, c, True) for i, c in enumerate(codes)], t)
    seg_d = [(0, 1_000_000), (1_000_000, text.size)]
    for i, c in enumerate(codes):
        lo, hi = seg_d[i % 2]
        assert got[i] == oracle.degenerate_count(text[lo:hi], c, True), c


REG_ALPHABETS = {
    "ACGT": b"ACGT",             # DNA: eight slots, 'N' in a slot of its own
    "ACGTN": b"ACGTN",           # 'N' a pattern byte
    "shift3": bytes([0x00, 0x08, 0x10, 0x18, 0x20]),  # bytes that differ only above bit 2
    "cased": b"acgtACGT",        # eight bytes no three-bit field separates: the class map
    "nine": b"ACGTNRYKM",        # more pattern bytes than slots: the class map
}


@pytest.mark.parametrize("alphabet", sorted(REG_ALPHABETS))
@pytest.mark.parametrize("step", [1, 2, 0])
@pytest.mark.parametrize("line", [32, 64])
def test_register_class_alphabets(alphabet, step, line):
    """Byte classes taken from registers where the patterns' bytes fit eight slots, else
    from the LDS class map: the text mixes the alphabet with other bytes, singly (so that
    the lanes of a wave split between the two) and in runs, and the counts must be the
    oracle's for one-byte and two-byte steps."""
    alpha = np.frombuffer(REG_ALPHABETS[alphabet], np.uint8)
    rng = np.random.default_rng([21, step, line, len(alpha), int(alpha[1])])
    n = 3_000_017
    text = rng.choice(alpha, n)
    idx = rng.integers(0, n, n // 300)
    text[idx] = rng.integers(0, 256, idx.size, dtype=np.uint8)
    for s in rng.integers(0, n - 6000, 24):
        text[s:s + int(rng.integers(1, 6000))] = ord("N") if alphabet != "ACGTN" else ord("n")
    pats = []
    while len(pats) < 24:  # drawn from the text where they use the alphabet only
        m = int(rng.integers(2, 41))
        at = int(rng.integers(0, n - m))
        p = text[at:at + m]
        if np.isin(p, alpha).all():
            pats.append(p.tobytes())
    pats += [rng.choice(alpha, int(rng.integers(1, 12))).tobytes() for _ in range(8)]
    t = api.tune(step_bytes=step, automaton_bytes=64 * 1024, line_bytes=line)
    seg_off = [0, n // 3, n]
    ps_ = [s for s in range(2) for _ in pats]
    pp_ = [j for _ in range(2) for j in range(len(pats))]
    got = check(text, seg_off, pats, ps_, pp_, t)
    say(alphabet, "step", step, "line", line, "matches", int(got.sum()))


def test_wide_alphabet_automata():
    """Automata with more than 128 byte classes keep state numbers in their tables and walk
    every wave on the guarded path; a long pattern of distinct bytes planted in random text,
    next to a DNA pattern set in another segment."""
    rng = np.random.default_rng(31)
    n = 2_000_003
    text = rng.integers(0, 256, n, dtype=np.uint8)
    wide = [bytes(range(1, 141)), bytes(range(96, 256)), bytes(range(255, 90, -1))]
    for p in wide:
        for at in rng.integers(0, n - 300, 40):
            text[at:at + len(p)] = np.frombuffer(p, np.uint8)
    dna = text.copy()
    dna[1_000_000:] = rng.choice(np.frombuffer(b"ACGT", np.uint8), n - 1_000_000)
    pats = wide + [dna[1_500_000:1_500_012].tobytes(), b"ACGTACG", b"A"]
    seg_off = [0, 1_000_000, n]
    got = check(dna, seg_off, pats, [0, 0, 0, 1, 1, 1, 0], [0, 1, 2, 3, 4, 5, 5])
    assert got[0] > 0 and got[1] > 0 and got[3] > 0
