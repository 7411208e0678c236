"""GPU parity of degenerate-pattern counting (IUPAC codes, optional reverse complement)
against the oracle's per-position definition: bit-exact."""
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


def table3_like(rng, k=9, m=8):
    """Random m-mers, each with one position replaced by a 3-way class (IUPAC B, D, H or V)."""
    out = []
    for i in range(k):
        s = list(synth.random_pattern(m, rng).decode())
        s[i % m] = "BDHV"[int(rng.integers(0, 4))]
        out.append("".join(s).encode())
    return out


def check(text, seg_off, queries):
    d = api.to_device(text)
    got = api.count_degenerate(d, seg_off, queries)
    want = np.array([oracle.degenerate_count(text[seg_off[s]:seg_off[s + 1]], code, both)
                     for s, code, both in queries], dtype=np.int64)
    assert np.array_equal(got, want), [(q, int(g), int(w)) for q, g, w in zip(queries, got, want) if g != w][:5]
    return got


def test_table3_structure_both_strands():
    text = synth.genome_like(4_000_000, 51, 0.02, 3000)
    rng = np.random.default_rng(1)
    codes = table3_like(rng) + [synth.random_pattern(8, rng)]
    seg_off = [0, 1_000_003, 1_000_003, 2_500_000, text.size]
    queries = [(s, c, True) for s in range(4) for c in codes]
    say("table-3-like queries", len(queries))
    got = check(text, seg_off, queries)
    assert got.sum() > 0


def test_longer_codes_single_and_both_strands():
    text = synth.genome_like(2_000_000, 52, 0.02, 2000)
    rng = np.random.default_rng(2)
    queries = []
    for i in range(12):
        m = int(rng.integers(6, 24))
        s = list(synth.random_pattern(m, rng).decode())
        for _ in range(int(rng.integers(1, 4))):
            s[int(rng.integers(0, m))] = "RYSWKMBDHVN"[int(rng.integers(0, 11))]
        queries.append((0, "".join(s).encode(), bool(i % 2)))
    check(text, [0, text.size], queries)


def test_many_expansions_and_palindromes():
    rng = np.random.default_rng(3)
    text = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, 600_000)].copy()
    queries = [(0, b"NNNNNN", False), (0, b"NNNNNN", True), (0, b"ACGT", True), (0, b"ACNGT", True),
               (0, b"A", True), (0, b"W", False)]
    got = check(text, [0, text.size], queries)
    assert got[0] == got[1] == text.size - 5
