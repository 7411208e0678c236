"""Pins of the oracle's multi-pattern automaton (oracle/ac.py).

The automaton is pinned to (a) the paper's worked table (Table 2, with the
one cell that contradicts Fig. 4 corrected; the file header says which), up
to state numbering and the merging of final states with equal rows, and (b)
the window-compare definition of an occurrence, on small random pattern sets.
"""
from __future__ import annotations

import importlib.util
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import ac

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE2 = os.path.join(HERE, "golden", "paper_table2_corrected.txt")
PATS = [b"ACG", b"ACT", b"CTA", b"TGA"]


def _minimize(table, finals, alphabet):
    """Moore partition refinement over the given columns: blocks of states that no
    input over the alphabet can tell apart (final or not)."""
    n = len(table)
    block = [1 if s in finals else 0 for s in range(n)]
    while True:
        sig = {}
        new = []
        for s in range(n):
            key = (block[s],) + tuple(block[table[s][c]] for c in alphabet)
            new.append(sig.setdefault(key, len(sig)))
        if len(set(new)) == len(set(block)):
            return new
        block = new


def _canon(step, finals, alphabet, start=0):
    """Relabel states in breadth-first order from the start state: two automata are the
    same up to numbering iff their canonical forms are equal."""
    order = {start: 0}
    queue = [start]
    rows = []
    while queue:
        s = queue.pop(0)
        row = []
        for c in alphabet:
            t = step(s, c)
            if t not in order:
                order[t] = len(order)
                queue.append(t)
            row.append(order[t])
        rows.append(tuple(row))
    return tuple(rows), frozenset(order[f] for f in finals if f in order)


def test_table2_corrected_is_the_minimal_total_count_automaton():
    a = ac.build(PATS)
    assert a.nstates == 11 and a.nstates - a.first_final == 4  # one state per prefix, one final per pattern
    # every byte outside the patterns' letters leads back to the start state
    other = [c for c in range(256) if c not in b"ACGT"]
    assert (a.table[:, other] == 0).all()
    finals = set(range(a.first_final, a.nstates))
    alphabet = list(b"ACGT")
    blk = _minimize(a.table, finals, alphabet)
    nb = max(blk) + 1
    qt = [[0] * 256 for _ in range(nb)]
    for s in range(a.nstates):
        for c in alphabet:
            qt[blk[s]][c] = blk[a.table[s, c]]
    qfinals = {blk[s] for s in finals}
    mine = _canon(lambda s, c: qt[s][c], qfinals, alphabet, blk[0])
    rows, gfinals = ac.total_count_table(TABLE2)
    assert len(rows) == 10 and gfinals == {6, 7, 8}
    golden = _canon(lambda s, c: ac.step_table(rows, s, c), gfinals, alphabet)
    assert nb == 10
    assert mine == golden


def _walk_total(rows, finals, text):
    q, n = 0, 0
    for c in text:
        q = ac.step_table(rows, q, c)
        n += q in finals
    return n


def test_table2_corrected_counts_every_short_text_exactly():
    rows, finals = ac.total_count_table(TABLE2)
    for L in range(0, 8):
        for t in itertools.product(b"ACGT", repeat=L):
            text = bytes(t)
            want = sum(oracle.count(np.frombuffer(text, np.uint8), p) for p in PATS) if L else 0
            assert _walk_total(rows, finals, text) == want, text


def test_table2_as_printed_miscounts():
    rows, finals = ac.total_count_table(TABLE2)
    printed = {k: dict(v) for k, v in rows.items() if k != 9}
    printed[3][ord("T")] = 5
    text = b"CTGA"  # holds tga once
    assert _walk_total(printed, finals, text) == 0
    assert _walk_total(rows, finals, text) == 1


def _random_set(rng, k, lo, hi, alphabet=b"ACGT"):
    out = []
    for _ in range(k):
        m = int(rng.integers(lo, hi + 1))
        out.append(bytes(rng.choice(list(alphabet), size=m).tolist()))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_ac_counts_equal_window_definition(seed):
    rng = np.random.default_rng(seed)
    pats = _random_set(rng, int(rng.integers(1, 9)), 1, 6)
    # nested and repeated patterns: a suffix, a prefix and a duplicate of the first one
    p0 = pats[0]
    pats += [p0[1:] or p0, p0[:-1] or p0, p0]
    if seed % 2:
        pats.append(b"N" + p0)  # a byte outside ACGT inside a pattern
    text = bytes(rng.choice(list(b"ACGTN"), size=3000, p=[0.27, 0.23, 0.23, 0.23, 0.04]).tolist())
    a = ac.build(pats)
    got = ac.counts(a, text, len(pats))
    want = np.array([oracle.count(np.frombuffer(text, np.uint8), p) for p in pats])
    assert np.array_equal(got, want)


def test_ac_structure():
    rng = np.random.default_rng(11)
    pats = _random_set(rng, 6, 2, 7)
    a = ac.build(pats)
    prefixes = {p[:i] for p in pats for i in range(len(p) + 1)}
    assert a.nstates == len(prefixes) and a.states[0] == b""
    for s, outs in zip(a.states, a.outputs):
        assert outs == [i for i, p in enumerate(pats) if s.endswith(p)]
    # finals numbered last
    isf = [bool(o) for o in a.outputs]
    assert isf == [i >= a.first_final for i in range(a.nstates)]
    # single pattern: the automaton is the single-pattern table of oracle.c
    p = b"ACAACG"
    one = ac.build([p])
    assert np.array_equal(one.table, oracle.transition_table(p).astype(np.int32))


MUTANTS = [
    # longest suffix -> shortest suffix
    ("for k in range(len(t), -1, -1):", "for k in range(0, len(t) + 1):"),
    # report patterns that are prefixes instead of suffixes
    ("if s.endswith(p)]", "if s.startswith(p)]"),
    # finals numbered first
    ("states = plain + finals", "states = finals + plain"),
    # drop the last byte of the suffix search window
    ("suf = t[len(t) - k:]", "suf = t[len(t) - k:len(t) - (1 if k else 0)]"),
]


@pytest.mark.parametrize("i", range(len(MUTANTS)))
def test_pins_catch_planted_mistakes(i, tmp_path):
    src = open(ac.__file__).read()
    old, new = MUTANTS[i]
    assert src.count(old) == 1
    path = tmp_path / f"ac_mut{i}.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"ac_mut{i}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = False
    try:
        a = mod.build(PATS)
        if a.nstates != 11 or a.nstates - a.first_final != 4:
            caught = True
        rng = np.random.default_rng(3)
        for _ in range(3):
            pats = _random_set(rng, 4, 1, 5)
            text = bytes(rng.choice(list(b"ACGT"), size=400).tolist())
            b = mod.build(pats)
            got = mod.counts(b, text, len(pats))
            want = np.array([oracle.count(np.frombuffer(text, np.uint8), p) for p in pats])
            if not np.array_equal(got, want) or any(bool(o) != (k >= b.first_final) for k, o in enumerate(b.outputs)):
                caught = True
    except Exception:
        caught = True
    assert caught
