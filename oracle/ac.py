"""Multi-pattern automaton by its definition (test infrastructure only).

The paper's improved Aho-Corasick automaton (Sec. "Implementation Aspects",
Fig. 4 and Table 2) has one state per distinct prefix of the patterns and a
transition for every byte: from state s on byte c it moves to the longest
suffix of s.c that is itself a prefix of some pattern (no failure links are
followed at scan time).  State s reports every pattern that is a suffix of s.
States that report something are numbered last, so "is final" is one
comparison against the first final state.

Everything here is brute force over strings -- states are kept as the prefix
strings themselves -- and meant for small pattern sets only.  Parity of the
GPU path is checked on per-pattern counts against the window-compare
definition in oracle.c; this module pins the automaton the batched path is
built from.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


class Automaton:
    def __init__(self, states, table, first_final, outputs):
        self.states = states            # list[bytes]: the prefix each state stands for
        self.table = table              # int32[nstates, 256]
        self.first_final = first_final  # states >= first_final report at least one pattern
        self.outputs = outputs          # list[list[int]]: pattern indices reported by each state

    @property
    def nstates(self) -> int:
        return len(self.states)


def build(patterns: Sequence[bytes]) -> Automaton:
    pats = [bytes(p) for p in patterns]
    prefixes = {b""}
    for p in pats:
        if not p:
            raise ValueError("empty pattern")
        for i in range(1, len(p) + 1):
            prefixes.add(p[:i])
    # states in order of prefix length, then bytes; the empty prefix is state 0
    order = sorted(prefixes, key=lambda s: (len(s), s))
    outputs_of = {s: [i for i, p in enumerate(pats) if s.endswith(p)] for s in order}
    plain = [s for s in order if not outputs_of[s]]
    finals = [s for s in order if outputs_of[s]]
    states = plain + finals
    index = {s: i for i, s in enumerate(states)}
    table = np.zeros((len(states), 256), dtype=np.int32)
    for s in states:
        for c in range(256):
            t = s + bytes([c])
            # longest suffix of t that is a prefix of some pattern (the empty one always is)
            for k in range(len(t), -1, -1):
                suf = t[len(t) - k:]
                if suf in index:
                    table[index[s], c] = index[suf]
                    break
    return Automaton(states, table, len(plain), [outputs_of[s] for s in states])


def counts(a: Automaton, text: bytes, npat: int) -> np.ndarray:
    """Per-pattern occurrence counts: walk the text from state 0 and add one to every
    pattern the state reports after each byte."""
    out = np.zeros(npat, dtype=np.int64)
    q = 0
    for c in bytes(text):
        q = int(a.table[q, c])
        if q >= a.first_final:
            for i in a.outputs[q]:
                out[i] += 1
    return out


def total_count_table(path: str):
    """Read a worked table file: rows "state next..." under a "#! columns" line naming the
    bytes of the columns, and a "#! finals" line.  Returns (rows as dict state ->
    {byte: next}, set of finals)."""
    rows, finals, cols = {}, set(), None
    for ln in open(path):
        ln = ln.strip()
        if ln.startswith("#! finals"):
            finals = {int(x) for x in ln.split()[2:]}
            continue
        if ln.startswith("#! columns"):
            cols = [ord(x) for x in ln.split()[2:]]
            continue
        if not ln or ln.startswith("#"):
            continue
        v = [int(x) for x in ln.split()]
        rows[v[0]] = dict(zip(cols, v[1:]))
    return rows, finals


def step_table(rows, q: int, c: int) -> int:
    """Next state of a worked table: the listed columns, state 0 for every other byte."""
    return rows[q].get(c, 0)


__all__: List[str] = ["Automaton", "build", "counts", "total_count_table", "step_table"]
