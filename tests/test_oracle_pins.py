"""Pins for the CPU oracle against things other than itself.

* Python's ``re`` engine with a zero-width lookahead, an independent library
  routine that reports every overlapping occurrence of a literal;
* textbook values: the string-matching automaton for "ababaca" and the prefix
  function of "ababababca" (Cormen et al., Introduction to Algorithms, 3rd ed.,
  Sections 32.3-32.4), stored under tests/golden/;
* closed forms on periodic texts, additivity over concatenation, reverse
  symmetry, absence by construction, planted occurrences and the expected
  count of a k-mer in i.i.d. text.

Each check takes an oracle instance so the last test can rebuild the oracle
with a plausible mistake planted in a copy of its C source and show that some
pin fails for every such mutant.
"""
from __future__ import annotations

import itertools
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from oracle import OracleLib
from paper_1506_08612_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def regex_starts(text: bytes, pat: bytes) -> np.ndarray:
    return np.array([mm.start() for mm in re.finditer(b"(?=" + re.escape(pat) + b")", text)],
                    dtype=np.int64)


def walk_state(table: np.ndarray, s: bytes) -> int:
    q = 0
    for b in s:
        q = int(table[q, b])
    return q


def rand_text(rng, n, alphabet=b"ACGT"):
    a = np.frombuffer(alphabet, dtype=np.uint8)
    return a[rng.integers(0, a.size, n)].tobytes()


# ----------------------------------------------------------------------------------------
# checks (each raises AssertionError on a violated pin)
# ----------------------------------------------------------------------------------------

def check_textbook_automaton(O):
    rows = [list(map(int, ln.split())) for ln in open(os.path.join(GOLDEN, "clrs_ababaca_delta.txt"))
            if ln.strip() and not ln.startswith("#")]
    tab = O.transition_table(b"ababaca")
    assert tab.shape == (8, 256)
    for q, a, b, c in rows:
        assert (tab[q, ord("a")], tab[q, ord("b")], tab[q, ord("c")]) == (a, b, c), q
    others = np.ones(256, bool)
    others[[ord("a"), ord("b"), ord("c")]] = False
    assert not tab[:, others].any()


def check_prefix_function(O):
    lines = [ln.strip() for ln in open(os.path.join(GOLDEN, "clrs_prefix_function.txt"))
             if ln.strip() and not ln.startswith("#")]
    pat = lines[0].encode()
    pi = list(map(int, lines[1].split()))
    tab = O.transition_table(pat)
    # the longest proper border of P[:q] is the longest prefix of P that is a suffix of P[1:q],
    # i.e. the state reached by reading P[1:q] from q0
    for q in range(1, len(pat) + 1):
        assert walk_state(tab, pat[1:q]) == pi[q - 1], q


def check_regex_exhaustive(O, maxlen=9):
    pats = [bytes(p) for L in range(1, 4) for p in itertools.product(b"AC", repeat=L)]
    tabs = {p: O.transition_table(p) for p in pats}
    for L in range(0, maxlen + 1):
        for t in itertools.product(b"AC", repeat=L):
            t = bytes(t)
            for p in pats:
                want = regex_starts(t, p)
                got = O.occurrences(t, p)
                assert np.array_equal(got, want), (t, p, got, want)
                assert np.array_equal(O.automaton_scan(tabs[p], t), want), (t, p)


def check_regex_random(O, cases=150, seed=11):
    rng = np.random.default_rng(seed)
    for k in range(cases):
        alpha = [b"AC", b"ACGT", b"ACGTN", bytes(range(256))][k % 4]
        n = int(rng.integers(0, 3000))
        t = rand_text(rng, n, alpha)
        m = int(rng.integers(1, 13))
        if n >= m and rng.random() < 0.5:
            o = int(rng.integers(0, n - m + 1))
            p = t[o:o + m]
        else:
            p = rand_text(rng, m, alpha[:4] if len(alpha) > 4 else alpha)
        want = regex_starts(t, p)
        assert np.array_equal(O.occurrences(t, p), want), (k, n, p)
        assert O.count(t, p) == want.size
        assert np.array_equal(O.automaton_scan(O.transition_table(p), t), want), (k, n, p)


def check_closed_forms(O):
    for n in (1, 5, 64, 1000):
        for m in (1, 2, 7, 64):
            got = O.occurrences(b"A" * n, b"A" * m)
            exp = np.arange(0, max(0, n - m + 1), dtype=np.int64)
            assert np.array_equal(got, exp), (n, m)
    for k in (1, 2, 3, 50, 777):
        t = b"AC" * k
        assert np.array_equal(O.occurrences(t, b"ACA"), np.arange(0, 2 * k - 3, 2)), k
        t = b"AAC" * k
        assert O.count(t, b"AACAA") == max(0, k - 1), k
        t = b"ACGT" * k
        for s in range(4):
            p = (b"ACGT" * 3)[s:s + 5]
            exp = [i for i in range(s, 4 * k - 4, 4) if i + 5 <= 4 * k]
            assert O.occurrences(t, p).tolist() == exp, (k, s)


def check_additivity(O, cases=60, seed=12):
    rng = np.random.default_rng(seed)
    for _ in range(cases):
        m = int(rng.integers(1, 10))
        a = rand_text(rng, int(rng.integers(0, 400)), b"AC")
        b = rand_text(rng, int(rng.integers(0, 400)), b"AC")
        p = rand_text(rng, m, b"AC")
        # occurrences that start in the last m-1 bytes of a and run into b
        border = a[max(0, len(a) - m + 1):] + b[:m - 1]
        bstart = max(0, len(a) - m + 1)
        cross = [bstart + i for i in regex_starts(border, p).tolist()
                 if bstart + i < len(a) < bstart + i + m]
        whole = O.occurrences(a + b, p).tolist()
        parts = O.occurrences(a, p).tolist() + sorted(cross) + \
            [len(a) + i for i in O.occurrences(b, p).tolist()]
        assert whole == parts, (a, b, p)


def check_reverse(O, cases=60, seed=13):
    rng = np.random.default_rng(seed)
    for _ in range(cases):
        n = int(rng.integers(0, 2000))
        m = int(rng.integers(1, 8))
        t = rand_text(rng, n, b"ACG")
        p = rand_text(rng, m, b"ACG")
        fwd = O.occurrences(t, p)
        bwd = O.occurrences(t[::-1], p[::-1])
        assert sorted((n - m - bwd).tolist()) == fwd.tolist()


def check_absent(O, seed=14):
    rng = np.random.default_rng(seed)
    t = rand_text(rng, 20000, b"ACG")
    for m in (1, 4, 16, 64):
        p = bytearray(rand_text(rng, m, b"ACG"))
        p[int(rng.integers(0, m))] = ord("T")
        assert O.count(t, bytes(p)) == 0
    # an 'N' run wider than the pattern separates two halves that each hold half of it
    p = rand_text(rng, 12, b"ACGT")
    t = p[:6] + b"N" * 50 + p[6:]
    assert O.count(t, p) == 0
    assert O.count(t, b"N" * 50) == 1 and O.count(t, b"N" * 51) == 0


def check_planted(O):
    w = synth.tiny_uniform(1 << 16, 8, seed=0)
    pos = O.occurrences(w.text, w.patterns[0])
    assert w.offsets[0] in pos.tolist()
    for i in pos.tolist():
        assert w.text[i:i + 8].tobytes() == w.patterns[0]


def check_table_structure(O, cases=40, seed=15):
    rng = np.random.default_rng(seed)
    for k in range(cases):
        m = int(rng.integers(1, 40)) if k else 255
        p = rand_text(rng, m, b"ACGT" if k % 2 else b"AC")
        tab = O.transition_table(p)
        assert tab.shape == (m + 1, 256)
        for q in range(m):
            assert tab[q, p[q]] == q + 1
        absent = np.ones(256, bool)
        absent[list(set(p))] = False
        assert not tab[:, absent].any()
        assert (tab <= np.minimum(np.arange(m + 1) + 1, m)[:, None]).all()
        # from the final state the automaton must keep finding overlapping matches
        assert np.array_equal(O.automaton_scan(tab, p + p), regex_starts(p + p, p))


def check_pair_counts(O, seed=16):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 700, size=9)
    seg_off = np.concatenate(([0], np.cumsum(lens))).astype(np.int64)
    text = rand_text(rng, int(seg_off[-1]), b"AC")
    pats = [rand_text(rng, int(rng.integers(1, 6)), b"AC") for _ in range(7)]
    ps, pp = [], []
    for s in range(lens.size):
        for j in rng.choice(len(pats), size=3, replace=False).tolist():
            ps.append(s)
            pp.append(j)
    got = O.pair_counts(text, seg_off, pats, ps, pp)
    for k, (s, j) in enumerate(zip(ps, pp)):
        seg = text[seg_off[s]:seg_off[s + 1]]
        assert got[k] == regex_starts(seg, pats[j]).size, (s, j)
    # a match that straddles a segment border belongs to neither segment
    got = O.pair_counts(b"ACGTAC" + b"GT", [0, 6, 8], [b"ACGT"], [0, 1], [0, 0])
    assert got.tolist() == [1, 0]


def check_edges(O):
    assert O.count(b"", b"A") == 0
    assert O.count(b"ACG", b"ACGT") == 0
    assert O.occurrences(b"ACGT", b"ACGT").tolist() == [0]
    with pytest.raises(ValueError):
        O.count(b"ACGT", b"")
    with pytest.raises(ValueError):
        O.transition_table(b"A" * 256)
    tab = O.transition_table(b"G")
    assert tab[0, ord("G")] == 1 and tab[1, ord("G")] == 1 and tab.sum() == 2


def check_expected_count(O, seed=17):
    # i.i.d. uniform text: a pattern with no proper border occurs (n-m+1)/4^m times on
    # average, with variance below the mean; allow 6 standard deviations
    n = 1 << 21
    rng = np.random.default_rng(seed)
    t = rand_text(rng, n)
    for p in (b"ACCCCC", b"AGTTTT", b"CAAAAG"[::-1][:5] + b"T"):
        e = (n - len(p) + 1) / 4 ** len(p)
        assert abs(O.count(t, p) - e) < 6 * np.sqrt(e) + 1, p


ALL_CHECKS = [check_textbook_automaton, check_prefix_function, check_regex_exhaustive,
              check_regex_random, check_closed_forms, check_additivity, check_reverse,
              check_absent, check_planted, check_table_structure, check_pair_counts,
              check_edges, check_expected_count]


@pytest.mark.parametrize("check", ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(check):
    check(oracle._load() if hasattr(oracle, "_load") else oracle.oracle._load())


# ----------------------------------------------------------------------------------------
# the pins catch plausible mistakes planted in a copy of the oracle
# ----------------------------------------------------------------------------------------

MUTANTS = [
    ("drop the last window", "i + m <= n", "i + m < n"),
    ("ignore the last pattern byte", "while (j < m && text", "while (j + 1 < m && text"),
    ("report the end instead of the start", "pos[count] = i;", "pos[count] = i + m - 1;"),
    ("non-overlapping matches", "if (count < cap) pos[count] = i;\n            ++count;",
     "if (count < cap) pos[count] = i;\n            ++count;\n            i += m - 1;"),
    ("never advance past q", "int64_t k = (q + 1 < m) ? q + 1 : m;",
     "int64_t k = (q < m) ? q : m;"),
    ("wrong border index", "pat[q - k + 1 + j]", "pat[q - k + j]"),
    ("wrong last-byte index", "if (pat[k - 1] != (uint8_t)b)", "if (pat[k] != (uint8_t)b)"),
    ("automaton reports the end", "pos[count] = c - m + 1;", "pos[count] = c - m;"),
    ("segment end off by one", "oracle_occurrences(text + lo, hi - lo,",
     "oracle_occurrences(text + lo, hi - lo - 1,"),
    ("segments read one byte early", "oracle_occurrences(text + lo, hi - lo,",
     "oracle_occurrences(text + lo - (lo > 0), hi - lo,"),
]


def _build_mutant(src: str, d: str, k: int) -> OracleLib:
    path = os.path.join(d, f"m{k}.c")
    open(path, "w").write(src)
    so = os.path.join(d, f"libm{k}.so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", so, path])
    return OracleLib(so)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_pins_catch_planted_mistakes():
    src = open(os.path.join(os.path.dirname(oracle.lib_path()), "oracle.c")).read()
    with tempfile.TemporaryDirectory() as d:
        for k, (name, old, new) in enumerate(MUTANTS):
            assert src.count(old) == 1, name
            O = _build_mutant(src.replace(old, new), d, k)
            failed = []
            for check in ALL_CHECKS:
                try:
                    if check is check_regex_exhaustive:
                        check(O, maxlen=7)
                    else:
                        check(O)
                except (AssertionError, ValueError, IndexError):
                    failed.append(check.__name__)
            assert failed, f"no pin caught the mutant '{name}'"
