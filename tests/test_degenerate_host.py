"""Host tests of degenerate (IUPAC) pattern expansion, dfa_degenerate_expand."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from paper_1506_08612_amd import api

CLASSES = {"A": "A", "C": "C", "G": "G", "T": "T", "R": "AG", "Y": "CT", "S": "CG", "W": "AT",
           "K": "GT", "M": "AC", "B": "CGT", "D": "AGT", "H": "ACT", "V": "ACG", "N": "ACGT"}
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def brute(code: str, both: bool):
    out = {"".join(t) for t in itertools.product(*[CLASSES[c] for c in code])}
    if both:
        out |= {"".join(COMP[b] for b in reversed(k)) for k in out}
    return sorted(k.encode() for k in out)


@pytest.mark.parametrize("seed", range(8))
def test_expansion_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    for _ in range(10):
        m = int(rng.integers(1, 9))
        code = "".join(rng.choice(list("ACGTRYSWKMBDHVN")) if rng.random() < 0.4 else rng.choice(list("ACGT"))
                       for _ in range(m))
        for both in (False, True):
            assert api.expand_degenerate(code.encode(), both) == brute(code, both), (code, both)


def test_palindromes_and_sizes():
    assert api.expand_degenerate(b"ACGT", True) == [b"ACGT"]          # its own reverse complement
    assert len(api.expand_degenerate(b"N" * 5, False)) == 4 ** 5
    assert len(api.expand_degenerate(b"N" * 5, True)) == 4 ** 5       # the set is closed under reverse complement
    assert api.expand_degenerate(b"AAAC", True) == [b"AAAC", b"GTTT"]


def test_expansion_errors():
    for bad in (b"", b"ACX", b"acg", b"N" * 11):  # empty, not a code, lower case, 4^11 > 2^20
        with pytest.raises(api.DfaError):
            api.expand_degenerate(bad, False)
    c = np.frombuffer(b"NN", np.uint8).copy()
    out = np.empty(2 * 3, np.uint8)
    assert api.lib.dfa_degenerate_expand(c.ctypes.data, 2, 0, out.ctypes.data, 3) == api.DFA_ENOSPACE
