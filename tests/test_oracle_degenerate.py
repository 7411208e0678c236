"""Pins of the oracle's degenerate-pattern count (IUPAC codes, optional reverse
complement strand): Python's regex engine with character classes and a zero-width
lookahead, brute-force expansion into plain k-mers, closed forms, and the
reverse-complement identities."""
from __future__ import annotations

import itertools
import re

import numpy as np
import pytest

import oracle

CLASSES = {"A": "A", "C": "C", "G": "G", "T": "T", "R": "AG", "Y": "CT", "S": "CG", "W": "AT",
           "K": "GT", "M": "AC", "B": "CGT", "D": "AGT", "H": "ACT", "V": "ACG", "N": "ACGT"}
COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def regex_of(code: str) -> str:
    return "".join(f"[{CLASSES[c]}]" for c in code)


def revcomp_code(code: str) -> str:
    # complement each code as a set of bases, then reverse
    inv = {v: k for k, v in CLASSES.items()}
    out = []
    for c in reversed(code):
        bases = "".join(sorted(COMP[b] for b in CLASSES[c]))
        out.append(inv[bases])
    return "".join(out)


def regex_count(text: bytes, code: str, both: bool) -> int:
    pat = regex_of(code)
    if both:
        pat = f"(?:{pat}|{regex_of(revcomp_code(code))})"
    return sum(1 for _ in re.finditer(f"(?={pat})", text.decode("latin-1")))


def random_code(rng, m, degenerate_frac=0.3):
    out = []
    for _ in range(m):
        if rng.random() < degenerate_frac:
            out.append(rng.choice(list("RYSWKMBDHVN")))
        else:
            out.append(rng.choice(list("ACGT")))
    return "".join(out)


@pytest.mark.parametrize("seed", range(10))
def test_matches_regex_engine(seed):
    rng = np.random.default_rng(seed)
    text = bytes(rng.choice(list(b"ACGTN"), size=4000, p=[0.28, 0.22, 0.22, 0.25, 0.03]).tolist())
    for _ in range(6):
        code = random_code(rng, int(rng.integers(1, 10)))
        for both in (False, True):
            assert oracle.degenerate_count(text, code.encode(), both) == regex_count(text, code, both), (code, both)


def test_equals_union_of_expanded_kmers():
    rng = np.random.default_rng(7)
    text = np.frombuffer(bytes(rng.choice(list(b"ACGT"), size=20000).tolist()), np.uint8)
    for _ in range(8):
        code = random_code(rng, 6, 0.4)
        kmers = {"".join(t) for t in itertools.product(*[CLASSES[c] for c in code])}
        kmers |= {"".join(t) for t in itertools.product(*[CLASSES[c] for c in revcomp_code(code)])}
        want = sum(oracle.count(text, k.encode()) for k in kmers)  # equal-length k-mers: at most one per position
        assert oracle.degenerate_count(text, code.encode(), True) == want, code


def test_closed_forms_and_identities():
    text = np.frombuffer(b"ACGT" * 1000, np.uint8)
    assert oracle.degenerate_count(text, b"N", False) == 4000
    assert oracle.degenerate_count(text, b"NNNN", True) == 3997
    assert oracle.degenerate_count(text, b"R", False) == 2000          # A or G
    assert oracle.degenerate_count(text, b"ACGT", False) == 1000
    assert oracle.degenerate_count(text, b"ACGT", True) == 1000        # ACGT is its own reverse complement
    assert oracle.degenerate_count(text, b"CGTA", True) == 999 + 999   # CGTA and its reverse complement TACG
    nn = np.frombuffer(b"NNNNACGTNNNN", np.uint8)
    assert oracle.degenerate_count(nn, b"N", False) == 4              # a text N is no base
    assert oracle.degenerate_count(nn, b"NN", False) == 3
    # reverse complement of the reverse complement is the code itself
    rng = np.random.default_rng(3)
    for _ in range(20):
        c = random_code(rng, 7, 0.5)
        assert revcomp_code(revcomp_code(c)) == c
        t = bytes(rng.choice(list(b"ACGT"), size=500).tolist())
        assert (oracle.degenerate_count(t, c.encode(), True) ==
                oracle.degenerate_count(t, revcomp_code(c).encode(), True))


def test_rejects_bad_codes():
    with pytest.raises(ValueError):
        oracle.degenerate_count(b"ACGT", b"AXG", False)
    with pytest.raises(ValueError):
        oracle.degenerate_count(b"ACGT", b"acg", False)


DEGENERATE_MUTANTS = [
    ("complement keeps the base", "if (b & 1) r |= 8;", "if (b & 1) r |= 1;"),
    ("reverse complement not reversed", "rc[m - 1 - j] = iupac_complement(pat[j]);", "rc[j] = iupac_complement(pat[j]);"),
    ("text N matches N", "    default: return 0;\n    }\n}\n\n/* The complement",
     "    case 'N': return 1 | 2 | 4 | 8;\n    default: return 0;\n    }\n}\n\n/* The complement"),
    ("both strands counted twice", "if (degenerate_at(text, i, pat, m) || (both_strands && degenerate_at(text, i, rc, m))) ++count;",
     "count += degenerate_at(text, i, pat, m) + (both_strands && degenerate_at(text, i, rc, m));"),
    ("R read as A or C", "case 'R': return 1 | 4;", "case 'R': return 1 | 2;"),
]


def test_degenerate_pins_catch_planted_mistakes(tmp_path):
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    src = open(oracle.lib_path().replace("liboracle.so", "oracle.c")).read()
    for k, (name, old, new) in enumerate(DEGENERATE_MUTANTS):
        assert src.count(old) == 1, name
        c = tmp_path / f"d{k}.c"
        c.write_text(src.replace(old, new))
        so = tmp_path / f"libd{k}.so"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", str(so), str(c)])
        O = oracle.OracleLib(str(so))
        failed = False
        rng = np.random.default_rng(k)
        try:
            for _ in range(12):
                text = bytes(rng.choice(list(b"ACGTN"), size=600, p=[0.27, 0.23, 0.23, 0.23, 0.04]).tolist())
                code = random_code(rng, int(rng.integers(1, 7)), 0.5)
                for both in (False, True):
                    if O.degenerate_count(text, code.encode(), both) != regex_count(text, code, both):
                        failed = True
        except ValueError:
            failed = True
        assert failed, f"no pin caught the mutant '{name}'"
