"""Pins of the oracle's FASTA normalisation (oracle/fasta.py): a worked example written
out by hand, invariance under line width and line endings, case folding against
bytes.upper(), and a round trip through a FASTA writer."""
from __future__ import annotations

import importlib.util

import numpy as np
import pytest

from oracle import fasta


def test_worked_example():
    raw = b">chr1 first\nACGTacgt\nNNac\n>chr2\r\ngg\r\nTT\n\n>empty\n>chr4\nA"
    seq, starts = fasta.normalize(raw)
    assert seq == b"ACGTACGTNNACGGTTA"
    assert starts == [0, 12, 16, 16]
    assert fasta.normalize(b"") == (b"", [])
    assert fasta.normalize(b"acgt\n>r\nAA") == (b"ACGTAA", [4])       # a preamble before the first header
    assert fasta.normalize(b"AC>GT\n") == (b"AC>GT", [])              # '>' inside a line is kept
    assert fasta.normalize(b">only a header") == (b"", [0])


def _write(records, width, crlf=False, lower_runs=()):
    nl = b"\r\n" if crlf else b"\n"
    out = bytearray()
    for k, (name, seq) in enumerate(records):
        s = bytearray(seq)
        for (a, b) in lower_runs:
            s[a:b] = s[a:b].lower()
        out += b">" + name + nl
        for i in range(0, len(s), width):
            out += bytes(s[i:i + width]) + nl
    return bytes(out)


@pytest.mark.parametrize("seed", range(5))
def test_round_trip_any_width_and_line_ending(seed):
    rng = np.random.default_rng(seed)
    recs = []
    for k in range(int(rng.integers(1, 6))):
        n = int(rng.integers(0, 3000))
        recs.append((f"seq{k} desc".encode(), bytes(rng.choice(list(b"ACGTN"), size=n).tolist())))
    want_seq = b"".join(s for _, s in recs)
    want_starts = list(np.cumsum([0] + [len(s) for _, s in recs])[:-1])
    for width in (1, 7, 60, 70, 80, 4096):
        for crlf in (False, True):
            raw = _write(recs, width, crlf, lower_runs=[(10, 50), (200, 260)])
            seq, starts = fasta.normalize(raw)
            assert seq == want_seq and starts == want_starts, (width, crlf)


def test_case_folding_matches_bytes_upper():
    rng = np.random.default_rng(9)
    body = bytes(rng.integers(32, 127, size=5000, dtype=np.uint8).tolist()).replace(b">", b"")
    seq, _ = fasta.normalize(b">h\n" + body)
    assert seq == body.upper()


MUTANTS = [
    ("headers kept", "            starts.append(len(out))\n            continue", "            starts.append(len(out))"),
    ("carriage returns kept", "            if b == 0x0D:  # '\\r'\n                continue\n", ""),
    ("no case folding", "                b -= 0x20", "                pass"),
    ("record start after the header's bytes", "starts.append(len(out))", "starts.append(len(out) + 1)"),
]


@pytest.mark.parametrize("i", range(len(MUTANTS)))
def test_pins_catch_planted_mistakes(i, tmp_path):
    src = open(fasta.__file__).read()
    name, old, new = MUTANTS[i]
    assert src.count(old) == 1, name
    p = tmp_path / f"fasta_mut{i}.py"
    p.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"fasta_mut{i}", p)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = False
    try:
        if mod.normalize(b">chr1 first\nACGTacgt\nNNac\n>chr2\r\ngg\r\nTT\n\n>empty\n>chr4\nA") != (
                b"ACGTACGTNNACGGTTA", [0, 12, 16, 16]):
            caught = True
    except Exception:
        caught = True
    assert caught, name
