"""CPU model of the device FASTA normaliser's decomposition, checked against the
oracle's definition (oracle/fasta.py).

The device cuts the text into fixed units (one per wave), summarises each unit
on its own (last line start with its header flag, bytes before the first line
start counted apart, kept bytes, header count), combines the summaries in text
order with an associative operator in two levels (blocks of units, then the
blocks before each block), and then writes each unit's kept bytes at the
offset the combination gives.  Its stores are whole aligned 16-byte blocks
in the middle of a unit's output and single bytes at the two partial ends.
This model follows those steps byte by byte with small units and blocks, so
that the order of the combination, its identity, units with no line start,
headers that span units and every output alignment are exercised."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import fasta as ofasta

NL, CR, GT = 0x0A, 0x0D, 0x3E
IDENT = (-1, 0, 0, 0)


def summarise(raw, u0, u1):
    """(last line start as 2 s + header or -1, pre, kept, headers) of raw[u0:u1]."""
    cur, last, pre, kept, hdr = None, -1, 0, 0, 0
    for i in range(u0, u1):
        x = raw[i]
        if i == 0 or raw[i - 1] == NL:
            cur = 2 * i + (x == GT)
            last = cur
            hdr += x == GT
        if x in (NL, CR):
            continue
        if cur is None:
            pre += 1
        elif not cur & 1:
            kept += 1
    return (last, pre, kept, hdr)


def combine(x, y):
    ls = y[0] if y[0] >= 0 else x[0]
    if x[0] < 0:
        return (ls, x[1] + y[1], x[2] + y[2], x[3] + y[3])
    return (ls, x[1], x[2] + (0 if x[0] & 1 else y[1]) + y[2], x[3] + y[3])


def fold(items):
    acc = IDENT
    for it in items:
        acc = combine(acc, it)
    return acc


def plan(sums, block):
    """Exclusive prefix of every unit: block totals, then each block's prefix
    (the blocks before it) combined with the exclusive scan inside it."""
    blocks = [fold(sums[b:b + block]) for b in range(0, len(sums), block)]
    out = []
    for bi, b in enumerate(range(0, len(sums), block)):
        cur = fold(blocks[:bi])
        for s in sums[b:b + block]:
            out.append(cur)
            cur = combine(cur, s)
    return out, fold(blocks)


def write_unit(raw, u0, u1, ls_before):
    """The unit's kept bytes and the offsets (within them) of its record starts."""
    cur = -1 if ls_before >= 0 and ls_before & 1 else -2
    kept, recs = bytearray(), []
    for i in range(u0, u1):
        x = raw[i]
        if i == 0 or raw[i - 1] == NL:
            cur = 2 * i + (x == GT)
            if x == GT:
                recs.append(len(kept))
        if x in (NL, CR) or cur & 1:
            continue
        kept.append(x - 0x20 if 0x61 <= x <= 0x7A else x)
    return bytes(kept), recs


def stores(o_start, o_end, base, round_ends):
    """The device's stores of one unit's output [o_start, o_end) for an output
    buffer at address `base`, flushing after each round (its running output
    end in round_ends): a list of (first byte, length) stores."""
    head_end = o_start + (-(base + o_start)) % 16
    f, head_done, out = o_start, head_end == o_start, []
    for o in round_ends:
        if not head_done and o >= head_end:
            out += [(q, 1) for q in range(o_start, head_end)]
            f, head_done = head_end, True
        if head_done:
            end = o - (base + o) % 16
            q = f
            while q < end:
                assert (base + q) % 16 == 0
                out.append((q, 16))
                q += 16
            f = max(f, end)
    out += [(q, 1) for q in range(f, o_end)]
    return out


def run_model(raw: bytes, unit: int, block: int, rnd: int, base: int):
    n = len(raw)
    units = [(u0, min(u0 + unit, n)) for u0 in range(0, n, unit)]
    sums = [summarise(raw, a, b) for a, b in units]
    pre, total = plan(sums, block)
    assert pre == [fold(sums[:k]) for k in range(len(sums))]  # the two-level order is the plain one
    out = bytearray(total[2] + total[1])
    written = np.zeros(len(out), np.int32)
    starts = []
    for (u0, u1), p in zip(units, pre):
        assert p[1] == 0  # byte 0 starts a line: nothing before the first line start
        kept, recs = write_unit(raw, u0, u1, p[0])
        o_start = p[2]
        out[o_start:o_start + len(kept)] = kept
        starts += [o_start + r for r in recs]
        # the running output end after each round of `rnd` input bytes
        ends, o = [], o_start
        for r0 in range(u0, u1, rnd):
            o += len(write_unit(raw, r0, min(r0 + rnd, u1), 1 if _line_flag(raw, r0) else -1)[0])
            ends.append(o)
        assert o == o_start + len(kept)
        for q, ln in stores(o_start, o_start + len(kept), base, ends):
            assert o_start <= q and q + ln <= o_start + len(kept)
            written[q:q + ln] += 1
    assert (written == 1).all()
    return bytes(out), starts, total


def _line_flag(raw, r0):
    """Whether the line open at byte r0 (started before it) is a header."""
    s = raw.rfind(b"\n", 0, r0)
    return r0 > 0 and raw[s + 1:s + 2] == b">"


def random_fasta(rng, n_rec, max_len):
    out = bytearray()
    if rng.random() < 0.3:
        out += b"acgtn\n"  # a preamble
    for k in range(n_rec):
        nl = b"\r\n" if rng.random() < 0.3 else b"\n"
        out += b">" + b"h" * int(rng.integers(0, 40)) + b" %d" % k + nl
        seq = rng.choice(np.frombuffer(b"ACGTacgtN>", np.uint8), size=int(rng.integers(0, max_len))).tobytes()
        w = int(rng.integers(1, 30))
        for i in range(0, len(seq), w):
            out += seq[i:i + w] + nl
        if rng.random() < 0.2:
            out += nl  # an empty line
    if out and rng.random() < 0.5:
        out = out[:-1]  # no final newline
    return bytes(out)


@pytest.mark.parametrize("seed", range(6))
def test_model_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    raw = random_fasta(rng, int(rng.integers(1, 12)), 300)
    want_seq, want_starts = ofasta.normalize(raw)
    for unit, block, rnd in ((16, 2, 16), (32, 3, 8), (64, 1, 64), (48, 5, 16)):
        for base in (0, 1, 7, 15):
            seq, starts, total = run_model(raw, unit, block, rnd, base)
            assert seq == want_seq and starts == want_starts
            assert total[2] + total[1] == len(want_seq) and total[3] == len(want_starts)


def test_model_edges():
    for raw in (b"", b">", b">only header", b"\n\n\n", b"AC>GT\nT", b">a\n>b\n>c\nA\n",
                b"acgt" * 40, b">" + b"H" * 100 + b"\nacgt", b"\r\n" * 50 + b">x\nA"):
        want = ofasta.normalize(raw)
        for unit in (16, 32):
            seq, starts, _ = run_model(raw, unit, 2, 16, 3)
            assert (seq, starts) == want


def test_combine_is_associative_with_identity():
    rng = np.random.default_rng(5)
    raw = random_fasta(rng, 6, 200)
    cuts = sorted(set(int(c) for c in rng.integers(0, len(raw), size=12)) | {0, len(raw)})
    parts = [summarise(raw, a, b) for a, b in zip(cuts, cuts[1:])]
    for x in parts:
        assert combine(IDENT, x) == x and combine(x, IDENT) == x
    for i in range(len(parts) - 2):
        x, y, z = parts[i:i + 3]
        assert combine(combine(x, y), z) == combine(x, combine(y, z))
    assert fold(parts) == summarise(raw, 0, len(raw))
