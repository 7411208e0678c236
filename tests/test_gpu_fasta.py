"""GPU parity of FASTA normalisation (dfa_fasta_normalize) against the oracle's
definition (oracle/fasta.py): kept bytes and record starts bit-exact, including
headers and line breaks that straddle the kernel's 32 KiB units (one per wave),
its 1 KiB rounds and 16-byte lane pieces, outputs at every alignment, texts
that span several blocks of the plan; then counts on the normalised records."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from oracle import fasta as ofasta
from paper_1506_08612_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1506_08612_amd import api  # noqa: E402

UNIT = 32 * 1024      # bytes per wave
ROUND = 1024          # bytes per wave and round
PLAN_BLOCK = 2048     # units per block of the plan
TWO = 2 * UNIT        # two units: every multiple of it is a unit border too


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def write_fasta(records, width, rng, crlf_frac=0.0, lower_frac=0.0):
    out = bytearray()
    for name, seq in records:
        nl = b"\r\n" if rng.random() < crlf_frac else b"\n"
        out += b">" + name + nl
        s = bytearray(seq)
        if lower_frac and len(s):
            for _ in range(3):
                a = int(rng.integers(0, len(s)))
                b = min(len(s), a + int(rng.integers(1, 5000)))
                s[a:b] = s[a:b].lower()
        for i in range(0, len(s), width):
            out += bytes(s[i:i + width]) + nl
    return bytes(out)


def check(raw: bytes, rec_cap=1 << 16, want=None):
    d = api.to_device(np.frombuffer(raw, np.uint8).copy() if raw else np.zeros(0, np.uint8))
    seq, rec, kept, nrec = api.fasta_normalize(d, rec_cap)
    want_seq, want_starts = want if want is not None else ofasta.normalize(raw)
    assert kept == len(want_seq) and nrec == len(want_starts)
    assert bytes(seq.cpu().numpy().tobytes()) == want_seq
    assert rec.cpu().numpy().tolist() == want_starts[:rec_cap]
    return seq, want_starts


@pytest.mark.parametrize("seed", range(4))
def test_random_genomes(seed):
    rng = np.random.default_rng(seed)
    recs = []
    for k in range(int(rng.integers(1, 40))):
        n = int(rng.choice([0, 1, 59, 60, 61, int(rng.integers(0, 200_000))]))
        recs.append((f"rec{k} some description {seed}".encode(), synth.iid_gc41(n, 100 * seed + k).tobytes()))
    for width in (60, 80, 7):
        raw = write_fasta(recs, width, rng, crlf_frac=0.3, lower_frac=0.5)
        say("seed", seed, "width", width, "bytes", len(raw))
        check(raw)


def test_unit_border_cases():
    # a header that starts exactly at a unit border, one that straddles one, a newline as a
    # unit's last byte, a header longer than two units, no final newline, a preamble
    body = b"ACGT" * (TWO // 4)
    raw = bytearray(b"acgtn\n")                       # preamble before the first header
    raw += body[:TWO - len(raw) - 1] + b"\n"            # this newline is a unit's last byte
    raw += b">at_unit_start\n" + body[:1000] + b"\n"
    pad = 2 * TWO - len(raw) - 3
    raw += body[:pad] + b"\n>s"                        # header straddling the second boundary
    raw += b"traddle header\n" + body[:5000] + b"\n"
    raw += b">" + b"H" * (TWO + 123) + b"\n"            # header longer than two units
    raw += body[:777] + b"\r\n>last\nAcGt"              # no final newline
    check(bytes(raw))


def test_edges():
    check(b"")
    check(b">only header")
    check(b"\n\n\n")
    check(b"AC>GT\nT")
    check(b">a\n>b\n>c\nA\n")
    rng = np.random.default_rng(7)
    recs = [(b"r%d" % k, b"A" * 3) for k in range(5000)]
    raw = write_fasta(recs, 60, rng)
    seq, starts = check(raw, rec_cap=100)               # more records than rec_cap
    assert len(starts) == 5000


def test_counts_on_normalised_records():
    rng = np.random.default_rng(11)
    recs = [(b"chr%d" % k, synth.genome_like(int(rng.integers(1000, 400_000)), 200 + k, 0.02, 500).tobytes())
            for k in range(12)]
    raw = write_fasta(recs, 70, rng, lower_frac=1.0)
    d = api.to_device(np.frombuffer(raw, np.uint8).copy())
    seq, rec, kept, nrec = api.fasta_normalize(d)
    seg_off = np.concatenate((rec.cpu().numpy(), [kept])).astype(np.int64)
    pats = [synth.random_pattern(int(m), rng) for m in rng.integers(4, 20, size=10)]
    pats += [recs[3][1][100:112]]
    pair_seg = np.repeat(np.arange(nrec), len(pats))
    pair_pat = np.tile(np.arange(len(pats)), nrec)
    got = api.count_merged(seq, seg_off, pats, pair_seg, pair_pat)
    text = b"".join(s for _, s in recs)
    want = oracle.pair_counts(np.frombuffer(text, np.uint8), seg_off, pats, pair_seg, pair_pat)
    assert np.array_equal(got, want)


def test_unit_round_and_piece_boundaries():
    # newlines and header starts on both sides of every kind of border: the last
    # byte of a lane's piece, of a round, of a unit; a header line that runs over
    # several units; CRLF split over a unit border
    rng = np.random.default_rng(21)
    body = synth.iid_gc41(4 * UNIT, 3).tobytes()
    raw = bytearray()
    for border in (16, ROUND, UNIT, 2 * UNIT, 3 * UNIT):
        for d in (-2, -1, 0, 1):
            target = border * (1 + len(raw) // border) + d
            raw += body[:max(0, target - len(raw) - 1)] + b"\n"
            raw += b">h%d\n" % d if d % 2 else b"acgt\r\n"
    raw += b">" + b"x" * (2 * UNIT + 77) + b"\r\n" + body[:UNIT - 3] + b"\r\n" + body[:100]
    for cut in (0, 1, 15, 16, 17, ROUND - 1, ROUND + 1):
        say("cut", cut, "bytes", len(raw) - cut)
        check(bytes(raw[:len(raw) - cut]))
    check(write_fasta([(b"r", body)], 61, rng, lower_frac=1.0))


def test_open_headers_in_sequence_rounds():
    # header lines of letters only, LF line ends: the rounds that hold a header's tail
    # have no byte below 0x40 but '\n', so they take the sequence-round path with a
    # header still open.  The header's '\n' lands on every offset around piece, round
    # and unit borders; a '>' inside a sequence line is kept.
    rng = np.random.default_rng(33)
    body = synth.iid_gc41(3 * UNIT, 8).tobytes()
    raw = bytearray(body[:100] + b"\n")
    for border in (16, ROUND, UNIT):
        for d in (-17, -16, -1, 0, 1, 15, 16, 300):
            target = border * (3 + len(raw) // border) + d   # index of the header's '\n'
            raw += b">" + b"H" * (target - len(raw) - 1) + b"\n"
            assert raw[target] == ord("\n")
            raw += body[:int(rng.integers(1, 2000))] + b"\n"
    raw += body[:500] + b">" + body[:40] + b"\n" + body[:3000]
    check(bytes(raw))
    recs = [(b"Name" + b"x" * int(rng.integers(0, 3000)), synth.iid_gc41(int(rng.integers(0, 5000)), 60 + k).tobytes())
            for k in range(50)]
    check(write_fasta(recs, 60, rng, lower_frac=0.5))


def test_output_alignments():
    # the kept bytes go to out + k for every k: whole 16-byte blocks in the middle
    # of a unit's output, bytes at its two ends
    rng = np.random.default_rng(5)
    recs = [(b"c%d" % k, synth.iid_gc41(int(rng.integers(0, 3 * UNIT)), 40 + k).tobytes()) for k in range(9)]
    raw = write_fasta(recs, 60, rng, crlf_frac=0.5, lower_frac=0.5)
    want_seq, want_starts = ofasta.normalize(raw)
    n = len(raw)
    d = api.to_device(np.frombuffer(raw, np.uint8).copy())
    big = torch.full((n + 64,), 0xA5, dtype=torch.uint8, device=d.device)
    rec = torch.empty(64, dtype=torch.int64, device=d.device)
    tot = torch.zeros(2, dtype=torch.int64, device=d.device)
    ws = torch.empty(max(256, api.lib.dfa_fasta_workspace_bytes(n)), dtype=torch.uint8, device=d.device)
    for k in range(17):
        say("output offset", k)
        big.fill_(0xA5)
        api._check(api.lib.dfa_fasta_normalize(d.data_ptr(), n, big.data_ptr() + k, rec.data_ptr(), 64,
                                               tot.data_ptr(), ws.data_ptr(), ws.numel(), api._stream_handle(None)))
        kept, nrec = (int(x) for x in tot.cpu().tolist())
        host = big.cpu().numpy()
        assert kept == len(want_seq) and nrec == len(want_starts)
        assert host[k:k + kept].tobytes() == want_seq
        assert (host[:k] == 0xA5).all() and (host[k + kept:] == 0xA5).all()   # nothing outside
        assert rec.cpu().numpy()[:nrec].tolist() == want_starts


def test_several_plan_blocks():
    # more units than one block of the plan combines: 2.3 blocks
    rng = np.random.default_rng(9)
    n_target = int(2.3 * PLAN_BLOCK * UNIT) // 1000 * 1000
    seq = synth.iid_gc41(n_target, 17)
    lines = seq.reshape(-1, 1000)
    width = lines.shape[1] + 1
    raw = np.full((lines.shape[0], width), ord("\n"), np.uint8)
    raw[:, :-1] = lines
    flat = raw.reshape(-1)
    # a header every ~4 MB, placed at line starts
    heads = sorted(set(int(x) for x in rng.integers(0, lines.shape[0], size=40)) | {0})
    parts, prev = [], 0
    for i, h in enumerate(heads):
        parts.append(flat[prev * width:h * width].tobytes())
        parts.append(b">rec%d\n" % i)
        prev = h
    parts.append(flat[prev * width:].tobytes())
    text = b"".join(parts)
    say("bytes", len(text), "units", -(-len(text) // UNIT))
    want_seq = seq.tobytes()
    check(text, want=(want_seq, [h * 1000 for h in heads]))


def test_genome_scale_round_trip():
    # the benchmark's FASTA workload at full size and in the launch it times: the 3.2 GB
    # genome-like text written as FASTA (24 records, 60 bases per line, 10 % soft-masked in
    # runs) normalises back to the text itself, with each record starting where the writer cut
    # the text; the first 4 MB of the FASTA are also checked against the oracle directly
    import bench
    n = 3_200_000_000
    text = synth.genome_like(n, 2, 0.05, 50_000)
    raw = bench.fasta_bytes(text)
    say("fasta bytes", raw.size)
    d = api.to_device(raw)
    seq, rec, kept, nrec = api.fasta_normalize(d, 64)
    del d
    assert kept == n and nrec == 24
    cuts = np.linspace(0, n, 25).astype(np.int64)[:-1]
    assert rec.cpu().numpy().tolist() == cuts.tolist()
    dtext = api.to_device(text)
    assert bool(torch.equal(seq, dtext))
    del dtext
    head = raw[:4_000_000].tobytes()
    want, _ = ofasta.normalize(head[:head.rfind(b"\n") + 1])
    assert seq[:len(want)].cpu().numpy().tobytes() == want
