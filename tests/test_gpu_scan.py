"""GPU parity of the single-pattern scan (dfa_count through the C ABI) against the
CPU oracle: counts and sorted positions must be bit-exact on every input.
"""
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


def gpu_result(dtext, pat: bytes, t=None):
    tab, m = api.device_table(pat)
    c = api.count(dtext, tab, m, t=t)
    c2, pos = api.positions(dtext, tab, m, t=t)
    assert c2 == c
    return c, pos.cpu().numpy()


def check(text: np.ndarray, pat: bytes, t=None, dtext=None):
    if dtext is None:
        dtext = api.to_device(text)
    want = oracle.occurrences(text, pat)
    c, pos = gpu_result(dtext, pat, t)
    assert c == want.size, (len(text), len(pat), c, want.size)
    assert np.array_equal(pos, want)
    return c


def gc_text(n, seed, n_frac=0.03, plant=None, every=997):
    t = synth.genome_like(n, seed, n_frac, n_run_mean=300)
    if plant is not None and n >= len(plant):
        for i in range(0, n - len(plant) + 1, every):
            t[i:i + len(plant)] = np.frombuffer(plant, np.uint8)
    return t


def test_tiny_uniform_workload():
    w = synth.tiny_uniform()
    say("tiny uniform n=1MiB m=8")
    c = check(w.text, w.patterns[0])
    assert c >= 1
    _, pos = gpu_result(api.to_device(w.text), w.patterns[0])
    assert w.offsets[0] in pos.tolist()


@pytest.mark.parametrize("m", [1, 2, 4, 8, 17, 18, 33, 34, 64, 255])
def test_ragged_sizes(m):
    rng = np.random.default_rng(m)
    pat = synth.random_pattern(m, rng)
    for n in [0, 1, 7, 15, 16, 17, 127, 128, 129, 255, 256, 1000, 4095, 4096, 4097, 65535,
              65536 + 7, (1 << 20) + 13]:
        say(f"ragged n={n} m={m}")
        check(gc_text(n, n + m, plant=pat, every=331 + m), pat)


TUNES = [
    dict(chain_bytes=16), dict(chain_bytes=48), dict(chain_bytes=128), dict(chain_bytes=1024),
    dict(chain_bytes=4096), dict(chain_bytes=65536),
    dict(line_bytes=64), dict(line_bytes=128), dict(chains_per_lane=2, line_bytes=64),
    dict(waves_per_group=1), dict(waves_per_group=2, line_bytes=64), dict(waves_per_group=8),
    dict(waves_per_group=16), dict(waves_per_group=16, chain_bytes=128),
    dict(waves_per_group=3, chain_bytes=2000 // 16 * 16, chains_per_lane=2, line_bytes=64),
]


@pytest.mark.parametrize("tn", TUNES, ids=lambda d: ",".join(f"{k}={v}" for k, v in d.items()))
def test_result_independent_of_launch_shape(tn):
    text = gc_text(3_000_017, 99)
    d = api.to_device(text)
    rng = np.random.default_rng(7)
    for m in (4, 8, 16, 32, 64, 200):
        pat, _ = synth.drawn_pattern(text, m, rng)
        say(f"tune {tn} m={m}")
        check(text, pat, api.tune(**tn), dtext=d)


def test_periodic_texts_dense_matches():
    n = (1 << 20) + 3
    text = np.full(n, ord("A"), np.uint8)
    d = api.to_device(text)
    for m in (1, 4, 64, 255):
        say(f"A^n m={m}")
        c, pos = gpu_result(d, b"A" * m)
        assert c == n - m + 1
        assert np.array_equal(pos, np.arange(n - m + 1))
    k = 300_001
    text = np.frombuffer(b"AC" * k, np.uint8).copy()
    c, pos = gpu_result(api.to_device(text), b"ACA")
    assert c == k - 1 and np.array_equal(pos, np.arange(0, 2 * k - 3, 2))


def test_match_bursts_between_sparse_stretches():
    """Matches packed together (every lane of a wave matching in the same bytes) between
    long stretches without any, so that the per-walk counting pass changes how it walks
    many times within one walk and one wave."""
    rng = np.random.default_rng(11)
    n = (1 << 21) + 45
    text = synth.genome_like(n, 12, 0.0, 300)
    for m in (2, 5, 12, 20, 40):
        pat = synth.random_pattern(m, rng)
        t = text.copy()
        starts = rng.integers(0, n - 4096, size=60)
        for s0 in starts:  # a burst: the pattern repeated back to back
            reps = int(rng.integers(1, 4096 // m))
            burst = np.frombuffer(pat * reps, np.uint8)
            t[s0:s0 + burst.size] = burst
        say(f"bursts m={m}")
        check(t, pat)


def test_all_byte_values():
    rng = np.random.default_rng(5)
    text = rng.integers(0, 256, size=(1 << 19) + 77, dtype=np.uint8)
    text[1000:1003] = [0, 255, 0]
    text[5000:5003] = [0, 255, 0]
    d = api.to_device(text)
    for pat in (bytes([0, 255, 0]), bytes([0]), bytes([255]), text[40000:40002].tobytes()):
        say(f"bytes pattern={list(pat)}")
        check(text, pat, dtext=d)


def test_positions_truncated_to_cap():
    text = np.full(100_000, ord("G"), np.uint8)
    d = api.to_device(text)
    tab, m = api.device_table(b"GG")
    c, pos = api.positions(d, tab, m, cap=1000)
    assert c == 99_999
    assert np.array_equal(pos.cpu().numpy(), np.arange(1000))


def test_positions_truncated_to_cap_long_pattern():
    """Patterns longer than 17 bytes count per wave and write positions from a second walk
    of the waves with a match; the cap holds there too, and the count stays exact."""
    text = np.full(300_000, ord("G"), np.uint8)
    d = api.to_device(text)
    for m in (18, 40, 100):
        tab, mm = api.device_table(b"G" * m)
        c, pos = api.positions(d, tab, mm, cap=1234)
        assert c == text.size - m + 1
        assert np.array_equal(pos.cpu().numpy(), np.arange(1234))


def test_positions_truncated_to_cap_sparse_long_pattern():
    """Per-wave plans with one or two matches per re-walked share (written from the counting
    walk's registers) and with more (written by a second walk): the first `cap` positions
    equal the oracle's, for caps that cut inside either kind of share."""
    rng = np.random.default_rng(17)
    n = 2_000_003
    for m in (12, 16, 24, 40):
        pat = synth.random_pattern(m, rng)
        t = synth.genome_like(n, 30 + m, 0.0, 300)
        for s0 in range(1000, n - 200, 45 + m):    # isolated matches, 45 + m bytes apart
            t[s0:s0 + m] = np.frombuffer(pat, np.uint8)
        if m <= 20:                                # and a burst of back-to-back repeats
            burst = np.frombuffer(pat * (3000 // m), np.uint8)
            t[500_000:500_000 + burst.size] = burst
        want = oracle.occurrences(t, pat)
        d = api.to_device(t)
        tab, mm = api.device_table(pat)
        for cap in (1, 2, 3, len(want) // 3, len(want) - 1):
            say(f"sparse cap m={m} cap={cap} of {len(want)}")
            c, pos = api.positions(d, tab, mm, cap=cap)
            assert c == len(want)
            assert np.array_equal(pos.cpu().numpy(), want[:cap])


def test_repeatable_bit_equal():
    text = gc_text(5_000_000, 3)
    d = api.to_device(text)
    pat = text[123456:123464].tobytes()
    a = gpu_result(d, pat)
    b = gpu_result(d, pat)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


@pytest.mark.slow
def test_paper_scale_genome():
    """3.2 GB genome-like text (GC 41 %, 5 % 'N' runs of mean 50 kb), patterns of length
    4..64 drawn from the text, scanned one per launch with the library's default launch
    shape (the shape the benchmark times)."""
    say("generating 3.2 GB genome-like text")
    w = synth.paper_scale()
    d = api.to_device(w.text)
    for pat, off in zip(w.patterns, w.offsets):
        say(f"paper scale m={len(pat)}")
        want = oracle.occurrences(w.text, pat)
        c, pos = gpu_result(d, pat)
        assert c == want.size
        assert np.array_equal(pos, want)
        assert off in set(pos[max(0, np.searchsorted(pos, off) - 1):np.searchsorted(pos, off) + 1].tolist())
    del d
    torch.cuda.empty_cache()


def test_binding_rejects_bad_tensors():
    # argument checks of the binding: no kernel is launched for any of these
    d = api.to_device(np.frombuffer(b"ACGT" * 64, np.uint8).copy())
    tab, m = api.device_table(b"ACGT")
    out = torch.zeros(1, dtype=torch.int64, device=d.device)
    pos = torch.zeros(8, dtype=torch.int64, device=d.device)
    with pytest.raises(ValueError, match="dtype"):
        api.count_async(d.view(torch.int8), tab, m, out)
    with pytest.raises(ValueError, match="contiguous"):
        api.count_async(d[::2], tab, m, out)
    with pytest.raises(ValueError, match="at least"):
        api.count_async(d, tab[:100], m, out)
    with pytest.raises(ValueError, match="dtype"):
        api.count_async(d, tab, m, out.view(torch.float64))
    with pytest.raises(ValueError, match="at least"):
        api.count_async(d, tab, m, out, pos, 9)
    with pytest.raises(ValueError, match="contiguous"):
        api.fasta_normalize(d[::2])
    assert api.count(d, tab, m) == 64  # the same tensors, well formed


@pytest.mark.parametrize("n,m,chain", [(1, 1, 0), (1000, 4, 0), ((1 << 20) + 13, 8, 0), ((1 << 20) + 13, 8, 4096),
                                        (50_000_017, 4, 0), (50_000_017, 32, 0), (3_000_001, 200, 512)])
def test_count_timed_matches_oracle(n, m, chain):
    """The load-balance study's entry point: its count equals the oracle's, every launched
    workgroup leaves an ordered, non-zero record, and a short record buffer is respected."""
    text = gc_text(n, 31 + n % 7, plant=None)
    pat = synth.drawn_pattern(text, m, np.random.default_rng(n + m))[0] or b"A" * m
    d = api.to_device(text)
    tab, mm = api.device_table(pat)
    t = api.tune(chain_bytes=chain) if chain else None
    c, rows = api.count_timed(d, tab, mm, t=t)
    assert c == oracle.count(text, pat), (n, m)
    assert c == api.count(d, tab, mm, t=t)
    nb = rows.shape[0]
    assert nb >= 1
    start, end, cyc = rows[:, 0], rows[:, 1], rows[:, 2]
    assert (start > 0).all() and (end >= start).all() and (cyc > 0).all(), (n, m)
    assert end.max() - start.min() < 10 * 100_000_000  # the launch spans under 10 s of the 100 MHz clock
    # room for only three workgroups: the count is unchanged and only those rows are written
    c3, rows3 = api.count_timed(d, tab, mm, t=t, wg_cap=3)
    assert c3 == c and rows3.shape[0] == min(3, nb) and (rows3[:, 2] > 0).all()


def test_calls_on_several_streams_with_their_own_workspaces():
    """dfa_count with positions issued in turn on three streams, each with its own
    workspace (the benchmark's step), then joined: every count and position equals the
    oracle's, for short (per-walk plan) and long (per-wave plan) patterns."""
    text = gc_text(40_000_000, 77, plant=None)
    rng = np.random.default_rng(78)
    pats = [synth.drawn_pattern(text, m, rng)[0] for m in (4, 8, 12, 16, 32, 64)]
    d = api.to_device(text)
    n = text.size
    streams = (torch.cuda.current_stream(), torch.cuda.Stream(), torch.cuda.Stream())
    wsb = max(api.count_workspace_bytes(n, len(p), True) for p in pats)
    wss = [torch.empty(wsb, dtype=torch.uint8, device=d.device) for _ in streams]
    want = [oracle.occurrences(text, p) for p in pats]
    tabs = [api.device_table(p)[0] for p in pats]
    cnts = [torch.empty(1, dtype=torch.int64, device=d.device) for _ in pats]
    poss = [torch.empty(max(1, w.size), dtype=torch.int64, device=d.device) for w in want]
    torch.cuda.synchronize()
    for rep in range(3):
        for i, p in enumerate(pats):
            s = (i + rep) % len(streams)
            api.count_async(d, tabs[i], len(p), cnts[i], poss[i], poss[i].numel(), wss[s], stream=streams[s])
        for st in streams[1:]:
            streams[0].wait_stream(st)
        torch.cuda.synchronize()
        for i, w in enumerate(want):
            assert int(cnts[i].item()) == w.size, (rep, len(pats[i]))
            assert np.array_equal(poss[i][:w.size].cpu().numpy(), w), (rep, len(pats[i]))
