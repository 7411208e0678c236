"""GPU tests of the orchestration layer: HIP graph capture and replay of the scan launches,
the autotuner, and the continuous-batching server.  Every result is compared with the
CPU oracle exactly; the server's answers must be identical alone and in the mix."""
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

from paper_1506_08612_amd import api, autotune, graph, serve  # noqa: E402


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_graph_replay_batch_tracks_text_changes():
    w = synth.uneven_segments(nseg=25, median=40_000, sigma=1.0, lo=100, hi=300_000, seed=21)
    d = api.to_device(w.text)
    ps = api.PatternSet(w.patterns)
    b = api.Batch(w.seg_off, ps, w.pair_seg, w.pair_pat)
    g = graph.GraphedBatch(d, b)
    rng = np.random.default_rng(2)
    text = w.text.copy()
    for rep in range(4):
        say(f"graph replay {rep}")
        got = g.replay().cpu().numpy()
        want = oracle.pair_counts(text, w.seg_off, w.patterns, w.pair_seg, w.pair_pat)
        assert np.array_equal(got, want), rep
        # eager work between replays: an unrelated scan and a rewrite of part of the text
        t2, m2 = api.device_table(b"ACGTACGT")
        api.count(d, t2, m2)
        lo = int(rng.integers(0, text.size - 5000))
        text[lo:lo + 5000] = synth.iid_gc41(5000, 100 + rep)
        d[lo:lo + 5000].copy_(torch.from_numpy(text[lo:lo + 5000]).to(d.device))
        torch.cuda.synchronize()


def test_graph_replay_single_pattern():
    text = synth.genome_like(4_000_000, 8, 0.02, 1000)
    d = api.to_device(text)
    pat = text[777:785].tobytes()
    tab, m = api.device_table(pat)
    g = graph.GraphedCount(d, tab, m)
    for rep in range(3):
        got = int(g.replay().item())
        assert got == oracle.count(text, pat), rep
        api.count(d, tab, m)  # eager launch between replays
        torch.cuda.synchronize()


def test_autotune_picks_a_correct_shape(tmp_path, monkeypatch):
    monkeypatch.setenv("DFA_TUNE_CACHE", str(tmp_path / "tune.json"))
    text = synth.genome_like(8_000_000, 9, 0.02, 1000)
    d = api.to_device(text)
    pat = text[100:116].tobytes()
    tab, m = api.device_table(pat)
    t, entry = autotune.tune_scan(d, tab, m, reps=1)
    assert len(entry["tried"]) >= 3
    assert api.count(d, tab, m, t=t) == oracle.count(text, pat)
    t2, entry2 = autotune.tune_scan(d, tab, m, reps=1)  # served from the cache
    assert entry2["tune"] == entry["tune"]
    assert (tmp_path / "tune.json").exists()
    w = synth.uneven_segments(nseg=20, median=50_000, sigma=1.0, lo=100, hi=300_000, seed=5)
    dw = api.to_device(w.text)
    ps = api.PatternSet(w.patterns)
    tb, eb = autotune.tune_batch(dw, w.seg_off, ps, w.pair_seg, w.pair_pat, reps=1)
    got = api.count_batch(dw, w.seg_off, ps, w.pair_seg, w.pair_pat, tb)
    assert np.array_equal(got, oracle.pair_counts(w.text, w.seg_off, w.patterns, w.pair_seg, w.pair_pat))


def _trace(nq, rate, seed, len_hi=2e6, pmax=16):
    return serve.make_trace(nq, rate, seed=seed, len_lo=1e4, len_hi=len_hi, pmax=pmax)


def _want(req):
    return np.array([oracle.count(req.text, p) for p in req.patterns], dtype=np.int64)


@pytest.mark.parametrize("mode", ["continuous", "fifo"])
def test_server_answers_match_oracle(mode):
    trace = _trace(24, rate=2000.0, seed=3)
    srv = serve.Server(arena_bytes=64 << 20)
    res = srv.serve(trace, mode=mode)
    srv.release_pinned()
    for req, r in zip(trace, res):
        assert r.qid == req.qid
        assert np.array_equal(r.counts, _want(req)), req.qid
        assert r.done >= r.launched >= r.admitted >= r.arrival - 1e-3
    s = serve.summarize(res)
    say(mode, s)
    assert s["queries"] == 24
    # served again after the pinned copies were released: pinned anew, same answers
    again = srv.serve([serve.Request(r.qid, r.text, r.patterns, 0.0) for r in trace[:3]], mode=mode)
    for a, r in zip(again, res[:3]):
        assert np.array_equal(a.counts, r.counts)


def test_server_alone_equals_in_mix_with_admission_pressure():
    """A small arena forces requests to wait for memory; every answer must equal the
    answer the same request gets when served alone."""
    trace = _trace(30, rate=5000.0, seed=4, len_hi=3e6)
    big = max(r.text.size for r in trace)
    srv = serve.Server(arena_bytes=int(big * 2.2) // 256 * 256 + 4096)
    mix = srv.serve(trace, mode="continuous")
    batches = {r.launched for r in mix}
    assert len(batches) > 1  # admission pressure split the requests over several launches
    for req, r in zip(trace, mix):
        alone = srv.serve([serve.Request(req.qid, req.text, req.patterns, 0.0)], mode="continuous")[0]
        assert np.array_equal(alone.counts, r.counts), req.qid
        assert np.array_equal(r.counts, _want(req)), req.qid


def test_server_edge_requests():
    rng = np.random.default_rng(9)
    reqs = [serve.Request(0, np.zeros(0, np.uint8), [b"ACGT"], 0.0),
            serve.Request(1, np.frombuffer(b"ACGTACGTAC", np.uint8).copy(), [b"ACGTACGTACG", b"AC"], 0.0),
            serve.Request(2, synth.iid_gc41(100_000, 3), [b"A", b"ACGT", b"TTTT"], 0.0),
            serve.Request(3, np.full(70_000, ord("A"), np.uint8), [b"A" * 64, b"A" * 4], 0.0)]
    srv = serve.Server(arena_bytes=1 << 20)
    res = srv.serve(reqs)
    for req, r in zip(reqs, res):
        assert np.array_equal(r.counts, _want(req)), req.qid
    del rng


def test_server_fuses_empty_request_after_text_at_offset_zero():
    """An empty request shares offset 0 with the text placed there; fused into one launch
    after it, both answers must be exact."""
    text = synth.iid_gc41(50_000, 11)
    reqs = [serve.Request(0, text, [b"ACGT", b"GATTACA", bytes(text[100:112])], 0.0),
            serve.Request(1, np.zeros(0, np.uint8), [b"ACGT", b"A"], 0.0)]
    srv = serve.Server(arena_bytes=1 << 20)
    srv.arena_buf[:text.size].copy_(torch.from_numpy(text))
    jobs = []
    for r in reqs:
        j = serve._Job()
        j.req, j.pinned, j.offset = r, None, 0
        j.admitted = j.launched = 0.0
        j.next_byte, j.pending_events = r.text.size, 0
        jobs.append(j)
    ev, counts, spans, keep = srv._launch(jobs)
    ev.synchronize()
    c = counts.cpu().numpy()
    for (a, b), r in zip(spans, reqs):
        assert np.array_equal(c[a:b], _want(r)), r.qid
