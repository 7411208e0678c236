"""CPU tests of the serving loop's host bookkeeping and of the autotuner's cache keys."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1506_08612_amd import synth
from paper_1506_08612_amd.serve import ALIGN, Arena, segments_for


def test_arena_first_fit_and_coalescing():
    a = Arena(10 * ALIGN)
    x = a.alloc(1)
    y = a.alloc(3 * ALIGN)
    z = a.alloc(2 * ALIGN + 5)
    assert (x, y, z) == (0, ALIGN, 4 * ALIGN)
    assert a.alloc(4 * ALIGN) is None          # only 3 blocks left at the end
    a.release(y, 3 * ALIGN)
    assert a.alloc(4 * ALIGN) is None          # the hole is 3 blocks
    w = a.alloc(2 * ALIGN)
    assert w == ALIGN                          # first fit reuses the hole
    a.release(x, 1)
    a.release(w, 2 * ALIGN)
    a.release(z, 2 * ALIGN + 5)
    assert a.free == [(0, 10 * ALIGN)] and a.used == 0


def test_arena_random_alloc_free_never_overlaps():
    rng = np.random.default_rng(0)
    a = Arena(1 << 20)
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            k = list(live)[int(rng.integers(0, len(live)))]
            off, n = live.pop(k)
            a.release(off, n)
        else:
            n = int(rng.integers(1, 40000))
            off = a.alloc(n)
            if off is not None:
                assert off % ALIGN == 0 and off + n <= a.size
                for o2, n2 in live.values():
                    assert off + n <= o2 or o2 + n2 <= off
                live[step] = (off, n)
    for off, n in live.values():
        a.release(off, n)
    assert a.free == [(0, 1 << 20)]


def test_segments_cover_texts_and_gaps():
    placed = [(1024, 100), (0, 300), (5000, 0), (4096, 10)]
    seg_off, seg_of = segments_for(placed, 1 << 20)
    assert (np.diff(seg_off) >= 0).all() and seg_off[0] == 0
    for (off, ln), s in zip(placed, seg_of):
        assert seg_off[s] == off and seg_off[s + 1] == off + ln


def test_segments_empty_text_sharing_offset_zero():
    # an empty text is placed at offset 0 without arena space; fused after a text that
    # starts at 0, the offsets must still be non-decreasing and both segments exact
    for placed in ([(0, 1000), (0, 0)], [(0, 0), (0, 1000)], [(0, 1000), (0, 0), (0, 0), (1024, 5)]):
        seg_off, seg_of = segments_for(placed, 1 << 20)
        assert (np.diff(seg_off) >= 0).all() and seg_off[0] == 0, placed
        for (off, ln), s in zip(placed, seg_of):
            assert seg_off[s] == off and seg_off[s + 1] == off + ln, placed


def test_query_trace_shape():
    tr = synth.query_trace(200, 50.0, seed=1, len_lo=1e4, len_hi=5e8)
    t = np.array([q.arrival_s for q in tr])
    assert (np.diff(t) > 0).all()
    assert abs(len(tr) / t[-1] - 50.0) < 15
    L = np.array([q.text_len for q in tr])
    assert L.min() >= 1e4 and L.max() <= 5e8
    k = np.array([len(q.pattern_lens) for q in tr])
    assert k.min() >= 1 and k.max() <= 64
    ms = np.concatenate([q.pattern_lens for q in tr])
    assert ms.min() >= 4 and ms.max() <= 64


def test_tune_cache_key_names_the_built_library(tmp_path, monkeypatch):
    from paper_1506_08612_amd import api, autotune
    key = autotune.device_key()
    assert key.endswith("|" + autotune._lib_hash()) and len(autotune._lib_hash()) == 12
    # another library file (different kernels) gives another key
    other = tmp_path / "libdfa.so"
    other.write_bytes(open(api.LIB_PATH, "rb").read() + b"\0")
    monkeypatch.setattr(api, "LIB_PATH", str(other))
    monkeypatch.setattr(autotune, "_LIB_HASH", None)
    assert autotune.device_key() != key
