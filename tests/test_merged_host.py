"""Host-side tests of the merged multi-pattern automata: the library's builder
(dfa_ac_build) against the oracle's automaton, argument checks of the merged
batch planner, and a CPU model of the merged scan's decomposition and
start-position ownership rule against the window-compare oracle."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
from oracle import ac as oac
from paper_1506_08612_amd import api


def _outputs_walk(step, outputs, text):
    q = 0
    seq = []
    for c in text:
        q = step(q, c)
        seq.append(sorted(outputs(q)))
    return seq


def _random_set(rng, k, lo, hi, alphabet=b"ACGT"):
    return [bytes(rng.choice(list(alphabet), size=int(rng.integers(lo, hi + 1))).tolist()) for _ in range(k)]


@pytest.mark.parametrize("seed", range(8))
def test_ac_build_matches_oracle_automaton(seed):
    rng = np.random.default_rng(100 + seed)
    alpha = b"ACGT" if seed % 2 == 0 else b"ACGTN#\x00\xff"
    pats = _random_set(rng, int(rng.integers(1, 12)), 1, 7, alpha)
    pats += [pats[0], pats[0][1:] or pats[0]]  # a repeat and a suffix
    mine = api.ac_build(pats)
    ref = oac.build(pats)
    assert mine.nstates == ref.nstates
    assert mine.first_final == ref.first_final
    # same behaviour on every short string and on a long random text: the same
    # reported patterns after every byte (the automata are equal up to numbering)
    texts = [bytes(rng.choice(list(alpha + b"Z"), size=2000).tolist())]
    for L in range(1, 4):
        for i in range(min(200, len(alpha) ** L)):
            texts.append(bytes(rng.choice(list(alpha), size=L).tolist()))
    for text in texts:
        a = _outputs_walk(lambda q, c: int(mine.table[q, c]), mine.outputs, text)
        b = _outputs_walk(lambda q, c: int(ref.table[q, c]), lambda q: ref.outputs[q], text)
        assert a == b
    # reporting states are numbered last and report at least one pattern
    for q in range(mine.nstates):
        assert (len(mine.outputs(q)) > 0) == (q >= mine.first_final)


def test_ac_build_table2_set():
    pats = [b"ACG", b"ACT", b"CTA", b"TGA"]
    t = api.ac_build(pats)
    assert t.nstates == 11 and t.nstates - t.first_final == 4
    other = [c for c in range(256) if c not in b"ACGT"]
    assert (t.table[:, other] == 0).all()


def test_ac_build_errors():
    blob = np.frombuffer(b"ACGT", np.uint8).copy()
    offs = np.zeros(1, np.int64)
    ff = ctypes.c_int32()
    for lens in ([0], [256]):
        ln = np.array(lens, np.int32)
        assert api.lib.dfa_ac_build(blob.ctypes.data, offs.ctypes.data, ln.ctypes.data, 1, None, 0, None, None, None,
                                    0, None) == api.DFA_EINVAL
    ln = np.array([4], np.int32)
    assert api.lib.dfa_ac_build(blob.ctypes.data, offs.ctypes.data, ln.ctypes.data, 0, None, 0, None, None, None, 0,
                                None) == api.DFA_EINVAL
    assert api.lib.dfa_ac_build(blob.ctypes.data, offs.ctypes.data, ln.ctypes.data, 1, None, 0, ctypes.byref(ff),
                                None, None, 0, None) == 5
    small = np.empty((4, 256), np.uint16)
    assert api.lib.dfa_ac_build(blob.ctypes.data, offs.ctypes.data, ln.ctypes.data, 1, small.ctypes.data, 4, None,
                                None, None, 0, None) == api.DFA_ENOSPACE
    out_off = np.empty(2, np.int32)
    out_pat = np.empty(1, np.int32)
    assert api.lib.dfa_ac_build(blob.ctypes.data, offs.ctypes.data, ln.ctypes.data, 1, None, 0, ctypes.byref(ff),
                                out_off.ctypes.data, out_pat.ctypes.data, 0, None) == api.DFA_ENOSPACE


def _prepare(seg_off, patterns, pair_seg, pair_pat, t=None):
    pats, blob, offs, lens = api._pack_patterns(patterns)
    so = np.ascontiguousarray(seg_off, np.int64)
    ps = np.ascontiguousarray(pair_seg, np.int32)
    pp = np.ascontiguousarray(pair_pat, np.int32)
    plan = api.MergedPlan()
    rc = api.lib.dfa_merged_prepare(so.ctypes.data, so.size - 1, blob.ctypes.data, offs.ctypes.data,
                                    lens.ctypes.data, len(pats), ps.ctypes.data, pp.ctypes.data, ps.size, None, 0,
                                    None, 0, api._tune_ptr(t), ctypes.byref(plan), None)
    return rc, plan


def test_merged_prepare_argument_checks():
    pats = [b"ACGT", b"GG"]
    ok, plan = _prepare([0, 1000, 5000], pats, [0, 1, 1], [0, 0, 1])
    assert ok == api.DFA_OK and plan.npairs == 3 and plan.nautomata == 2 and plan.nitems >= 2
    assert plan.workspace_bytes > 0 and plan.text_bytes == 5000
    bad = [
        ([0, 1000], pats, [1], [0], None),                      # segment out of range
        ([0, 1000], pats, [0], [2], None),                      # pattern out of range
        ([0, 1000, 500], pats, [0], [0], None),                 # decreasing offsets
        ([0, 1000], pats, [0], [0], api.tune(chain_bytes=192)),  # span not a multiple of 128
        ([0, 1000], pats, [0], [0], api.tune(automaton_bytes=1000)),
        ([0, 1000], pats, [0], [0], api.tune(waves_per_group=17)),
        ([0, 1000], pats, [0], [0], api.tune(line_bytes=128)),    # rounds of 32 or 64 bytes only
        ([0, 1000], [b""], [0], [0], None),                     # empty pattern
        ([0, 1000], [b"A" * 256], [0], [0], None),              # too long
    ]
    for so, p, s, q, t in bad:
        rc, _ = _prepare(so, p, s, q, t)
        assert rc == api.DFA_EINVAL, (so, p, s, q)


def test_merged_prepare_splits_by_budget():
    rng = np.random.default_rng(5)
    pats = _random_set(rng, 300, 20, 40)
    n = len(pats)
    _, big = _prepare([0, 1 << 20], pats, [0] * n, list(range(n)), api.tune(automaton_bytes=120 * 1024))
    _, small = _prepare([0, 1 << 20], pats, [0] * n, list(range(n)), api.tune(automaton_bytes=8 * 1024))
    assert big.nautomata < small.nautomata
    # a budget that no single pattern fits still gets one automaton per pattern
    _, tiny = _prepare([0, 1 << 20], [b"ACGT" * 60], [0], [0], api.tune(automaton_bytes=4096))
    assert tiny.nautomata == 1


# ---------------------------------------------------------------------------
# CPU model of the merged scan's decomposition (same rules as the kernel)
# ---------------------------------------------------------------------------

def _model_counts(text, seg_off, patterns, pair_seg, pair_pat, S, walks_per_tile):
    """Walks on the 128-byte grid of each segment; each walk starts in state 0 at its
    first byte inside the segment, owns the starts of its span, reads max(m) - 1 bytes
    past it, and counts a match that ends past the span only if it starts inside it."""
    counts = np.zeros(len(pair_seg), np.int64)
    for s in range(len(seg_off) - 1):
        ks = [k for k in range(len(pair_seg)) if pair_seg[k] == s]
        lo, hi = int(seg_off[s]), int(seg_off[s + 1])
        if not ks or hi <= lo:
            continue
        pats = [patterns[pair_pat[k]] for k in ks]
        t = api.ac_build(pats)
        maxm = max(len(p) for p in pats)
        base = lo & ~127
        tile = S * walks_per_tile
        for ts in range(base, hi, tile):
            own_end = min(hi, ts + tile)
            for w in range(walks_per_tile):
                ws = ts + w * S
                lo_w = min(max(lo - ws, 0), S)
                own = min(max(own_end - ws, 0), S)
                if own <= lo_w:
                    continue
                ln = min(own + maxm - 1, hi - ws)
                q = 0
                for j in range(lo_w, ln):
                    q = int(t.table[q, text[ws + j]])
                    for i in t.outputs(q):
                        if j < own or j + 1 < own + len(pats[i]):
                            counts[ks[i]] += 1
    return counts


@pytest.mark.parametrize("seed", range(4))
def test_merged_decomposition_model_matches_oracle(seed):
    rng = np.random.default_rng(40 + seed)
    nseg = 5
    lens = rng.integers(0, 3000, size=nseg)
    lens[0] = 1
    seg_off = np.zeros(nseg + 1, np.int64)
    seg_off[1:] = np.cumsum(lens) + 37  # the first segment does not start on a line
    seg_off[0] = 37
    n = int(seg_off[-1]) + 50
    text = rng.choice(np.frombuffer(b"ACGT", np.uint8), size=n)
    pats = _random_set(rng, 12, 1, 9)
    pats.append(text[int(seg_off[2]) + 3:int(seg_off[2]) + 11].tobytes())  # occurs
    pair_seg, pair_pat = [], []
    for s in range(nseg):
        for j in rng.choice(len(pats), size=6, replace=False):
            pair_seg.append(s)
            pair_pat.append(int(j))
    want = oracle.pair_counts(text, seg_off, pats, np.array(pair_seg), np.array(pair_pat))
    for S, wpt in ((128, 2), (256, 3), (1024, 1)):
        got = _model_counts(text, seg_off, pats, pair_seg, pair_pat, S, wpt)
        assert np.array_equal(got, want), (S, wpt)


def test_merged_prepare_pair_automata():
    """Pair automata (two bytes per step): only when step_bytes=2 asks for them (one
    byte per step is the default and step_bytes=1), packing patterns so that every
    automaton fits as one; their items are planned first."""
    rng = np.random.default_rng(6)
    pats = _random_set(rng, 6, 6, 12)
    n = len(pats)
    _, dflt = _prepare([0, 1 << 20], pats, [0] * n, list(range(n)))
    assert dflt.pair_items == 0 and dflt.nitems > 0
    _, two = _prepare([0, 1 << 20], pats, [0] * n, list(range(n)), api.tune(step_bytes=2))
    assert two.pair_items == two.nitems == dflt.nitems   # every item's automaton is a pair automaton
    _, one = _prepare([0, 1 << 20], pats, [0] * n, list(range(n)), api.tune(step_bytes=1))
    assert one.pair_items == 0 and one.nitems == dflt.nitems
    many = _random_set(rng, 300, 20, 40)
    m = len(many)
    _, single = _prepare([0, 1 << 20], many, [0] * m, list(range(m)))
    _, paired = _prepare([0, 1 << 20], many, [0] * m, list(range(m)), api.tune(step_bytes=2))
    assert single.pair_items == 0                       # large automata stay one-step
    assert paired.nautomata > single.nautomata and paired.pair_items == paired.nitems
    # more byte classes than a pair automaton takes: one-step only
    wide = [bytes(range(i, i + 12)) for i in range(0, 240, 12)]
    _, w = _prepare([0, 1 << 20], wide, [0] * len(wide), list(range(len(wide))), api.tune(step_bytes=2))
    assert w.pair_items == 0
    rc, _ = _prepare([0, 1000], pats, [0], [0], api.tune(step_bytes=3))
    assert rc == api.DFA_EINVAL


def test_merged_prepare_round_bytes():
    """Rounds of 32 or 64 bytes per walk: the plan records the choice for the run, and the
    larger rounds' transpose buffers leave less LDS for workgroups with large automata."""
    rng = np.random.default_rng(9)
    pats = _random_set(rng, 300, 20, 40)
    n = len(pats)
    _, r32 = _prepare([0, 1 << 24], pats, [0] * n, list(range(n)), api.tune(line_bytes=32, waves_per_group=8))
    _, r64 = _prepare([0, 1 << 24], pats, [0] * n, list(range(n)), api.tune(line_bytes=64, waves_per_group=8))
    assert int(r32.reserved[1]) == 32 and int(r64.reserved[1]) == 64
    assert r32.nitems == r64.nitems and r32.nautomata == r64.nautomata
    assert r64.lds_bytes - r32.lds_bytes == r64.waves_per_group * 64 * 32
    _, dflt = _prepare([0, 1 << 24], pats, [0] * n, list(range(n)))
    assert int(dflt.reserved[1]) in (32, 64)


def test_merged_prepare_waves_per_workgroup():
    """16-wave workgroups where they hold more resident waves (one copy of a large automaton
    shared by twice the waves), 8 where small automata fit four workgroups per CU anyway; a
    tile holds waves x 64 walks; more than 16 waves is refused."""
    rng = np.random.default_rng(12)
    big = _random_set(rng, 1024, 4, 64)
    n = len(big)
    _, p16 = _prepare([0, 1 << 26], big, [0] * n, list(range(n)))
    assert p16.waves_per_group == 16 and p16.nautomata > 1
    _, p8 = _prepare([0, 1 << 26], big, [0] * n, list(range(n)), api.tune(waves_per_group=8))
    assert p8.waves_per_group == 8 and p8.nautomata == p16.nautomata
    assert p8.nitems == 2 * p16.nitems
    small = _random_set(rng, 6, 6, 12)
    _, ps = _prepare([0, 1 << 26], small, [0] * 6, list(range(6)))
    assert ps.waves_per_group == 8
    rc, _ = _prepare([0, 1000], small, [0], [0], api.tune(waves_per_group=17))
    assert rc == api.DFA_EINVAL
