"""CPU tests of the library's host side: exported ABI, automaton build, argument
checks, workspace sizing, and a CPU model of the scan's decomposition.

No compute call reaches a GPU here: every dfa_count call below fails its
argument checks, which run before anything is launched.
"""
from __future__ import annotations

import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_1506_08612_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "dfa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dfa_\w+)\s*\(", src)))


def test_library_exports_every_header_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", api.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(dfa_\w+)", out))
    declared = header_functions()
    assert declared, "no declarations parsed"
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    # the binding wraps exactly what the header declares
    assert sorted(api.exported_symbols()) == declared
    for f in declared:
        assert hasattr(api.lib, f)


def test_version_and_error_string():
    assert b"gfx950" in api.lib.dfa_version()
    assert api.lib.dfa_table_bytes(0) == api.DFA_EINVAL
    assert "m=0" in api.last_error()


@pytest.mark.parametrize("alphabet", [b"AC", b"ACGT", b"ACGTN", bytes(range(256))])
def test_build_matches_oracle_definition(alphabet):
    rng = np.random.default_rng(len(alphabet))
    a = np.frombuffer(alphabet, np.uint8)
    for m in list(range(1, 20)) + [31, 32, 63, 64, 65, 100, 128, 200, 254, 255]:
        p = a[rng.integers(0, a.size, m)].tobytes()
        got = api.build_table(p)
        want = oracle.transition_table(p)
        assert np.array_equal(got, want), (m, p)


def test_build_periodic_and_single():
    for p in (b"A", b"AAAA", b"ACACA", b"ababaca", b"N" * 255, b"ACGT" * 16):
        assert np.array_equal(api.build_table(p), oracle.transition_table(p)), p


def test_table_bytes():
    assert api.table_bytes(1) == 512
    assert api.table_bytes(64) == 65 * 256
    assert api.table_bytes(255) == 256 * 256
    for bad in (0, -1, 256):
        assert api.lib.dfa_table_bytes(bad) == api.DFA_EINVAL


def test_build_rejects_bad_args():
    buf = (ctypes.c_uint8 * 1024)()
    pat = (ctypes.c_uint8 * 300)()
    assert api.lib.dfa_build(None, 4, buf) == api.DFA_EINVAL
    assert api.lib.dfa_build(pat, 4, None) == api.DFA_EINVAL
    assert api.lib.dfa_build(pat, 0, buf) == api.DFA_EINVAL
    assert api.lib.dfa_build(pat, 256, buf) == api.DFA_EINVAL


def test_count_argument_checks_run_before_launch():
    # bogus but non-null "device" pointers: the checks reject them before any HIP call
    fake = 1 << 20
    L = api.lib
    assert L.dfa_count(fake, -1, fake, 8, fake, None, 0, None, 0, None, None) == api.DFA_EINVAL
    assert L.dfa_count(fake, 10, fake, 0, fake, None, 0, None, 0, None, None) == api.DFA_EINVAL
    assert L.dfa_count(fake, 10, fake, 256, fake, None, 0, None, 0, None, None) == api.DFA_EINVAL
    assert L.dfa_count(None, 10, fake, 8, fake, None, 0, None, 0, None, None) == api.DFA_EINVAL
    assert L.dfa_count(fake, 10, None, 8, fake, None, 0, None, 0, None, None) == api.DFA_EINVAL
    assert L.dfa_count(fake, 10, fake, 8, None, None, 0, None, 0, None, None) == api.DFA_EINVAL
    assert L.dfa_count(fake + 1, 10, fake, 8, fake, None, 0, None, 0, None, None) == api.DFA_EINVAL
    assert "aligned" in api.last_error()
    assert L.dfa_count(fake, 10, fake, 8, fake, fake, -1, None, 0, None, None) == api.DFA_EINVAL
    t = api.tune(chain_bytes=24)
    assert L.dfa_count(fake, 10, fake, 8, fake, None, 0, None, 0, ctypes.byref(t), None) == api.DFA_EINVAL
    t = api.tune(chains_per_lane=3)
    assert L.dfa_count(fake, 10, fake, 8, fake, None, 0, None, 0, ctypes.byref(t), None) == api.DFA_EINVAL
    t = api.tune(chains_per_lane=2, line_bytes=128)  # a shape the library does not build
    assert L.dfa_count(fake, 10, fake, 8, fake, None, 0, None, 0, ctypes.byref(t), None) == api.DFA_EINVAL
    t = api.tune(line_bytes=96)
    assert L.dfa_count(fake, 10, fake, 8, fake, None, 0, None, 0, ctypes.byref(t), None) == api.DFA_EINVAL
    # 16 waves per workgroup: only with one walk per lane and 64-byte rounds
    for bad in (dict(waves_per_group=17), dict(waves_per_group=16, line_bytes=128),
                dict(waves_per_group=16, chains_per_lane=2, line_bytes=64)):
        t = api.tune(**bad)
        assert L.dfa_count(fake, 10, fake, 8, fake, None, 0, None, 0, ctypes.byref(t), None) == api.DFA_EINVAL, bad
    t = api.tune(waves_per_group=16)
    assert api.lib.dfa_count_workspace_bytes(1 << 20, 8, 1, ctypes.byref(t)) > 0
    t = api.tune()
    t.reserved[1] = 5
    assert L.dfa_count(fake, 10, fake, 8, fake, None, 0, None, 0, ctypes.byref(t), None) == api.DFA_EINVAL
    # positions requested with too small a workspace
    assert L.dfa_count(fake, 1 << 20, fake, 8, fake, fake, 10, fake, 16, None, None) == api.DFA_ENOSPACE


def test_fasta_argument_checks_run_before_launch():
    fake = 1 << 20
    L = api.lib
    ws = L.dfa_fasta_workspace_bytes(1000)
    assert ws > 0 and L.dfa_fasta_workspace_bytes(0) == 0
    assert L.dfa_fasta_workspace_bytes(-1) == api.DFA_EINVAL
    # raw must be 16-byte aligned (whole-piece loads); out may have any alignment
    for off in (1, 4, 8):
        assert L.dfa_fasta_normalize(fake + off, 1000, fake, fake, 4, fake, fake, ws, None) == api.DFA_EINVAL
        assert "aligned" in api.last_error()
    assert L.dfa_fasta_normalize(fake, 1000, fake, fake, 4, fake + 4, fake, ws, None) == api.DFA_EINVAL
    assert L.dfa_fasta_normalize(fake, 1000, None, fake, 4, fake, fake, ws, None) == api.DFA_EINVAL
    assert L.dfa_fasta_normalize(fake, 1000, fake, None, 4, fake, fake, ws, None) == api.DFA_EINVAL
    assert L.dfa_fasta_normalize(fake, 1000, fake, fake, 4, fake, fake, ws - 1, None) == api.DFA_ENOSPACE
    assert L.dfa_fasta_normalize(fake, 1000, fake, fake, 4, fake, fake + 16, ws, None) == api.DFA_ENOSPACE


def test_binding_rejects_host_tensors_before_any_call():
    import torch
    tab = torch.zeros(9 * 256, dtype=torch.uint8)
    out = torch.zeros(1, dtype=torch.int64)
    with pytest.raises(ValueError, match="device tensor"):
        api.count_async(torch.zeros(100, dtype=torch.uint8), tab, 8, out)
    with pytest.raises(TypeError, match="torch tensor"):
        api.count_async(np.zeros(100, np.uint8), tab, 8, out)
    with pytest.raises(ValueError, match="device tensor"):
        api.fasta_normalize(torch.zeros(100, dtype=torch.uint8))


def test_workspace_bytes():
    assert api.count_workspace_bytes(1 << 30, 8, False) == 0
    a = api.count_workspace_bytes(1 << 30, 8, True)
    b = api.count_workspace_bytes(1 << 30, 8, True, api.tune(chain_bytes=4096))
    assert a > b > 0
    assert api.count_workspace_bytes(0, 8, True) == 0
    assert api.lib.dfa_count_workspace_bytes(-1, 8, 1, None) == api.DFA_EINVAL


# ----------------------------------------------------------------------------------------
# CPU model of the decomposition (Sec. III.A): walk g owns starts [gS, (g+1)S) and reads
# m-1 bytes past them; summing what the walks report must give every match exactly once,
# for every span length, including spans shorter than the pattern.
# ----------------------------------------------------------------------------------------

def model_scan(text: bytes, pat: bytes, S: int):
    tab = oracle.transition_table(pat)
    m, n = len(pat), len(text)
    out = []
    for start in range(0, n, S):
        end = min(n, start + S + m - 1)
        out.extend(start + p for p in oracle.automaton_scan(tab, text[start:end]).tolist())
    return out


@pytest.mark.parametrize("S", [1, 2, 3, 5, 16, 17, 64, 128, 1000])
def test_decomposition_counts_every_match_once(S):
    rng = np.random.default_rng(S)
    for _ in range(30):
        n = int(rng.integers(0, 1500))
        t = np.frombuffer(b"AC", np.uint8)[rng.integers(0, 2, n)].tobytes()
        m = int(rng.integers(1, 12))
        p = np.frombuffer(b"AC", np.uint8)[rng.integers(0, 2, m)].tobytes()
        assert model_scan(t, p, S) == oracle.occurrences(t, p).tolist()


# ----------------------------------------------------------------------------------------
# batched scans: planning and argument checks run on the host (workspace == NULL is a size
# query that launches nothing)
# ----------------------------------------------------------------------------------------

def _plan(seg_off, ms, pair_seg, pair_pat, t=None):
    seg_off = np.asarray(seg_off, np.int64)
    ms = np.asarray(ms, np.int32)
    toff = np.zeros(ms.size, np.int64)
    if ms.size > 1:
        toff[1:] = np.cumsum((ms.astype(np.int64) + 1) * 256)[:-1]
    ps = np.asarray(pair_seg, np.int32)
    pp = np.asarray(pair_pat, np.int32)
    plan = api.BatchPlan()
    rc = api.lib.dfa_batch_prepare(seg_off.ctypes.data, seg_off.size - 1, toff.ctypes.data, ms.ctypes.data,
                                   ms.size, ps.ctypes.data, pp.ctypes.data, ps.size, None, 0,
                                   ctypes.byref(t) if t is not None else None, ctypes.byref(plan), None)
    return rc, plan


def test_batch_plan_groups_and_items():
    # one 1 MB segment, 20 patterns of length 30 (31 rows each): 4 per group by default,
    # 8 per group fit 255 rows
    rc, plan = _plan([0, 1 << 20], [30] * 20, [0] * 20, list(range(20)))
    assert rc == api.DFA_OK, api.last_error()
    assert plan.ngroups == 5 and plan.npairs == 20 and plan.text_bytes == 1 << 20
    assert plan.nitems % plan.ngroups == 0 and plan.nitems >= plan.ngroups
    assert plan.workspace_bytes > 0 and plan.dfas_per_group == 4
    rc, plan = _plan([0, 1 << 20], [30] * 20, [0] * 20, list(range(20)), api.tune(dfas_per_group=8))
    assert rc == api.DFA_OK and plan.ngroups == 3 and plan.dfas_per_group == 8
    # rows cap the group: patterns of length 126 take 127 rows, two per group (255 rows
    # are usable)
    rc, plan = _plan([0, 4096], [126] * 5, [0] * 5, list(range(5)))
    assert rc == api.DFA_OK and plan.ngroups == 3
    rc, plan = _plan([0, 4096], [127] * 4, [0] * 4, list(range(4)))
    assert rc == api.DFA_OK and plan.ngroups == 4
    # segments of length 0 contribute no work
    rc, plan = _plan([0, 0, 0], [4], [0, 1], [0, 0])
    assert rc == api.DFA_OK and plan.nitems == 0 and plan.npairs == 2
    rc, plan = _plan([0, 1000], [8] * 3, [0] * 3, [0, 1, 2], api.tune(dfas_per_group=4, waves_per_group=2))
    assert rc == api.DFA_OK and plan.dfas_per_group == 4 and plan.waves_per_group == 2


def test_batch_plan_rejects_bad_arguments():
    assert _plan([0, 10, 5], [4], [0], [0])[0] == api.DFA_EINVAL          # seg_off decreasing
    assert _plan([0, 10], [0], [0], [0])[0] == api.DFA_EINVAL             # m < 1
    assert _plan([0, 10], [256], [0], [0])[0] == api.DFA_EINVAL           # m > 255
    assert _plan([0, 10], [255], [0], [0])[0] == api.DFA_EINVAL           # batched: m <= 254
    assert _plan([0, 10], [4], [1], [0])[0] == api.DFA_EINVAL             # segment out of range
    assert _plan([0, 10], [4], [0], [3])[0] == api.DFA_EINVAL             # pattern out of range
    assert _plan([0, 10], [4], [0], [0], api.tune(dfas_per_group=5))[0] == api.DFA_EINVAL
    assert _plan([0, 10], [4], [0], [0], api.tune(waves_per_group=9))[0] == api.DFA_EINVAL
    plan = api.BatchPlan()
    assert api.lib.dfa_batch_run(None, 0, None, 0, None, ctypes.byref(plan), None, None) == api.DFA_EINVAL
    rc, plan = _plan([0, 100], [4], [0], [0])
    assert plan.tables_bytes == 5 * 256
    fake = 1 << 20
    # text shorter than the segments span
    assert api.lib.dfa_batch_run(fake, 50, fake, 4096, fake, ctypes.byref(plan), fake, None) == api.DFA_EINVAL
    # tables buffer shorter than the tables the plan refers to
    assert api.lib.dfa_batch_run(fake, 100, fake, 1000, fake, ctypes.byref(plan), fake, None) == api.DFA_EINVAL


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch must still leave one HIP runtime mapped:
    torch's copy and the system's are distinct files, and a second runtime in the
    process sees no device."""
    code = ("from paper_1506_08612_amd import api\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


def test_scan_events_hook_arguments():
    """dfa_set_scan_events takes both events or neither (no GPU call is made)."""
    assert api.lib.dfa_set_scan_events(None, None) == api.DFA_OK
    assert api.lib.dfa_set_scan_events(ctypes.c_void_p(16), None) == api.DFA_EINVAL
    assert "both events" in api.last_error()
    assert api.lib.dfa_set_scan_events(None, ctypes.c_void_p(16)) == api.DFA_EINVAL
    assert api.lib.dfa_set_scan_events(None, None) == api.DFA_OK


def test_noalloc_scratch_limit_checked_on_the_host():
    """dfa_count_noalloc refuses, before touching any device, positions whose workspace
    would not fit the library's scratch; the binding's constant is the header's."""
    src = open(os.path.join(ROOT, "include", "dfa.h")).read()
    m = re.search(r"#define DFA_NOALLOC_SCRATCH_BYTES \((\d+)LL << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == api.NOALLOC_SCRATCH_BYTES
    n = 1_000_000_000
    assert api.count_workspace_bytes(n, 8, True) > api.NOALLOC_SCRATCH_BYTES
    fake = 1 << 20  # never dereferenced: the size check comes first
    rc = api.lib.dfa_count_noalloc(fake, n, fake, 8, fake, fake, 1, None, None)
    assert rc == api.DFA_ENOSPACE and "scratch" in api.last_error()
    # bad arguments are still EINVAL
    assert api.lib.dfa_count_noalloc(fake, -1, fake, 8, fake, fake, 1, None, None) == api.DFA_EINVAL
    assert api.lib.dfa_count_noalloc(fake, 100, fake, 0, fake, fake, 1, None, None) == api.DFA_EINVAL


def test_lds_probe_argument_checks_run_before_launch():
    fake = 1 << 20
    L = api.lib
    ok_args = (2, 1, 16, 4, fake, None)
    for i, bad in ((0, 3), (1, 3), (1, -1), (2, 0), (2, (1 << 20) + 1), (3, 0), (3, (1 << 24) + 1)):
        a = list(ok_args)
        a[i] = bad
        assert L.dfa_lds_probe(*a) == api.DFA_EINVAL, (i, bad)
    assert L.dfa_lds_probe(2, 1, 16, 4, None, None) == api.DFA_EINVAL
    assert L.dfa_lds_probe(2, 1, 16, 4, fake + 4, None) == api.DFA_EINVAL  # sink not 8-byte aligned
