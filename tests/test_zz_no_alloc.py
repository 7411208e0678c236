"""dfa_count_noalloc -- dfa_count whose positions workspace is the library's own device
scratch, for callers that cannot allocate -- against dfa_count with a caller-owned
workspace, through the C ABI: two calls in a row, the second on a smaller input, counts and
sorted positions bit-exact (both plans of the positions path: per-walk counts for short
patterns, per-wave counts from m = 12 on)."""
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


def with_workspace(d, tab, m):
    """dfa_count with a caller workspace (the existing entry point)."""
    c, pos = api.positions(d, tab, m)
    return c, pos.cpu().numpy()


def without_allocation(d, tab, m, cap):
    cnt = torch.full((1,), -7, dtype=torch.int64, device=d.device)
    pos = torch.full((max(1, cap),), -7, dtype=torch.int64, device=d.device)
    api.count_noalloc_async(d, tab, m, cnt, pos, cap)
    torch.cuda.synchronize()
    c = int(cnt.item())
    return c, pos[:min(c, cap)].cpu().numpy()


@pytest.mark.parametrize("m,sizes", [(4, (700_000_000, 3_000_017)), (8, (120_000_000, 1_000_003)),
                                     (16, (400_000_000, 2_500_001)), (33, (64_000_000, 77_777))])
def test_noalloc_equals_dfa_count_two_calls_second_smaller(m, sizes):
    for k, n in enumerate(sizes):
        text = synth.genome_like(n, 70 + k + m, 0.05, n_run_mean=20_000)
        pat, off = synth.drawn_pattern(text, m, np.random.default_rng(n))
        if m >= 12:  # plant a few copies so that the re-walk of the per-wave plan runs
            for i in range(1, 40):
                j = (i * 7_919_993) % (n - m)
                text[j:j + m] = np.frombuffer(pat, np.uint8)
        say(f"noalloc m={m} call {k + 1}: n={n}")
        d = api.to_device(text)
        tab, mm = api.device_table(pat)
        need = api.count_workspace_bytes(n, mm, True)
        assert need <= api.NOALLOC_SCRATCH_BYTES
        c_ref, p_ref = with_workspace(d, tab, mm)
        c, p = without_allocation(d, tab, mm, max(1, c_ref))
        assert c == c_ref and np.array_equal(p, p_ref), (m, n)
        assert off in p.tolist()
        # a cap below the count: count stays exact, the first cap positions
        cap = max(1, c_ref // 3)
        c2, p2 = without_allocation(d, tab, mm, cap)
        assert c2 == c_ref and np.array_equal(p2, p_ref[:cap])
        # count only
        c3, _ = without_allocation(d, tab, mm, 0)
        assert c3 == c_ref
        if n < 5_000_000:
            assert np.array_equal(p, oracle.occurrences(text, pat))
        del d


def test_noalloc_refuses_positions_beyond_its_scratch():
    n = 800_000_000
    assert api.count_workspace_bytes(n, 8, True) > api.NOALLOC_SCRATCH_BYTES
    d = torch.zeros(n, dtype=torch.uint8, device="cuda")
    tab, m = api.device_table(b"ACGTACGT")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    pos = torch.zeros(16, dtype=torch.int64, device="cuda")
    with pytest.raises(api.DfaError) as e:
        api.count_noalloc_async(d, tab, m, cnt, pos, 16)
    assert e.value.rc == api.DFA_ENOSPACE
    # count only needs no scratch at any size
    api.count_noalloc_async(d, tab, m, cnt)
    assert int(cnt.item()) == 0
