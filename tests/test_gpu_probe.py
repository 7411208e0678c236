"""The LDS read probe (dfa_lds_probe) on the device: every width and mode runs to its end,
reports the reads it made, and never writes its sink (the checksum it guards cannot occur)."""
from __future__ import annotations

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1506_08612_amd import api  # noqa: E402


@pytest.mark.parametrize("mode", sorted(api.LDS_PROBE_MODES))
@pytest.mark.parametrize("width", [1, 2])
def test_probe_runs_and_reports_its_reads(width, mode):
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    blocks, iters = 300, 64
    reads = api.lds_probe(width, mode, blocks, iters, sink)
    torch.cuda.synchronize()
    assert reads == blocks * 512 * iters * 8
    assert int(sink.item()) == 0
