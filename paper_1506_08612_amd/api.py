"""ctypes binding over libdfa.so (include/dfa.h).

Argument marshalling only: every step of the scan runs in the HIP library.
PyTorch provides device memory and streams.  Importing this module loads the
library and raises if it has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdfa.so")

DFA_OK = 0
DFA_EINVAL = -1
DFA_EHIP = -2
DFA_ENOSPACE = -3
MAX_M = 255
ALPHABET = 256


class DfaError(RuntimeError):
    def __init__(self, rc: int, msg: str):
        super().__init__(f"libdfa error {rc}: {msg}")
        self.rc = rc


class Tune(ctypes.Structure):
    """dfa_tune: launch shape; zero fields mean "library default"."""
    _fields_ = [
        ("chain_bytes", ctypes.c_int64),
        ("waves_per_group", ctypes.c_int32),
        ("chains_per_lane", ctypes.c_int32),
        ("dfas_per_group", ctypes.c_int32),
        ("tile_bytes", ctypes.c_int32),
        ("line_bytes", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_vp = ctypes.c_void_p
_TuneP = ctypes.POINTER(Tune)

# name -> (restype, argtypes); mirrors include/dfa.h
SIGNATURES = {
    "dfa_last_error": (ctypes.c_char_p, []),
    "dfa_version": (ctypes.c_char_p, []),
    "dfa_table_bytes": (_i64, [_i32]),
    "dfa_build": (ctypes.c_int, [_vp, _i32, _vp]),
    "dfa_count_workspace_bytes": (_i64, [_i64, _i32, _i32, _TuneP]),
    "dfa_count": (ctypes.c_int, [_vp, _i64, _vp, _i32, _vp, _vp, _i64, _vp, _i64, _TuneP, _vp]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1506_08612_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return lib.dfa_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise DfaError(rc, last_error())
    return rc


def tune(chain_bytes: int = 0, waves_per_group: int = 0, chains_per_lane: int = 0,
         dfas_per_group: int = 0, tile_bytes: int = 0, line_bytes: int = 0) -> Tune:
    return Tune(chain_bytes, waves_per_group, chains_per_lane, dfas_per_group, tile_bytes,
                line_bytes)


def _tune_ptr(t: Optional[Tune]):
    return ctypes.byref(t) if t is not None else None


def table_bytes(m: int) -> int:
    return _check(lib.dfa_table_bytes(m))


def build_table(pattern: bytes) -> np.ndarray:
    """Host automaton build: (m+1, 256) uint8 transition table."""
    p = np.frombuffer(bytes(pattern), dtype=np.uint8)
    m = p.size
    if m < 1 or m > MAX_M:
        raise DfaError(DFA_EINVAL, f"pattern length {m} outside [1, {MAX_M}]")
    out = np.empty((m + 1, ALPHABET), dtype=np.uint8)
    _check(lib.dfa_build(p.ctypes.data, m, out.ctypes.data))
    return out


# ---------------------------------------------------------------------------
# device-side helpers (torch is only the allocator and stream provider)
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def to_device(arr, device="cuda") -> "torch.Tensor":
    """Copy a host byte array into a new device tensor (the text stays resident)."""
    torch = _torch()
    a = np.ascontiguousarray(arr)
    t = torch.from_numpy(a.view(np.uint8).reshape(-1))
    return t.to(device, non_blocking=False)


def device_table(pattern: bytes, device="cuda"):
    """Build on the host, upload once: returns (table tensor, m)."""
    tab = build_table(pattern)
    return to_device(tab, device), tab.shape[0] - 1


def count_workspace_bytes(n: int, m: int, want_positions: bool, t: Optional[Tune] = None) -> int:
    return _check(lib.dfa_count_workspace_bytes(n, m, int(bool(want_positions)), _tune_ptr(t)))


def count_async(text, table, m: int, count_out, positions_out=None, cap: int = 0,
                workspace=None, t: Optional[Tune] = None, stream=None) -> None:
    """Enqueue dfa_count on the stream.  All tensors are device tensors:
    text uint8[n], table uint8[(m+1)*256], count_out int64[1], positions_out int64[cap]."""
    n = text.numel()
    wsp = workspace.data_ptr() if workspace is not None else None
    wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    pos = positions_out.data_ptr() if positions_out is not None else None
    _check(lib.dfa_count(text.data_ptr() if n else None, n, table.data_ptr(), m, count_out.data_ptr(),
                         pos, int(cap), wsp, wsb, _tune_ptr(t), _stream_handle(stream)))


def count(text, table, m: int, t: Optional[Tune] = None, stream=None) -> int:
    """Exact overlapping match count (synchronises the stream)."""
    torch = _torch()
    out = torch.empty(1, dtype=torch.int64, device=text.device)
    count_async(text, table, m, out, t=t, stream=stream)
    return int(out.item())


def positions(text, table, m: int, cap: Optional[int] = None, t: Optional[Tune] = None,
              stream=None):
    """(count, sorted int64 start offsets).  If cap is None the count is taken
    first and the output sized from it; otherwise at most cap positions."""
    torch = _torch()
    n = text.numel()
    dev = text.device
    out = torch.empty(1, dtype=torch.int64, device=dev)
    if cap is None:
        count_async(text, table, m, out, t=t, stream=stream)
        cap = int(out.item())
    pos = torch.empty(max(int(cap), 1), dtype=torch.int64, device=dev)
    wsb = count_workspace_bytes(n, m, True, t)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    count_async(text, table, m, out, pos, cap, ws, t=t, stream=stream)
    c = int(out.item())
    return c, pos[:min(c, int(cap))]


def exported_symbols() -> Sequence[str]:
    return list(SIGNATURES)
