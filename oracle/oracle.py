"""ctypes wrapper around oracle.c -- the plain CPU reference (test infrastructure).

Each function restates the definition it computes; the C file carries the
same statements.  See oracle.c for the paper passages each one follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc -O2 (plain single-threaded C)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


class OracleLib:
    """The oracle's C functions loaded from one shared object (the default build, or a
    deliberately mutated copy built by the pin tests to show that the pins catch it)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        lib.oracle_occurrences.restype = ctypes.c_int64
        lib.oracle_occurrences.argtypes = [_u8p, ctypes.c_int64, _u8p, ctypes.c_int64,
                                           _i64p, ctypes.c_int64]
        lib.oracle_transition_table.restype = ctypes.c_int
        lib.oracle_transition_table.argtypes = [_u8p, ctypes.c_int64, _u8p]
        lib.oracle_automaton_scan.restype = ctypes.c_int64
        lib.oracle_automaton_scan.argtypes = [_u8p, ctypes.c_int64, _u8p, ctypes.c_int64,
                                              _i64p, ctypes.c_int64]
        lib.oracle_pair_counts.restype = ctypes.c_int
        lib.oracle_pair_counts.argtypes = [_u8p, _i64p, ctypes.c_int64, _u8p, _i64p, _i64p,
                                           ctypes.c_int64, _i64p, _i64p, ctypes.c_int64, _i64p]
        lib.oracle_degenerate_count.restype = ctypes.c_int64
        lib.oracle_degenerate_count.argtypes = [_u8p, ctypes.c_int64, _u8p, ctypes.c_int64, ctypes.c_int]
        self.lib = lib

    # -- definitions (see oracle.c) ------------------------------------------------------
    def occurrences(self, text, pattern) -> np.ndarray:
        """Ascending 0-based start offsets i with text[i:i+m] == pattern (overlaps included)."""
        t, p = _as_u8(text), _as_u8(pattern)
        c = self.lib.oracle_occurrences(_p(t, _u8p), t.size, _p(p, _u8p), p.size, None, 0)
        if c < 0:
            raise ValueError("pattern length must be >= 1")
        out = np.empty(max(c, 1), dtype=np.int64)
        c2 = self.lib.oracle_occurrences(_p(t, _u8p), t.size, _p(p, _u8p), p.size,
                                         _p(out, _i64p), c)
        assert c2 == c
        return out[:c]

    def count(self, text, pattern) -> int:
        """Number of (overlapping) occurrences of pattern in text."""
        t, p = _as_u8(text), _as_u8(pattern)
        c = self.lib.oracle_occurrences(_p(t, _u8p), t.size, _p(p, _u8p), p.size, None, 0)
        if c < 0:
            raise ValueError("pattern length must be >= 1")
        return int(c)

    def transition_table(self, pattern) -> np.ndarray:
        """(m+1, 256) uint8: entry (q, b) = longest prefix of P that is a suffix of P[:q] + b."""
        p = _as_u8(pattern)
        out = np.zeros((p.size + 1, 256), dtype=np.uint8)
        if self.lib.oracle_transition_table(_p(p, _u8p), p.size, _p(out, _u8p)) != 0:
            raise ValueError("pattern length must be in [1, 255]")
        return out

    def automaton_scan(self, table: np.ndarray, text) -> np.ndarray:
        """Start offsets reported by walking the (m+1, 256) automaton from q0 over text."""
        tab = np.ascontiguousarray(table, dtype=np.uint8)
        m = tab.shape[0] - 1
        t = _as_u8(text)
        c = self.lib.oracle_automaton_scan(_p(tab, _u8p), m, _p(t, _u8p), t.size, None, 0)
        out = np.empty(max(c, 1), dtype=np.int64)
        self.lib.oracle_automaton_scan(_p(tab, _u8p), m, _p(t, _u8p), t.size,
                                       _p(out, _i64p), c)
        return out[:c]

    def pair_counts(self, text, seg_off, patterns, pair_seg, pair_pat) -> np.ndarray:
        """Occurrence count of patterns[pair_pat[k]] inside segment pair_seg[k] for every k."""
        t = _as_u8(text)
        so = np.ascontiguousarray(seg_off, dtype=np.int64)
        pats = [bytes(p) for p in patterns]
        lens = np.array([len(p) for p in pats], dtype=np.int64)
        offs = np.zeros(len(pats), dtype=np.int64)
        if len(pats) > 1:
            offs[1:] = np.cumsum(lens)[:-1]
        blob = np.frombuffer(b"".join(pats) or b"\0", dtype=np.uint8).copy()
        ps = np.ascontiguousarray(pair_seg, dtype=np.int64)
        pp = np.ascontiguousarray(pair_pat, dtype=np.int64)
        out = np.zeros(ps.size, dtype=np.int64)
        rc = self.lib.oracle_pair_counts(_p(t, _u8p), _p(so, _i64p), so.size - 1,
                                         _p(blob, _u8p), _p(offs, _i64p), _p(lens, _i64p),
                                         len(pats), _p(ps, _i64p), _p(pp, _i64p), ps.size,
                                         _p(out, _i64p))
        if rc != 0:
            raise ValueError("bad pair / segment / pattern index")
        return out


    def degenerate_count(self, text, pattern, both_strands: bool = False) -> int:
        """Start positions where the IUPAC pattern (or, with both_strands, its reverse
        complement) matches; one count per position."""
        t = _as_u8(text)
        p = _as_u8(pattern)
        r = self.lib.oracle_degenerate_count(_p(t, _u8p), t.size, _p(p, _u8p), p.size, 1 if both_strands else 0)
        if r < 0:
            raise ValueError("bad degenerate pattern")
        return int(r)


def _load() -> OracleLib:
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            _lib = OracleLib(_LIB)
    return _lib


def _as_u8(buf) -> np.ndarray:
    if isinstance(buf, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(buf), dtype=np.uint8)
    a = np.ascontiguousarray(buf)
    if a.dtype != np.uint8:
        raise TypeError("expected uint8 data")
    return a


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def occurrences(text, pattern) -> np.ndarray:
    return _load().occurrences(text, pattern)


def count(text, pattern) -> int:
    return _load().count(text, pattern)


def transition_table(pattern) -> np.ndarray:
    return _load().transition_table(pattern)


def automaton_scan(table, text) -> np.ndarray:
    return _load().automaton_scan(table, text)


def pair_counts(text, seg_off, patterns, pair_seg, pair_pat) -> np.ndarray:
    return _load().pair_counts(text, seg_off, patterns, pair_seg, pair_pat)


def degenerate_count(text, pattern, both_strands: bool = False) -> int:
    return _load().degenerate_count(text, pattern, both_strands)
