"""FASTA normalisation by its definition (test infrastructure only).

The paper scans GenBank genomes (Table 1), which come as FASTA text: records
that each start with a header line ("> ..."), the sequence wrapped over lines
of any width, lower-case letters for soft-masked regions.  The scan itself
wants one plain byte string per record.  The definition used here:

* a line is the bytes up to and including the next '\\n' (the last line may
  lack it);
* a line whose first byte is '>' is a header: it starts a new record and none
  of its bytes are kept;
* every other byte is kept, except '\\n' and '\\r', with 'a'..'z' turned into
  'A'..'Z';
* record k's sequence starts where the kept bytes stood when its header was
  read; kept bytes before the first header form a preamble (normally empty).

Plain Python over lines; small inputs only.
"""
from __future__ import annotations

from typing import List, Tuple


def normalize(raw: bytes) -> Tuple[bytes, List[int]]:
    """(kept bytes, start offset of every record's sequence in them)."""
    out = bytearray()
    starts = []
    for line in bytes(raw).split(b"\n"):
        if line[:1] == b">":
            starts.append(len(out))
            continue
        for b in line:
            if b == 0x0D:  # '\r'
                continue
            if 0x61 <= b <= 0x7A:  # 'a'..'z'
                b -= 0x20
            out.append(b)
    return bytes(out), starts


__all__ = ["normalize"]
