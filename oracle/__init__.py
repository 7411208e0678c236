"""CPU oracle for exact k-mer matching (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product library.

``oracle.ac`` builds the paper's multi-pattern automaton by its definition
(brute force over prefix strings, small pattern sets only).
"""
from .oracle import (  # noqa: F401
    build,
    occurrences,
    count,
    transition_table,
    automaton_scan,
    pair_counts,
    degenerate_count,
    lib_path,
    OracleLib,
)
from . import ac, fasta  # noqa: F401,E402
