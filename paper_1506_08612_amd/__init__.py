"""MI355X-native exact k-mer matching with finite automata.

The hot path (automaton build, device-resident text, domain-decomposed
automaton walk on gfx950, count reduction, sorted match positions, batched
and segmented scans) lives in the HIP library ``libdfa.so`` built from
``csrc/``; ``api`` is the thin ctypes binding over its C ABI.  Importing this
package loads nothing; ``api`` loads the library on first use and raises if it
is missing.
"""
__all__ = ["api", "synth"]
