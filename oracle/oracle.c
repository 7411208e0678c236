/*
 * oracle.c -- plain, slow, obviously correct CPU reference for exact k-mer
 * matching with a finite automaton (Memeti & Pllana, "Accelerating DNA
 * Sequence Analysis using Intel Xeon Phi", 2015).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * Every function below is the plain definition of what it computes, written
 * out with no blocking, threading, vectorisation or reordering:
 *
 *   oracle_occurrences      -- Sec. II.A: all i with T[i..i+m-1] = P,
 *                              overlapping occurrences included (Sec. II.A,
 *                              Aho-Corasick paragraph).  Positions are
 *                              0-based START offsets; the paper prints the
 *                              1-based index of the LAST character (Alg. 1),
 *                              which is start + m in 1-based terms.
 *   oracle_transition_table -- Sec. III.B: the failure-free ("improved AC")
 *                              automaton for one pattern stored as a sparse
 *                              state transition table with one column per
 *                              byte value (256 columns); bytes that lead
 *                              nowhere go to the start state q0.  The entry
 *                              for (q, b) is, by definition, the length of
 *                              the longest prefix of P that is a suffix of
 *                              (the q characters matched so far) followed by
 *                              b.  State q = "q pattern characters matched";
 *                              the only final state is m, numbered last, so
 *                              the paper's "q >= a-b" test is q == m.
 *   oracle_automaton_scan   -- Alg. 1 with one worker and one lane (the
 *                              paper's sequential form): q <- delta(q, T[c]),
 *                              report when q is final.
 *   oracle_pair_counts      -- the occurrence count of Sec. II.A applied to
 *                              every (text segment, pattern) pair of a batch.
 *
 * Parity pins (tests/test_oracle_pins.py): Python's regex engine with a
 * lookahead (an independent library routine for overlapping matches),
 * closed forms on periodic texts, additivity over concatenation, reverse
 * symmetry, absence by construction, planted occurrences, the textbook
 * string-matching automaton for "ababaca" (tests/golden/) and the expected
 * count of a k-mer in i.i.d. text.
 *
 * Build: gcc -O2 -shared -fPIC -o liboracle.so oracle.c   (see build.py)
 */
#include <stdint.h>
#include <string.h>

#define ORACLE_ALPHABET 256

/* All 0 <= i <= n-m with text[i..i+m-1] == pat[0..m-1].  Returns the number
 * of occurrences (or -1 when m < 1 or n < 0) and writes the first
 * min(count, cap) start positions, ascending, to pos (pos may be NULL when
 * cap == 0). */
int64_t oracle_occurrences(const uint8_t *text, int64_t n, const uint8_t *pat,
                           int64_t m, int64_t *pos, int64_t cap)
{
    int64_t count = 0;
    if (m < 1 || n < 0) return -1;
    for (int64_t i = 0; i + m <= n; ++i) {
        int64_t j = 0;
        while (j < m && text[i + j] == pat[j]) ++j;
        if (j == m) {
            if (count < cap) pos[count] = i;
            ++count;
        }
    }
    return count;
}

/* Does pat[0..k-1] equal the last k characters of (pat[0..q-1] . b)? */
static int prefix_is_suffix(const uint8_t *pat, int64_t q, int b, int64_t k)
{
    if (k == 0) return 1;
    if (pat[k - 1] != (uint8_t)b) return 0;
    /* pat[0..k-2] must equal pat[q-k+1 .. q-1] */
    for (int64_t j = 0; j < k - 1; ++j)
        if (pat[j] != pat[q - k + 1 + j]) return 0;
    return 1;
}

/* table[q*256 + b] for q = 0..m, b = 0..255: the longest k <= m such that
 * pat[0..k-1] is a suffix of pat[0..q-1] followed by the byte b.  States are
 * 0..m and m is the only final state.  Returns 0, or -1 if m < 1 or m > 255
 * (the state must fit one byte). */
int oracle_transition_table(const uint8_t *pat, int64_t m, uint8_t *table)
{
    if (m < 1 || m > 255) return -1;
    for (int64_t q = 0; q <= m; ++q) {
        for (int b = 0; b < ORACLE_ALPHABET; ++b) {
            /* the string read so far has length q + 1, and no state exceeds m */
            int64_t k = (q + 1 < m) ? q + 1 : m;
            while (!prefix_is_suffix(pat, q, b, k)) --k;
            table[q * ORACLE_ALPHABET + b] = (uint8_t)k;
        }
    }
    return 0;
}

/* Run the automaton of a (m+1) x 256 table over text, starting in q0, and
 * report a match whenever the final state m is entered.  The match that ends
 * at c starts at c - m + 1.  Returns the count and writes min(count, cap)
 * start positions. */
int64_t oracle_automaton_scan(const uint8_t *table, int64_t m,
                              const uint8_t *text, int64_t n,
                              int64_t *pos, int64_t cap)
{
    int64_t count = 0;
    int64_t q = 0;
    if (m < 1 || n < 0) return -1;
    for (int64_t c = 0; c < n; ++c) {
        q = table[q * ORACLE_ALPHABET + text[c]];
        if (q == m) {
            if (count < cap) pos[count] = c - m + 1;
            ++count;
        }
    }
    return count;
}

/* Batched counts: for each pair p, the number of occurrences of pattern
 * pair_pat[p] inside the segment text[seg_off[s] .. seg_off[s+1]-1] with
 * s = pair_seg[p].  Patterns are stored back to back: pattern j occupies
 * pats[pat_off[j] .. pat_off[j] + pat_len[j] - 1].  A match never spans two
 * segments.  Returns 0, or -1 on a bad argument. */
int oracle_pair_counts(const uint8_t *text, const int64_t *seg_off,
                       int64_t nseg, const uint8_t *pats,
                       const int64_t *pat_off, const int64_t *pat_len,
                       int64_t npat, const int64_t *pair_seg,
                       const int64_t *pair_pat, int64_t npairs,
                       int64_t *counts)
{
    for (int64_t p = 0; p < npairs; ++p) {
        int64_t s = pair_seg[p], j = pair_pat[p];
        if (s < 0 || s >= nseg || j < 0 || j >= npat) return -1;
        int64_t lo = seg_off[s], hi = seg_off[s + 1];
        if (hi < lo) return -1;
        counts[p] = oracle_occurrences(text + lo, hi - lo, pats + pat_off[j],
                                       pat_len[j], (int64_t *)0, 0);
        if (counts[p] < 0) return -1;
    }
    return 0;
}
