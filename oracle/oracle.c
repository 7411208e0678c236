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
 *   oracle_degenerate_count -- start positions where a degenerate pattern
 *                              (IUPAC nucleotide codes) or, on request, its
 *                              reverse complement matches: the structure of
 *                              the paper's pattern table (Table 3), where
 *                              each 8-mer is paired with its reverse
 *                              complement and carries a 3-way alternative.
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

/* The bases an IUPAC code stands for, as a bit set (A=1, C=2, G=4, T=8); 0 for
 * a byte that is not a code.  A text byte matches a code iff it is one of the
 * bases A, C, G, T in the code's set: a text 'N' (an unknown base) matches
 * nothing. */
static int iupac_bases(uint8_t c)
{
    switch (c) {
    case 'A': return 1;
    case 'C': return 2;
    case 'G': return 4;
    case 'T': return 8;
    case 'R': return 1 | 4;          /* purine */
    case 'Y': return 2 | 8;          /* pyrimidine */
    case 'S': return 2 | 4;
    case 'W': return 1 | 8;
    case 'K': return 4 | 8;
    case 'M': return 1 | 2;
    case 'B': return 2 | 4 | 8;      /* not A */
    case 'D': return 1 | 4 | 8;      /* not C */
    case 'H': return 1 | 2 | 8;      /* not G */
    case 'V': return 1 | 2 | 4;      /* not T */
    case 'N': return 1 | 2 | 4 | 8;
    default: return 0;
    }
}

static int base_bit(uint8_t x)
{
    switch (x) {
    case 'A': return 1;
    case 'C': return 2;
    case 'G': return 4;
    case 'T': return 8;
    default: return 0;
    }
}

/* The complement of a code: the code of the complementary bases (A<->T, C<->G). */
static uint8_t iupac_complement(uint8_t c)
{
    int b = iupac_bases(c), r = 0;
    if (b & 1) r |= 8;
    if (b & 8) r |= 1;
    if (b & 2) r |= 4;
    if (b & 4) r |= 2;
    static const char code_of[16] = {0, 'A', 'C', 'M', 'G', 'R', 'S', 'V',
                                     'T', 'W', 'Y', 'H', 'K', 'D', 'B', 'N'};
    return (uint8_t)code_of[r];
}

/* Does the degenerate pattern p[0..m-1] match text[i..i+m-1]? */
static int degenerate_at(const uint8_t *text, int64_t i, const uint8_t *p, int64_t m)
{
    for (int64_t j = 0; j < m; ++j)
        if (!(iupac_bases(p[j]) & base_bit(text[i + j]))) return 0;
    return 1;
}

/* Number of start positions i (0 <= i <= n-m) where the degenerate pattern
 * matches, or (both_strands != 0) where it or its reverse complement matches
 * -- one count per position.  Returns -1 for m < 1, m > 255 or a byte of pat
 * that is not an IUPAC code. */
int64_t oracle_degenerate_count(const uint8_t *text, int64_t n, const uint8_t *pat,
                                int64_t m, int both_strands)
{
    uint8_t rc[255];
    if (m < 1 || m > 255 || n < 0) return -1;
    for (int64_t j = 0; j < m; ++j) {
        if (!iupac_bases(pat[j])) return -1;
        rc[m - 1 - j] = iupac_complement(pat[j]);
    }
    int64_t count = 0;
    for (int64_t i = 0; i <= n - m; ++i)
        if (degenerate_at(text, i, pat, m) || (both_strands && degenerate_at(text, i, rc, m))) ++count;
    return count;
}
