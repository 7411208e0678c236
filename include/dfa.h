/*
 * dfa.h -- C ABI of libdfa.so: exact k-mer matching with finite automata on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: S. Memeti and S. Pllana, "Accelerating DNA Sequence Analysis using
 * Intel Xeon Phi" (PBio at ISPA 2015).  The library builds the single-pattern
 * failure-free automaton as a 256-column state transition table (Sec. III.B)
 * and runs Algorithm 1's domain-decomposed scan (Sec. III.A): the text is split
 * into chunks, every chunk is read with m-1 extra characters so that matches
 * crossing a border are found, each worker starts in q0, steps
 * q <- delta(q, T[c]) once per character and reports whenever q is final.
 *
 * Conventions for every entry point:
 *   - plain C types only; every size and offset is int64_t (texts exceed 2^31);
 *   - "device" pointers are GPU memory of the current HIP device, "host"
 *     pointers are CPU memory; the caller owns all memory, nothing is
 *     allocated by the library;
 *   - arguments are checked synchronously before anything is launched; a bad
 *     argument returns DFA_EINVAL and launches nothing;
 *   - device work is enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream) and is asynchronous: results are valid once the stream is
 *     synchronised;
 *   - no exception crosses the ABI; on failure dfa_last_error() returns a
 *     message (thread-local, valid until the next call on that thread).
 *
 * Match semantics (Sec. II.A): the text T[0..n-1] and pattern P[0..m-1] are
 * byte strings; an occurrence is every i with 0 <= i <= n-m and
 * T[i..i+m-1] == P, overlapping occurrences included.  Positions are 0-based
 * START offsets (Algorithm 1 prints the index of the last character, which is
 * start + m - 1).  Comparison is byte-exact over all 256 byte values: a byte
 * that does not occur in P sends the automaton to q0 (Sec. III.B, sparse STT).
 */
#ifndef DFA_H
#define DFA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DFA_OK 0
#define DFA_EINVAL (-1)  /* bad argument: null pointer, size out of range, misalignment */
#define DFA_EHIP (-2)    /* HIP runtime or launch error; see dfa_last_error() */
#define DFA_ENOSPACE (-3) /* workspace smaller than dfa_*_workspace_bytes() */

#define DFA_MAX_M 255    /* states are one byte: q in 0..m */
#define DFA_ALPHABET 256 /* one table column per byte value (Sec. III.B) */

/* Launch shape.  Pass NULL for the library's choice.  A zero field means
 * "choose for me".  Results never depend on these values, only speed does. */
typedef struct dfa_tune {
    int64_t chain_bytes;     /* bytes of text one automaton walk owns (multiple of 16) */
    int32_t waves_per_group; /* 64-lane waves per workgroup, 1..8 */
    int32_t chains_per_lane; /* independent walks interleaved in one lane: 1 (or 2 with
                              * 64-byte rounds) */
    int32_t dfas_per_group;  /* batched scans: automata walked together: 2, 4, 8 or 16 */
    int32_t tile_bytes;      /* unused, must be zero */
    int32_t line_bytes;      /* bytes of every walk fetched per round: 64 or 128 */
    int32_t reserved[3];     /* must be zero */
} dfa_tune;

/* Message for the last failed call on this thread ("" if none). */
const char *dfa_last_error(void);

/* Library version string. */
const char *dfa_version(void);

/* ------------------------------------------------------------------------ */
/* Automaton build (Sec. III.B: failure transitions folded into delta;      */
/* sparse 256-column STT; final state numbered last).                       */
/* ------------------------------------------------------------------------ */

/* Size in bytes of the transition table of a length-m pattern:
 * (m+1) * 256, or DFA_EINVAL if m < 1 or m > DFA_MAX_M. */
int64_t dfa_table_bytes(int32_t m);

/* Host-only.  Writes the (m+1) x 256 uint8 table, row-major by state, to
 * `table` (host, dfa_table_bytes(m) bytes).  State q means "the last q bytes
 * read equal P[0..q-1] and no longer prefix of P ends here"; entry (q, b) is
 * the state after reading byte b in state q.  The only final state is m, the
 * highest number, so "q is final" is q == m.  Entries for bytes absent from P
 * are 0.  Returns DFA_OK or DFA_EINVAL (null pointer, m out of range). */
int dfa_build(const uint8_t *pattern, int32_t m, uint8_t *table);

/* ------------------------------------------------------------------------ */
/* Single pattern, one text (Algorithm 1).                                  */
/* ------------------------------------------------------------------------ */

/* Device workspace needed by dfa_count for this (n, m, want_positions, tune):
 * 0 when want_positions == 0; otherwise the per-walk match counts and their
 * prefix sums.  Returns bytes, or DFA_EINVAL. */
int64_t dfa_count_workspace_bytes(int64_t n, int32_t m, int32_t want_positions,
                                  const dfa_tune *tune);

/* Count every occurrence of the pattern whose table is `table` in text[0..n-1].
 *   text       device, n bytes, 16-byte aligned, read-only; n >= 0 (n < m -> 0)
 *   table      device, dfa_table_bytes(m) bytes from dfa_build, 4-byte aligned
 *   count      device, one int64, OVERWRITTEN with the exact number of matches
 *   positions  device or NULL; if non-NULL and cap > 0, receives the first
 *              min(count, cap) start offsets in ascending order (count stays
 *              exact when it exceeds cap: size the buffer from it and retry)
 *   workspace  device, >= dfa_count_workspace_bytes(...) bytes, 256-byte
 *              aligned; may be NULL when positions == NULL
 * Returns DFA_OK, DFA_EINVAL, DFA_ENOSPACE or DFA_EHIP. */
int dfa_count(const uint8_t *text, int64_t n, const uint8_t *table, int32_t m,
              int64_t *count, int64_t *positions, int64_t cap,
              void *workspace, int64_t workspace_bytes,
              const dfa_tune *tune, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched: many patterns over many texts in one launch.                    */
/* ------------------------------------------------------------------------ */

/* Texts are segments of one buffer: segment s is text[seg_off[s] .. seg_off[s+1]-1]
 * and no match crosses a segment border.  Patterns are given by their tables
 * from dfa_build, stored back to back on the device: pattern j has length m[j]
 * (1..254) and its table starts at byte table_off[j] (a multiple of 4) of
 * `tables`.
 * Work pair k asks for the number of occurrences of pattern pair_pat[k] in
 * segment pair_seg[k].  Every pattern keeps its own automaton and its own
 * m-1 overlap, so patterns of different lengths are counted exactly (the
 * equal-length restriction of the merged automaton of Sec. III.A does not
 * apply).  Segments of the same pattern group are read once per workgroup for
 * all automata of the group.
 *
 * Two steps, so that the second can be captured in a HIP graph and replayed:
 *   dfa_batch_prepare  host: validates the arrays (all host memory), packs
 *                      patterns into groups and tiles into work items, and
 *                      uploads that plan into `workspace` (device, 256-byte
 *                      aligned).  With workspace == NULL it only fills `plan`
 *                      (including plan->workspace_bytes).  Synchronises `stream`.
 *   dfa_batch_run      device only: zeroes counts[0..npairs-1] (int64, device)
 *                      and launches the scan.  `text` (device, n >= plan->text_bytes
 *                      bytes, 16-byte aligned) and `tables` (device, tables_bytes
 *                      >= plan->tables_bytes) must be the buffers the plan
 *                      describes; the workspace must hold the plan.  Asynchronous,
 *                      allocates nothing, no memset nodes.
 * dfa_count_batch = prepare + run.  All return DFA_OK, DFA_EINVAL,
 * DFA_ENOSPACE or DFA_EHIP. */
typedef struct dfa_batch_plan {
    int64_t nitems;          /* work items: (tile of a segment, pattern group) */
    int64_t ngroups;         /* pattern groups */
    int64_t npairs;          /* counters written by dfa_batch_run */
    int64_t text_bytes;      /* bytes the segments span (seg_off[nseg]) */
    int64_t tables_bytes;    /* bytes of `tables` the referenced tables span */
    int64_t workspace_bytes; /* device bytes the plan occupies */
    int64_t items_offset;    /* layout of the plan inside the workspace */
    int32_t dfas_per_group;  /* automata walked together per work item */
    int32_t waves_per_group; /* 64-lane waves per workgroup */
    int32_t reserved[4];
} dfa_batch_plan;

int dfa_batch_prepare(const int64_t *seg_off, int32_t nseg, const int64_t *table_off,
                      const int32_t *m, int32_t npat, const int32_t *pair_seg,
                      const int32_t *pair_pat, int64_t npairs, void *workspace,
                      int64_t workspace_bytes, const dfa_tune *tune, dfa_batch_plan *plan,
                      void *stream);

int dfa_batch_run(const uint8_t *text, int64_t n, const uint8_t *tables, int64_t tables_bytes,
                  const void *workspace, const dfa_batch_plan *plan, int64_t *counts, void *stream);

int dfa_count_batch(const uint8_t *text, int64_t n, const int64_t *seg_off, int32_t nseg,
                    const uint8_t *tables, int64_t tables_bytes, const int64_t *table_off,
                    const int32_t *m, int32_t npat,
                    const int32_t *pair_seg, const int32_t *pair_pat, int64_t npairs,
                    int64_t *counts, void *workspace, int64_t workspace_bytes,
                    const dfa_tune *tune, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DFA_H */
