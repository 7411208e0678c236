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
    int32_t waves_per_group; /* 64-lane waves per workgroup, 1..8 (1..16 for merged scans
                              * and for the single-pattern scan with one walk per lane
                              * and 64-byte rounds) */
    int32_t chains_per_lane; /* independent walks interleaved in one lane: 1 (or 2 with
                              * 64-byte rounds) */
    int32_t dfas_per_group;  /* batched scans: automata walked together: 2, 4, 8 or 16 */
    int32_t automaton_bytes; /* merged scans: LDS bytes one merged automaton may take
                              * (its table, byte-class map and final-state counters);
                              * decides how many patterns share one automaton */
    int32_t line_bytes;      /* bytes of every walk fetched per round: 64 or 128 (merged
                              * scans: 32 or 64) */
    int32_t step_bytes;      /* merged scans: text bytes per automaton step, 1 or 2 (a pair
                              * table, where it fits automaton_bytes); other scans ignore it */
    int32_t reserved[2];     /* must be zero */
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
 * 0 when want_positions == 0; otherwise per walk (or per wave of 64 walks)
 * its match count, output offset and first 16 match starts, and per
 * workgroup its total, flags and a prefix level (about 44 bytes per walk of
 * 512 text bytes).  Returns bytes, or DFA_EINVAL. */
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

/* Measurement hook for per-kernel timing: while set, every dfa_count call
 * made from the calling thread records `begin` on its stream right before
 * the launch of its walk over the whole text (the count-only scan, or with
 * positions the per-walk counting pass) and `end` right after it, so that
 * the two events bracket that one kernel.  Both are hipEvent_t handles the
 * caller created (with timing); NULL, NULL clears the hook.  A dfa_count
 * that fails before that launch records neither.  Returns DFA_OK, or
 * DFA_EINVAL if exactly one of the two is NULL. */
int dfa_set_scan_events(void *begin, void *end);

/* Measurement hook for load-balance studies: dfa_count's count-only scan
 * (n >= 1, no positions) where workgroup b also writes, for b < wg_cap,
 * wg_times[3b] = its start and wg_times[3b+1] = its end on the device's
 * constant-rate wall clock (hipDeviceAttributeWallClockRate) and
 * wg_times[3b+2] = its length in shader cycles (device, 8-byte aligned).
 * Returns the number of workgroups launched, or DFA_EINVAL / DFA_EHIP. */
int64_t dfa_count_timed(const uint8_t *text, int64_t n, const uint8_t *table, int32_t m,
                        int64_t *count, unsigned long long *wg_times, int64_t wg_cap,
                        const dfa_tune *tune, void *stream);

/* Measurement only: the LDS read rate of the current GPU, the ceiling of the
 * table reads every automaton step makes (Alg. 1; the sparse transition
 * table of Sec. III.B, held in LDS here).  Launches `blocks` workgroups of 512
 * threads; each thread makes iters x 8 reads of `width` bytes (1 or 2) from a
 * 16 KiB LDS table, at
 *   mode 0: scattered addresses independent of the values read (the gather
 *           rate when lanes of a wave meet in the same bank),
 *   mode 1: addresses computed, in 8 chains per thread, from the chain's
 *           previous value as value x row + column (an automaton step's
 *           dependent read), rows of 61 bytes or of 5 two-byte entries,
 *   mode 2: addresses where lane l of each half-wave reads dword l of a row
 *           (no two lanes of a half-wave in one bank: the conflict-free rate).
 * `sink` (device, 8 bytes, 8-byte aligned) is written only in a case that
 * does not occur; it keeps the reads.  Returns the number of reads launched
 * (time the launch on `stream` to get the rate), or DFA_EINVAL (width, mode,
 * blocks in [1, 2^20] or iters in [1, 2^24] out of range, null or misaligned
 * sink) / DFA_EHIP. */
int64_t dfa_lds_probe(int32_t width, int32_t mode, int32_t blocks, int64_t iters,
                      unsigned long long *sink, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dfa_count
 * with the positions workspace taken from a buffer the library itself holds
 * in device memory, DFA_NOALLOC_SCRATCH_BYTES per GPU, kept from the first
 * call on that GPU until the process ends.  The call allocates nothing.
 * Arguments, results and errors are dfa_count's (same kernels, same output),
 * without workspace / workspace_bytes; the scratch belongs to the device
 * current on the calling thread.  When positions are asked for and
 * dfa_count_workspace_bytes(n, m, 1, tune) exceeds DFA_NOALLOC_SCRATCH_BYTES
 * (with the default tune: n above about 770 MB), it returns DFA_ENOSPACE and
 * launches nothing.  Every call on one GPU uses the same scratch: calls that
 * overlap on a GPU (on different streams, or from different threads without
 * ordering) race and give undefined results; calls ordered on one stream are
 * safe, each one initialises what it reads. */
#define DFA_NOALLOC_SCRATCH_BYTES (64LL << 20)
int dfa_count_noalloc(const uint8_t *text, int64_t n, const uint8_t *table, int32_t m,
                      int64_t *count, int64_t *positions, int64_t cap,
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

/* ------------------------------------------------------------------------ */
/* Merged multi-pattern automata (Sec. "Implementation Aspects", Fig. 4,    */
/* Table 2): one automaton advances many patterns per byte.                 */
/* ------------------------------------------------------------------------ */

#define DFA_AC_MAX_STATES 65535 /* merged states are 16-bit */

/* Host-only.  Builds the paper's improved Aho-Corasick automaton for patterns
 * p_i = patterns[pat_off[i] .. pat_off[i] + pat_len[i] - 1], i < npat
 * (1 <= pat_len[i] <= DFA_MAX_M; repeats allowed): one state per distinct
 * prefix of the patterns, state 0 the empty prefix; entry (q, b) is the state
 * of the longest suffix of (prefix of q) + b that is a prefix of some pattern,
 * so failure links never have to be followed; every byte that occurs in no
 * pattern leads to state 0.  States that report at least one pattern (a
 * pattern is a suffix of their prefix) are numbered last, from *first_final on.
 *   table        host, max_states x 256 uint16, row-major by state, or NULL
 *                for a size query
 *   first_final  host int32 or NULL: receives the first reporting state
 *   out_off      host or NULL: nstates - first_final + 1 int32; the patterns
 *   out_pat      reported by state f are out_pat[out_off[f - first_final] ..
 *                out_off[f - first_final + 1] - 1] (indices i), room for out_cap
 *   n_out        host int64 or NULL: receives the number of out_pat entries
 * Returns the number of states (>= 2), or DFA_EINVAL (bad arguments, more
 * than DFA_AC_MAX_STATES states) or DFA_ENOSPACE (table or out_pat too small). */
int64_t dfa_ac_build(const uint8_t *patterns, const int64_t *pat_off, const int32_t *pat_len,
                     int32_t npat, uint16_t *table, int64_t max_states, int32_t *first_final,
                     int32_t *out_off, int32_t *out_pat, int64_t out_cap, int64_t *n_out);

#define DFA_MERGED_GROUPS 8
typedef struct dfa_merged_plan {
    int64_t nitems;          /* work items: (tile of a segment, merged automaton) */
    int64_t nautomata;       /* merged automata built */
    int64_t nstates;         /* states over all automata */
    int64_t nfinal;          /* reporting states over all automata */
    int64_t npairs;          /* (segment, pattern) pairs */
    int64_t ncounts;         /* counters written by dfa_merged_run */
    int64_t text_bytes;      /* bytes the segments span (seg_off[nseg]) */
    int64_t workspace_bytes; /* device bytes the plan occupies (automata, items, visit counters) */
    int64_t items_offset;    /* layout of the plan inside the workspace */
    int64_t outputs_offset;
    int64_t entries_offset;
    int64_t visits_offset;
    int32_t waves_per_group; /* 64-lane waves per workgroup */
    int32_t lds_bytes;       /* dynamic LDS of the largest scan launch */
    int32_t reserved[4];
    /* the scan's launches, in order: group g runs the next group_items[g]
     * work items with group_lds[g] bytes of LDS, over pair automata (two
     * text bytes per step) if group_pair[g] != 0 */
    int64_t group_items[DFA_MERGED_GROUPS];
    int32_t group_lds[DFA_MERGED_GROUPS];
    int32_t group_pair[DFA_MERGED_GROUPS];
} dfa_merged_plan;

/* Batched counting with merged automata: same question as the dfa_batch_*
 * calls (pair k asks for the occurrences of pattern pair_pat[k] inside
 * segment pair_seg[k]; pair_dst, if not NULL, sends pair k's count to
 * counter pair_dst[k] < ncounts, where the counts of all pairs sent to one
 * counter add up -- with NULL, counter k is pair k and ncounts must be 0 or
 * npairs), but the patterns are passed as bytes
 * (patterns[pat_off[j] ..], pat_len[j] in 1..DFA_MAX_M, host) and the pairs
 * of each segment are merged into as few automata as the LDS budget
 * (tune->automaton_bytes) allows, so that one table lookup per text byte
 * advances all patterns of an automaton.  Each automaton is stored as a
 * 256-entry byte-class map plus a 16-bit table with one column per class
 * (every byte that occurs in none of its patterns is one class): the same
 * transitions as the 256-column table of dfa_ac_build, in the space that lets
 * thousands of states share LDS.  A walk owns the match starts of its span and
 * reads max(m) - 1 bytes past it; a match that ends in that overlap is
 * counted only if it starts inside the span (the start-position rule that
 * makes patterns of unequal lengths exact).
 *   dfa_merged_prepare  host: validates, builds the automata, plans the work
 *                       and uploads everything into `workspace` (device,
 *                       256-byte aligned); with workspace == NULL only fills
 *                       `plan`.  Synchronises `stream`.
 *   dfa_merged_run      device only: clears the counters it owns, zeroes
 *                       counts[0..ncounts-1] (int64, device, 8-byte aligned) and
 *                       launches the scan and the count reduction; `text`
 *                       (device, n >= plan->text_bytes, 16-byte aligned).
 *                       Asynchronous, allocates nothing, no memset nodes; the
 *                       workspace is written (calls that share it must not
 *                       overlap).
 * Both return DFA_OK, DFA_EINVAL, DFA_ENOSPACE or DFA_EHIP. */
int dfa_merged_prepare(const int64_t *seg_off, int32_t nseg, const uint8_t *patterns,
                       const int64_t *pat_off, const int32_t *pat_len, int32_t npat,
                       const int32_t *pair_seg, const int32_t *pair_pat, int64_t npairs,
                       const int32_t *pair_dst, int64_t ncounts,
                       void *workspace, int64_t workspace_bytes, const dfa_tune *tune,
                       dfa_merged_plan *plan, void *stream);

int dfa_merged_run(const uint8_t *text, int64_t n, void *workspace, const dfa_merged_plan *plan,
                   int64_t *counts, void *stream);

/* ------------------------------------------------------------------------ */
/* Degenerate patterns (the structure of Table 3: IUPAC codes, both strands) */
/* ------------------------------------------------------------------------ */

#define DFA_DEGENERATE_MAX_KMERS (1 << 20)

/* Host-only.  Expands code[0..m-1] (IUPAC nucleotide codes A C G T R Y S W K
 * M B D H V N, upper case; 1 <= m <= DFA_MAX_M) into the distinct plain
 * k-mers over A, C, G, T it matches -- and, if both_strands, those its
 * reverse complement matches -- sorted, m bytes each, back to back in `out`
 * (host, room for out_cap k-mers; NULL for a size query).  A text position
 * matches the degenerate pattern (on either strand) iff exactly one of these
 * k-mers starts there, so its count is the sum of theirs; a text byte that is
 * not A, C, G or T (e.g. 'N') matches no code.  Returns the number of k-mers,
 * DFA_EINVAL (bad code or length, more than DFA_DEGENERATE_MAX_KMERS) or
 * DFA_ENOSPACE. */
int64_t dfa_degenerate_expand(const uint8_t *code, int32_t m, int32_t both_strands, uint8_t *out,
                              int64_t out_cap);

/* ------------------------------------------------------------------------ */
/* FASTA input (the paper's genomes, Table 1, are FASTA text)                */
/* ------------------------------------------------------------------------ */

/* Device workspace for dfa_fasta_normalize on n bytes (0 for n == 0). */
int64_t dfa_fasta_workspace_bytes(int64_t n);

/* Device-only.  Turns FASTA text raw[0..n-1] (device, 16-byte aligned) into
 * plain sequence: a line whose first byte is '>' is a header (it starts a
 * record; none of its bytes are kept); every other byte is kept except '\n'
 * and '\r', with 'a'..'z' made upper case (soft-masking dropped).
 *   out        device, room for n bytes, any alignment: the kept bytes, in
 *              order (no byte of out past them is written)
 *   rec_start  device int64, room for rec_cap entries: where each record's
 *              sequence starts in `out` (the first rec_cap records)
 *   totals     device int64[2]: {kept bytes, records} (exact even past rec_cap)
 *   workspace  device, dfa_fasta_workspace_bytes(n) bytes, 256-byte aligned
 * Kept bytes before the first header (normally none) precede record 0.  With
 * seg_off = {rec_start..., totals[0]} the records are the segments of the
 * batched scans.  Asynchronous; returns DFA_OK, DFA_EINVAL, DFA_ENOSPACE or
 * DFA_EHIP. */
int dfa_fasta_normalize(const uint8_t *raw, int64_t n, uint8_t *out, int64_t *rec_start,
                        int64_t rec_cap, int64_t *totals, void *workspace, int64_t workspace_bytes,
                        void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DFA_H */
