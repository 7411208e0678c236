// Single-pattern automaton scan for gfx950 (CDNA4): Algorithm 1 of Memeti &
// Pllana, re-decomposed for 64-lane waves.
//
// Decomposition (Sec. III.A).  The text is cut into equal spans of S bytes,
// one per "walk".  Walk g owns the match starts [g*S, (g+1)*S) and reads
// T[g*S .. min(n, (g+1)*S + m - 1) - 1]: the m-1 extra bytes are the overlap
// of Algorithm 1, so a match that crosses a span border is found by the walk
// in which it starts, and by no other (a walk that restarts in q0 at g*S
// cannot reach the final state before it has read m bytes of its own span).
// Every lane of a wave runs K independent walks, interleaved for latency
// hiding; the 64*K walks of a wave are consecutive spans of the text.
// Spans are whole 128-byte lines, so a walk's loads never share a line with
// another round's.
//
// Data movement.  A wave reads its walks' text as whole 128-byte lines with
// coalesced 16-byte loads (8 lanes read one line; non-temporal), each line
// two 64-byte rounds (128-byte rounds as a tune).  A round goes to a
// wave-private LDS buffer and is read back transposed, so that every lane
// holds the round's bytes of its own walk in registers; the next lines'
// loads are in flight while the current rounds are walked.  HBM traffic is
// the text once: a walk's m-1 overlap bytes are the first bytes of the next
// walk's span, which each lane copies out of the wave's staged first round and
// keeps in registers (only the wave's last walk loads them, from the next
// wave's first line).
//
// Automaton step (Sec. III.B).  The (m+1) x 256 byte-indexed table lives in
// LDS with rows padded to 280 bytes, so the rows of the low, most visited
// states start in different LDS banks.  One step is q <- tab[q*280 + c] (one
// LDS byte gather) followed by the final-state test q == m.  Matches are
// counted per wave with ballot + popcount, summed over the workgroup in LDS,
// and added to the result with one 64-bit atomic per workgroup.
//
// Positions.  Sorted positions are produced without sorting: walks are in
// text order, and inside a walk matches are found in increasing order.  A
// first pass records each walk's match count; an exclusive prefix sum gives
// each walk its output offset; a second pass re-walks only spans that hold a
// match and writes start offsets (end - m + 1) in order.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>

#include "dfa.h"
#include "dfa_internal.h"
#include "launch_util.h"
#include "walk_common.h"

namespace {

using namespace dfa_dev;

// kCount: one wave-wide count, one atomic per workgroup.  kCountPerWalk: a
// count and the first kBuffered match starts per walk.  kPositions: the
// positions of the walks past their buffer.  kCountPerWave: the count-only
// walk, one count per wave (the positions of its waves with a match come
// from k_rewalk).
enum Mode { kCount = 0, kCountPerWalk = 1, kPositions = 2, kCountPerWave = 3 };

struct ScanParams {
    const uint8_t *text;
    int64_t n;
    const uint8_t *table;
    int32_t m;
    int32_t rounds;    // ceil((S + m - 1) / LINE)
    int64_t S;         // span bytes per walk (multiple of 16)
    int64_t nwalks;
    unsigned long long *total;    // kCount: += matches
    uint32_t *walk_count;         // kCountPerWalk: matches per walk, written by waves with a match
                                  // (read back by kPositions); kCountPerWave: matches per wave
    uint16_t *walk_buf;           // kCountPerWalk: start offsets (within the walk) of its first kStaged matches
    uint16_t *walk_buf1;          //   and of the next kBuffered - kStaged
    unsigned long long *wg_part;  // kCountPerWalk, kCountPerWave: matches per workgroup
    uint32_t *wg_waves;           // kCountPerWalk, kCountPerWave: bit w set when wave w of the
                                  // workgroup had a match (read back by kPositions)
    int32_t stage;                // kCountPerWalk: stage records in LDS (plans for short patterns)
    uint32_t rec_lds;             // in the kernel: LDS address of the wave's staged records (or 0)
    const uint32_t *wg_flag;      // kPositions: nonzero for a workgroup with a walk past its buffer
    const int64_t *walk_off;      // kPositions: output offset per walk (walks past their buffer only)
    int64_t *positions;         // kPositions
    int64_t cap;
    unsigned long long *wg_times;  // measurement only (kCount): 3 words per workgroup, or null
    int64_t wg_cap;                // workgroups with room in wg_times
};

// matches per walk whose start offsets the counting pass keeps (in the
// workspace); walks with more are walked again by the positions pass.  The
// first kStaged of them and the rest live in two arrays of kStaged entries
// per walk, so that the first halves of consecutive walks are contiguous.
constexpr int kBuffered = 16;
constexpr int kStaged = 8;
// Short patterns, one walk per lane: the per-walk counting pass keeps each
// walk's first kStaged records in LDS ([record][lane] 16-bit, 1 KiB per wave)
// and stores them in one 16-byte store per lane at the end of the walk.
// Records stored to HBM as they are found land in lines that leave L2 before
// the walk is done, and every such partial line costs a write of its own; the
// staging costs LDS, i.e. resident waves.  It pays where matches are dense:
// on a 4-letter text a pattern of m <= 6 bytes is expected about once per
// 4^m <= 4096 bytes, several times per walk; longer ones mostly not at all.
constexpr int kRecBytes = kStaged * kWave * 2;
constexpr int kStageMaxM = 6;
__host__ __device__ constexpr bool stages_records(int K, int MODE, int H) {
    return MODE == kCountPerWalk && K == 1 && H == 1;
}
// buffered matches are kept as 16-bit start offsets within the walk (a walk
// owns the starts of its span): the positions path needs S <= 65536
constexpr int64_t kMaxPositionsSpan = 65536;

__host__ __device__ inline int table_lds_bytes(int m) { return table_lds_rows_bytes(m + 1); }

// The per-walk counting pass and the positions pass with one walk per lane
// (used for m < kPerWaveMinM) keep a MARKED table in LDS: entry 2 q + f, f = 1
// iff q = m is the final state, every row stored twice (rows 2 q and 2 q + 1
// are state q's), so that the walk register holds the entry itself and one
// funnel shift per byte records whether it is final.  The final test is
// entry == 2 m + 1.
__host__ __device__ constexpr bool marked_table(int K, int mode) { return K == 1 && (mode == 1 || mode == 2); }
__host__ __device__ inline int scan_table_bytes(int m, int K, int mode) {
    return marked_table(K, mode) ? table_lds_rows_bytes(2 * (m + 1)) : table_lds_bytes(m);
}

struct WalkLane {
    int64_t wstart;  // first byte of the walk
    uint32_t len;    // bytes the walk reads (span + m - 1, clipped at the text end)
    uint32_t cnt;    // matches (per-walk counting pass)
    int64_t off;     // next output slot (positions pass)
};

typedef __attribute__((address_space(3))) uint16_t lds_u16w;

// Record `idx` (< kBuffered) of walk s of this lane.  p.walk_buf and
// p.walk_buf1 point at the wave's first walk in the per-walk counting pass,
// so the lane's own entries follow from the lane index alone (no pointer
// held per lane); p.rec_lds is nonzero when the first kStaged wait in LDS.
__device__ __forceinline__ void put_record(const ScanParams &p, int s, uint32_t idx, uint16_t v) {
    const uint32_t w = uint32_t(s * kWave) + __lane_id();
    if (idx < uint32_t(kStaged)) {
        if (p.rec_lds)
            *reinterpret_cast<lds_u16w *>(uintptr_t(p.rec_lds + 2u * (idx * kWave + __lane_id()))) = v;
        else
            p.walk_buf[w * kStaged + idx] = v;
    } else {
        p.walk_buf1[w * kStaged + idx - kStaged] = v;
    }
}

// The start offsets of a lane's matches in one unit, in increasing order,
// into the walk's buffer, from a marked walk's mask (walk16_marks: byte i of
// the unit in bit i; a match ending at byte j starts at j - (m - 1)).
__device__ __forceinline__ void record_marks(uint32_t hm, uint32_t jb, uint32_t m, WalkLane &w, const ScanParams &p) {
    while (hm) {
        const int b = __builtin_ctz(hm);
        if (w.cnt < uint32_t(kBuffered)) put_record(p, 0, w.cnt, uint16_t(jb + uint32_t(b) - (m - 1)));
        ++w.cnt;
        hm &= hm - 1u;
    }
}

// Walk 16 bytes: byte b of word w is byte jb + 4w + b of the walk.  GUARD:
// only bytes below the walk's length count.  kCount: ballot + scalar count.
// kCountPerWalk: per-walk count and the first kBuffered match starts (the
// total is summed from the per-walk counts at the end).  kPositions: write
// the start offset of every match.
template <int K, int MODE, bool GUARD>
__device__ __forceinline__ void walk_unit(const v4u (&t)[K], uint32_t (&q)[K], uint32_t m, uint32_t mhit, uint32_t jb,
                                          uint32_t &acc, WalkLane (&wl)[K], const ScanParams &p) {
    if constexpr (MODE == kCount && !GUARD && K == 1) {
        walk16_count(q[0], t[0], acc, mhit);
        return;
    }

    if constexpr (MODE == kCountPerWalk && !GUARD && K == 1) {
        // Each wave picks per unit how to walk it.  While its last unit had no
        // match it walks like the count-only scan (one wave-wide count in a
        // scalar register) and walks the unit again, from the state it started
        // in, with per-lane hit masks only if that count is nonzero; after a
        // unit with matches it walks the next one with hit masks directly.
        // `acc` carries the choice (nonzero: hit masks); the per-walk counts
        // live in wl and `acc` is rewritten with their sum at the end.
        // (one walk per lane: the table is marked, see marked_table)
        uint32_t hm;
        if (__builtin_amdgcn_readfirstlane(acc)) {
            walk16_marks(q[0], t[0], hm);
            const bool any = __ballot(hm != 0) != 0;
            if (any) record_marks(hm, jb, m, wl[0], p);
            acc = any ? 1u : 0u;
        } else {
            const uint32_t q0 = q[0];
            uint32_t a = 0;
            walk16_count(q[0], t[0], a, mhit);
            if (__builtin_amdgcn_readfirstlane(a)) {
                q[0] = q0;
                walk16_marks(q[0], t[0], hm);
                record_marks(hm, jb, m, wl[0], p);
                acc = 1u;
            }
        }
        return;
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
            for (int s = 0; s < K; ++s) {
                const uint32_t c = (t[s][w] >> (8 * b)) & 0xffu;
                const uint32_t j = jb + uint32_t(4 * w + b);
                q[s] = table_step(q[s], c);
                bool hit = q[s] == mhit;
                if (GUARD) hit = hit && (j < wl[s].len);
                if (MODE == kCount) {
                    add_hits(acc, hit);
                } else if (MODE == kCountPerWalk) {
                    if (hit) {
                        if (wl[s].cnt < uint32_t(kBuffered)) put_record(p, s, wl[s].cnt, uint16_t(j - (m - 1)));
                        ++wl[s].cnt;
                    }
                } else if (hit) {
                    if (wl[s].off < p.cap) p.positions[wl[s].off] = wl[s].wstart + j - (m - 1);
                    ++wl[s].off;
                }
            }
        }
    }
}

// One overlap unit on the whole-wave path, where every walk of the wave reads
// the same number of overlap bytes: `nvalid` (1..16, wave-uniform) of its 16
// bytes belong to the walk.  With one walk per lane and a counting mode the
// 16 steps run as in the span and the hit mask drops the bytes past the
// overlap (the count-only mode adds the lane's hits to `extra`, summed over
// the wave at the end); otherwise the byte loop with its length check.
template <int K, int MODE>
__device__ __forceinline__ void walk_overlap_unit(const v4u (&t)[K], uint32_t (&q)[K], uint32_t m, uint32_t mhit,
                                                  uint32_t jb, uint32_t nvalid, uint32_t &acc, uint32_t &extra,
                                                  WalkLane (&wl)[K], const ScanParams &p) {
    if constexpr (K == 1 && MODE == kCount) {
        uint32_t hm;
        walk16_hits(q[0], t[0], hm, m);
        hm &= 0xffffu & ~((1u << (16u - nvalid)) - 1u);  // byte i of the unit is bit 15 - i
        extra += uint32_t(__popc(hm));
    } else if constexpr (K == 1 && MODE == kCountPerWalk) {
        uint32_t hm;
        walk16_marks(q[0], t[0], hm);
        hm &= (1u << nvalid) - 1u;  // byte i of the unit is bit i
        if (__ballot(hm != 0)) record_marks(hm, jb, m, wl[0], p);
    } else {
        walk_unit<K, MODE, true>(t, q, m, mhit, jb, acc, wl, p);
    }
}

// Walk one staged round: its units stream from LDS, the next one in flight
// while the current one is walked.  `nbytes` (wave-uniform) bytes of the round
// belong to every walk when GUARD is false; with GUARD, each walk's own length
// decides.
template <int K, int LINE, int MODE, bool GUARD>
__device__ __forceinline__ void walk_round(const v4u *xb, int lane, uint32_t (&q)[K], uint32_t m, uint32_t mhit,
                                           uint32_t rb, int nbytes, uint32_t &acc, WalkLane (&wl)[K],
                                           const ScanParams &p) {
    using G = Geo<LINE>;
    const int units = GUARD ? G::U : (nbytes + 15) / 16;
    v4u cur[K], nxt[K];
#pragma unroll
    for (int s = 0; s < K; ++s) cur[s] = unit_of<LINE>(xb, s, lane, 0);
    for (int u = 0; u < units; ++u) {
        if (u + 1 < units) {
#pragma unroll
            for (int s = 0; s < K; ++s) nxt[s] = unit_of<LINE>(xb, s, lane, u + 1);
        }
        const uint32_t jb = rb + uint32_t(16 * u);
        if (GUARD || 16 * (u + 1) > nbytes)
            walk_unit<K, MODE, true>(cur, q, m, mhit, jb, acc, wl, p);
        else
            walk_unit<K, MODE, false>(cur, q, m, mhit, jb, acc, wl, p);
#pragma unroll
        for (int s = 0; s < K; ++s) cur[s] = nxt[s];
    }
}

// Overlap units loaded ahead (H): 1 unit covers m <= 17, 2 units m <= 33,
// 4 units m <= 65.  Every unit held costs 4 registers for the whole walk, so
// the default shape (one walk per lane, 64-byte rounds) is instantiated for
// all three and the others for 1 and 4.
constexpr int halo_units_for(int m) { return m <= 17 ? 1 : m <= 33 ? 2 : 4; }

// The default counting kernels (one walk per lane, 64-byte rounds) are asked
// to fit 6 waves per SIMD (at most 80 registers): the per-walk counting pass
// with 4 overlap units would otherwise need 81 (the compiler then keeps one
// overlap unit in scratch between the first round and the end of the walk).
// A budget of 64 registers (8 waves per SIMD) for the count-only and
// count-per-wave walks measured slower where it changed the code: with 2
// overlap units the compiler keeps the second in scratch, and m = 32 walked
// 3.2 GB in 0.60 ms against 0.54 ms, in workgroups of 8 or of 16 waves (32
// resident per CU instead of 24); with 1 unit the count-only walk (64
// registers instead of 72) took 0.49-0.59 ms against 0.50-0.55.
template <int K, int LINE, int MODE>
constexpr int scan_waves_per_eu() {
    return (K == 1 && LINE == 64 && (MODE == kCount || MODE == kCountPerWalk || MODE == kCountPerWave)) ? 6 : 1;
}

// The walks of one wave (64 x K of them, from walk g0) over their spans and
// overlaps: the whole-wave path when every load lies inside the text, else
// the guarded one.  WM is the walking mode: kCount, kCountPerWalk or
// kPositions.
template <int K, int LINE, int WM, int H>
__device__ __forceinline__ void walk_wave(const ScanParams &p, v4u *xb, int lane, int64_t g0, uint32_t m,
                                          uint32_t mhit, uint32_t lane_off, uint32_t (&q)[K], uint32_t &acc,
                                          WalkLane (&wl)[K]) {
    using G = Geo<LINE>;
    // whole wave in bounds: every load of every round lies inside the text
    const int64_t glast = g0 + kWave * K - 1;
    const bool full = glast < p.nwalks && glast * p.S + int64_t(p.rounds) * LINE <= p.n;

    if (full) {
        // The span [0, S) streams in R rounds; the overlap [S, S + m - 1) is
        // the start of the next span, which the neighbouring lane (the next
        // walk) receives in round 0.  Right after round 0 is staged, each lane
        // copies the first H units of its neighbour's row out of the wave's
        // buffer and keeps them in registers until the end of the walk; only
        // the wave's last walk, whose neighbour belongs to another wave,
        // loads them from memory.  Fetching the overlap at the end of the
        // walk instead would miss in L2 and cost a whole line of HBM per
        // walk.  Units past H (m > 65) are loaded at the end.
        const int R = int((p.S + LINE - 1) / LINE);
        const int rlast = R - 1;
        const int lastlen = int(p.S - int64_t(rlast) * LINE);  // bytes of the last round (LINE unless S is not a
                                                               // multiple of LINE)
        // Loads run two rounds ahead of the walk: pa holds even rounds, pb odd
        // ones.  A short last round fetches only the units it walks: lanes past
        // them repeat the last unit's address, a load of the same line.  A
        // fetch past the last round reads the first line of the text instead
        // (always cached), so that both buffers are always written and stay
        // in registers without touching another line of HBM.  With 64-byte
        // rounds, rounds r + 2 and r + 3 are the two halves of the walks' next
        // 128-byte lines; both are requested back to back so that the second
        // half finds the line still in L2 (requested one round apart, the
        // shared line is evicted first and read twice).
        const uint32_t ulast = uint32_t(lastlen + 15) / 16;
        const uint32_t lane_unit = uint32_t(lane % G::U);
        const uint32_t off_last = lane_off - 16u * lane_unit + 16u * (lane_unit < ulast ? lane_unit : ulast - 1);
        const uint32_t off_none = 16u * lane_unit;
        const int64_t wb = g0 * p.S;
        const int hu = (p.m - 1 + 15) / 16;  // overlap units
        v4u halo[K][H];
        if (LINE == 64 && (p.S & 127) == 0) {
            // Spans of whole 128-byte lines (every default span): rounds r
            // and r + 1 arrive together as whole lines (fetch_pair), half the
            // lanes holding each, and are staged one after the other.  Fetches,
            // stages and walks come in the same order as in the other branch
            // with 64-byte rounds; here R is even and at least 2.
            v4u pp[K][8];
            const uint32_t pair_off = uint32_t(lane / 8) * uint32_t(p.S) + 16u * uint32_t(lane % 8);
            fetch_pair<K>(pp, p.text, wb, p.S, pair_off, lane, 0, rlast);
            stage_pair<K, 0>(pp, xb, lane);
            grab_halo<K, LINE, H>(halo, xb, lane, p.text, wb, p.S, hu, G::U);
            walk_round<K, LINE, WM, false>(xb, lane, q, m, mhit, 0u, LINE, acc, wl, p);
            stage_pair<K, 1>(pp, xb, lane);
            fetch_pair<K>(pp, p.text, wb, p.S, pair_off, lane, 2, rlast);
            walk_round<K, LINE, WM, false>(xb, lane, q, m, mhit, uint32_t(LINE), LINE, acc, wl, p);
            for (int r = 2; r < R; r += 2) {
                stage_pair<K, 0>(pp, xb, lane);
                walk_round<K, LINE, WM, false>(xb, lane, q, m, mhit, uint32_t(r * LINE), LINE, acc, wl, p);
                stage_pair<K, 1>(pp, xb, lane);
                fetch_pair<K>(pp, p.text, wb, p.S, pair_off, lane, r + 2, rlast);
                walk_round<K, LINE, WM, false>(xb, lane, q, m, mhit, uint32_t((r + 1) * LINE), LINE, acc, wl, p);
            }
        } else {
            v4u pa[K][G::U], pb[K][G::U];
            fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, 0, rlast);
            fetch_round_or_none<K, LINE>(pb, p.text, wb, p.S, lane_off, off_last, off_none, 1, rlast);
            // round 0 (and 1), then the steady state from round 2
            stage_round<K, LINE>(pa, xb, lane);
            grab_halo<K, LINE, H>(halo, xb, lane, p.text, wb, p.S, hu, rlast == 0 ? int(ulast) : G::U);
            if (LINE == 128) fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, 2, rlast);
            walk_round<K, LINE, WM, false>(xb, lane, q, m, mhit, 0u, rlast == 0 ? lastlen : LINE, acc, wl, p);
            if (rlast >= 1) {
                stage_round<K, LINE>(pb, xb, lane);
                if (LINE == 64) fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, 2, rlast);
                fetch_round_or_none<K, LINE>(pb, p.text, wb, p.S, lane_off, off_last, off_none, 3, rlast);
                walk_round<K, LINE, WM, false>(xb, lane, q, m, mhit, uint32_t(LINE), rlast == 1 ? lastlen : LINE, acc, wl,
                                                 p);
            }
            for (int r = 2; r < R; r += 2) {
                stage_round<K, LINE>(pa, xb, lane);
                if (LINE == 128)
                    fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, r + 2, rlast);
                walk_round<K, LINE, WM, false>(xb, lane, q, m, mhit, uint32_t(r * LINE), r == rlast ? lastlen : LINE,
                                                 acc, wl, p);
                if (r + 1 > rlast) break;
                stage_round<K, LINE>(pb, xb, lane);
                if (LINE == 64)
                    fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, r + 2, rlast);
                fetch_round_or_none<K, LINE>(pb, p.text, wb, p.S, lane_off, off_last, off_none, r + 3, rlast);
                walk_round<K, LINE, WM, false>(xb, lane, q, m, mhit, uint32_t((r + 1) * LINE),
                                                 r + 1 == rlast ? lastlen : LINE, acc, wl, p);
            }
        }
        // the overlap, from registers, then (m > 65) the rest of it from memory
        const uint32_t hb = uint32_t(p.S);
        uint32_t extra = 0;
#pragma unroll
        for (int u = 0; u < H; ++u) {
            if (u < hu) {
                v4u t[K];
#pragma unroll
                for (int s = 0; s < K; ++s) t[s] = halo[s][u];
                const uint32_t nv = m - 1 - 16u * u;
                walk_overlap_unit<K, WM>(t, q, m, mhit, hb + 16u * u, nv < 16u ? nv : 16u, acc, extra, wl, p);
            }
        }
        for (int u = H; u < hu; ++u) {
            v4u t[K];
#pragma unroll
            for (int s = 0; s < K; ++s)
                t[s] = *reinterpret_cast<const v4u *>(p.text + (g0 + s * kWave + lane + 1) * p.S + 16 * u);
            const uint32_t nv = m - 1 - 16u * u;
            walk_overlap_unit<K, WM>(t, q, m, mhit, hb + 16u * u, nv < 16u ? nv : 16u, acc, extra, wl, p);
        }
        if (WM == kCount && K == 1) {
            // the overlap's hits, summed over the wave
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) extra += uint32_t(__shfl_xor(int(extra), o));
            acc = uint32_t(__builtin_amdgcn_readfirstlane(int(acc))) +
                  uint32_t(__builtin_amdgcn_readfirstlane(int(extra)));
        }
    } else {
        v4u pf[K][G::U];
        fetch_round<K, LINE, true>(pf, p.text, p.n, g0 * p.S, p.S, lane_off, 0);
        for (int r = 0; r < p.rounds; ++r) {
            stage_round<K, LINE>(pf, xb, lane);
            if (r + 1 < p.rounds) fetch_round<K, LINE, true>(pf, p.text, p.n, g0 * p.S, p.S, lane_off, r + 1);
            walk_round<K, LINE, WM, true>(xb, lane, q, m, mhit, uint32_t(r * LINE), LINE, acc, wl, p);
        }
    }

}

// Workgroups of up to 16 waves for the default shape (one walk per lane,
// 64-byte rounds: at most 80 registers, so 16 waves fit a CU), 8 for the
// others (whose larger register files would not).
template <int K, int LINE>
constexpr int scan_max_waves() {
    return (K == 1 && LINE == 64) ? 16 : 8;
}

template <int K, int LINE, int MODE, int H>
__global__ __launch_bounds__((scan_max_waves<K, LINE>() * kWave))
    __attribute__((amdgpu_waves_per_eu(scan_waves_per_eu<K, LINE, MODE>()))) void k_scan(ScanParams p) {  // by value: the per-walk counting pass moves p.walk_buf to its wave
    using G = Geo<LINE>;
    extern __shared__ __align__(16) unsigned char smem[];
    // measurement hook: the workgroup's start (constant-rate wall clock) and cycles
    const bool timed = MODE == kCount && p.wg_times != nullptr && int64_t(blockIdx.x) < p.wg_cap;
    const unsigned long long t_wall = timed ? wall_clock64() : 0ull;
    const unsigned long long t_cyc = timed ? clock64() : 0ull;
    const int lane = threadIdx.x & (kWave - 1);
    // wave index, known to the compiler as uniform so that per-wave addresses
    // live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    const int nwaves = blockDim.x / kWave;
    // table first (LDS address 0), then one transpose buffer per wave
    constexpr bool kMarked = marked_table(K, MODE);
    const int tbytes = scan_table_bytes(p.m, K, MODE);
    v4u *xb = reinterpret_cast<v4u *>(smem + tbytes + wave * (K * kWave * LINE));

    // only walks whose matches did not all fit the counting pass's buffer are
    // walked again: a workgroup without any leaves before loading the table
    if (MODE == kPositions && p.wg_flag[blockIdx.x] == 0) return;

    // table -> LDS, rows padded to kRow bytes (marked: entries 2 q + [q == m],
    // each row twice)
    {
        const uint32_t *tg = reinterpret_cast<const uint32_t *>(p.table);
        const int words = (p.m + 1) * (DFA_ALPHABET / 4);
        for (int i = threadIdx.x; i < words; i += blockDim.x) {
            const uint32_t w = tg[i];
            if (kMarked) {
                uint32_t e = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t b = (w >> (8 * k)) & 0xffu;
                    e |= (2u * b + (b == uint32_t(p.m) ? 1u : 0u)) << (8 * k);
                }
                *reinterpret_cast<uint32_t *>(smem + (2 * (i >> 6)) * kRow + 4 * (i & 63)) = e;
                *reinterpret_cast<uint32_t *>(smem + (2 * (i >> 6) + 1) * kRow + 4 * (i & 63)) = e;
            } else {
                *reinterpret_cast<uint32_t *>(smem + (i >> 6) * kRow + 4 * (i & 63)) = w;
            }
        }
    }
    __syncthreads();

    const int64_t g0 = (int64_t(blockIdx.x) * nwaves + wave) * (kWave * K);
    if (MODE == kCountPerWalk) {
        p.walk_buf += g0 * kStaged;
        p.walk_buf1 += g0 * kStaged;
        p.rec_lds = stages_records(K, MODE, H) && p.stage
                        ? uint32_t(tbytes + nwaves * (K * kWave * LINE) + wave * kRecBytes)
                        : 0u;
    }
    const uint32_t m = uint32_t(p.m);
    const uint32_t mhit = kMarked ? 2u * m + 1u : m;  // the final state's table entry
    const uint32_t lane_off = uint32_t(lane / G::U) * uint32_t(p.S) + 16u * uint32_t(lane % G::U);

    // per-lane walk bookkeeping
    WalkLane wl[K];
    uint32_t q[K];
    bool any_work = false;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int64_t g = g0 + s * kWave + lane;
        const int64_t start = g * p.S;
        int64_t len = 0;
        if (g < p.nwalks) {
            len = p.n - start;
            if (len > p.S + p.m - 1) len = p.S + p.m - 1;
        }
        wl[s].wstart = start;
        wl[s].len = uint32_t(len);
        wl[s].cnt = 0;
        wl[s].off = 0;
        q[s] = 0;
        if (MODE == kPositions) {
            // only walks whose matches did not all fit the counting pass's buffer
            // (the other lanes walk along without writing: their offset is past
            // any capacity)
            const bool has = g < p.nwalks && ((p.wg_waves[blockIdx.x] >> wave) & 1u) &&
                             p.walk_count[g] > uint32_t(kBuffered);
            wl[s].off = has ? p.walk_off[g] : (int64_t(1) << 62);
            any_work |= has;
        }
    }
    if (MODE == kPositions && __ballot(any_work) == 0) return;  // nothing left to write in this wave

    uint32_t acc = 0;
    walk_wave<K, LINE, MODE == kCountPerWave ? int(kCount) : MODE, H>(p, xb, lane, g0, m, mhit, lane_off, q, acc,
                                                                       wl);

    if (MODE == kPositions) return;

    if (MODE == kCountPerWave && lane == 0 && g0 < p.nwalks) p.walk_count[g0 / (kWave * K)] = acc;

    if (MODE == kCountPerWalk) {
        uint32_t c = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) c += wl[s].cnt;
        // only a wave with a match writes its walks' counts (and its staged
        // records); the workgroup's wave mask says which did
        if (__ballot(c != 0)) {
#pragma unroll
            for (int s = 0; s < K; ++s) {
                const int64_t g = g0 + s * kWave + lane;
                if (g < p.nwalks) p.walk_count[g] = wl[s].cnt;
            }
            if (stages_records(K, MODE, H) && p.rec_lds && g0 + lane < p.nwalks) {
                // entries past the walk's count are stale and never read
                uint32_t r[kStaged / 2];
#pragma unroll
                for (int k = 0; k < kStaged / 2; ++k) {
                    const uint32_t a = p.rec_lds + 2u * (uint32_t(2 * k) * kWave + uint32_t(lane));
                    const uint32_t lo = *reinterpret_cast<const lds_u16w *>(uintptr_t(a));
                    const uint32_t hi = *reinterpret_cast<const lds_u16w *>(uintptr_t(a + 2u * kWave));
                    r[k] = lo | (hi << 16);
                }
                const v4u rec = {r[0], r[1], r[2], r[3]};
                __builtin_nontemporal_store(rec, reinterpret_cast<v4u *>(p.walk_buf + lane * kStaged));
            }
        }
        // the wave's matches, summed over its lanes
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) c += uint32_t(__shfl_xor(int(c), o));
        acc = uint32_t(__builtin_amdgcn_readfirstlane(int(c)));
    }
    // workgroup sum in LDS (reusing the first transpose buffer): one atomic,
    // or (per-walk counting) the workgroup's total for the placement scan
    unsigned long long *red = reinterpret_cast<unsigned long long *>(smem + tbytes);
    __syncthreads();
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int w = 0; w < nwaves; ++w) sum += red[w];
        if (MODE == kCountPerWalk || MODE == kCountPerWave) {
            p.wg_part[blockIdx.x] = sum;
            uint32_t mask = 0;
            for (int w = 0; w < nwaves; ++w) mask |= red[w] ? 1u << w : 0u;
            p.wg_waves[blockIdx.x] = mask;
        } else if (sum) {
            atomicAdd(p.total, sum);
        }
        if (timed) {
            unsigned long long *t = p.wg_times + 3 * int64_t(blockIdx.x);
            t[0] = t_wall;
            t[1] = wall_clock64();
            t[2] = clock64() - t_cyc;
        }
    }
}

// ---------------------------------------------------------------------------
// Placement of the positions.  The counting pass leaves, per walk, its match
// count and the start offsets of its first kBuffered matches, and per
// workgroup its total.  One scan of the workgroup totals gives every
// workgroup's first output slot; then one block per counting workgroup (one
// thread per walk) scans its walks' counts, writes the buffered positions in
// order, the output offsets of the walks with more matches than the buffer
// holds, and whether the workgroup has any: the positions pass walks only
// those workgroups again.
// ---------------------------------------------------------------------------

__global__ void k_zero_u64(unsigned long long *x) { *x = 0; }

constexpr int kMaxGroupWalks = 1024;  // walks of one counting workgroup: 8 waves x 64 lanes x 2 walks

__device__ __forceinline__ unsigned long long wave_inclusive_scan(unsigned long long v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const unsigned long long u = __shfl_up(v, d);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive scan of one value per thread over the block (any multiple of 64
// threads up to 1024); `sh` holds 16 scratch slots in LDS; *total receives
// the block total.
__device__ __forceinline__ unsigned long long block_exclusive_scan(unsigned long long v, unsigned long long *sh,
                                                                   unsigned long long *total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    const unsigned long long inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) sh[w] = inc;
    __syncthreads();
    unsigned long long before = 0, all = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) before += sh[i];
        all += sh[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// Output slots are handed out in two levels: the workgroup totals fall in
// super-blocks of kSuper consecutive workgroups; one block sums every
// super-block and scans those sums, and each placement block adds the totals
// of the workgroups before its own inside its super-block.  Every kernel
// here synchronises its block a fixed number of times, whatever the text size.
constexpr int kSuper = 1024;
constexpr int kPartsThreads = 1024;

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// Block-wide sum (any multiple of 64 threads up to 1024); `sh` holds 16 slots.
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v, unsigned long long *sh) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    v = wave_sum(v);
    if (lane == 0) sh[w] = v;
    __syncthreads();
    unsigned long long all = 0;
    for (int i = 0; i < int(blockDim.x / kWave); ++i) all += sh[i];
    __syncthreads();
    return all;
}

// One block of kPartsThreads: sup[k] = exclusive prefix of the super-block
// sums (nsup = ceil(nb / kSuper) of them); *count = the total.
__global__ __launch_bounds__(kPartsThreads) void k_scan_parts(const unsigned long long *part, int64_t nb,
                                                              unsigned long long *sup, int64_t *count,
                                                              uint32_t *list_count) {
    __shared__ unsigned long long sh[kPartsThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t nsup = (nb + kSuper - 1) / kSuper;
    // wave w sums super-blocks w, w + 16, ...: 16 coalesced loads per lane, one wave reduction
    for (int64_t sb = w; sb < nsup; sb += kPartsThreads / kWave) {
        unsigned long long x = 0;
#pragma unroll
        for (int k = 0; k < kSuper / kWave; ++k) {
            const int64_t i = sb * kSuper + k * kWave + lane;
            x += i < nb ? part[i] : 0ull;
        }
        x = wave_sum(x);
        if (lane == 0) sup[sb] = x;
    }
    __syncthreads();
    // exclusive scan of the nsup sums: each thread a run of consecutive ones
    // (the writes above are visible to the block after the barrier)
    const int64_t per = (nsup + kPartsThreads - 1) / kPartsThreads;
    const int64_t i0 = int64_t(threadIdx.x) * per, i1 = i0 + per < nsup ? i0 + per : nsup;
    unsigned long long mine = 0;
    for (int64_t i = i0; i < i1; ++i) mine += sup[i];
    unsigned long long total;
    unsigned long long run = block_exclusive_scan(mine, sh, &total);
    for (int64_t i = i0; i < i1; ++i) {
        const unsigned long long x = sup[i];
        sup[i] = run;
        run += x;
    }
    if (threadIdx.x == 0) {
        *count = int64_t(total);
        if (list_count) *list_count = 0u;  // (per-wave plans) the placement pass appends to the list
    }
}

// One block of kPlaceThreads per `per_block` consecutive counting workgroups
// (at most kPlaceWalks walks), kPlacePerThread consecutive walks per thread,
// so that each thread's loads are all issued before the block first waits.
// The block's first output slot is its super-block's prefix plus the totals
// of the workgroups before it in that super-block.  A single scan then
// carries two sums packed in 64 bits: the matches before each thread's walks
// (high half: at most 2048 walks x (65536 + 255)) and the buffered matches
// before them (low half: at most 2048 x kBuffered).  A walk's count is read
// only when its wave had a match (the wave mask of its workgroup); the other
// counts are zero and their memory may hold an earlier call's.  Every
// counting workgroup gets a flag: nonzero when one of its walks has more
// matches than its buffer holds.
constexpr int kPlaceThreads = 256;
constexpr int kPlacePerThread = 8;
constexpr int kPlaceWalks = kPlaceThreads * kPlacePerThread;
constexpr int kPlaceUnroll = 4;  // buffered matches a thread places per iteration

__global__ __launch_bounds__(kPlaceThreads) void k_place(const uint32_t *walk_count, const uint16_t *walk_buf,
                                                         const uint16_t *walk_buf1, const uint32_t *wg_waves,
                                                         const unsigned long long *part,
                                                         const unsigned long long *sup, int64_t nwalks, int64_t nb,
                                                         int group_walks, int wave_walks, int per_block, int64_t S,
                                                         int64_t *walk_off, uint32_t *wg_flag, int64_t *positions,
                                                         int64_t cap) {
    __shared__ unsigned long long sh[kPlaceThreads / kWave];
    __shared__ uint32_t first[kPlaceWalks];  // buffered matches before each walk of the block
    __shared__ int64_t out[kPlaceWalks];     // output offset of each walk
    __shared__ uint32_t over[kPlaceWalks / kWave];  // per workgroup of the block: a walk past its buffer
    const int t = threadIdx.x;
    const int64_t wg0 = int64_t(blockIdx.x) * per_block;
    const int64_t g0 = wg0 * group_walks;
    const int bw = per_block * group_walks;  // walks of the block (a multiple of 64)
    // loads first: this thread's walk counts, the totals before wg0 in its super-block
    uint32_t c[kPlacePerThread];
    const int64_t gt = g0 + t * kPlacePerThread;
    // the thread's walks lie in one wave (wave_walks is a multiple of 64)
    const int lw = t * kPlacePerThread / group_walks;
    const bool wrote = t * kPlacePerThread < bw && wg0 + lw < nb &&
                       ((wg_waves[wg0 + lw] >> (t * kPlacePerThread % group_walks / wave_walks)) & 1u);
    if (!wrote) {
#pragma unroll
        for (int k = 0; k < kPlacePerThread; ++k) c[k] = 0u;
    } else if (gt + kPlacePerThread <= nwalks) {
        // 32 aligned bytes (g0 is a multiple of 64 walks)
        const uint4 lo = *reinterpret_cast<const uint4 *>(walk_count + gt);
        const uint4 hi = *reinterpret_cast<const uint4 *>(walk_count + gt + 4);
        c[0] = lo.x; c[1] = lo.y; c[2] = lo.z; c[3] = lo.w;
        c[4] = hi.x; c[5] = hi.y; c[6] = hi.z; c[7] = hi.w;
    } else {
#pragma unroll
        for (int k = 0; k < kPlacePerThread; ++k) {
            const int idx = t * kPlacePerThread + k;
            c[k] = (idx < bw && g0 + idx < nwalks) ? walk_count[g0 + idx] : 0u;
        }
    }
    const int64_t sb = wg0 / kSuper * kSuper;
    unsigned long long before = 0;
    for (int64_t i = sb + t; i < wg0; i += kPlaceThreads) before += part[i];
    const unsigned long long sup0 = sup[wg0 / kSuper];
    if (t < per_block) over[t] = 0u;
    const int64_t base = int64_t(sup0 + block_sum(before, sh));

    uint32_t tc = 0, tb = 0;
#pragma unroll
    for (int k = 0; k < kPlacePerThread; ++k) {
        tc += c[k];
        tb += c[k] <= uint32_t(kBuffered) ? c[k] : 0u;
    }
    unsigned long long total;
    const unsigned long long ex = block_exclusive_scan((uint64_t(tc) << 32) | tb, sh, &total);
    int64_t run = base + int64_t(ex >> 32);
    uint32_t runb = uint32_t(ex);
    const uint32_t nbuf = uint32_t(total);
#pragma unroll
    for (int k = 0; k < kPlacePerThread; ++k) {
        const int idx = t * kPlacePerThread + k;
        if (idx < bw) {
            if (nbuf) {  // the walk table is only read when there are buffered matches
                first[idx] = runb;
                out[idx] = run;
            }
            if (c[k] > uint32_t(kBuffered)) {
                walk_off[g0 + idx] = run;
                over[idx / group_walks] = 1u;  // every writer stores the same value
            }
        }
        run += c[k];
        runb += c[k] <= uint32_t(kBuffered) ? c[k] : 0u;
    }
    __syncthreads();
    if (t < per_block && wg0 + t < nb) wg_flag[wg0 + t] = over[t];
    // Buffered match k goes to the walk holding it: the last w with
    // first[w] <= k (first[0] = 0 and first never decreases), found in a
    // fixed number of halving steps.  Consecutive threads write consecutive
    // positions (a thread writing a run of its own would scatter partial lines
    // across the wave); each thread takes kPlaceUnroll matches per iteration,
    // so that their searches interleave and their record loads are in flight
    // together.
    for (uint32_t k0 = t; k0 < nbuf; k0 += kPlaceUnroll * kPlaceThreads) {
        int lo[kPlaceUnroll];
#pragma unroll
        for (int u = 0; u < kPlaceUnroll; ++u) {
            const uint32_t k = k0 + uint32_t(u * kPlaceThreads);
            int l = 0;
#pragma unroll
            for (int step = kPlaceWalks / 2; step > 0; step >>= 1)
                if (l + step < bw && first[l + step] <= k) l += step;
            lo[u] = l;
        }
        int64_t dst[kPlaceUnroll];
        uint32_t rec[kPlaceUnroll];
#pragma unroll
        for (int u = 0; u < kPlaceUnroll; ++u) {
            const uint32_t k = k0 + uint32_t(u * kPlaceThreads);
            const uint32_t i = k - first[lo[u]];
            const int64_t gw = g0 + lo[u];
            dst[u] = out[lo[u]] + i;
            rec[u] = 0;
            if (k < nbuf && dst[u] < cap)
                rec[u] = i < uint32_t(kStaged) ? walk_buf[gw * kStaged + i] : walk_buf1[gw * kStaged + i - kStaged];
        }
#pragma unroll
        for (int u = 0; u < kPlaceUnroll; ++u) {
            const uint32_t k = k0 + uint32_t(u * kPlaceThreads);
            if (k < nbuf && dst[u] < cap)
                __builtin_nontemporal_store((g0 + lo[u]) * S + int64_t(rec[u]), positions + dst[u]);
        }
    }
}

// Per-wave plans: one thread per counting wave, kPlaceThreads waves of whole
// counting workgroups per block (per_block of them, wpg waves each): the
// output slot of every wave with a match, from the same two-level prefix.
__global__ __launch_bounds__(kPlaceThreads) void k_place_waves(const uint32_t *wave_count,
                                                               const unsigned long long *part,
                                                               const unsigned long long *sup, int64_t nwaves,
                                                               int wpg, int per_block, int64_t *wave_off,
                                                               uint32_t *list, uint32_t *list_count) {
    __shared__ unsigned long long sh[kPlaceThreads / kWave];
    const int t = threadIdx.x;
    const int64_t wg0 = int64_t(blockIdx.x) * per_block;
    const int64_t w = wg0 * wpg + t;
    const uint32_t c = (t < per_block * wpg && w < nwaves) ? wave_count[w] : 0u;
    const int64_t sb = wg0 / kSuper * kSuper;
    unsigned long long before = 0;
    for (int64_t i = sb + t; i < wg0; i += kPlaceThreads) before += part[i];
    const int64_t base = int64_t(sup[wg0 / kSuper] + block_sum(before, sh));
    unsigned long long total;
    const unsigned long long ex = block_exclusive_scan(c, sh, &total);
    if (c) {
        wave_off[w] = base + int64_t(ex);
        list[atomicAdd(list_count, 1u)] = uint32_t(w);  // any order: each wave knows its slot
    }
}

// Positions of per-wave plans.  A fixed grid of kRewalkGroups workgroups of
// kRewalkThreads goes through the list of waves with a match (written by the
// placement pass; its length was set before the grid starts, so every loop
// ends).  Each such wave's 64 spans (64 S bytes from the wave's first walk)
// are split into shares of 64 S / kRewalkThreads bytes (rounded up to 16),
// each walked with the m - 1 bytes after it from the start state, counting
// the matches that start in it and keeping the first two; after a block scan
// of the counts gives each share its output slot (after the wave's), a share
// with at most two matches writes them from registers and one with more walks
// again, writing as it goes (for m >= 12 a share rarely has more than one).
// The table is read
// through a pointer into dynamic LDS (the block scan's slots follow it
// there).  256 groups (one per CU) cost less to launch than 1024 when the
// list is short (a few microseconds per call) and measured the same on a
// dense list (160 million matches, every N-run wave listed); 64 were twice
// as slow there.
constexpr int kRewalkThreads = 1024;
constexpr int kRewalkGroups = 256;

// One thread's share: the matches starting in [a, b), walking bytes
// [a, min(n, b + m - 1)) from the start state (a match ends m - 1 bytes after
// it starts; from the start state at a, no match that starts before a can be
// completed).  WRITE: the k-th of them goes to positions[off + k] (below cap).
// a is a multiple of 4.  The bytes come 16 at a time as four words, the next
// 16 requested before the current ones are walked, from the text in global
// memory, or (STAGED) from the wave's bytes staged in LDS, byte j at
// staged[j - base].
template <bool STAGED>
__device__ __forceinline__ void rewalk_fetch(const uint8_t *text, int64_t n, const uint8_t *staged, int64_t base,
                                             int64_t j0, int64_t lim, uint32_t (&w)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t j = j0 + 4 * k;
        if (j >= lim) {
            w[k] = 0;
        } else if (STAGED) {
            w[k] = *reinterpret_cast<const uint32_t *>(staged + (j - base));  // staged up to lim, padded to 16
        } else if (j + 4 <= n) {
            w[k] = *reinterpret_cast<const uint32_t *>(text + j);
        } else {
            uint32_t v = 0;
            for (int i = 0; j + i < n; ++i) v |= uint32_t(text[j + i]) << (8 * i);
            w[k] = v;
        }
    }
}

template <bool WRITE, bool STAGED>
__device__ __forceinline__ uint32_t rewalk_share(const uint8_t *text, int64_t n, const uint8_t *staged, int64_t base,
                                                 const unsigned char *tab, uint32_t m, int64_t a, int64_t b,
                                                 int64_t off, int64_t *positions, int64_t cap, int64_t &s0,
                                                 int64_t &s1) {
    const int64_t lim = b + int64_t(m) - 1 < n ? b + int64_t(m) - 1 : n;
    uint32_t q = 0, c = 0;
    uint32_t cur[4], nxt[4];
    rewalk_fetch<STAGED>(text, n, staged, base, a, lim, cur);
    for (int64_t j0 = a; j0 < lim; j0 += 16) {
        rewalk_fetch<STAGED>(text, n, staged, base, j0 + 16, lim, nxt);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            q = tab[q * uint32_t(kRow) + ((cur[k / 4] >> (8 * (k % 4))) & 0xffu)];
            if (q == m && j0 + k < lim) {
                const int64_t st = j0 + k - int64_t(m - 1);
                if (WRITE) {
                    if (off + c < cap) positions[off + c] = st;
                } else if (c == 0) {
                    s0 = st;
                } else if (c == 1) {
                    s1 = st;
                }
                ++c;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) cur[k] = nxt[k];
    }
    return c;
}

// LDS of k_rewalk: the table, the block scan's slots, and (staged) one listed
// wave's bytes: its 64 spans plus the m - 1 after them, padded to 16
__host__ __device__ inline int64_t rewalk_stage_offset(int m) { return table_lds_bytes(m) + 256; }
__host__ __device__ inline int64_t rewalk_lds_bytes(int m, int64_t S, bool staged) {
    return rewalk_stage_offset(m) + (staged ? (kWave * S + m - 1 + 15) / 16 * 16 + 16 : 0);
}

// STAGED: each listed wave's bytes are first copied to LDS with coalesced
// 16-byte loads by the whole workgroup, so that the shares (a few dozen bytes
// each, overlapping by m - 1) are walked from LDS instead of each thread
// waiting on its own chain of global loads.
template <bool STAGED>
__global__ __launch_bounds__(kRewalkThreads) void k_rewalk(const uint8_t *text, int64_t n, const uint8_t *table,
                                                           int32_t m, int64_t S, const uint32_t *list,
                                                           const uint32_t *list_count, const int64_t *wave_off,
                                                           int64_t *positions, int64_t cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t nlist = *list_count;
    if (blockIdx.x >= nlist) return;
    const int t = threadIdx.x;
    {
        const uint32_t *tg = reinterpret_cast<const uint32_t *>(table);
        const int words = (m + 1) * (DFA_ALPHABET / 4);
        for (int i = t; i < words; i += kRewalkThreads)
            *reinterpret_cast<uint32_t *>(smem + (i >> 6) * kRow + 4 * (i & 63)) = tg[i];
    }
    unsigned long long *sh = reinterpret_cast<unsigned long long *>(smem + table_lds_bytes(m));
    uint8_t *staged = smem + rewalk_stage_offset(m);
    __syncthreads();
    int64_t share = (kWave * S / kRewalkThreads + 15) / 16 * 16;  // S is a multiple of 16
    if (share < 16) share = 16;
    for (uint32_t i = blockIdx.x; i < nlist; i += gridDim.x) {  // uniform over the workgroup
        const int64_t gw = list[i];
        const int64_t start = gw * kWave * S;
        const int64_t end = start + kWave * S < n ? start + kWave * S : n;
        if (STAGED) {
            // bytes [start, min(n, end + m - 1)): start is 16-byte aligned; past n zeros
            const int64_t lim = end + m - 1 < n ? end + m - 1 : n;
            __syncthreads();  // the previous wave's shares are walked
            for (int64_t k = int64_t(t) * 16; start + k < lim; k += int64_t(kRewalkThreads) * 16) {
                v4u v;
                if (start + k + 16 <= n) {
                    v = *reinterpret_cast<const v4u *>(text + start + k);
                } else {
                    uint32_t w4[4] = {0u, 0u, 0u, 0u};
                    for (int e = 0; start + k + e < n; ++e) w4[e / 4] |= uint32_t(text[start + k + e]) << (8 * (e % 4));
                    v = v4u{w4[0], w4[1], w4[2], w4[3]};
                }
                *reinterpret_cast<v4u *>(staged + k) = v;
            }
            __syncthreads();
        }
        const int64_t a = start + t * share;
        const int64_t b = a + share < end ? a + share : end;
        int64_t s0 = 0, s1 = 0;  // the first two match starts, kept by the counting walk
        const uint32_t c = a < b ? rewalk_share<false, STAGED>(text, n, staged, start, smem, uint32_t(m), a, b, 0,
                                                               nullptr, 0, s0, s1)
                                 : 0u;
        unsigned long long total;
        const int64_t off = wave_off[gw] + int64_t(block_exclusive_scan(c, sh, &total));
        if (c > 2) {
            rewalk_share<true, STAGED>(text, n, staged, start, smem, uint32_t(m), a, b, off, positions, cap, s0, s1);
        } else {
            if (c > 0 && off < cap) positions[off] = s0;
            if (c > 1 && off + 1 < cap) positions[off + 1] = s1;
        }
    }
}

// ---------------------------------------------------------------------------
// Host side: planning and the C ABI
// ---------------------------------------------------------------------------

struct Plan {
    int64_t S = 0;
    int K = 1;
    int line = 128;
    int wpg = 4;
    int rounds = 0;
    int64_t nwalks = 0;
    int64_t blocks = 0;
    size_t lds = 0;
};

template <int K, int LINE, int H>
const void *scan_fn(int mode) {
    if (mode == kCount) return reinterpret_cast<const void *>(&k_scan<K, LINE, kCount, H>);
    if (mode == kCountPerWalk) return reinterpret_cast<const void *>(&k_scan<K, LINE, kCountPerWalk, H>);
    if (mode == kPositions) return reinterpret_cast<const void *>(&k_scan<K, LINE, kPositions, H>);
    if constexpr (K == 1) {
        if (mode == kCountPerWave) return reinterpret_cast<const void *>(&k_scan<K, LINE, kCountPerWave, H>);
    }
    return nullptr;
}

// the (walks per lane, bytes per round) shapes compiled into the library, each
// with the overlap prefetch depth for the pattern length
const void *pick_scan(int K, int line, int mode, int m) {
    const int h = halo_units_for(m);
    if (K == 1 && line == 128) return h == 1 ? scan_fn<1, 128, 1>(mode) : scan_fn<1, 128, 4>(mode);
    if (K == 1 && line == 64)
        return h == 1 ? scan_fn<1, 64, 1>(mode) : h == 2 ? scan_fn<1, 64, 2>(mode) : scan_fn<1, 64, 4>(mode);
    if (K == 2 && line == 64) return scan_fn<2, 64, 4>(mode);
    return nullptr;
}

// LDS of one workgroup of a plan made for `mode`: the table, one transpose
// buffer per wave and, where the per-walk counting pass stages its records,
// 1 KiB more per wave (the positions pass runs with the same plan and size).
bool plan_stages(int K, int m, int mode) { return stages_records(K, mode, halo_units_for(m)) && m <= kStageMaxM; }

// Positions plans for patterns of at least kPerWaveMinM bytes, one walk per
// lane, count per wave: their walk is the count-only one (per-walk counts and
// records cost registers, i.e. resident waves, and at m > 33 spill), and such
// matches are rarely dense -- on a 4-letter text a 12-mer is expected once per
// 4^12 ~ 17 million bytes, one wave's 32 KiB of spans in ~500 -- so walking
// the few waves with a match twice more costs less than per-walk bookkeeping
// in every wave.  Shorter patterns keep the per-walk plan: an 8-mer lands in
// about every second wave.
constexpr int kPerWaveMinM = 12;
bool per_wave_plan(int K, int m) { return K == 1 && m >= kPerWaveMinM; }

size_t scan_lds_bytes(int wpg, int K, int line, int m, int mode) {
    const bool rec = plan_stages(K, m, mode);
    // the positions pass runs with the counting pass's plan: size its table as marked too
    const int tmode = mode == kPositions ? int(kCountPerWalk) : mode;
    return size_t(wpg) * (K * kWave * line + (rec ? kRecBytes : 0)) + size_t(scan_table_bytes(m, K, tmode));
}

// Default span of one walk, in whole 128-byte lines: 512 bytes up to m = 16,
// 1024 up to m = 64, 2048 beyond.  Short walks make short workgroups, which
// the hardware dispatcher balances well (the launch's tail, while the last
// workgroups finish, shrinks with them); the span grows with m so that the
// overlap (m - 1 bytes walked twice) stays small.
constexpr int64_t kSpanMin = 512;
constexpr int64_t kSpanMax = 2048;

// The shortest span a plan for this tune can use (sizes the positions workspace).
int64_t min_span(const dfa_tune *t) { return (t && t->chain_bytes > 0) ? t->chain_bytes : kSpanMin; }

// gfx950 compute unit: 4 SIMDs, 512 vector registers per lane per SIMD, at
// most 8 waves per SIMD, 160 KiB of LDS
constexpr int kSimdsPerCu = 4;
constexpr int kVgprsPerLane = 512;
constexpr int kMaxWavesPerSimd = 8;
constexpr size_t kLdsPerCu = 160 * 1024;

constexpr int kDefaultK = 1;
constexpr int kDefaultLine = 64;
constexpr int kDefaultWpg = 4;


bool check_tune(const dfa_tune *t) {
    if (!t) return true;
    if (t->chain_bytes < 0 || (t->chain_bytes % 16) != 0) {
        dfa::set_error("tune.chain_bytes=%lld must be a positive multiple of 16 (or 0)",
                       (long long)t->chain_bytes);
        return false;
    }
    if (t->chain_bytes > (int64_t(1) << 24)) {
        dfa::set_error("tune.chain_bytes=%lld above 2^24", (long long)t->chain_bytes);
        return false;
    }
    if (t->line_bytes != 0 && t->line_bytes != 64 && t->line_bytes != 128) {
        dfa::set_error("tune.line_bytes=%d must be 64 or 128 (or 0)", t->line_bytes);
        return false;
    }
    const int line = t->line_bytes ? t->line_bytes : kDefaultLine;
    const int K = t->chains_per_lane ? t->chains_per_lane : kDefaultK;
    const int max_waves = (K == 1 && line == 64) ? 16 : 8;
    if (t->waves_per_group < 0 || t->waves_per_group > max_waves) {
        dfa::set_error("tune.waves_per_group=%d outside [1, %d] for this shape", t->waves_per_group, max_waves);
        return false;
    }
    if (t->chains_per_lane < 0 || !pick_scan(K, line, kCount, 1)) {
        dfa::set_error("tune: chains_per_lane=%d with line_bytes=%d is not a built shape "
                       "(1 with 64 or 128, 2 with 64)", t->chains_per_lane, line);
        return false;
    }
    if (t->dfas_per_group < 0 || t->automaton_bytes < 0) {
        dfa::set_error("tune: negative field");
        return false;
    }
    if (t->step_bytes < 0 || t->step_bytes > 2) {
        dfa::set_error("tune.step_bytes=%d must be 1 or 2 (or 0)", t->step_bytes);
        return false;
    }
    for (int i = 0; i < 2; ++i)
        if (t->reserved[i]) {
            dfa::set_error("tune.reserved must be zero");
            return false;
        }
    return true;
}

// Upper bound on the number of walks for any plan of (n, tune): used to size
// the workspace without a device query.
int64_t max_walks(int64_t n, const dfa_tune *t) { return n > 0 ? dfa::ceil_div(n, min_span(t)) : 0; }

// workspace layout: walk counts u32[nw] | walk offsets i64[nw] | workgroup
// totals u64[nb] | super-block prefixes u64[nb / kSuper] | workgroup flags
// (per-wave plans: the list of waves with a match) u32[nb] | workgroup wave
// masks u32[nb] | the list's length u32 | first kStaged match starts
// u16[nw * kStaged] | the next ones u16[nw * kStaged], with nb sized for the
// smallest workgroup (64 walks), i.e. the number of waves
struct WsLayout {
    int64_t cnt = 0, off = 0, part = 0, sup = 0, flag = 0, waves = 0, ctr = 0, buf = 0, buf1 = 0, total = 0;
};
WsLayout ws_layout(int64_t nw) {
    WsLayout L;
    if (nw <= 0) return L;
    const int64_t nb = dfa::ceil_div(nw, kWave);
    L.cnt = 0;
    L.off = L.cnt + dfa::round_up(nw * 4, 256);
    L.part = L.off + dfa::round_up(nw * 8, 256);
    L.sup = L.part + dfa::round_up(nb * 8, 256);
    L.flag = L.sup + dfa::round_up(dfa::ceil_div(nb, kSuper) * 8, 256);
    L.waves = L.flag + dfa::round_up(nb * 4, 256);
    L.ctr = L.waves + dfa::round_up(nb * 4, 256);
    L.buf = L.ctr + 256;
    L.buf1 = L.buf + dfa::round_up(nw * 2 * kStaged, 256);
    L.total = L.buf1 + dfa::round_up(nw * 2 * (kBuffered - kStaged), 256);
    return L;
}
int64_t workspace_for(int64_t nw) { return ws_layout(nw).total; }

// Vector registers per lane of a compiled kernel (0 if unknown).
int kernel_vgprs(const void *fn) {
    static std::mutex mu;
    static std::map<const void *, int> seen;
    std::lock_guard<std::mutex> lk(mu);
    auto it = seen.find(fn);
    if (it != seen.end()) return it->second;
    hipFuncAttributes a{};
    const int regs = hipFuncGetAttributes(&a, fn) == hipSuccess ? a.numRegs : 0;
    if (regs <= 0) (void)hipGetLastError();
    seen[fn] = regs;
    return regs;
}

// Default waves per workgroup: of 4 and 8, the one that keeps more waves
// resident on a CU (4 on a tie), given the registers per wave and the LDS
// each workgroup needs (its transpose buffers plus its own copy of the
// table).  Smaller workgroups refill a CU at a finer grain; larger ones share
// one table among more waves, which matters once the table is large (long
// patterns).  Workgroups of 5 to 7 waves measured slower than both even where
// they fit more waves (m = 32: 0.59-0.61 ms for 3.2 GB against 0.54 in 4 or
// 8), and so did 16 (a tune's choice for the default shape) where registers
// allow only one such workgroup per CU: m = 32, 16 resident waves, 0.68 ms.
int default_wpg(const void *fn, int K, int line, int m, int mode) {
    const int regs = kernel_vgprs(fn);
    if (regs <= 0) return kDefaultWpg;
    const int per_simd = std::min(kMaxWavesPerSimd, kVgprsPerLane / int(dfa::round_up(regs, 8)));
    const int by_regs = kSimdsPerCu * std::max(1, per_simd);
    const int cand[2] = {4, 8};
    int waves[2];
    for (int i = 0; i < 2; ++i) {
        const int groups = int(kLdsPerCu / scan_lds_bytes(cand[i], K, line, m, mode));
        waves[i] = std::min(by_regs, groups * cand[i]);
    }
    return waves[1] > waves[0] ? cand[1] : cand[0];
}

bool make_plan(int64_t n, int m, int mode, const dfa_tune *t, Plan &pl) {
    pl.K = (t && t->chains_per_lane) ? t->chains_per_lane : kDefaultK;
    pl.line = (t && t->line_bytes) ? t->line_bytes : kDefaultLine;
    if (t && t->waves_per_group) {
        pl.wpg = t->waves_per_group;
    } else {
        const void *fn = pick_scan(pl.K, pl.line, mode, m);
        pl.wpg = fn ? default_wpg(fn, pl.K, pl.line, m, mode) : kDefaultWpg;
    }
    pl.lds = scan_lds_bytes(pl.wpg, pl.K, pl.line, m, mode);
    if (pl.lds > kLdsPerCu) {
        dfa::set_error("%d waves per workgroup with m=%d need %zu bytes of LDS (%zu per CU)", pl.wpg, m, pl.lds,
                       kLdsPerCu);
        return false;
    }
    if (t && t->chain_bytes > 0) {
        pl.S = t->chain_bytes;
    } else {
        // whole lines: every walk starts on a 128-byte boundary (the text is
        // 16-byte aligned, torch and hipMalloc give 256), so each round's
        // loads cover exactly one cache line per walk.  A span that is not a
        // multiple of the line makes every round straddle two lines; with
        // hundreds of streaming waves per XCD the shared line is evicted from
        // L2 before the next round needs it, and HBM reads double.  Longer
        // patterns take longer spans (m = 32 and 64 measured faster at 1024
        // than at 512 bytes, shorter ones slower).
        pl.S = m <= 16 ? kSpanMin : (m <= 64 ? 2 * kSpanMin : kSpanMax);
    }
    pl.rounds = int(dfa::ceil_div(pl.S + m - 1, pl.line));
    pl.nwalks = n > 0 ? dfa::ceil_div(n, pl.S) : 0;
    const int64_t walks_per_block = int64_t(pl.wpg) * kWave * pl.K;
    pl.blocks = dfa::ceil_div(pl.nwalks, walks_per_block);
    return true;
}

using dfa::hip_ok;

int launch_scan(const Plan &pl, int mode, const ScanParams &sp, hipStream_t st) {
    const void *fn = pick_scan(pl.K, pl.line, mode, sp.m);
    if (!fn) {
        dfa::set_error("no kernel for K=%d line=%d", pl.K, pl.line);
        return DFA_EINVAL;
    }
    // allow any plan's LDS (make_plan keeps it within a CU's)
    if (!dfa::allow_lds(fn, int(kLdsPerCu))) return DFA_EHIP;
    void *args[] = {const_cast<ScanParams *>(&sp)};
    if (!hip_ok(hipLaunchKernel(fn, dim3(unsigned(pl.blocks)), dim3(pl.wpg * kWave), args, pl.lds, st),
                "k_scan launch"))
        return DFA_EHIP;
    return DFA_OK;
}

// dfa_set_scan_events: events bracketing the text walk of this thread's calls
thread_local hipEvent_t t_scan_begin = nullptr, t_scan_end = nullptr;

// The walk over the whole text, bracketed by the measurement events if set.
int launch_walk(const Plan &pl, int mode, const ScanParams &sp, hipStream_t st) {
    if (t_scan_begin && !hip_ok(hipEventRecord(t_scan_begin, st), "hipEventRecord")) return DFA_EHIP;
    const int rc = launch_scan(pl, mode, sp, st);
    if (rc == DFA_OK && t_scan_end && !hip_ok(hipEventRecord(t_scan_end, st), "hipEventRecord")) return DFA_EHIP;
    return rc;
}

}  // namespace

extern "C" int dfa_set_scan_events(void *begin, void *end) {
    if ((begin == nullptr) != (end == nullptr)) {
        dfa::set_error("dfa_set_scan_events: give both events or neither");
        return DFA_EINVAL;
    }
    t_scan_begin = reinterpret_cast<hipEvent_t>(begin);
    t_scan_end = reinterpret_cast<hipEvent_t>(end);
    dfa::clear_error();
    return DFA_OK;
}

extern "C" int64_t dfa_count_workspace_bytes(int64_t n, int32_t m, int32_t want_positions,
                                             const dfa_tune *tune) {
    if (n < 0 || m < 1 || m > DFA_MAX_M || !check_tune(tune)) {
        if (n < 0 || m < 1 || m > DFA_MAX_M) dfa::set_error("dfa_count_workspace_bytes: bad n or m");
        return DFA_EINVAL;
    }
    if (!want_positions) return 0;
    return workspace_for(max_walks(n, tune));
}

extern "C" int dfa_count(const uint8_t *text, int64_t n, const uint8_t *table, int32_t m,
                         int64_t *count, int64_t *positions, int64_t cap, void *workspace,
                         int64_t workspace_bytes, const dfa_tune *tune, void *stream) {
    if (n < 0 || m < 1 || m > DFA_MAX_M) {
        dfa::set_error("dfa_count: n=%lld m=%d out of range", (long long)n, m);
        return DFA_EINVAL;
    }
    if ((!text && n > 0) || !table || !count) {
        dfa::set_error("dfa_count: null text, table or count");
        return DFA_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(text) & 15) || (reinterpret_cast<uintptr_t>(table) & 3) ||
        (reinterpret_cast<uintptr_t>(count) & 7)) {
        dfa::set_error("dfa_count: text must be 16-byte, table 4-byte, count 8-byte aligned");
        return DFA_EINVAL;
    }
    if (cap < 0 || (positions && (reinterpret_cast<uintptr_t>(positions) & 7))) {
        dfa::set_error("dfa_count: cap < 0 or misaligned positions");
        return DFA_EINVAL;
    }
    if (!check_tune(tune)) return DFA_EINVAL;
    const bool want_pos = positions != nullptr && cap > 0;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);

    if (want_pos) {
        const int64_t need = workspace_for(max_walks(n, tune));
        if (workspace_bytes < need || (need > 0 && !workspace) ||
            (reinterpret_cast<uintptr_t>(workspace) & 255)) {
            dfa::set_error("dfa_count: workspace of %lld bytes (256-aligned) needed, got %lld",
                           (long long)need, (long long)workspace_bytes);
            return DFA_ENOSPACE;
        }
    }

    if (n == 0 || !want_pos) {
        // the count-only scan adds into *count; the positions path writes it
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, reinterpret_cast<unsigned long long *>(count));
        if (!hip_ok(hipGetLastError(), "k_zero_u64 launch")) return DFA_EHIP;
    }
    if (n == 0) {
        dfa::clear_error();
        return DFA_OK;
    }

    const int K = (tune && tune->chains_per_lane) ? tune->chains_per_lane : kDefaultK;
    const bool per_wave = want_pos && per_wave_plan(K, m);
    const int count_mode = !want_pos ? kCount : per_wave ? kCountPerWave : kCountPerWalk;
    Plan pl;
    if (!make_plan(n, m, count_mode, tune, pl)) return DFA_EINVAL;
    if (want_pos && pl.S > kMaxPositionsSpan) {
        dfa::set_error("dfa_count: positions need chain_bytes <= %lld", (long long)kMaxPositionsSpan);
        return DFA_EINVAL;
    }

    ScanParams sp{};
    sp.text = text;
    sp.n = n;
    sp.table = table;
    sp.m = m;
    sp.rounds = pl.rounds;
    sp.S = pl.S;
    sp.nwalks = pl.nwalks;
    sp.total = reinterpret_cast<unsigned long long *>(count);
    sp.cap = cap;

    if (!want_pos) {
        int rc = launch_walk(pl, kCount, sp, st);
        if (rc == DFA_OK) dfa::clear_error();
        return rc;
    }

    uint8_t *ws = reinterpret_cast<uint8_t *>(workspace);
    const int64_t nw = pl.nwalks;
    const int group_walks = pl.wpg * kWave * pl.K;  // walks of one workgroup of both passes
    const WsLayout L = ws_layout(nw);
    uint32_t *wcnt = reinterpret_cast<uint32_t *>(ws + L.cnt);
    int64_t *woff = reinterpret_cast<int64_t *>(ws + L.off);
    unsigned long long *part = reinterpret_cast<unsigned long long *>(ws + L.part);
    unsigned long long *sup = reinterpret_cast<unsigned long long *>(ws + L.sup);
    uint32_t *flag = reinterpret_cast<uint32_t *>(ws + L.flag);
    uint32_t *waves = reinterpret_cast<uint32_t *>(ws + L.waves);
    uint32_t *list_count = reinterpret_cast<uint32_t *>(ws + L.ctr);
    uint16_t *wbuf = reinterpret_cast<uint16_t *>(ws + L.buf);
    uint16_t *wbuf1 = reinterpret_cast<uint16_t *>(ws + L.buf1);
    if (group_walks > kMaxGroupWalks || pl.blocks > dfa::ceil_div(nw, kWave)) {
        dfa::set_error("dfa_count: %d walks per workgroup (at most %d)", group_walks, kMaxGroupWalks);
        return DFA_EINVAL;
    }

    sp.walk_count = wcnt;
    sp.wg_part = part;
    sp.wg_waves = waves;
    if (per_wave) {
        // count per wave (walk_count / walk_off hold one entry per wave), then
        // the waves with a match are walked again to write their positions
        int rc = launch_walk(pl, kCountPerWave, sp, st);
        if (rc != DFA_OK) return rc;
        hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kPartsThreads), 0, st, (const unsigned long long *)part,
                           pl.blocks, sup, count, list_count);
        const int per_block = kPlaceThreads / pl.wpg;  // counting workgroups per placement block
        hipLaunchKernelGGL(k_place_waves, dim3(unsigned(dfa::ceil_div(pl.blocks, per_block))), dim3(kPlaceThreads), 0,
                           st, (const uint32_t *)wcnt, (const unsigned long long *)part,
                           (const unsigned long long *)sup, dfa::ceil_div(nw, kWave), pl.wpg, per_block, woff, flag,
                           list_count);
        if (!hip_ok(hipGetLastError(), "placement launch")) return DFA_EHIP;
        // the listed waves' bytes staged in LDS when they fit next to the table
        const bool staged = rewalk_lds_bytes(m, pl.S, true) <= int64_t(kLdsPerCu);
        const void *rw = staged ? reinterpret_cast<const void *>(&k_rewalk<true>)
                                : reinterpret_cast<const void *>(&k_rewalk<false>);
        if (!dfa::allow_lds(rw, int(kLdsPerCu))) return DFA_EHIP;
        const dim3 rw_grid(unsigned(std::min<int64_t>(kRewalkGroups, dfa::ceil_div(nw, kWave))));
        const size_t rw_lds = size_t(rewalk_lds_bytes(m, pl.S, staged));
        if (staged)
            hipLaunchKernelGGL(k_rewalk<true>, rw_grid, dim3(kRewalkThreads), rw_lds, st, text, n, table, m, pl.S,
                               (const uint32_t *)flag, (const uint32_t *)list_count, (const int64_t *)woff, positions,
                               cap);
        else
            hipLaunchKernelGGL(k_rewalk<false>, rw_grid, dim3(kRewalkThreads), rw_lds, st, text, n, table, m, pl.S,
                               (const uint32_t *)flag, (const uint32_t *)list_count, (const int64_t *)woff, positions,
                               cap);
        if (!hip_ok(hipGetLastError(), "k_rewalk launch")) return DFA_EHIP;
        dfa::clear_error();
        return DFA_OK;
    }
    sp.stage = plan_stages(pl.K, m, kCountPerWalk) ? 1 : 0;
    sp.walk_buf = wbuf;
    sp.walk_buf1 = wbuf1;
    int rc = launch_walk(pl, kCountPerWalk, sp, st);
    if (rc != DFA_OK) return rc;
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kPartsThreads), 0, st, (const unsigned long long *)part, pl.blocks,
                       sup, count, nullptr);
    const int per_block = kPlaceWalks / group_walks;  // counting workgroups per placement block
    hipLaunchKernelGGL(k_place, dim3(unsigned(dfa::ceil_div(pl.blocks, per_block))), dim3(kPlaceThreads), 0, st,
                       (const uint32_t *)wcnt, (const uint16_t *)wbuf, (const uint16_t *)wbuf1,
                       (const uint32_t *)waves, (const unsigned long long *)part, (const unsigned long long *)sup, nw,
                       pl.blocks, group_walks, kWave * pl.K, per_block, pl.S, woff, flag, positions, cap);
    if (!hip_ok(hipGetLastError(), "placement launch")) return DFA_EHIP;
    sp.wg_flag = flag;
    sp.walk_off = woff;
    sp.positions = positions;
    rc = launch_scan(pl, kPositions, sp, st);
    if (rc == DFA_OK) dfa::clear_error();
    return rc;
}

// ---------------------------------------------------------------------------
// dfa_count without a caller workspace: the positions workspace lives in a
// device array of the library, one copy per GPU.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol):
// the device address of the current GPU's copy is looked up once per device
// and used everywhere instead.  The positions path initialises every part of
// its workspace it reads (workgroup totals, wave masks, prefixes, the list
// length and the flags are written by the kernels of each call before they
// are read), so the contents a previous call left behind do not matter.
// ---------------------------------------------------------------------------

namespace {

static __device__ __align__(256) uint8_t scratch[DFA_NOALLOC_SCRATCH_BYTES];

// Device address of the current GPU's scratch, or nullptr (error set).
void *scratch_on_current_device() {
    static std::mutex mu;
    static std::map<int, void *> addr;  // device ordinal -> address of its copy
    int dev = -1;
    if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void *ptr = nullptr;
    if (!hip_ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) return nullptr;
    if (!ptr) {
        dfa::set_error("hipGetSymbolAddress(scratch) returned a null address");
        return nullptr;
    }
    addr[dev] = ptr;
    return ptr;
}

}  // namespace

extern "C" int dfa_count_noalloc(const uint8_t *text, int64_t n, const uint8_t *table, int32_t m,
                                 int64_t *count, int64_t *positions, int64_t cap, const dfa_tune *tune,
                                 void *stream) {
    const bool want_pos = positions != nullptr && cap > 0;
    int64_t need = 0;
    if (want_pos) {
        need = dfa_count_workspace_bytes(n, m, 1, tune);
        if (need < 0) return int(need);  // bad n, m or tune: message set
        if (need > DFA_NOALLOC_SCRATCH_BYTES) {
            dfa::set_error("dfa_count_noalloc: positions of n=%lld need %lld bytes of workspace, above the "
                           "library's %lld-byte scratch (use dfa_count with a caller workspace)",
                           (long long)n, (long long)need, (long long)DFA_NOALLOC_SCRATCH_BYTES);
            return DFA_ENOSPACE;
        }
    }
    void *ws = nullptr;
    if (need > 0) {
        ws = scratch_on_current_device();
        if (!ws) return DFA_EHIP;
    }
    return dfa_count(text, n, table, m, count, positions, cap, ws, need, tune, stream);
}

extern "C" int64_t dfa_count_timed(const uint8_t *text, int64_t n, const uint8_t *table, int32_t m, int64_t *count,
                                   unsigned long long *wg_times, int64_t wg_cap, const dfa_tune *tune, void *stream) {
    if (n <= 0 || m < 1 || m > DFA_MAX_M || !text || !table || !count || wg_cap < 0 || (wg_cap > 0 && !wg_times)) {
        dfa::set_error("dfa_count_timed: bad arguments");
        return DFA_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(text) & 15) || (reinterpret_cast<uintptr_t>(table) & 3) ||
        (reinterpret_cast<uintptr_t>(count) & 7) || (reinterpret_cast<uintptr_t>(wg_times) & 7)) {
        dfa::set_error("dfa_count_timed: misaligned argument");
        return DFA_EINVAL;
    }
    if (!check_tune(tune)) return DFA_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, reinterpret_cast<unsigned long long *>(count));
    if (!hip_ok(hipGetLastError(), "k_zero_u64 launch")) return DFA_EHIP;
    Plan pl;
    if (!make_plan(n, m, kCount, tune, pl)) return DFA_EINVAL;
    ScanParams sp{};
    sp.text = text;
    sp.n = n;
    sp.table = table;
    sp.m = m;
    sp.rounds = pl.rounds;
    sp.S = pl.S;
    sp.nwalks = pl.nwalks;
    sp.total = reinterpret_cast<unsigned long long *>(count);
    sp.wg_times = wg_times;
    sp.wg_cap = wg_cap;
    const int rc = launch_scan(pl, kCount, sp, st);
    if (rc != DFA_OK) return rc;
    dfa::clear_error();
    return pl.blocks;
}