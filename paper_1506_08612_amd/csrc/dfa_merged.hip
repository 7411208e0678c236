// Batched counting with merged multi-pattern automata for gfx950.
//
// The paper's improved Aho-Corasick automaton (Sec. "Implementation Aspects",
// Fig. 4, Table 2) advances every pattern of a set with one table lookup per
// text byte.  Here the pairs (segment, pattern) of each segment are merged
// into as few automata as fit the LDS budget; one work item is (one tile of
// a segment, one automaton); every lane walks its own span of the tile.
//
// Table layout.  The paper stores 256 columns per state so that a byte is its
// own column.  With thousands of states per automaton that is 512 bytes per
// state and no automaton worth merging fits LDS, so each automaton is kept as
// a byte-class map (256 entries; every byte that occurs in none of its
// patterns is one class, on which every state returns to the start) and a
// 16-bit table with one column per class.  A step is the class of the byte
// (independent of the state, so off the dependent chain) and one LDS read of
// the next state.  For DNA-like alphabets the class comes from registers (a
// v_perm over an 8-entry table in two registers, four bytes at a time, see
// reg_classes); other bytes take one more LDS read of the class map.
// Reporting states are numbered last (first_final on),
// so "is final" is one compare; visits of each reporting state are counted in
// an LDS histogram and turned into per-pair counts at the end through the
// per-state output lists.
//
// Pair automata (on request: tune step_bytes = 2).  Where an automaton has
// few byte classes (DNA patterns have five: A, C, G, T and everything else)
// its table over PAIRS of classes, the state after two bytes, takes ncls^2
// columns per state, and a full wave's rounds then take one dependent table
// read per two bytes.  A pair entry carries one more bit: whether the state
// after the first byte reports, so that visits stay exact (the rare pair with
// one recomputes that state with the one-step table).  Their larger images
// leave room for fewer workgroups per CU, and at the occupancy the one-step
// walk reaches they measured slower.
//
// Ownership.  A walk owns the match starts of its span [w, w + S) and reads
// max(m) - 1 bytes past it (clipped at the segment end).  A match that ends
// inside the span starts inside it (the walk starts in the start state at w);
// a match that ends in the overlap is counted only if it starts before w + S,
// checked per reported pattern.  This start-position rule makes patterns of
// unequal lengths exact, where a single m - 1 overlap (Sec. III.A) would count
// some matches twice.
//
// Data movement follows the single-pattern scan: walks start on 128-byte
// boundaries (the first walk of a segment may start before the segment and
// skips the bytes in front of it), rounds of 32 or 64 bytes of every walk
// staged through a wave-private LDS transpose (32-byte rounds take half the
// LDS, so that a workgroup with a large automaton leaves room for another;
// 64-byte rounds are fetched as whole lines, non-temporal, where no tile is
// walked by a second automaton), the overlap read from memory after the
// rounds.  Items are ordered so that consecutive items on one XCD walk the
// same tile with different automata, whose later reads of it then find it in
// that XCD's L2 while it holds it.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ac_build.h"
#include "dfa.h"
#include "dfa_internal.h"
#include "launch_util.h"
#include "walk_common.h"

namespace {

using namespace dfa_dev;

constexpr int kWavesPerSimd = 8;                 // register budget of the scan kernels (64 VGPRs)
constexpr int kXcds = 8;                         // workgroups are dealt to the XCDs in turn
constexpr int64_t kMinSpan = 256;                // span bounds (multiples of 128)
constexpr int64_t kMaxSpan = 1024;
// Longest span of a segment walked by a single automaton: 72 8-mers over 1 GB
// in 0.267-0.269 ms at 768 bytes against 0.279-0.284 at 1024 (same box); where
// several automata walk each tile (and read it from L2 after the first),
// 1024-byte spans measured faster (1 GB x 1024 patterns: 1.83 against 1.90 ms).
constexpr int64_t kMaxSpanOne = 768;
constexpr int kMaxWaves = 16;                    // waves per workgroup (the kernel's launch bound)
// LDS budget of one merged automaton: with 16-wave workgroups and 32-byte
// rounds, two workgroups of 64 KiB automata fit a CU (1 GB x 1024 patterns,
// before short patterns were packed first: 7 automata, 1.86 ms; 56 KiB: 8,
// 2.19 ms; 80 KiB: 6 at one workgroup of 16 or two of 8 waves, 2.35 ms)
constexpr int kDefaultAutomatonBytes = 64 * 1024;
constexpr int kMinAutomatonBytes = 4 * 1024;
constexpr int kLdsPerCu = 160 * 1024;
constexpr int kCmapBytes = 512;                  // 256 x u16: twice the class of each byte

typedef __attribute__((address_space(3))) const uint16_t lds_u16;

// An automaton's LDS image (copied from the workspace to LDS address 0; its
// visit counters follow it).  One-step automata: the nstates x ncls u16 table
// at 0, then the 16-bit class map.  Pair automata: a byte map of c at 0,
// the nstates x ncls^2 u16 pair table at kPairMaps, the one-step table, then
// the 16-bit class map, whose entries hold the one-step table's LDS offset
// plus 2 c, so that one-step reads need no base either.
struct MAuto {
    int64_t table_off;  // offset of the image in the workspace
    int64_t fin_base;   // global index of this automaton's first reporting state
    int32_t nstates;
    int32_t first_final;
    int32_t ncls;
    int32_t maxm;
    int32_t image_bytes;  // bytes of the image (16-byte multiple)
    int32_t cmap_off;     // LDS offset of the 16-bit class map
    int32_t pair;         // nonzero: pair automaton
    int32_t cls_shift;    // register classes: a byte's slot is bits [s, s + 3) of it
    uint32_t lut_lo;      // register classes: byte h of (lut_hi:lut_lo) is the class of the byte in slot h
    uint32_t lut_hi;
    uint32_t key_lo;      // byte h of (key_hi:key_lo): the one byte slot h's lut entry holds
    uint32_t key_hi;
    int32_t scaled;       // one-step entries are byte offsets of the next state's row (else state numbers)
    uint32_t magic;       // ceil(2^32 / row bytes): a row offset's state number is its high product
};

struct MItem {
    int64_t tile_start;  // first byte of the tile's first walk
    int64_t seg_lo;      // segment start: bytes before it are skipped
    int64_t own_end;     // the tile owns match starts below this
    int64_t seg_end;     // segment end: nothing is read past it
    int32_t automaton;
    int32_t span;        // S, a multiple of 128
};

struct OutEntry {
    int32_t pair;  // the counter the pattern's matches go to
    int32_t m;
};

struct MParams {
    const uint8_t *text;
    int64_t n;
    const uint8_t *ws;  // workspace base (tables)
    const MAuto *autos;
    const MItem *items;
    const int32_t *out_off;  // per global reporting state: its entries
    const OutEntry *out_ent;
    unsigned long long *visits;  // per global reporting state
    unsigned long long *counts;  // per pair
};

// Per lane: bytes before the segment (skipped), owned starts, bytes that count.
struct MLane {
    uint32_t lo, own, len;
};

struct MCtx {
    uint32_t row2;   // bytes per one-step table row
    uint32_t rowp;   // bytes per pair table row (pair automata)
    uint32_t cmap;   // LDS address of the 16-bit class map
    uint32_t hist;   // LDS address of the visit counters
    uint32_t F;      // first reporting state
    int64_t fin_base;
    uint32_t cs, lut_lo, lut_hi, key_lo, key_hi;  // register classes (MAuto)
    uint32_t wts0, wts1;  // pair automata: byte weights (2 ncls, 2) of each pair of a text word
    // one-step table entries: e = q qrow, a row at byte e qscale (qrow qscale = row2),
    // the first reporting entry Fx = F qrow
    uint32_t qrow, qscale, Fx, magic;
};

// Pair automata: the byte map sits at LDS 0 and the pair table at kPairMaps,
// so every address of a pair step is a sum of per-lane terms and a constant
// the reads take as their offset.  A pair entry is the state after both
// bytes, with bit 15 set when the state after the first byte reports (states
// stay below 2^15).
constexpr uint32_t kPairMaps = 256;
constexpr uint32_t kMidReports = 0x8000u;
typedef __attribute__((address_space(3))) const uint8_t lds_u8c;

// Register classes.  Where an automaton's pattern bytes (those of classes 1
// and up) are at most eight and differ in three consecutive bits [s, s + 3),
// those bits of a text byte name its slot, and one v_perm over the 8-byte
// register table (lut_hi:lut_lo) gives the class bytes of all four bytes of
// a word at once (2 c, a column's byte offset, for one-step automata; c for
// pair automata); the same v_perm over (key_hi:key_lo) gives the byte each
// slot stands for.  A word whose four bytes equal their slots' bytes is classed in
// registers; any other word (a default-class byte in a slot that stands for
// another byte) takes the LDS class map.  Slots that no pattern byte takes
// stand for a default-class byte ('N' where it can), with c = 0.  An
// automaton whose pattern bytes do not fit has keys that no byte matches.
__device__ __forceinline__ bool reg_classes(uint32_t w, const MCtx &x, uint32_t &P) {
    const uint32_t h = (w >> x.cs) & 0x07070707u;
    P = __builtin_amdgcn_perm(x.lut_hi, x.lut_lo, h);
    return __builtin_amdgcn_perm(x.key_hi, x.key_lo, h) == w;
}

// The class bytes of the four bytes of w, byte b of the result for byte b of
// w: from registers, else from the LDS maps.  Pair automata: c (the byte map
// at 0).  One-step automata: 2 c, the byte offset of the class's column (the
// 16-bit map at cmap; their table is at 0 and has at most 128 classes where
// this is called).
template <bool PAIR>
__device__ __forceinline__ uint32_t word_classes(uint32_t w, const MCtx &x) {
    uint32_t P;
    if (!reg_classes(w, x, P)) {
        P = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t byte = (w >> (8 * b)) & 0xffu;
            const uint32_t c = PAIR ? uint32_t(*reinterpret_cast<lds_u8c *>(uintptr_t(byte)))
                                    : uint32_t(*reinterpret_cast<lds_u16 *>(uintptr_t(x.cmap + 2u * byte)));
            P |= c << (8 * b);
        }
    }
    return P;
}

// Index among the automaton's reporting states of a one-step table entry
// e >= Fx (a row offset's state number is a high product with the magic
// reciprocal, exact for offsets below 2^16 that are multiples of row2).
__device__ __forceinline__ uint32_t fin_index(uint32_t e, const MCtx &x) {
    return x.qrow == 1u ? e - x.Fx : __umulhi(e - x.Fx, x.magic);
}

// A reporting state (index f) reached at byte j of the overlap: count each
// reported pattern whose match starts inside the span (j - m + 1 < own).
__device__ __forceinline__ void overlap_hit(const MParams &p, const MCtx &x, uint32_t f, uint32_t j, uint32_t own) {
    const int64_t g = x.fin_base + int64_t(f);
    const int32_t e1 = p.out_off[g + 1];
    for (int32_t e = p.out_off[g]; e < e1; ++e) {
        const OutEntry oe = p.out_ent[e];
        if (j + 1 < own + uint32_t(oe.m)) atomicAdd(p.counts + oe.pair, 1ull);
    }
}

// Walk 16 bytes one byte per step with the lane's [lo, own, len) deciding
// (edge waves and every overlap); byte b of word w is byte jb + 4w + b of the
// walk, q a one-step table entry.  Per half of the unit: its 8 column
// offsets first (they do not depend on the state: from registers where the
// entries are row offsets of a one-step automaton, else 8 reads of the class
// map in flight together), then the 8 steps, then one test of the largest
// entry reached before the visits are counted.  Only a segment's first walk
// skips bytes (fewer than 128, in front of the segment), so the start state
// is forced only in the walk's first 128 bytes.
template <bool PAIR>
__device__ __forceinline__ void mwalk16_guarded(const v4u &t, uint32_t &q, uint32_t jb, const MCtx &x,
                                                const MLane &L, unsigned char *smem, const MParams &p) {
    uint32_t *hist = reinterpret_cast<uint32_t *>(smem + x.hist);
    const bool lo_guard = jb < 128u;  // wave-uniform
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint32_t qs[8];
        if (!PAIR && x.qrow != 1u) {
            const uint32_t P0 = word_classes<false>(t[2 * h], x), P1 = word_classes<false>(t[2 * h + 1], x);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                q = *reinterpret_cast<lds_u16 *>(uintptr_t(q + (((i < 4 ? P0 : P1) >> (8 * (i % 4))) & 0xffu)));
                if (lo_guard && jb + uint32_t(8 * h + i) < L.lo) q = 0;  // in front of the segment
                qs[i] = q;
            }
        } else {
            uint32_t k2[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                k2[i] = *reinterpret_cast<lds_u16 *>(
                    uintptr_t(x.cmap + 2u * ((t[2 * h + i / 4] >> (8 * (i % 4))) & 0xffu)));
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                q = *reinterpret_cast<lds_u16 *>(uintptr_t(__umul24(q, x.qscale) + k2[i]));
                if (lo_guard && jb + uint32_t(8 * h + i) < L.lo) q = 0;  // in front of the segment
                qs[i] = q;
            }
        }
        uint32_t top = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) top = max(top, qs[i]);
        if (top >= x.Fx) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t j = jb + uint32_t(8 * h + i);
                if (qs[i] >= x.Fx) {
                    if (j < L.own)
                        atomicAdd(hist + fin_index(qs[i], x), 1u);
                    else if (j < L.len)
                        overlap_hit(p, x, fin_index(qs[i], x), j, L.own);
                }
            }
        }
    }
}

// Walk 16 bytes of a full wave one byte per step (one-step automata whose
// entries are row offsets).  Per text word: the column offsets 2 c of its
// bytes, then its 4 steps, each one add (the row offset plus a byte of the
// column offsets) and the transition read, then one test of the largest
// entry reached against Fx (reporting states are numbered last) before the
// visits are counted.
__device__ __forceinline__ void mwalk16_full(const v4u &t, uint32_t &q, const MCtx &x, uint32_t *hist) {
#pragma unroll
    for (int wd = 0; wd < 4; ++wd) {
        const uint32_t P = word_classes<false>(t[wd], x);
        uint32_t qs[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            q = *reinterpret_cast<lds_u16 *>(uintptr_t(q + ((P >> (8 * i)) & 0xffu)));
            qs[i] = q;
        }
        if (max(max(qs[0], qs[1]), max(qs[2], qs[3])) >= x.Fx) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (qs[i] >= x.Fx) atomicAdd(hist + fin_index(qs[i], x), 1u);
        }
    }
}

// A pair whose entry e is at least F (a reporting state after its second
// byte, or bit 15: after its first) counts its visits; qp is the state before
// the pair and c1 its first byte.
__device__ __forceinline__ void pair_visits(uint32_t e, uint32_t qp, uint32_t c1, const MCtx &x, uint32_t *hist) {
    if (e & kMidReports) {  // the one-step table's entry after c1
        const uint32_t k2 = *reinterpret_cast<lds_u16 *>(uintptr_t(x.cmap + 2u * c1));
        const uint32_t mid = *reinterpret_cast<lds_u16 *>(uintptr_t(__umul24(qp, x.row2) + k2));
        atomicAdd(hist + fin_index(mid, x), 1u);
    }
    const uint32_t q = e & (kMidReports - 1u);
    if (q >= x.F) atomicAdd(hist + (q - x.F), 1u);
}

// Walk 16 bytes of a full wave two bytes per step (pair automata).  Per text
// word: the classes of its bytes, then 2 dependent pair reads, each at row q
// and column ncls c1 + c2 (a v_dot4 of the word's class bytes with weights
// 2 ncls and 2 gives the byte offset), then one test of the larger entry
// against F (bit 15 exceeds every state).
__device__ __forceinline__ void mwalk16_pair(const v4u &t, uint32_t &q, const MCtx &x, uint32_t *hist) {
#pragma unroll
    for (int wd = 0; wd < 4; ++wd) {
        const uint32_t w = t[wd];
        const uint32_t P = word_classes<true>(w, x);
        const uint32_t q0 = q;
        const uint32_t e0 = *reinterpret_cast<lds_u16 *>(
            uintptr_t(kPairMaps + __builtin_amdgcn_udot4(P, x.wts0, __umul24(q, x.rowp), false)));
        const uint32_t q1 = e0 & (kMidReports - 1u);
        const uint32_t e1 = *reinterpret_cast<lds_u16 *>(
            uintptr_t(kPairMaps + __builtin_amdgcn_udot4(P, x.wts1, __umul24(q1, x.rowp), false)));
        q = e1 & (kMidReports - 1u);
        if (max(e0, e1) >= x.F) {
            if (e0 >= x.F) pair_visits(e0, q0, w & 0xffu, x, hist);
            if (e1 >= x.F) pair_visits(e1, q1, (w >> 16) & 0xffu, x, hist);
        }
    }
}

// The units of a staged round of a full wave, the next one read from LDS
// while the current one is walked.
template <int LINE, bool PAIR>
__device__ __forceinline__ void mwalk_round(const v4u *xb, int lane, uint32_t &q, const MCtx &x, uint32_t *hist) {
    using G = Geo<LINE>;
    v4u cur = unit_of<LINE>(xb, 0, lane, 0), nxt = cur;
#pragma unroll
    for (int u = 0; u < G::U; ++u) {
        if (u + 1 < G::U) nxt = unit_of<LINE>(xb, 0, lane, u + 1);
        if (PAIR)
            mwalk16_pair(cur, q, x, hist);
        else
            mwalk16_full(cur, q, x, hist);
        cur = nxt;
    }
}

// The rounds and overlap of a full wave (every walk inside its segment, its
// span owned and its overlap inside the segment and the text).  S is a
// multiple of 128: the rounds come in pairs.  NT (64-byte rounds only): each
// pair of rounds is fetched as whole 128-byte lines with non-temporal loads,
// for plans where no tile is walked by a second automaton (whose reads would
// want the lines kept in L2).  The overlap goes one byte per step (it counts
// only matches that start inside the span), its units read from memory after
// the rounds: the first H unrolled, the rest in a loop.
template <int H, bool PAIR, int LINE, bool NT>
__device__ __forceinline__ void walk_full(const MParams &p, v4u *xb, int lane, int64_t wbase, int64_t wstart,
                                          int64_t S, uint32_t lane_off, int maxm, uint32_t &q, const MCtx &x,
                                          const MLane &L, unsigned char *smem) {
    static_assert(!NT || LINE == 64, "whole-line fetches take 64-byte rounds");
    using G = Geo<LINE>;
    uint32_t *hist = reinterpret_cast<uint32_t *>(smem + x.hist);
    const int R = int(S / LINE);
    const int rlast = R - 1;
    if constexpr (NT) {
        const uint32_t pair_off = uint32_t(lane / 8) * uint32_t(S) + 16u * uint32_t(lane % 8);
        v4u pp[1][8];
        fetch_pair<1>(pp, p.text, wbase, S, pair_off, lane, 0, rlast);
        for (int r = 0; r < R; r += 2) {
            stage_pair<1, 0>(pp, xb, lane);
            mwalk_round<LINE, PAIR>(xb, lane, q, x, hist);
            stage_pair<1, 1>(pp, xb, lane);
            fetch_pair<1>(pp, p.text, wbase, S, pair_off, lane, r + 2, rlast);
            mwalk_round<LINE, PAIR>(xb, lane, q, x, hist);
        }
    } else {
        const uint32_t off_none = 16u * uint32_t(lane % G::U);
        v4u pa[1][G::U], pb[1][G::U];
        fetch_round_or_none<1, LINE>(pa, p.text, wbase, S, lane_off, lane_off, off_none, 0, rlast);
        fetch_round_or_none<1, LINE>(pb, p.text, wbase, S, lane_off, lane_off, off_none, 1, rlast);
        for (int r = 0; r < R; r += 2) {
            stage_round<1, LINE>(pa, xb, lane);
            mwalk_round<LINE, PAIR>(xb, lane, q, x, hist);
            stage_round<1, LINE>(pb, xb, lane);
            fetch_round_or_none<1, LINE>(pa, p.text, wbase, S, lane_off, lane_off, off_none, r + 2, rlast);
            fetch_round_or_none<1, LINE>(pb, p.text, wbase, S, lane_off, lane_off, off_none, r + 3, rlast);
            mwalk_round<LINE, PAIR>(xb, lane, q, x, hist);
        }
    }
    if (PAIR) q *= x.qrow;  // the pair walk's state as a one-step table entry
    const int hu = (maxm - 1 + 15) / 16;
    const uint8_t *ov = p.text + wstart + S;
    v4u halo[H];
#pragma unroll
    for (int u = 0; u < H; ++u)
        if (u < hu) halo[u] = *reinterpret_cast<const v4u *>(ov + 16 * u);
#pragma unroll
    for (int u = 0; u < H; ++u)
        if (u < hu) mwalk16_guarded<PAIR>(halo[u], q, uint32_t(S) + 16u * u, x, L, smem, p);
    for (int u = H; u < hu; ++u) {
        const v4u t = *reinterpret_cast<const v4u *>(ov + 16 * u);
        mwalk16_guarded<PAIR>(t, q, uint32_t(S) + 16u * u, x, L, smem, p);
    }
}

// H: overlap units unrolled (1 where every pattern has at most 17 bytes,
// else 4; longer overlaps loop).  PAIR: every item's automaton is a pair
// automaton (the plan puts those items in launches of their own, so that
// each kernel keeps only its own path's registers).  LINE: bytes of every
// walk staged per round (32 or 64).  NT: 64-byte rounds fetched as whole
// lines with non-temporal loads.
template <int H, bool PAIR, int LINE, bool NT>
__global__ __launch_bounds__(kMaxWaves * kWave) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd))) void k_merged(
    MParams p) {
    using G = Geo<LINE>;
    extern __shared__ __align__(16) unsigned char smem[];
    const MItem it = p.items[blockIdx.x];
    const MAuto au = p.autos[it.automaton];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    const uint32_t ib = uint32_t(__builtin_amdgcn_readfirstlane(au.image_bytes));
    const uint32_t F = uint32_t(__builtin_amdgcn_readfirstlane(au.first_final));
    const uint32_t nst = uint32_t(__builtin_amdgcn_readfirstlane(au.nstates));
    const uint32_t ncls = uint32_t(__builtin_amdgcn_readfirstlane(au.ncls));
    const uint32_t nfin = nst - F;
    const int maxm = __builtin_amdgcn_readfirstlane(au.maxm);

    // LDS: the automaton's image (from address 0), visit counters, transpose buffers
    MCtx x;
    x.row2 = 2u * ncls;
    x.rowp = 2u * ncls * ncls;
    x.cmap = uint32_t(__builtin_amdgcn_readfirstlane(au.cmap_off));
    x.hist = ib;
    x.F = F;
    const bool scaled = __builtin_amdgcn_readfirstlane(au.scaled) != 0;
    x.qrow = scaled ? x.row2 : 1u;
    x.qscale = scaled ? 1u : x.row2;
    x.Fx = F * x.qrow;
    x.magic = uint32_t(__builtin_amdgcn_readfirstlane(int(au.magic)));
    x.fin_base = au.fin_base;
    x.cs = uint32_t(__builtin_amdgcn_readfirstlane(au.cls_shift));
    x.lut_lo = uint32_t(__builtin_amdgcn_readfirstlane(int(au.lut_lo)));
    x.lut_hi = uint32_t(__builtin_amdgcn_readfirstlane(int(au.lut_hi)));
    x.key_lo = uint32_t(__builtin_amdgcn_readfirstlane(int(au.key_lo)));
    x.key_hi = uint32_t(__builtin_amdgcn_readfirstlane(int(au.key_hi)));
    // lut_lo and key_lo kept in vector registers: a v_perm reads one scalar operand
    asm volatile("v_mov_b32 %0, %1" : "=v"(x.lut_lo) : "s"(x.lut_lo));
    asm volatile("v_mov_b32 %0, %1" : "=v"(x.key_lo) : "s"(x.key_lo));
    x.wts0 = (2u * ncls) | (2u << 8);
    x.wts1 = (2u * ncls << 16) | (2u << 24);
    const uint32_t stage = (x.hist + 4u * nfin + 15u) & ~15u;
    v4u *xb = reinterpret_cast<v4u *>(smem + stage + wave * (kWave * LINE));
    {
        const v4u *src = reinterpret_cast<const v4u *>(p.ws + au.table_off);
        const uint32_t chunks = ib / 16u;
        for (uint32_t i = threadIdx.x; i < chunks; i += blockDim.x) reinterpret_cast<v4u *>(smem)[i] = src[i];
        uint32_t *hist = reinterpret_cast<uint32_t *>(smem + x.hist);
        for (uint32_t i = threadIdx.x; i < nfin; i += blockDim.x) hist[i] = 0;
    }
    __syncthreads();

    const int64_t S = it.span;
    const int64_t wbase = it.tile_start + int64_t(wave) * kWave * S;
    const int64_t wstart = wbase + int64_t(lane) * S;
    MLane L;
    {
        int64_t lo = it.seg_lo - wstart, own = it.own_end - wstart;
        lo = lo < 0 ? 0 : (lo > S ? S : lo);
        own = own < 0 ? 0 : (own > S ? S : own);
        int64_t len = 0;
        if (own > lo) {
            len = own + maxm - 1;
            if (wstart + len > it.seg_end) len = it.seg_end - wstart;
        }
        L.lo = uint32_t(lo);
        L.own = uint32_t(own);
        L.len = uint32_t(len);
    }
    uint32_t q = 0;
    const uint32_t lane_off = uint32_t(lane / G::U) * uint32_t(S) + 16u * uint32_t(lane % G::U);
    const int rounds_all = int((S + maxm - 1 + LINE - 1) / LINE);
    const int64_t wlast = wbase + int64_t(kWave - 1) * S;
    // (one-step automata take the full-wave path where their entries are row offsets)
    const bool full = (PAIR || scaled) && wbase >= it.seg_lo && wlast + S <= it.own_end &&
                      wlast + S + maxm - 1 <= it.seg_end &&
                      wlast + int64_t(rounds_all) * LINE <= p.n;

    if (full) {
        walk_full<H, PAIR, LINE, NT>(p, xb, lane, wbase, wstart, S, lane_off, maxm, q, x, L, smem);
    } else if (__builtin_amdgcn_ballot_w64(L.own > L.lo) != 0) {
        // edge waves (the segment's first or last walks, or the text's end): one byte per
        // step, the rounds up to the longest walk of the wave; a wave none of whose walks
        // owns a byte (past the segment's end in a tile sized for the workgroup's waves)
        // has nothing to walk
        int need = int((L.len + uint32_t(LINE) - 1u) / uint32_t(LINE));
        for (int o = kWave / 2; o > 0; o >>= 1) need = max(need, __shfl_xor(need, o));
        const int rounds = __builtin_amdgcn_readfirstlane(min(need, rounds_all));
        v4u pf[1][G::U];
        fetch_round<1, LINE, true>(pf, p.text, p.n, wbase, S, lane_off, 0);
        for (int r = 0; r < rounds; ++r) {
            stage_round<1, LINE>(pf, xb, lane);
            if (r + 1 < rounds) fetch_round<1, LINE, true>(pf, p.text, p.n, wbase, S, lane_off, r + 1);
#pragma unroll
            for (int u = 0; u < G::U; ++u)
                mwalk16_guarded<PAIR>(unit_of<LINE>(xb, 0, lane, u), q, uint32_t(r * LINE + 16 * u), x, L, smem, p);
        }
    }

    // visit counters -> global, one atomic per nonzero counter
    __syncthreads();
    const uint32_t *hist = reinterpret_cast<const uint32_t *>(smem + x.hist);
    for (uint32_t i = threadIdx.x; i < nfin; i += blockDim.x) {
        const uint32_t v = hist[i];
        if (v) atomicAdd(p.visits + au.fin_base + i, (unsigned long long)v);
    }
}

__global__ void k_merged_zero(unsigned long long *counts, int64_t npairs, unsigned long long *visits, int64_t nfinal) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < npairs + nfinal; i += stride) {
        if (i < npairs)
            counts[i] = 0;
        else
            visits[i - npairs] = 0;
    }
}

// counts[pair] += visits of every reporting state that reports the pair's pattern
__global__ void k_visits_to_counts(const unsigned long long *visits, const int32_t *out_off, const OutEntry *out_ent,
                                   int64_t nfinal, unsigned long long *counts) {
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < nfinal;
         g += int64_t(gridDim.x) * blockDim.x) {
        const unsigned long long v = visits[g];
        if (!v) continue;
        for (int32_t e = out_off[g]; e < out_off[g + 1]; ++e) atomicAdd(counts + out_ent[e].pair, v);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

using dfa::hip_ok;

template <int LINE, bool NT>
const void *merged_fn_line(int H, bool pair) {
    if (H == 1) return pair ? reinterpret_cast<const void *>(&k_merged<1, true, LINE, NT>)
                            : reinterpret_cast<const void *>(&k_merged<1, false, LINE, NT>);
    return pair ? reinterpret_cast<const void *>(&k_merged<4, true, LINE, NT>)
                : reinterpret_cast<const void *>(&k_merged<4, false, LINE, NT>);
}

const void *merged_fn(int H, bool pair, int line, bool nt) {
    if (line == 64) return nt ? merged_fn_line<64, true>(H, pair) : merged_fn_line<64, false>(H, pair);
    return merged_fn_line<32, false>(H, pair);
}

struct MHostPlan {
    std::vector<MAuto> autos;
    std::vector<MItem> items;
    std::vector<int32_t> out_off{0};
    std::vector<OutEntry> out_ent;
    std::vector<uint8_t> area;  // tables and class maps
    int waves = 0;  // waves per workgroup (0: the plan chooses)
    int line = 0;  // bytes of every walk staged per round (0: the plan chooses)
    bool nt = false;  // whole-line non-temporal fetches (64-byte rounds, no tile shared by automata)
    int H = 1;
    int lds = 0;  // dynamic LDS of the largest launch
    // launch groups (pair automata, then one-step automata, each by the
    // workgroups per CU their LDS leaves room for: 4 or more, 3, 2, 1): items
    // and LDS of each
    int64_t group_items[DFA_MERGED_GROUPS] = {};
    int group_lds[DFA_MERGED_GROUPS] = {};
    int64_t text_bytes = 0;
    int64_t nstates = 0;
    int64_t ncounts = 0;
    const int32_t *pair_dst = nullptr;  // counter of each pair (null: the pair itself)
    bool allow_pair = true;             // pair automata where they fit the budget
    bool pack_pairs = false;            // pack patterns so that automata fit the budget as pair automata
    int budget = kDefaultAutomatonBytes;
};

// Pair automata: at most kPairMaxCls byte classes (a state's row of ncls^2
// entries grows fast; the weight 2 ncls of a pair's column sum is a byte),
// states below 2^15, every image offset below 64 KiB (the 16-bit class map
// holds the one-step table's offset).
constexpr int kPairMaxCls = 11;

int64_t auto_lds_bytes(const MAuto &a) {
    return a.image_bytes + dfa::round_up(int64_t(a.nstates - a.first_final) * 4, 16);
}

// LDS is handed to workgroups in blocks; counted in whole kLdsBlock units so
// that a third of the CU's LDS really fits three workgroups.
constexpr int64_t kLdsBlock = 2048;

// Workgroups that fit a CU when each needs `need` bytes of LDS (by LDS, and
// by registers: kWavesPerSimd per SIMD, 4 SIMDs per CU).
int64_t groups_for(int64_t need, int waves) {
    const int64_t by_lds = kLdsPerCu / dfa::round_up(need, kLdsBlock);
    return std::max<int64_t>(1, std::min<int64_t>(by_lds, 4 * kWavesPerSimd / waves));
}

// LDS of one wave's transpose buffer: a round of each of its 64 walks
int64_t stage_bytes_per_wave(int line) { return int64_t(kWave) * line; }

// ... with an automaton of `bytes` plus one transpose buffer per wave
int64_t groups_per_cu(int64_t bytes, int waves, int line) {
    return groups_for(bytes + int64_t(waves) * stage_bytes_per_wave(line), waves);
}

// Register classes of an automaton (the device side's reg_classes), each
// slot holding factor x its byte's class (2 c, the column's byte offset, for
// one-step automata; c for pair automata): the first shift s that gives its
// pattern bytes distinct slots, preferring one where 'N' (an assembly gap, of
// the default class unless a pattern holds it) gets a slot of its own; else
// keys that no byte matches.
void set_reg_classes(const dfa::AcAutomaton &a, int factor, MAuto &m) {
    std::vector<int> pb;
    for (int b = 0; b < 256; ++b)
        if (a.cls[b]) pb.push_back(b);
    auto slot = [](int b, int s) { return (b >> s) & 7; };
    int shift = -1;
    for (int pass = 0; pass < 2 && shift < 0 && pb.size() <= 8; ++pass)
        for (int s = 0; s <= 5 && shift < 0; ++s) {
            unsigned seen = 0;
            bool ok = true;
            for (int b : pb) {
                ok = ok && !((seen >> slot(b, s)) & 1u);
                seen |= 1u << slot(b, s);
            }
            if (ok && (pass == 1 || a.cls['N'] || !((seen >> slot('N', s)) & 1u))) shift = s;
        }
    uint8_t lut[8] = {}, key[8] = {};
    if (shift < 0) {
        m.cls_shift = 0;
        for (int h = 0; h < 8; ++h) key[h] = uint8_t((h + 1) & 7);  // slot of key[h] is not h: never equal
    } else {
        m.cls_shift = shift;
        bool used[8] = {};
        for (int b : pb) {
            key[slot(b, shift)] = uint8_t(b);
            lut[slot(b, shift)] = uint8_t(factor * a.cls[b]);
            used[slot(b, shift)] = true;
        }
        for (int h = 0; h < 8; ++h) {
            if (used[h]) continue;
            int pick = -1;
            for (int b : {int('N'), int('n')})
                if (pick < 0 && slot(b, shift) == h && !a.cls[b]) pick = b;
            for (int b = 0; b < 256 && pick < 0; ++b)
                if (slot(b, shift) == h && !a.cls[b]) pick = b;
            key[h] = uint8_t(pick);  // a default-class byte: c = 0
        }
    }
    auto pack = [](const uint8_t *v) {
        return uint32_t(v[0]) | uint32_t(v[1]) << 8 | uint32_t(v[2]) << 16 | uint32_t(v[3]) << 24;
    };
    m.lut_lo = pack(lut);
    m.lut_hi = pack(lut + 4);
    m.key_lo = pack(key);
    m.key_hi = pack(key + 4);
}

int add_automaton(const std::vector<int64_t> &ks, const int32_t *pair_pat, const uint8_t *patterns,
                  const int64_t *pat_off, const int32_t *pat_len, MHostPlan &hp) {
    std::vector<const uint8_t *> pats;
    std::vector<int32_t> lens;
    int maxm = 0;
    for (int64_t k : ks) {
        const int32_t j = pair_pat[k];
        pats.push_back(patterns + pat_off[j]);
        lens.push_back(pat_len[j]);
        maxm = std::max(maxm, int(pat_len[j]));
    }
    dfa::AcAutomaton a;
    if (!dfa::ac_build(pats, lens, DFA_AC_MAX_STATES, a)) {
        dfa::set_error("dfa_merged: an automaton would need more than %d states", DFA_AC_MAX_STATES);
        return DFA_EINVAL;
    }
    MAuto m{};
    m.nstates = a.nstates;
    m.first_final = a.first_final;
    m.ncls = a.ncls;
    m.maxm = maxm;
    m.table_off = int64_t(hp.area.size());
    m.fin_base = int64_t(hp.out_off.size()) - 1;
    const int64_t ns = a.nstates, nc = a.ncls;
    const int64_t one = dfa::round_up(ns * nc * 2, 16);      // one-step table
    const int64_t pairs = dfa::round_up(ns * nc * nc * 2, 16);  // pair table
    const int64_t hist = dfa::round_up((ns - a.first_final) * 4, 16);
    const int64_t pair_image = int64_t(kPairMaps) + pairs + one + kCmapBytes;
    const bool pair_ok = hp.allow_pair && nc <= kPairMaxCls && ns < int64_t(kMidReports) &&
                         pair_image + hist <= hp.budget && pair_image <= 65536;
    // A pair automaton halves the dependent table reads per byte of a full
    // wave's rounds, but at the occupancy the one-step kernel reaches (8 waves
    // per SIMD, classes from registers) it was slower everywhere measured:
    // 2000 segments of 1 kB - 250 MB with 1-16 patterns of 6-48 bytes, 0.56
    // ms against 0.45 ms one-step; 72 8-mers over 1 GB, 0.32 against 0.30 ms.
    // Taken only when the plan asks for two bytes per step.
    m.pair = pair_ok && hp.pack_pairs;
    set_reg_classes(a, m.pair ? 1 : 2, m);
    // one-step entries as row offsets where they fit 16 bits and 2 c a byte
    m.scaled = (ns * 2 * nc <= 65536 && nc <= 128) ? 1 : 0;
    m.magic = uint32_t(((uint64_t(1) << 32) + uint64_t(2 * nc) - 1) / uint64_t(2 * nc));
    const int64_t tab1 = m.pair ? int64_t(kPairMaps) + pairs : 0;  // LDS offset of the one-step table
    m.cmap_off = int32_t(tab1 + one);
    m.image_bytes = int32_t(tab1 + one + kCmapBytes);
    hp.area.resize(hp.area.size() + size_t(m.image_bytes), 0);
    uint8_t *img = hp.area.data() + m.table_off;
    uint16_t *tab = reinterpret_cast<uint16_t *>(img + tab1);
    for (size_t i = 0; i < a.next.size(); ++i) tab[i] = uint16_t(m.scaled ? a.next[i] * 2 * nc : a.next[i]);
    uint16_t *cm = reinterpret_cast<uint16_t *>(img + m.cmap_off);
    for (int b = 0; b < 256; ++b) cm[b] = uint16_t(tab1 + 2 * a.cls[b]);
    if (m.pair) {
        // byte map: c; entry (q, c1 c2) = the state after both bytes, bit 15
        // if the one after c1 reports
        for (int b = 0; b < 256; ++b) img[b] = uint8_t(a.cls[b]);
        uint16_t *pt = reinterpret_cast<uint16_t *>(img + kPairMaps);
        for (int64_t q = 0; q < ns; ++q)
            for (int64_t c1 = 0; c1 < nc; ++c1) {
                const int32_t mid = a.next[size_t(q * nc + c1)];
                for (int64_t c2 = 0; c2 < nc; ++c2) {
                    const int32_t end = a.next[size_t(int64_t(mid) * nc + c2)];
                    pt[q * nc * nc + c1 * nc + c2] =
                        uint16_t(end | (mid >= a.first_final ? int32_t(kMidReports) : 0));
                }
            }
    }
    for (int32_t f = 0; f < a.nstates - a.first_final; ++f) {
        for (int32_t e = a.out_off[size_t(f)]; e < a.out_off[size_t(f) + 1]; ++e) {
            const int64_t k = ks[size_t(a.out_pat[size_t(e)])];
            const int32_t dst = hp.pair_dst ? hp.pair_dst[k] : int32_t(k);
            hp.out_ent.push_back(OutEntry{dst, pat_len[pair_pat[k]]});
        }
        if (hp.out_ent.size() > size_t(0x7fffffff)) {
            dfa::set_error("dfa_merged: too many output entries");
            return DFA_EINVAL;
        }
        hp.out_off.push_back(int32_t(hp.out_ent.size()));
    }
    hp.nstates += a.nstates;
    hp.autos.push_back(m);
    return DFA_OK;
}

int plan_merged(const int64_t *seg_off, int32_t nseg, const uint8_t *patterns, const int64_t *pat_off,
                const int32_t *pat_len, int32_t npat, const int32_t *pair_seg, const int32_t *pair_pat, int64_t npairs,
                const int32_t *pair_dst, int64_t ncounts, const dfa_tune *t, MHostPlan &hp) {
    if (!pair_dst) {
        if (ncounts != 0 && ncounts != npairs) {
            dfa::set_error("dfa_merged: without pair_dst, ncounts must be 0 or npairs");
            return DFA_EINVAL;
        }
        ncounts = npairs;
    }
    if (ncounts < 0 || ncounts > 0x7fffffff) {
        dfa::set_error("dfa_merged: ncounts=%lld out of range", (long long)ncounts);
        return DFA_EINVAL;
    }
    for (int64_t k = 0; pair_dst && k < npairs; ++k)
        if (pair_dst[k] < 0 || pair_dst[k] >= ncounts) {
            dfa::set_error("dfa_merged: pair_dst[%lld]=%d outside [0, %lld)", (long long)k, pair_dst[k],
                           (long long)ncounts);
            return DFA_EINVAL;
        }
    hp.ncounts = ncounts;
    hp.pair_dst = pair_dst;
    if (nseg < 0 || npat < 0 || npairs < 0 || (nseg > 0 && !seg_off) ||
        (npat > 0 && (!patterns || !pat_off || !pat_len)) || (npairs > 0 && (!pair_seg || !pair_pat))) {
        dfa::set_error("dfa_merged: bad counts or null arrays");
        return DFA_EINVAL;
    }
    int budget = kDefaultAutomatonBytes;
    int64_t fixed_span = 0;
    if (t) {
        for (int i = 0; i < 2; ++i)
            if (t->reserved[i]) {
                dfa::set_error("tune.reserved must be zero");
                return DFA_EINVAL;
            }
        if (t->step_bytes < 0 || t->step_bytes > 2) {
            dfa::set_error("tune.step_bytes=%d must be 1 or 2 (or 0)", t->step_bytes);
            return DFA_EINVAL;
        }
        if (t->line_bytes != 0 && t->line_bytes != 32 && t->line_bytes != 64) {
            dfa::set_error("tune.line_bytes=%d: merged scans take 32 or 64 (or 0)", t->line_bytes);
            return DFA_EINVAL;
        }
        if (t->line_bytes) hp.line = t->line_bytes;
        if (t->step_bytes == 1) hp.allow_pair = false;
        if (t->step_bytes == 2) hp.pack_pairs = true;
        if (t->waves_per_group < 0 || t->waves_per_group > kMaxWaves) {
            dfa::set_error("tune.waves_per_group=%d outside [1, %d]", t->waves_per_group, kMaxWaves);
            return DFA_EINVAL;
        }
        if (t->chain_bytes < 0 || t->chain_bytes % 128 || t->chain_bytes > (1 << 20)) {
            dfa::set_error("tune.chain_bytes=%lld: merged scans take a multiple of 128 up to 2^20 (or 0)",
                           (long long)t->chain_bytes);
            return DFA_EINVAL;
        }
        if (t->automaton_bytes < 0 || (t->automaton_bytes && t->automaton_bytes < kMinAutomatonBytes)) {
            dfa::set_error("tune.automaton_bytes=%d below %d", t->automaton_bytes, kMinAutomatonBytes);
            return DFA_EINVAL;
        }
        if (t->waves_per_group) hp.waves = t->waves_per_group;
        if (t->automaton_bytes) budget = t->automaton_bytes;
        hp.budget = budget;
        fixed_span = t->chain_bytes;
    }
    for (int32_t s = 0; s < nseg; ++s)
        if (seg_off[s + 1] < seg_off[s] || seg_off[s] < 0) {
            dfa::set_error("dfa_merged: seg_off must be nondecreasing and >= 0");
            return DFA_EINVAL;
        }
    hp.text_bytes = nseg > 0 ? seg_off[nseg] : 0;
    for (int32_t j = 0; j < npat; ++j)
        if (pat_len[j] < 1 || pat_len[j] > DFA_MAX_M || pat_off[j] < 0) {
            dfa::set_error("dfa_merged: pattern %d has length %d (1..%d) or offset %lld", j, pat_len[j], DFA_MAX_M,
                           (long long)pat_off[j]);
            return DFA_EINVAL;
        }
    std::vector<std::vector<int64_t>> by_seg(size_t(std::max(nseg, 0)));
    for (int64_t k = 0; k < npairs; ++k) {
        if (pair_seg[k] < 0 || pair_seg[k] >= nseg || pair_pat[k] < 0 || pair_pat[k] >= npat) {
            dfa::set_error("dfa_merged: pair %lld refers to segment %d / pattern %d out of range", (long long)k,
                           pair_seg[k], pair_pat[k]);
            return DFA_EINVAL;
        }
        by_seg[size_t(pair_seg[k])].push_back(k);
    }
    std::vector<int32_t> order;
    for (int32_t s = 0; s < nseg; ++s)
        if (!by_seg[size_t(s)].empty() && seg_off[s + 1] > seg_off[s]) order.push_back(s);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return seg_off[a + 1] - seg_off[a] > seg_off[b + 1] - seg_off[b];
    });
    // Patterns of at most kHotLen bytes first (they match often: on DNA a
    // 4-mer every 256 bytes), then by bytes so that neighbours share trie
    // prefixes.  A segment split over several automata then has its frequent
    // visits in one of them: an automaton's visit counters take one LDS
    // atomic per byte position where any lane of a wave reports, so hits
    // spread over every automaton cost each of them nearly one per position.
    constexpr int32_t kHotLen = 6;
    auto pat_less = [&](int64_t a, int64_t b) {
        const int32_t ja = pair_pat[a], jb = pair_pat[b];
        const bool ha = pat_len[ja] <= kHotLen, hb = pat_len[jb] <= kHotLen;
        if (ha != hb) return ha;
        const int32_t n = std::min(pat_len[ja], pat_len[jb]);
        const int c = std::memcmp(patterns + pat_off[ja], patterns + pat_off[jb], size_t(n));
        return c ? c < 0 : pat_len[ja] < pat_len[jb];
    };
    // pass 1: the automata of every segment
    int maxm_all = 1;
    std::vector<std::pair<size_t, size_t>> seg_autos;  // [first, end) automata of order[i]
    for (int32_t s : order) {
        // this segment's pairs in that order
        std::vector<int64_t> ks = by_seg[size_t(s)];
        std::stable_sort(ks.begin(), ks.end(), pat_less);
        bool used[256] = {};
        for (int64_t k : ks) {
            const int32_t j = pair_pat[k];
            for (int32_t i = 0; i < pat_len[j]; ++i) used[patterns[pat_off[j] + i]] = true;
        }
        int ncls = 1;
        for (int b = 0; b < 256; ++b) ncls += used[b];
        // add patterns while the trie (counted incrementally from the common
        // prefix with the previous pattern) fits the budget
        // LDS per state: one-step table row and visit counter, and with pair
        // packing the pair table row too (plus the byte map per automaton);
        // a pair automaton's image (without its counters) stays below 64 KiB
        const bool pp = hp.pack_pairs && ncls <= kPairMaxCls;
        const int64_t per_state = 2 * ncls + 4 + (pp ? 2 * ncls * ncls : 0);
        const int64_t fixed = kCmapBytes + (pp ? int64_t(kPairMaps) : 0);
        const int64_t pack_budget = pp ? std::min<int64_t>(budget, (65536 - 32 - fixed) / (per_state - 4) *
                                                                       per_state + fixed)
                                       : budget;
        // one-step entries stay row offsets (16 bits) while the table is at most 64 KiB
        const int64_t max_states = ncls <= 128 ? 65536 / (2 * ncls) : int64_t(DFA_AC_MAX_STATES);
        const size_t a_first = hp.autos.size();
        std::vector<int64_t> cur;
        int64_t states = 1;
        for (int64_t k : ks) {
            const int32_t j = pair_pat[k];
            maxm_all = std::max(maxm_all, int(pat_len[j]));
            int32_t common = 0;
            if (!cur.empty()) {
                const int32_t jp = pair_pat[cur.back()];
                const int32_t n = std::min(pat_len[j], pat_len[jp]);
                while (common < n && patterns[pat_off[j] + common] == patterns[pat_off[jp] + common]) ++common;
            }
            const int64_t add = pat_len[j] - common;
            if (!cur.empty() && ((states + add) * per_state + fixed > pack_budget ||
                                 states + add > DFA_AC_MAX_STATES || states + add > max_states)) {
                const int rc = add_automaton(cur, pair_pat, patterns, pat_off, pat_len, hp);
                if (rc != DFA_OK) return rc;
                cur.clear();
                states = 1;
            }
            states += cur.empty() ? pat_len[j] : add;
            cur.push_back(k);
        }
        if (!cur.empty()) {
            const int rc = add_automaton(cur, pair_pat, patterns, pat_off, pat_len, hp);
            if (rc != DFA_OK) return rc;
        }
        seg_autos.emplace_back(a_first, hp.autos.size());
    }
    hp.H = maxm_all <= 17 ? 1 : 4;
    int64_t auto_max = 0;
    for (const MAuto &a : hp.autos) auto_max = std::max(auto_max, auto_lds_bytes(a));
    if (!hp.line || !hp.waves) {
        // The scan is bound by the latency of its dependent table reads, so the
        // shape is chosen for resident waves per CU, weighting each automaton
        // by the bytes it walks: 64-byte rounds (whole halves of a line per
        // load: the faster reads) unless 32-byte rounds, whose transpose
        // buffers take half the LDS, fit more; 8 waves per workgroup unless 16,
        // which share one copy of the automaton among twice the waves, fit
        // more.  (1 GB x 1024 patterns in 48 KiB automata: 2.5 ms with 32-byte
        // rounds and 3 workgroups of 8 waves per CU against 3.3 ms with 64 and
        // 2.)
        double best = -1;
        int best_line = 64, best_waves = 8;
        for (int line : {64, 32})
            for (int waves : {8, 16}) {
                if ((hp.line && line != hp.line) || (hp.waves && waves != hp.waves)) continue;
                if (auto_max + int64_t(waves) * stage_bytes_per_wave(line) > kLdsPerCu) continue;
                double occ = 0;
                for (size_t oi = 0; oi < order.size(); ++oi) {
                    const double len = double(seg_off[order[oi] + 1] - seg_off[order[oi]]);
                    for (size_t a = seg_autos[oi].first; a < seg_autos[oi].second; ++a)
                        occ += len * double(waves * groups_per_cu(auto_lds_bytes(hp.autos[a]), waves, line));
                }
                if (occ > best) {
                    best = occ;
                    best_line = line;
                    best_waves = waves;
                }
            }
        if (!hp.line) hp.line = best_line;
        if (!hp.waves) hp.waves = best_waves;
    }
    // whole-line non-temporal fetches where every segment has one automaton:
    // 2000 segments 0.426 -> 0.410 ms, 72 8-mers over 1 GB 0.286 -> 0.282 ms
    hp.nt = hp.line == 64;
    for (size_t oi = 0; oi < order.size(); ++oi)
        if (seg_autos[oi].second - seg_autos[oi].first > 1) hp.nt = false;
    // fewer waves per workgroup if the largest automaton leaves too little room
    const int64_t per_wave = stage_bytes_per_wave(hp.line);
    while (hp.waves > 1 && auto_max + int64_t(hp.waves) * per_wave > kLdsPerCu) --hp.waves;
    if (auto_max + int64_t(hp.waves) * per_wave > kLdsPerCu) {
        dfa::set_error("dfa_merged: an automaton needs %lld bytes of LDS", (long long)auto_max);
        return DFA_EINVAL;
    }
    // pass 2: work items, (tile, automaton), on the 128-byte grid of the text;
    // short segments get short spans, long ones at most kMaxSpan (kMaxSpanOne
    // when one automaton walks the segment)
    const int64_t walks_per_tile = int64_t(hp.waves) * kWave;
    for (size_t oi = 0; oi < order.size(); ++oi) {
        const int32_t s = order[oi];
        const int64_t lo = seg_off[s], hi = seg_off[s + 1];
        const int64_t a_first = int64_t(seg_autos[oi].first);
        const int64_t na = int64_t(seg_autos[oi].second) - a_first;
        const int64_t base = lo & ~int64_t(127);
        const int64_t len = hi - base;
        int64_t S = fixed_span;
        if (!S) {
            S = dfa::round_up(dfa::ceil_div(len, walks_per_tile), 128);
            S = std::min(std::max(S, kMinSpan), na > 1 ? kMaxSpan : kMaxSpanOne);
        }
        const int64_t tile = S * walks_per_tile;
        const int64_t ntiles = dfa::ceil_div(len, tile);
        for (int64_t tb = 0; tb < ntiles; tb += kXcds) {
            const int64_t nt = std::min<int64_t>(kXcds, ntiles - tb);
            for (int64_t a = 0; a < na; ++a)
                for (int64_t ti = 0; ti < nt; ++ti) {
                    MItem it{};
                    it.tile_start = base + (tb + ti) * tile;
                    it.seg_lo = lo;
                    it.own_end = std::min(hi, it.tile_start + tile);
                    it.seg_end = hi;
                    it.automaton = int32_t(a_first + a);
                    it.span = int32_t(S);
                    hp.items.push_back(it);
                }
        }
    }
    if (hp.items.size() > size_t(0x7fffffff)) {
        dfa::set_error("dfa_merged: too many work items");
        return DFA_EINVAL;
    }
    // launch groups, each with the LDS its largest automaton needs: pair
    // automata by how many workgroups per CU they leave room for (4 or more,
    // 3, 2, 1), then the one-step ones the same way; items keep their order
    // inside a group
    const int64_t staging = int64_t(hp.waves) * per_wave;
    auto group_of = [&](const MItem &it) {
        const MAuto &a = hp.autos[size_t(it.automaton)];
        const int64_t g = groups_for(auto_lds_bytes(a) + staging, hp.waves);
        return (a.pair ? 0 : DFA_MERGED_GROUPS / 2) + (g >= 4 ? 0 : 4 - int(g));
    };
    std::stable_sort(hp.items.begin(), hp.items.end(),
                     [&](const MItem &x, const MItem &y) { return group_of(x) < group_of(y); });
    for (const MItem &it : hp.items) {
        const int g = group_of(it);
        hp.group_items[g] += 1;
        hp.group_lds[g] = std::max(hp.group_lds[g], int(auto_lds_bytes(hp.autos[size_t(it.automaton)]) + staging));
    }
    hp.lds = int(auto_max + staging);
    return DFA_OK;
}

struct WsLayout {
    int64_t autos = 0, items = 0, out_off = 0, out_ent = 0, visits = 0, area = 0, total = 0;
};

WsLayout ws_layout(const MHostPlan &hp) {
    WsLayout L;
    const int64_t nfin = int64_t(hp.out_off.size()) - 1;
    L.autos = 0;
    L.items = L.autos + dfa::round_up(int64_t(hp.autos.size() * sizeof(MAuto)), 256);
    L.out_off = L.items + dfa::round_up(int64_t(hp.items.size() * sizeof(MItem)), 256);
    L.out_ent = L.out_off + dfa::round_up(int64_t(hp.out_off.size() * sizeof(int32_t)), 256);
    L.visits = L.out_ent + dfa::round_up(int64_t(hp.out_ent.size() * sizeof(OutEntry)), 256);
    L.area = L.visits + dfa::round_up(nfin * 8, 256);
    L.total = L.area + dfa::round_up(int64_t(hp.area.size()), 256);
    return L;
}

}  // namespace

extern "C" int dfa_merged_prepare(const int64_t *seg_off, int32_t nseg, const uint8_t *patterns,
                                  const int64_t *pat_off, const int32_t *pat_len, int32_t npat,
                                  const int32_t *pair_seg, const int32_t *pair_pat, int64_t npairs,
                                  const int32_t *pair_dst, int64_t ncounts, void *workspace,
                                  int64_t workspace_bytes, const dfa_tune *tune, dfa_merged_plan *plan,
                                  void *stream) {
    if (!plan) {
        dfa::set_error("dfa_merged_prepare: null plan");
        return DFA_EINVAL;
    }
    MHostPlan hp;
    int rc = plan_merged(seg_off, nseg, patterns, pat_off, pat_len, npat, pair_seg, pair_pat, npairs, pair_dst,
                         ncounts, tune, hp);
    if (rc != DFA_OK) return rc;
    // the automata's table offsets are relative to the area: make them workspace offsets
    const WsLayout L = ws_layout(hp);
    for (MAuto &a : hp.autos) a.table_off += L.area;
    std::memset(plan, 0, sizeof(*plan));
    plan->nitems = int64_t(hp.items.size());
    plan->nautomata = int64_t(hp.autos.size());
    plan->nstates = hp.nstates;
    plan->nfinal = int64_t(hp.out_off.size()) - 1;
    plan->npairs = npairs;
    plan->ncounts = hp.ncounts;
    plan->text_bytes = hp.text_bytes;
    plan->workspace_bytes = L.total;
    plan->items_offset = L.items;
    plan->outputs_offset = L.out_off;
    plan->entries_offset = L.out_ent;
    plan->visits_offset = L.visits;
    plan->waves_per_group = hp.waves;
    plan->lds_bytes = hp.lds;
    plan->reserved[0] = hp.H;
    plan->reserved[1] = hp.line;
    plan->reserved[2] = hp.nt ? 1 : 0;
    for (int g = 0; g < DFA_MERGED_GROUPS; ++g) {
        plan->group_items[g] = hp.group_items[g];
        plan->group_lds[g] = hp.group_lds[g];
        plan->group_pair[g] = g < DFA_MERGED_GROUPS / 2 ? 1 : 0;
    }
    if (!workspace) {
        dfa::clear_error();
        return DFA_OK;  // size query
    }
    if (workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        dfa::set_error("dfa_merged_prepare: workspace of %lld bytes (256-aligned) needed, got %lld",
                       (long long)L.total, (long long)workspace_bytes);
        return DFA_ENOSPACE;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = reinterpret_cast<uint8_t *>(workspace);
    struct Part {
        int64_t off;
        const void *src;
        size_t bytes;
    } parts[] = {
        {L.autos, hp.autos.data(), hp.autos.size() * sizeof(MAuto)},
        {L.items, hp.items.data(), hp.items.size() * sizeof(MItem)},
        {L.out_off, hp.out_off.data(), hp.out_off.size() * sizeof(int32_t)},
        {L.out_ent, hp.out_ent.data(), hp.out_ent.size() * sizeof(OutEntry)},
        {L.area, hp.area.data(), hp.area.size()},
    };
    for (const Part &pt : parts)
        if (pt.bytes && !hip_ok(hipMemcpyAsync(ws + pt.off, pt.src, pt.bytes, hipMemcpyHostToDevice, st),
                                "merged plan upload"))
            return DFA_EHIP;
    // the host arrays are freed on return: make sure the copies are done
    if (!hip_ok(hipStreamSynchronize(st), "merged plan upload")) return DFA_EHIP;
    dfa::clear_error();
    return DFA_OK;
}

extern "C" int dfa_merged_run(const uint8_t *text, int64_t n, void *workspace, const dfa_merged_plan *plan,
                              int64_t *counts, void *stream) {
    if (!plan || n < 0 || (!text && n > 0) || (plan->ncounts > 0 && !counts) || (plan->nitems > 0 && !workspace)) {
        dfa::set_error("dfa_merged_run: null argument or n < 0");
        return DFA_EINVAL;
    }
    if (plan->text_bytes > n) {
        dfa::set_error("dfa_merged_run: segments span %lld bytes, text has %lld", (long long)plan->text_bytes,
                       (long long)n);
        return DFA_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(text) & 15) || (reinterpret_cast<uintptr_t>(counts) & 7) ||
        (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        dfa::set_error("dfa_merged_run: text must be 16-byte, counts 8-byte, workspace 256-byte aligned");
        return DFA_EINVAL;
    }
    const int H = plan->reserved[0];
    const int line = plan->reserved[1];
    const int nt = plan->reserved[2];
    int64_t grouped = 0;
    bool groups_ok = true;
    for (int g = 0; g < DFA_MERGED_GROUPS; ++g) {
        groups_ok &= plan->group_items[g] >= 0 && plan->group_lds[g] >= 0 && plan->group_lds[g] <= kLdsPerCu;
        grouped += plan->group_items[g];
    }
    if ((H != 1 && H != 4) || (line != 32 && line != 64) || (nt != 0 && nt != 1) || (nt && line != 64) ||
        plan->waves_per_group < 1 || plan->waves_per_group > kMaxWaves || plan->lds_bytes < 0 ||
        plan->lds_bytes > kLdsPerCu || !groups_ok || grouped != plan->nitems) {
        dfa::set_error("dfa_merged_run: plan not made by dfa_merged_prepare");
        return DFA_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = reinterpret_cast<uint8_t *>(workspace);
    unsigned long long *visits = reinterpret_cast<unsigned long long *>(ws + plan->visits_offset);
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(counts);
    if (plan->ncounts + plan->nfinal > 0) {
        const int64_t want = dfa::ceil_div(plan->ncounts + plan->nfinal, 256);
        hipLaunchKernelGGL(k_merged_zero, dim3(unsigned(std::min<int64_t>(want, 4096))), dim3(256), 0, st, cnt,
                           plan->ncounts, visits, plan->nfinal);
        if (!hip_ok(hipGetLastError(), "k_merged_zero launch")) return DFA_EHIP;
    }
    if (plan->nitems == 0) {
        dfa::clear_error();
        return DFA_OK;
    }
    MParams mp{};
    mp.text = text;
    mp.n = n;
    mp.ws = ws;
    mp.autos = reinterpret_cast<const MAuto *>(ws);
    mp.items = reinterpret_cast<const MItem *>(ws + plan->items_offset);
    mp.out_off = reinterpret_cast<const int32_t *>(ws + plan->outputs_offset);
    mp.out_ent = reinterpret_cast<const OutEntry *>(ws + plan->entries_offset);
    mp.visits = visits;
    mp.counts = cnt;
    // one launch per group of items
    for (int64_t g = 0, first = 0; g < DFA_MERGED_GROUPS; first += plan->group_items[g], ++g) {
        const int64_t count = plan->group_items[g];
        if (count == 0) continue;
        const void *fn = merged_fn(H, plan->group_pair[g] != 0, line, nt != 0);
        if (!dfa::allow_lds(fn, kLdsPerCu)) return DFA_EHIP;
        MParams kp = mp;
        kp.items = mp.items + first;
        void *args[] = {&kp};
        if (!hip_ok(hipLaunchKernel(fn, dim3(unsigned(count)), dim3(plan->waves_per_group * kWave), args,
                                    size_t(plan->group_lds[g]), st),
                    "k_merged launch"))
            return DFA_EHIP;
    }
    if (plan->nfinal > 0) {
        const int64_t want = dfa::ceil_div(plan->nfinal, 256);
        hipLaunchKernelGGL(k_visits_to_counts, dim3(unsigned(std::min<int64_t>(want, 4096))), dim3(256), 0, st, visits,
                           mp.out_off, mp.out_ent, plan->nfinal, cnt);
        if (!hip_ok(hipGetLastError(), "k_visits_to_counts launch")) return DFA_EHIP;
    }
    dfa::clear_error();
    return DFA_OK;
}
