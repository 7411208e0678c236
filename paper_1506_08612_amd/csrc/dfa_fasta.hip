// FASTA normalisation on the device (gfx950).
//
// The paper's inputs are GenBank genomes (Table 1): FASTA text whose records
// start with a header line ('>' first), whose sequence is wrapped over lines,
// and whose lower-case letters mark soft-masked regions.  The scan wants one
// plain byte string per record.  Rule: a line whose first byte is '>' is a
// header -- it starts a record and none of its bytes are kept; every other
// byte is kept except '\n' and '\r', with 'a'..'z' made upper case; record k
// starts where the kept bytes stood when its header was read.
//
// Whether a byte is kept depends on the first byte of its line, which may lie
// far back, so the text is cut into 32 KiB units, one per wave, and processed
// in three steps:
//   A  per unit: its last line start (with whether that line is a header),
//      its header count, and its kept bytes -- those before its first line
//      start counted apart, as their line began in an earlier unit;
//   B  the unit summaries combined in text order by an associative operator
//      (one kernel for the totals of blocks of 2048 units, one for each
//      block's prefix and its units' own): the line each unit starts in, its
//      output offset and its first record index;
//   C  per unit again: the kept bytes written, compacted, at their offsets,
//      and the record starts.
// A wave takes 1 KiB per round, 16 bytes per lane (one 16-byte load;
// consecutive lanes read consecutive pieces), with the next two rounds'
// loads in flight.  A line start s is held as 2 s + (byte s is '>'), relative
// to the unit, so that one wave-wide prefix max per round gives every byte
// both where its line began and whether that line is a header; in C one
// wave-wide prefix sum gives the lanes' output offsets.  The scans are DPP
// row shifts and row broadcasts, so the waves of a workgroup never wait for
// each other.  C stages a round's kept bytes in a per-wave LDS ring indexed
// by output address and stores whole aligned 16-byte blocks; the partial
// blocks at a unit's two ends, shared with the neighbouring units, are
// stored byte by byte.  C's text loads and block stores are non-temporal:
// each byte is read or written once.  A round in which no byte below 0x40
// but '\n' occurs (no header can start in it, no '\r' is dropped: almost
// every round of a genome) takes a short path in A and C: its line starts
// come from the newlines alone and carry no header flag, so one ballot of
// the lanes holding a line start replaces the wave-wide prefix max, and only
// a header line left open by an earlier round can drop bytes.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "dfa.h"
#include "dfa_internal.h"
#include "launch_util.h"

namespace {

constexpr int kWaveSize = 64;
constexpr int kWaves = 4;                       // waves (units) per workgroup in A and C
constexpr int kThreads = kWaves * kWaveSize;
constexpr int kPer = 16;                        // bytes per lane per round
constexpr int kRound = kWaveSize * kPer;        // bytes per wave per round
constexpr int64_t kUnit = 32 * 1024;            // bytes per wave
constexpr int kRing = 4096;                     // LDS staging ring per wave in C
constexpr int kPlanThreads = 256;
constexpr int kPlanPer = 8;                     // units per thread in B
constexpr int64_t kPlanUnits = int64_t(kPlanThreads) * kPlanPer;
constexpr int32_t kNone = INT32_MIN;            // no line start seen

static_assert(kUnit % kRound == 0, "a unit is whole rounds");
static_assert(kRing >= 2 * kRound + 2 * kPer, "the ring holds a round and the unstored tail");

struct UnitSummary {
    int64_t last_ls;     // last line start in the unit, as 2 s + header, or -1
    uint32_t pre;        // bytes before its first line start that a sequence line would keep
    uint32_t kept;       // kept bytes from its first line start on
    uint32_t headers;    // header lines starting in the unit
    uint32_t pad;
};

// A run of text summarised as a UnitSummary, with 64-bit counts.
struct Agg {
    int64_t ls;
    unsigned long long pre, kept, hdr;
};

struct UnitPlan {
    int64_t ls_before;   // last line start before the unit (2 s + header), or -1
    int64_t out_off;     // kept bytes before the unit
    int64_t rec_off;     // records before the unit
};

constexpr uint32_t kNl = '\n', kCr = '\r', kGt = '>';

// ---- wave-wide scans (DPP: row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143, wave_shr:1 = 0x138; lanes without a source keep `old`)

constexpr int kRowShr = 0x110, kBcast15 = 0x142, kBcast31 = 0x143, kWaveShr1 = 0x138;

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int32_t dpp_i32(int32_t old, int32_t v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROW_MASK, 0xf, false);
}

// inclusive prefix max over the wave's 64 lanes (all lanes active)
__device__ __forceinline__ int32_t wave_incl_max(int32_t v) {
    v = max(v, dpp_i32<kRowShr + 1, 0xf>(kNone, v));
    v = max(v, dpp_i32<kRowShr + 2, 0xf>(kNone, v));
    v = max(v, dpp_i32<kRowShr + 4, 0xf>(kNone, v));
    v = max(v, dpp_i32<kRowShr + 8, 0xf>(kNone, v));
    v = max(v, dpp_i32<kBcast15, 0xa>(kNone, v));
    v = max(v, dpp_i32<kBcast31, 0xc>(kNone, v));
    return v;
}

// inclusive prefix sum over the wave's 64 lanes (all lanes active)
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    int32_t v = int32_t(x);
    v += dpp_i32<kRowShr + 1, 0xf>(0, v);
    v += dpp_i32<kRowShr + 2, 0xf>(0, v);
    v += dpp_i32<kRowShr + 4, 0xf>(0, v);
    v += dpp_i32<kRowShr + 8, 0xf>(0, v);
    v += dpp_i32<kBcast15, 0xa>(0, v);
    v += dpp_i32<kBcast31, 0xc>(0, v);
    return uint32_t(v);
}

// v of the previous lane; lane 0 gets `first`
__device__ __forceinline__ int32_t from_prev_lane(int32_t v, int32_t first) {
    return dpp_i32<kWaveShr1, 0xf>(first, v);
}

__device__ __forceinline__ int32_t lane63(int32_t v) { return __builtin_amdgcn_readlane(v, 63); }

// ---- one lane's 16 bytes of a round

struct Piece {
    uint32_t w[4];       // byte j is byte j % 4 of w[j / 4]
    uint32_t valid;      // bit j: byte j lies below the end of the unit
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The 16 bytes at p, all present (raw + p is 16-byte aligned).  NT: a
// non-temporal load (the write pass, whose whole-line reads and 16-byte block
// stores stream faster non-temporal; the summary pass measured no difference).
template <bool NT>
__device__ __forceinline__ Piece load_full(const uint8_t *raw, int64_t p) {
    const u32x4 v = NT ? __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(raw + p))
                       : *reinterpret_cast<const u32x4 *>(raw + p);
    Piece x;
    x.w[0] = v.x;
    x.w[1] = v.y;
    x.w[2] = v.z;
    x.w[3] = v.w;
    x.valid = 0xffffu;
    return x;
}

// Bytes p .. p+15 of the last, partial round of a unit: those at or past
// `end` absent (read as '\n', not valid).
__device__ __forceinline__ Piece load_tail(const uint8_t *raw, int64_t end, int64_t p) {
    Piece x;
    x.valid = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) x.w[q] = kNl * 0x01010101u;
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        if (p + j < end) {
            const int s = 8 * (j & 3);
            x.w[j >> 2] = (x.w[j >> 2] & ~(0xffu << s)) | (uint32_t(raw[p + j]) << s);
            x.valid |= 1u << j;
        }
    return x;
}

// bit j set iff byte j differs from c.  Per dword: 0x80 in each byte that
// differs (exact: the low seven bits are added without carrying into the next
// byte), then one 4-way byte dot product with weights 1, 2, 4, 8 (or 16 .. 128)
// gathers the four flags into bits of the result.
__device__ __forceinline__ uint32_t ne_mask(const Piece &x, uint32_t c) {
    const uint32_t cc = c * 0x01010101u;
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t y = x.w[q] ^ cc;
        const uint32_t t = (((y & 0x7f7f7f7fu) + 0x7f7f7f7fu) | y) & 0x80808080u;
        const uint32_t wgt = (q & 1) ? 0x80402010u : 0x08040201u;
        if (q < 2)
            lo = __builtin_amdgcn_udot4(t, wgt, lo, false);
        else
            hi = __builtin_amdgcn_udot4(t, wgt, hi, false);
    }
    return (lo >> 7) | (hi << 1);  // lo, hi = 0x80 x the masks of bytes 0..7, 8..15
}

// bit j set iff byte j is below 0x40 (its two top bits clear): '\n', '\r' and
// '>' are, sequence letters are not.  Same gathering as ne_mask.
__device__ __forceinline__ uint32_t low_mask(const Piece &x) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t t = ~(x.w[q] | (x.w[q] << 1)) & 0x80808080u;
        const uint32_t wgt = (q & 1) ? 0x80402010u : 0x08040201u;
        if (q < 2)
            lo = __builtin_amdgcn_udot4(t, wgt, lo, false);
        else
            hi = __builtin_amdgcn_udot4(t, wgt, hi, false);
    }
    return (lo >> 7) | (hi << 1);
}

// the 16 bytes with 'a'..'z' made upper case (four at a time; bytes >= 0x80
// are left alone, and no byte carries into the next)
__device__ __forceinline__ void upper_case(const Piece &x, uint32_t (&up)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t lo7 = x.w[q] & 0x7f7f7f7fu;
        const uint32_t lower = (lo7 + 0x1f1f1f1fu) & ~(lo7 + 0x05050505u) & ~x.w[q] & 0x80808080u;
        up[q] = x.w[q] - (lower >> 2);
    }
}

struct Lines {
    uint32_t starts;     // bit j: a line starts at byte j
    uint32_t hs;         // bit j: a header line starts at byte j
    uint32_t elig;       // bit j: byte j is present and neither '\n' nor '\r'
    uint32_t fill;       // bit j: the last line start at or before byte j in the piece is a header
    uint32_t open;       // bit j: no line starts in the piece at or before byte j
};

// nl: bit j set iff byte j is '\n'; prev_nl: the byte before the piece is
// '\n' (or the piece starts the text)
__device__ __forceinline__ Lines analyse(const Piece &x, uint32_t nl, uint32_t prev_nl) {
    Lines L;
    L.starts = ((nl << 1) | prev_nl) & x.valid;
    L.hs = L.starts & ~ne_mask(x, kGt);
    L.elig = x.valid & ~nl & ne_mask(x, kCr);
    // copy each start's header flag forward to the bytes of its line
    uint32_t v = L.hs, open = ~L.starts & 0xffffu;
#pragma unroll
    for (int s = 1; s < kPer; s <<= 1) {
        v |= (v << s) & open;
        open &= (open << s) | ((1u << s) - 1u);
    }
    L.fill = v & 0xffffu;
    L.open = open & 0xffffu;
    return L;
}

// the piece's last line start (2 s + header, s relative to the unit), or kNone
__device__ __forceinline__ int32_t last_start(const Lines &L, int32_t prel) {
    if (!L.starts) return kNone;
    const int j = 31 - __clz(L.starts);
    return 2 * (prel + j) + int32_t((L.hs >> j) & 1u);
}

// Rounds of one unit, with the loads of the next two whole rounds in flight:
// three pieces in fixed registers, each reloaded right after its round is
// done, so that no piece is copied (a copy would wait for the load just
// issued).  Every reload is issued, those past the unit's whole rounds from
// its last whole piece again (a cache hit), so that the loads in flight are
// the same on every path and each round waits for its own load only.  A last,
// partial round (the end of the text) comes after them.
template <bool NT, class Step>
__device__ __forceinline__ void unit_rounds(const uint8_t *raw, int64_t u0, int64_t u1, Step &&step) {
    const int full = int((u1 - u0) / kRound);
    const int64_t lp = int64_t(__lane_id()) * kPer;
    if (full > 0) {
        const auto at = [&](int r) { return u0 + int64_t(r < full ? r : full - 1) * kRound + lp; };
        Piece a = load_full<NT>(raw, at(0)), b = load_full<NT>(raw, at(1)), c = load_full<NT>(raw, at(2));
        for (int r = 0; r < full; r += 3) {
            step(a, r);
            a = load_full<NT>(raw, at(r + 3));
            if (r + 1 < full) step(b, r + 1);
            b = load_full<NT>(raw, at(r + 4));
            if (r + 2 < full) step(c, r + 2);
            c = load_full<NT>(raw, at(r + 5));
        }
    }
    if (u0 + int64_t(full) * kRound < u1) step(load_tail(raw, u1, u0 + int64_t(full) * kRound + lp), full);
}

// Pass A: one wave per unit
__global__ __launch_bounds__(kThreads) void k_fasta_summary(const uint8_t *raw, int64_t n, int64_t nunits,
                                                            UnitSummary *sum) {
    const int lane = __lane_id();
    const int64_t u = int64_t(blockIdx.x) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    if (u >= nunits) return;
    const int64_t u0 = u * kUnit, u1 = std::min(u0 + kUnit, n);
    int32_t carry_nl = u0 == 0 ? 1 : int32_t(raw[u0 - 1] == kNl);
    int32_t carry = kNone;
    uint32_t pre = 0, kept = 0, hdr = 0;
    unit_rounds<false>(raw, u0, u1, [&](const Piece &x, int r) {
        const uint32_t nl = ~ne_mask(x, kNl) & 0xffffu;
        const uint32_t prev = uint32_t(from_prev_lane(int32_t(nl >> 15), carry_nl));
        carry_nl = lane63(int32_t(nl >> 15)) & 1;
        if (__builtin_amdgcn_ballot_w64((low_mask(x) & ~nl & x.valid) != 0) == 0) {
            // No byte of the round is below 0x40 except '\n' (the usual
            // sequence round): no '\r', no header starts, every present byte
            // that is not '\n' kept unless its line is an open header.  The
            // last line start before a lane's piece is the carry unless an
            // earlier lane of the round has one (never a header).
            const uint32_t starts = ((nl << 1) | prev) & x.valid;
            const uint32_t open = starts ? (1u << __builtin_ctz(starts)) - 1u : 0xffffu;
            const uint32_t elig = x.valid & ~nl;
            const unsigned long long sb = __builtin_amdgcn_ballot_w64(starts != 0);
            const bool before = __builtin_amdgcn_mbcnt_hi(uint32_t(sb >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(sb), 0u)) != 0u;
            if (!before && carry == kNone) {
                pre += __popc(elig & open);
                kept += __popc(elig & ~open);
            } else {
                kept += __popc(elig & ~((!before && (carry & 1)) ? open : 0u));
            }
            if (sb) {
                const int h = 63 - __builtin_clzll(sb);
                const int32_t ls = 2 * (r * kRound + lane * kPer + 31 - __clz(starts | 1u));
                carry = __builtin_amdgcn_readlane(ls, h);
            }
            return;
        }
        const Lines L = analyse(x, nl, prev);
        const int32_t incl = wave_incl_max(last_start(L, r * kRound + lane * kPer));
        const int32_t ex = max(from_prev_lane(incl, kNone), carry);
        if (ex == kNone) {
            pre += __popc(L.elig & L.open);
            kept += __popc(L.elig & ~L.open & ~L.fill);
        } else {
            kept += __popc(L.elig & ~(L.fill | ((ex & 1) ? L.open : 0u)));
        }
        hdr += __popc(L.hs);
        carry = max(carry, lane63(incl));
    });
    pre = uint32_t(lane63(int32_t(wave_incl_sum(pre))));
    kept = uint32_t(lane63(int32_t(wave_incl_sum(kept))));
    hdr = uint32_t(lane63(int32_t(wave_incl_sum(hdr))));
    if (lane == 0) {
        UnitSummary s;
        s.last_ls = carry == kNone ? -1 : 2 * u0 + carry;
        s.pre = pre;
        s.kept = kept;
        s.headers = hdr;
        s.pad = 0;
        sum[u] = s;
    }
}

// ---- pass B: ordered combination of unit summaries

__device__ __forceinline__ Agg agg_identity() { return Agg{-1, 0ull, 0ull, 0ull}; }

__device__ __forceinline__ Agg agg_of(const UnitSummary &s) { return Agg{s.last_ls, s.pre, s.kept, s.headers}; }

// x followed by y
__device__ __forceinline__ Agg combine(const Agg &x, const Agg &y) {
    Agg r;
    r.ls = y.ls >= 0 ? y.ls : x.ls;
    r.hdr = x.hdr + y.hdr;
    if (x.ls < 0) {  // y's leading bytes continue the line x's leading bytes are in
        r.pre = x.pre + y.pre;
        r.kept = x.kept + y.kept;
    } else {         // they continue x's last line
        r.pre = x.pre;
        r.kept = x.kept + ((x.ls & 1) ? 0ull : y.pre) + y.kept;
    }
    return r;
}

__device__ __forceinline__ Agg shfl_up_agg(const Agg &a, int d) {
    Agg r;
    r.ls = __shfl_up(a.ls, d);
    r.pre = __shfl_up(a.pre, d);
    r.kept = __shfl_up(a.kept, d);
    r.hdr = __shfl_up(a.hdr, d);
    return r;
}

// exclusive ordered scan over the block; *total = the whole block's
__device__ Agg block_scan_excl(Agg v, Agg *sh, Agg *total) {
    const int lane = threadIdx.x & (kWaveSize - 1), w = threadIdx.x / kWaveSize;
    const int nw = blockDim.x / kWaveSize;
    Agg inc = v;
#pragma unroll
    for (int d = 1; d < kWaveSize; d <<= 1) {
        const Agg u = shfl_up_agg(inc, d);
        if (lane >= d) inc = combine(u, inc);
    }
    Agg ex = shfl_up_agg(inc, 1);
    if (lane == 0) ex = agg_identity();
    if (lane == kWaveSize - 1) sh[w] = inc;
    __syncthreads();
    Agg before = agg_identity(), tot = agg_identity();
    for (int i = 0; i < nw; ++i) {
        if (i < w) before = combine(before, sh[i]);
        tot = combine(tot, sh[i]);
    }
    __syncthreads();
    *total = tot;
    return combine(before, ex);
}

// the thread's kPlanPer units of block `b`, combined
__device__ __forceinline__ Agg thread_units(const UnitSummary *sum, int64_t nunits, int64_t b) {
    const int64_t k0 = b * kPlanUnits + int64_t(threadIdx.x) * kPlanPer;
    Agg a = agg_identity();
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i)
        if (k0 + i < nunits) a = combine(a, agg_of(sum[k0 + i]));
    return a;
}

// B1: the combined summary of each block of kPlanUnits units
__global__ __launch_bounds__(kPlanThreads) void k_fasta_blocks(const UnitSummary *sum, int64_t nunits, Agg *blk) {
    __shared__ Agg sh[kPlanThreads / kWaveSize];
    Agg tot;
    block_scan_excl(thread_units(sum, nunits, blockIdx.x), sh, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

// B2: each block's prefix (the blocks before it), then its units' plans; the
// last block writes the totals.  One block with no units writes zero totals.
__global__ __launch_bounds__(kPlanThreads) void k_fasta_offsets(const UnitSummary *sum, int64_t nunits,
                                                                const Agg *blk, int64_t nblk, UnitPlan *plan,
                                                                int64_t *totals) {
    __shared__ Agg sh[kPlanThreads / kWaveSize];
    const int64_t b = blockIdx.x;
    if (nunits == 0) {
        if (threadIdx.x == 0) {
            totals[0] = 0;
            totals[1] = 0;
        }
        return;
    }
    // prefix over blocks 0 .. b-1, a contiguous run of them per thread
    const int64_t per = (b + kPlanThreads - 1) / kPlanThreads;
    Agg run = agg_identity();
    for (int64_t i = int64_t(threadIdx.x) * per; i < std::min(b, int64_t(threadIdx.x + 1) * per); ++i)
        run = combine(run, blk[i]);
    Agg prefix;
    block_scan_excl(run, sh, &prefix);
    Agg tot;
    const Agg ex = block_scan_excl(thread_units(sum, nunits, b), sh, &tot);
    Agg cur = combine(prefix, ex);
    const int64_t k0 = b * kPlanUnits + int64_t(threadIdx.x) * kPlanPer;
#pragma unroll
    for (int i = 0; i < kPlanPer; ++i) {
        const int64_t k = k0 + i;
        if (k >= nunits) break;
        UnitPlan p;
        p.ls_before = cur.ls;
        p.out_off = int64_t(cur.kept + cur.pre);  // pre is 0: byte 0 starts a line
        p.rec_off = int64_t(cur.hdr);
        plan[k] = p;
        cur = combine(cur, agg_of(sum[k]));
    }
    if (b == nblk - 1 && threadIdx.x == 0) {
        const Agg all = combine(prefix, tot);
        totals[0] = int64_t(all.kept + all.pre);
        totals[1] = int64_t(all.hdr);
    }
}

// Pass C: one wave per unit
__global__ __launch_bounds__(kThreads) void k_fasta_write(const uint8_t *raw, int64_t n, int64_t nunits,
                                                          const UnitPlan *plan, uint8_t *out, int64_t *rec_start,
                                                          int64_t rec_cap) {
    __shared__ __align__(16) uint8_t ring_all[kWaves][kRing];
    const int lane = __lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveSize);
    const int64_t u = int64_t(blockIdx.x) * kWaves + wv;
    if (u >= nunits) return;
    uint8_t *ring = ring_all[wv];
    constexpr uint32_t kMask = kRing - 1;
    const int64_t u0 = u * kUnit, u1 = std::min(u0 + kUnit, n);
    const UnitPlan pl = plan[u];
    int32_t carry_nl = u0 == 0 ? 1 : int32_t(raw[u0 - 1] == kNl);
    // before any start in the unit: -1 if the open line is a header, else -2
    int32_t carry = (pl.ls_before >= 0 && (pl.ls_before & 1)) ? -1 : -2;
    int64_t o = pl.out_off, rec = pl.rec_off;
    // output byte q sits at ring[(abase + q) & kMask]: ring blocks of 16 line up with out's
    const uint32_t abase = uint32_t(reinterpret_cast<uintptr_t>(out));
    const int64_t o_start = o;
    const int64_t head_end = o_start + ((16u - ((abase + uint32_t(o_start)) & 15u)) & 15u);
    int64_t f = o_start;  // output below f is stored
    bool head_done = head_end == o_start;
    unit_rounds<true>(raw, u0, u1, [&](const Piece &x, int r) {
        const uint32_t nl = ~ne_mask(x, kNl) & 0xffffu;
        const uint32_t prev = uint32_t(from_prev_lane(int32_t(nl >> 15), carry_nl));
        carry_nl = lane63(int32_t(nl >> 15)) & 1;
        uint32_t keep, hs;
        int32_t next_carry;
        if (__builtin_amdgcn_ballot_w64((low_mask(x) & ~nl & x.valid) != 0) == 0) {
            // a sequence round, read as in the summary pass
            const uint32_t starts = ((nl << 1) | prev) & x.valid;
            const uint32_t open = starts ? (1u << __builtin_ctz(starts)) - 1u : 0xffffu;
            const unsigned long long sb = __builtin_amdgcn_ballot_w64(starts != 0);
            const bool before = __builtin_amdgcn_mbcnt_hi(uint32_t(sb >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(sb), 0u)) != 0u;
            keep = x.valid & ~nl & ~((!before && (carry & 1)) ? open : 0u);
            hs = 0;
            next_carry = carry;
            if (sb) {
                const int h = 63 - __builtin_clzll(sb);
                next_carry = __builtin_amdgcn_readlane(2 * (r * kRound + lane * kPer + 31 - __clz(starts | 1u)), h);
            }
        } else {
            const Lines L = analyse(x, nl, prev);
            const int32_t incl = wave_incl_max(last_start(L, r * kRound + lane * kPer));
            const int32_t ex = max(from_prev_lane(incl, kNone), carry);
            keep = L.elig & ~(L.fill | ((ex & 1) ? L.open : 0u));
            hs = L.hs;
            next_carry = max(carry, lane63(incl));
        }
        // kept bytes and header starts of the lane, packed (each <= 16, wave sums <= 1024)
        const uint32_t packed = uint32_t(__popc(keep)) | (uint32_t(__popc(hs)) << 16);
        const uint32_t pin = wave_incl_sum(packed);
        const uint32_t pex = pin - packed;
        const uint32_t tot = uint32_t(lane63(int32_t(pin)));
        // stage the kept bytes, upper-cased
        uint32_t up[4];
        upper_case(x, up);
        uint32_t pos = abase + uint32_t(o) + (pex & 0xffffu);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if ((keep >> j) & 1u) {
                ring[pos & kMask] = uint8_t(up[j >> 2] >> (8 * (j & 3)));
                ++pos;
            }
        }
        // record starts: the kept bytes before each header start
        for (uint32_t hm = hs, k = 0; hm; hm &= hm - 1u, ++k) {
            const int j = __builtin_ctz(hm);
            const int64_t h = rec + int64_t(pex >> 16) + k;
            if (h >= 0 && h < rec_cap) rec_start[h] = o + int64_t(pex & 0xffffu) + __popc(keep & ((1u << j) - 1u));
        }
        o += int64_t(tot & 0xffffu);
        rec += int64_t(tot >> 16);
        carry = next_carry;
        __builtin_amdgcn_wave_barrier();
        // store: the head bytes once they are all staged, then whole 16-byte blocks
        if (!head_done && o >= head_end) {
            const int64_t q = o_start + lane;
            if (q >= 0 && q < head_end && q < n) out[q] = ring[(abase + uint32_t(q)) & kMask];
            f = head_end;
            head_done = true;
        }
        if (head_done) {
            const int64_t end = o - int64_t((abase + uint32_t(o)) & 15u);
            for (int64_t k = lane; f + 16 * k < end; k += kWaveSize) {
                const int64_t q = f + 16 * k;
                const u32x4 v = *reinterpret_cast<const u32x4 *>(ring + ((abase + uint32_t(q)) & kMask));
                if (q >= 0 && q + 16 <= n) __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(out + q));
            }
            f = std::max(f, end);
        }
    });
    // the unit's last partial block (or all of its output, if shorter than its head)
    for (int64_t q = f + lane; q < o; q += kWaveSize)
        if (q >= 0 && q < n) out[q] = ring[(abase + uint32_t(q)) & kMask];
}

using dfa::hip_ok;

int64_t nunits_of(int64_t n) { return n > 0 ? dfa::ceil_div(n, kUnit) : 0; }

struct Layout {
    int64_t nunits, nblk, sum_bytes, blk_bytes, plan_bytes;
};

Layout layout_of(int64_t n) {
    Layout l;
    l.nunits = nunits_of(n);
    l.nblk = dfa::ceil_div(l.nunits, kPlanUnits);
    l.sum_bytes = dfa::round_up(l.nunits * int64_t(sizeof(UnitSummary)), 256);
    l.blk_bytes = dfa::round_up(l.nblk * int64_t(sizeof(Agg)), 256);
    l.plan_bytes = dfa::round_up(l.nunits * int64_t(sizeof(UnitPlan)), 256);
    return l;
}

}  // namespace

extern "C" int64_t dfa_fasta_workspace_bytes(int64_t n) {
    if (n < 0) {
        dfa::set_error("dfa_fasta_workspace_bytes: n < 0");
        return DFA_EINVAL;
    }
    const Layout l = layout_of(n);
    return l.sum_bytes + l.blk_bytes + l.plan_bytes;
}

extern "C" int dfa_fasta_normalize(const uint8_t *raw, int64_t n, uint8_t *out, int64_t *rec_start, int64_t rec_cap,
                                   int64_t *totals, void *workspace, int64_t workspace_bytes, void *stream) {
    if (n < 0 || (n > 0 && (!raw || !out)) || !totals || rec_cap < 0 || (rec_cap > 0 && !rec_start)) {
        dfa::set_error("dfa_fasta_normalize: null argument or negative size");
        return DFA_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(raw) & 15) || (reinterpret_cast<uintptr_t>(totals) & 7) ||
        (reinterpret_cast<uintptr_t>(rec_start) & 7)) {
        dfa::set_error("dfa_fasta_normalize: raw must be 16-byte, totals and rec_start 8-byte aligned");
        return DFA_EINVAL;
    }
    const int64_t need = dfa_fasta_workspace_bytes(n);
    if (need > 0 && (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))) {
        dfa::set_error("dfa_fasta_normalize: workspace of %lld bytes (256-aligned) needed, got %lld", (long long)need,
                       (long long)workspace_bytes);
        return DFA_ENOSPACE;
    }
    const Layout l = layout_of(n);
    if (dfa::ceil_div(l.nunits, kWaves) > 0x7fffffff) {
        dfa::set_error("dfa_fasta_normalize: text too large");
        return DFA_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = reinterpret_cast<uint8_t *>(workspace);
    UnitSummary *sum = reinterpret_cast<UnitSummary *>(ws);
    Agg *blk = reinterpret_cast<Agg *>(ws + l.sum_bytes);
    UnitPlan *plan = reinterpret_cast<UnitPlan *>(ws + l.sum_bytes + l.blk_bytes);
    const unsigned groups = unsigned(dfa::ceil_div(l.nunits, kWaves));
    if (l.nunits > 0) {
        hipLaunchKernelGGL(k_fasta_summary, dim3(groups), dim3(kThreads), 0, st, raw, n, l.nunits, sum);
        hipLaunchKernelGGL(k_fasta_blocks, dim3(unsigned(l.nblk)), dim3(kPlanThreads), 0, st,
                           (const UnitSummary *)sum, l.nunits, blk);
    }
    hipLaunchKernelGGL(k_fasta_offsets, dim3(unsigned(std::max<int64_t>(1, l.nblk))), dim3(kPlanThreads), 0, st,
                       (const UnitSummary *)sum, l.nunits, (const Agg *)blk, l.nblk, plan, totals);
    if (l.nunits > 0)
        hipLaunchKernelGGL(k_fasta_write, dim3(groups), dim3(kThreads), 0, st, raw, n, l.nunits,
                           (const UnitPlan *)plan, out, rec_start, rec_cap);
    if (!hip_ok(hipGetLastError(), "fasta launch")) return DFA_EHIP;
    dfa::clear_error();
    return DFA_OK;
}
