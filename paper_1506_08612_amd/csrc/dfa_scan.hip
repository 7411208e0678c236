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
// Data movement.  Each round a wave fetches the next 128 bytes of each of its
// walks with coalesced 16-byte loads (8 lanes read one 128-byte line), writes
// them to a wave-private LDS buffer, and reads them back transposed so that
// every lane holds 128 consecutive bytes of its own walk in registers.  The
// loads for round r+1 are in flight while round r is walked.  HBM traffic is
// the text once plus the m-1 overlap bytes per walk (fetched as the first
// ceil((m-1)/16) units of the next span's first line).
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

enum Mode { kCount = 0, kCountPerWalk = 1, kPositions = 2 };

struct ScanParams {
    const uint8_t *text;
    int64_t n;
    const uint8_t *table;
    int32_t m;
    int32_t rounds;    // ceil((S + m - 1) / LINE)
    int64_t S;         // span bytes per walk (multiple of 16)
    int64_t nwalks;
    unsigned long long *total;  // kCount / kCountPerWalk: += matches
    uint32_t *walk_count;       // kCountPerWalk: matches per walk
    uint16_t *walk_buf;         // kCountPerWalk: start offsets (within the walk) of its first kBuffered matches
    const int64_t *walk_off;    // kPositions: output offset per walk
    int64_t *positions;         // kPositions
    int64_t cap;
    unsigned long long *wg_times;  // measurement only (kCount): 3 words per workgroup, or null
    int64_t wg_cap;                // workgroups with room in wg_times
};

// matches per walk whose end offsets the counting pass keeps (in the
// workspace); walks with more are walked again by the positions pass
constexpr int kBuffered = 16;
// buffered matches are kept as 16-bit start offsets within the walk (a walk
// owns the starts of its span): the positions path needs S <= 65536
constexpr int64_t kMaxPositionsSpan = 65536;

__host__ __device__ inline int table_lds_bytes(int m) { return table_lds_rows_bytes(m + 1); }

struct WalkLane {
    int64_t wstart;  // first byte of the walk
    uint32_t len;    // bytes the walk reads (span + m - 1, clipped at the text end)
    uint32_t cnt;    // matches (per-walk counting pass)
    uint16_t *buf;   // its kBuffered start offsets (per-walk counting pass)
    int64_t off;     // next output slot (positions pass)
};

// The start offsets of a lane's matches in one unit (hit mask from
// walk16_hits, first byte in bit 15; a match ending at byte j starts at
// j - (m - 1)), in increasing order, into the walk's buffer.
__device__ __forceinline__ void record_hits(uint32_t hm, uint32_t jb, uint32_t m, WalkLane &w) {
    while (hm) {
        const int b = 31 - __clz(hm);
        if (w.cnt < uint32_t(kBuffered)) w.buf[w.cnt] = uint16_t(jb + uint32_t(15 - b) - (m - 1));
        ++w.cnt;
        hm ^= 1u << b;
    }
}

// Walk 16 bytes: byte b of word w is byte jb + 4w + b of the walk.  GUARD:
// only bytes below the walk's length count.  kCount: ballot + scalar count.
// kCountPerWalk: per-walk count and the first kBuffered match ends (the
// total is summed from the per-walk counts at the end).  kPositions: write
// the start offset of every match.
template <int K, int MODE, bool GUARD>
__device__ __forceinline__ void walk_unit(const v4u (&t)[K], uint32_t (&q)[K], uint32_t m, uint32_t jb,
                                          uint32_t &acc, WalkLane (&wl)[K], const ScanParams &p) {
    if constexpr (MODE == kCount && !GUARD && K == 1) {
        walk16_count(q[0], t[0], acc, m);
        return;
    }
    if constexpr (MODE == kCountPerWalk && !GUARD && K == 1) {
        uint32_t hm;
        walk16_hits(q[0], t[0], hm, m);
        if (__ballot(hm != 0)) record_hits(hm, jb, m, wl[0]);
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
                bool hit = q[s] == m;
                if (GUARD) hit = hit && (j < wl[s].len);
                if (MODE == kCount) {
                    add_hits(acc, hit);
                } else if (MODE == kCountPerWalk) {
                    if (hit) {
                        if (wl[s].cnt < uint32_t(kBuffered)) wl[s].buf[wl[s].cnt] = uint16_t(j - (m - 1));
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

// Walk one staged round: its units stream from LDS, the next one in flight
// while the current one is walked.  `nbytes` (wave-uniform) bytes of the round
// belong to every walk when GUARD is false; with GUARD, each walk's own length
// decides.
template <int K, int LINE, int MODE, bool GUARD>
__device__ __forceinline__ void walk_round(const v4u *xb, int lane, uint32_t (&q)[K], uint32_t m,
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
            walk_unit<K, MODE, true>(cur, q, m, jb, acc, wl, p);
        else
            walk_unit<K, MODE, false>(cur, q, m, jb, acc, wl, p);
#pragma unroll
        for (int s = 0; s < K; ++s) cur[s] = nxt[s];
    }
}

// Overlap units loaded ahead (H): 1 unit covers m <= 17, 4 units m <= 65.
// The kernel is instantiated for both so that short patterns keep 12 more
// registers free (one more wave per SIMD).
constexpr int halo_units_for(int m) { return m <= 17 ? 1 : 4; }

// The default counting kernels (one walk per lane, 64-byte rounds) are asked
// to fit 6 waves per SIMD (at most 80 registers): the per-walk counting pass
// with 4 overlap units would otherwise need 81 (the compiler then keeps one
// overlap unit in scratch between the first round and the end of the walk).
template <int K, int LINE, int MODE>
constexpr int scan_waves_per_eu() { return (K == 1 && LINE == 64 && MODE != kPositions) ? 6 : 1; }

template <int K, int LINE, int MODE, int H>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(scan_waves_per_eu<K, LINE, MODE>())))
void k_scan(ScanParams p) {
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
    v4u *xb = reinterpret_cast<v4u *>(smem + table_lds_bytes(p.m) + wave * (K * kWave * LINE));

    if (MODE == kPositions) {
        // only walks whose matches did not all fit the counting pass's buffer
        // are walked again: a workgroup without any leaves before loading the
        // table.  The vote goes through the first word of each wave's
        // transpose buffer (no static LDS: the table must start at address 0).
        const int64_t gw0 = (int64_t(blockIdx.x) * nwaves + wave) * (kWave * K);
        bool mine = false;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int64_t g = gw0 + s * kWave + lane;
            mine |= g < p.nwalks && p.walk_count[g] > uint32_t(kBuffered);
        }
        const bool wave_has = __ballot(mine) != 0;
        uint32_t *vote = reinterpret_cast<uint32_t *>(smem + table_lds_bytes(p.m));
        const int stride = K * kWave * LINE / 4;  // words per wave buffer
        if (lane == 0) vote[wave * stride] = wave_has ? 1u : 0u;
        __syncthreads();
        bool any = false;
        for (int w = 0; w < nwaves; ++w) any |= vote[w * stride] != 0;
        if (!any) return;  // uniform over the workgroup
        // the table load below ends with a barrier before any buffer is restaged
    }

    // table -> LDS, rows padded to kRow bytes
    {
        const uint32_t *tg = reinterpret_cast<const uint32_t *>(p.table);
        const int words = (p.m + 1) * (DFA_ALPHABET / 4);
        for (int i = threadIdx.x; i < words; i += blockDim.x)
            *reinterpret_cast<uint32_t *>(smem + (i >> 6) * kRow + 4 * (i & 63)) = tg[i];
    }
    __syncthreads();

    const int64_t g0 = (int64_t(blockIdx.x) * nwaves + wave) * (kWave * K);
    const uint32_t m = uint32_t(p.m);
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
        wl[s].buf = MODE == kCountPerWalk ? p.walk_buf + g * kBuffered : nullptr;
        q[s] = 0;
        if (MODE == kPositions) {
            // only walks whose matches did not all fit the counting pass's buffer
            // (the other lanes walk along without writing: their offset is past
            // any capacity)
            const bool has = g < p.nwalks && p.walk_count[g] > uint32_t(kBuffered);
            wl[s].off = has ? p.walk_off[g] : (int64_t(1) << 62);
            any_work |= has;
        }
    }
    if (MODE == kPositions && __ballot(any_work) == 0) return;  // nothing left to write in this wave

    // whole wave in bounds: every load of every round lies inside the text
    const int64_t glast = g0 + kWave * K - 1;
    const bool full = glast < p.nwalks && glast * p.S + int64_t(p.rounds) * LINE <= p.n;
    uint32_t acc = 0;

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
        v4u pa[K][G::U], pb[K][G::U];
        fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, 0, rlast);
        fetch_round_or_none<K, LINE>(pb, p.text, wb, p.S, lane_off, off_last, off_none, 1, rlast);
        const int hu = (p.m - 1 + 15) / 16;  // overlap units
        v4u halo[K][H];
        // round 0 (and 1), then the steady state from round 2
        stage_round<K, LINE>(pa, xb, lane);
        grab_halo<K, LINE, H>(halo, xb, lane, p.text, wb, p.S, hu, rlast == 0 ? int(ulast) : G::U);
        if (LINE == 128) fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, 2, rlast);
        walk_round<K, LINE, MODE, false>(xb, lane, q, m, 0u, rlast == 0 ? lastlen : LINE, acc, wl, p);
        if (rlast >= 1) {
            stage_round<K, LINE>(pb, xb, lane);
            if (LINE == 64) fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, 2, rlast);
            fetch_round_or_none<K, LINE>(pb, p.text, wb, p.S, lane_off, off_last, off_none, 3, rlast);
            walk_round<K, LINE, MODE, false>(xb, lane, q, m, uint32_t(LINE), rlast == 1 ? lastlen : LINE, acc, wl,
                                             p);
        }
        for (int r = 2; r < R; r += 2) {
            stage_round<K, LINE>(pa, xb, lane);
            if (LINE == 128)
                fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, r + 2, rlast);
            walk_round<K, LINE, MODE, false>(xb, lane, q, m, uint32_t(r * LINE), r == rlast ? lastlen : LINE,
                                             acc, wl, p);
            if (r + 1 > rlast) break;
            stage_round<K, LINE>(pb, xb, lane);
            if (LINE == 64)
                fetch_round_or_none<K, LINE>(pa, p.text, wb, p.S, lane_off, off_last, off_none, r + 2, rlast);
            fetch_round_or_none<K, LINE>(pb, p.text, wb, p.S, lane_off, off_last, off_none, r + 3, rlast);
            walk_round<K, LINE, MODE, false>(xb, lane, q, m, uint32_t((r + 1) * LINE),
                                             r + 1 == rlast ? lastlen : LINE, acc, wl, p);
        }
        // the overlap, from registers, then (m > 65) the rest of it from memory
        const uint32_t hb = uint32_t(p.S);
#pragma unroll
        for (int u = 0; u < H; ++u) {
            if (u < hu) {
                v4u t[K];
#pragma unroll
                for (int s = 0; s < K; ++s) t[s] = halo[s][u];
                walk_unit<K, MODE, true>(t, q, m, hb + 16u * u, acc, wl, p);
            }
        }
        for (int u = H; u < hu; ++u) {
            v4u t[K];
#pragma unroll
            for (int s = 0; s < K; ++s)
                t[s] = *reinterpret_cast<const v4u *>(p.text + (g0 + s * kWave + lane + 1) * p.S + 16 * u);
            walk_unit<K, MODE, true>(t, q, m, hb + 16u * u, acc, wl, p);
        }
    } else {
        v4u pf[K][G::U];
        fetch_round<K, LINE, true>(pf, p.text, p.n, g0 * p.S, p.S, lane_off, 0);
        for (int r = 0; r < p.rounds; ++r) {
            stage_round<K, LINE>(pf, xb, lane);
            if (r + 1 < p.rounds) fetch_round<K, LINE, true>(pf, p.text, p.n, g0 * p.S, p.S, lane_off, r + 1);
            walk_round<K, LINE, MODE, true>(xb, lane, q, m, uint32_t(r * LINE), LINE, acc, wl, p);
        }
    }

    if (MODE == kPositions) return;

    if (MODE == kCountPerWalk) {
        uint32_t c = 0;
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int64_t g = g0 + s * kWave + lane;
            if (g < p.nwalks) p.walk_count[g] = wl[s].cnt;
            c += wl[s].cnt;
        }
        // the wave's matches, summed over its lanes
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) c += uint32_t(__shfl_xor(int(c), o));
        acc = uint32_t(__builtin_amdgcn_readfirstlane(int(c)));
    }
    // workgroup sum in LDS (reusing the first transpose buffer), one atomic
    unsigned long long *red = reinterpret_cast<unsigned long long *>(smem + table_lds_bytes(p.m));
    __syncthreads();
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int w = 0; w < nwaves; ++w) sum += red[w];
        if (sum) atomicAdd(p.total, sum);
        if (timed) {
            unsigned long long *t = p.wg_times + 3 * int64_t(blockIdx.x);
            t[0] = t_wall;
            t[1] = wall_clock64();
            t[2] = clock64() - t_cyc;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-walk offsets and the buffered positions.  Blocks of 256 threads; every
// global access is a coalesced pass over consecutive walks, staged in LDS.
// ---------------------------------------------------------------------------

__global__ void k_zero_u64(unsigned long long *x) { *x = 0; }

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 4;
constexpr int kScanBlock = kScanThreads * kScanPerThread;  // walks per block of the offset passes

__device__ __forceinline__ unsigned long long wave_inclusive_scan(unsigned long long v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const unsigned long long u = __shfl_up(v, d);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive scan of one value per thread over a 256-thread block; `sh` holds
// 4 scratch slots in LDS; *total receives the block total.
__device__ __forceinline__ unsigned long long block_exclusive_scan(unsigned long long v, unsigned long long *sh,
                                                                   unsigned long long *total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const unsigned long long inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) sh[w] = inc;
    __syncthreads();
    unsigned long long before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        if (i < w) before += sh[i];
        all += sh[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// part[b] = matches of the walks of block b
__global__ __launch_bounds__(kScanThreads) void k_walk_sums(const uint32_t *cnt, int64_t nw,
                                                            unsigned long long *part) {
    __shared__ unsigned long long sh[kScanThreads / kWave];
    const int64_t base = int64_t(blockIdx.x) * kScanBlock;
    unsigned long long v = 0;
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) {
        const int64_t g = base + i * kScanThreads + threadIdx.x;
        if (g < nw) v += cnt[g];
    }
    unsigned long long total;
    block_exclusive_scan(v, sh, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// one block: exclusive scan of the nb block totals; total match count to *count.
// Each thread first sums kPartsPerThread consecutive totals, so one pass of the
// block covers 1024 x 8 of them.
constexpr int kPartsThreads = 1024;
constexpr int kPartsPerThread = 8;

__global__ __launch_bounds__(kPartsThreads) void k_scan_parts(unsigned long long *part, int64_t nb,
                                                              int64_t *count) {
    __shared__ unsigned long long sh[kPartsThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    unsigned long long carry = 0;
    for (int64_t base = 0; base < nb; base += int64_t(kPartsThreads) * kPartsPerThread) {
        const int64_t i0 = base + int64_t(threadIdx.x) * kPartsPerThread;
        unsigned long long v[kPartsPerThread], mine = 0;
#pragma unroll
        for (int k = 0; k < kPartsPerThread; ++k) {
            v[k] = i0 + k < nb ? part[i0 + k] : 0ull;
            mine += v[k];
        }
        const unsigned long long inc = wave_inclusive_scan(mine);
        if (lane == kWave - 1) sh[w] = inc;
        __syncthreads();
        unsigned long long before = 0, tot = 0;
        for (int k = 0; k < kPartsThreads / kWave; ++k) {
            if (k < w) before += sh[k];
            tot += sh[k];
        }
        __syncthreads();
        unsigned long long run = carry + before + inc - mine;
#pragma unroll
        for (int k = 0; k < kPartsPerThread; ++k) {
            if (i0 + k < nb) part[i0 + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *count = int64_t(carry);
}

// off[g] = output offset of walk g: the block's counts are staged in LDS,
// each thread scans 4 consecutive walks, and the offsets leave through LDS.
__global__ __launch_bounds__(kScanThreads) void k_walk_offsets(const uint32_t *cnt, int64_t nw,
                                                               const unsigned long long *part, int64_t *off) {
    __shared__ unsigned long long sh[kScanThreads / kWave];
    __shared__ uint32_t c_sh[kScanBlock];
    __shared__ int64_t o_sh[kScanBlock];
    const int64_t base = int64_t(blockIdx.x) * kScanBlock;
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) {
        const int k = i * kScanThreads + threadIdx.x;
        c_sh[k] = base + k < nw ? cnt[base + k] : 0u;
    }
    __syncthreads();
    unsigned long long v = 0;
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) v += c_sh[threadIdx.x * kScanPerThread + i];
    unsigned long long total;
    unsigned long long run = part[blockIdx.x] + block_exclusive_scan(v, sh, &total);
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) {
        const int k = threadIdx.x * kScanPerThread + i;
        o_sh[k] = int64_t(run);
        run += c_sh[k];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanPerThread; ++i) {
        const int k = i * kScanThreads + threadIdx.x;
        if (base + k < nw) off[base + k] = o_sh[k];
    }
}

// Positions of the walks with 1..kBuffered matches, from the counting pass's
// buffer: start = walk start + buffered start offset.  One block per 256 walks
// enumerates the block's buffered matches in order (a scan of the buffered
// counts in LDS) so that consecutive threads write consecutive positions;
// the slots of walks with more matches are left to the positions pass.
__global__ __launch_bounds__(kScanThreads) void k_scatter_buffered(const uint32_t *walk_count, const uint16_t *walk_buf,
                                                                   const int64_t *walk_off, int64_t nwalks, int64_t S,
                                                                   int32_t m, int64_t *positions, int64_t cap) {
    __shared__ unsigned long long sh[kScanThreads / kWave];
    __shared__ uint32_t first[kScanThreads + 1];  // buffered matches before each walk of the block
    __shared__ int64_t out[kScanThreads];         // output offset of each walk
    const int64_t g0 = int64_t(blockIdx.x) * kScanThreads;
    const int64_t g = g0 + threadIdx.x;
    uint32_t c = 0;
    int64_t o = 0;
    if (g < nwalks) {
        c = walk_count[g];
        o = walk_off[g];
    }
    const uint32_t b = c <= uint32_t(kBuffered) ? c : 0u;
    unsigned long long total;
    first[threadIdx.x] = uint32_t(block_exclusive_scan(b, sh, &total));
    out[threadIdx.x] = o;
    if (threadIdx.x == 0) first[kScanThreads] = uint32_t(total);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < uint32_t(total); k += kScanThreads) {
        // the walk holding buffered match k: the last w with first[w] <= k
        int lo = 0, hi = kScanThreads - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (first[mid] <= k) lo = mid; else hi = mid - 1;
        }
        const uint32_t i = k - first[lo];
        const int64_t dst = out[lo] + i;
        const int64_t gw = g0 + lo;
        if (dst < cap) positions[dst] = gw * S + int64_t(walk_buf[gw * kBuffered + i]);
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
    return reinterpret_cast<const void *>(&k_scan<K, LINE, kPositions, H>);
}

// the (walks per lane, bytes per round) shapes compiled into the library, each
// with the overlap prefetch depth for the pattern length
const void *pick_scan(int K, int line, int mode, int m) {
    const bool h1 = halo_units_for(m) == 1;
    if (K == 1 && line == 128) return h1 ? scan_fn<1, 128, 1>(mode) : scan_fn<1, 128, 4>(mode);
    if (K == 1 && line == 64) return h1 ? scan_fn<1, 64, 1>(mode) : scan_fn<1, 64, 4>(mode);
    if (K == 2 && line == 64) return scan_fn<2, 64, 4>(mode);
    return nullptr;
}

size_t scan_lds_bytes(int wpg, int K, int line, int m) {
    return size_t(wpg) * K * kWave * line + size_t(table_lds_bytes(m));
}

// Default span of one walk: 8 m rounded up to whole lines, at least 512 and
// at most 2048 bytes.  Short walks make short workgroups, which the hardware
// dispatcher balances well (the launch's tail, while the last workgroups
// finish, shrinks with them); the span stays long against m so that the
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
    if (t->waves_per_group < 0 || t->waves_per_group > 8) {
        dfa::set_error("tune.waves_per_group=%d outside [1, 8]", t->waves_per_group);
        return false;
    }
    if (t->line_bytes != 0 && t->line_bytes != 64 && t->line_bytes != 128) {
        dfa::set_error("tune.line_bytes=%d must be 64 or 128 (or 0)", t->line_bytes);
        return false;
    }
    const int line = t->line_bytes ? t->line_bytes : kDefaultLine;
    const int K = t->chains_per_lane ? t->chains_per_lane : kDefaultK;
    if (t->chains_per_lane < 0 || !pick_scan(K, line, kCount, 1)) {
        dfa::set_error("tune: chains_per_lane=%d with line_bytes=%d is not a built shape "
                       "(1 with 64 or 128, 2 with 64)", t->chains_per_lane, line);
        return false;
    }
    if (t->dfas_per_group < 0 || t->automaton_bytes < 0) {
        dfa::set_error("tune: negative field");
        return false;
    }
    for (int i = 0; i < 3; ++i)
        if (t->reserved[i]) {
            dfa::set_error("tune.reserved must be zero");
            return false;
        }
    return true;
}

// Upper bound on the number of walks for any plan of (n, tune): used to size
// the workspace without a device query.
int64_t max_walks(int64_t n, const dfa_tune *t) { return n > 0 ? dfa::ceil_div(n, min_span(t)) : 0; }

// workspace layout: walk counts u32[nw] | walk offsets i64[nw] | block
// partials u64[nb] | buffered match ends u16[nw * kBuffered]
struct WsLayout {
    int64_t cnt = 0, off = 0, part = 0, buf = 0, total = 0;
};
WsLayout ws_layout(int64_t nw) {
    WsLayout L;
    if (nw <= 0) return L;
    const int64_t nb = dfa::ceil_div(nw, kScanBlock);
    L.cnt = 0;
    L.off = L.cnt + dfa::round_up(nw * 4, 256);
    L.part = L.off + dfa::round_up(nw * 8, 256);
    L.buf = L.part + dfa::round_up(nb * 8, 256);
    L.total = L.buf + dfa::round_up(nw * 2 * kBuffered, 256);
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

// Default waves per workgroup: the smaller of 4 and 8 whose workgroups keep
// at least 90% of the waves a CU can hold by registers resident, given the
// LDS each one needs (its transpose buffers plus its own copy of the table).
// Smaller workgroups refill a CU at a finer grain; larger ones share one table
// among more waves, which matters once the table is large (long patterns).
int default_wpg(const void *fn, int K, int line, int m) {
    const int regs = kernel_vgprs(fn);
    if (regs <= 0) return kDefaultWpg;
    const int per_simd = std::min(kMaxWavesPerSimd, kVgprsPerLane / int(dfa::round_up(regs, 8)));
    const int by_regs = kSimdsPerCu * std::max(1, per_simd);
    int waves[2], best = 0;
    const int cand[2] = {4, 8};
    for (int i = 0; i < 2; ++i) {
        const int groups = int(kLdsPerCu / scan_lds_bytes(cand[i], K, line, m));
        waves[i] = std::min(by_regs, groups * cand[i]);
        best = std::max(best, waves[i]);
    }
    for (int i = 0; i < 2; ++i)
        if (10 * waves[i] >= 9 * best) return cand[i];
    return kDefaultWpg;
}

bool make_plan(int64_t n, int m, int mode, const dfa_tune *t, Plan &pl) {
    pl.K = (t && t->chains_per_lane) ? t->chains_per_lane : kDefaultK;
    pl.line = (t && t->line_bytes) ? t->line_bytes : kDefaultLine;
    if (t && t->waves_per_group) {
        pl.wpg = t->waves_per_group;
    } else {
        const void *fn = pick_scan(pl.K, pl.line, mode, m);
        pl.wpg = fn ? default_wpg(fn, pl.K, pl.line, m) : kDefaultWpg;
    }
    pl.lds = scan_lds_bytes(pl.wpg, pl.K, pl.line, m);
    if (t && t->chain_bytes > 0) {
        pl.S = t->chain_bytes;
    } else {
        // whole lines: every walk starts on a 128-byte boundary (the text is
        // 16-byte aligned, torch and hipMalloc give 256), so each round's
        // loads cover exactly one cache line per walk.  A span that is not a
        // multiple of the line makes every round straddle two lines; with
        // hundreds of streaming waves per XCD the shared line is evicted from
        // L2 before the next round needs it, and HBM reads double.
        pl.S = std::min<int64_t>(kSpanMax, std::max<int64_t>(kSpanMin, dfa::round_up(int64_t(8) * m, 128)));
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
    // allow the largest table (m = 255) with the largest workgroup
    if (!dfa::allow_lds(fn, int(scan_lds_bytes(8, 1, 128, DFA_MAX_M)))) return DFA_EHIP;
    void *args[] = {const_cast<ScanParams *>(&sp)};
    if (!hip_ok(hipLaunchKernel(fn, dim3(unsigned(pl.blocks)), dim3(pl.wpg * kWave), args, pl.lds, st),
                "k_scan launch"))
        return DFA_EHIP;
    return DFA_OK;
}

}  // namespace

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

    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, reinterpret_cast<unsigned long long *>(count));
    if (!hip_ok(hipGetLastError(), "k_zero_u64 launch")) return DFA_EHIP;
    if (n == 0) {
        dfa::clear_error();
        return DFA_OK;
    }

    Plan pl;
    if (!make_plan(n, m, want_pos ? kCountPerWalk : kCount, tune, pl)) return DFA_EHIP;
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
        int rc = launch_scan(pl, kCount, sp, st);
        if (rc == DFA_OK) dfa::clear_error();
        return rc;
    }

    uint8_t *ws = reinterpret_cast<uint8_t *>(workspace);
    const int64_t nw = pl.nwalks;
    const int64_t nb = dfa::ceil_div(nw, kScanBlock);
    const WsLayout L = ws_layout(nw);
    uint32_t *wcnt = reinterpret_cast<uint32_t *>(ws + L.cnt);
    int64_t *woff = reinterpret_cast<int64_t *>(ws + L.off);
    unsigned long long *part = reinterpret_cast<unsigned long long *>(ws + L.part);
    uint16_t *wbuf = reinterpret_cast<uint16_t *>(ws + L.buf);

    sp.walk_count = wcnt;
    sp.walk_buf = wbuf;
    int rc = launch_scan(pl, kCountPerWalk, sp, st);
    if (rc != DFA_OK) return rc;
    hipLaunchKernelGGL(k_walk_sums, dim3(unsigned(nb)), dim3(kScanThreads), 0, st, wcnt, nw, part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kPartsThreads), 0, st, part, nb, count);
    hipLaunchKernelGGL(k_walk_offsets, dim3(unsigned(nb)), dim3(kScanThreads), 0, st, wcnt, nw,
                       (const unsigned long long *)part, woff);
    hipLaunchKernelGGL(k_scatter_buffered, dim3(unsigned(dfa::ceil_div(nw, kScanThreads))), dim3(kScanThreads), 0, st,
                       (const uint32_t *)wcnt, (const uint16_t *)wbuf, (const int64_t *)woff, nw, pl.S, m, positions,
                       cap);
    if (!hip_ok(hipGetLastError(), "prefix-sum launch")) return DFA_EHIP;
    sp.walk_off = woff;
    sp.positions = positions;
    rc = launch_scan(pl, kPositions, sp, st);
    if (rc == DFA_OK) dfa::clear_error();
    return rc;
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
    if (!make_plan(n, m, kCount, tune, pl)) return DFA_EHIP;
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