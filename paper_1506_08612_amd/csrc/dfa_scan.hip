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
//
// Data movement.  Each round a wave fetches the next 128 bytes of each of its
// walks with coalesced 16-byte loads (8 lanes read one 128-byte line), writes
// them to a wave-private LDS buffer, and reads them back transposed so that
// every lane holds 128 consecutive bytes of its own walk in registers.  The
// loads for round r+1 are in flight while round r is walked.  HBM traffic is
// the text once plus the m-1 overlap bytes per walk.
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

#include <cstdint>
#include <mutex>

#include "dfa.h"
#include "dfa_internal.h"

namespace {

constexpr int kLine = 128;              // bytes of one walk fetched per round
constexpr int kUnits = kLine / 16;      // 16-byte units per round
constexpr int kRow = DFA_ALPHABET + 24;  // LDS bytes per table row
constexpr int kWave = 64;
constexpr int kXbufBytes = kWave * kLine;  // wave-private transpose buffer

enum Mode { kCount = 0, kCountPerWalk = 1, kPositions = 2 };
enum Guard { kNoGuard = 0, kWaveLimit = 1, kLaneLimit = 2 };

struct ScanParams {
    const uint8_t *text;
    int64_t n;
    const uint8_t *table;
    int32_t m;
    int32_t rounds;    // ceil((S + m - 1) / kLine)
    int64_t S;         // span bytes per walk (multiple of 16)
    int64_t nwalks;
    unsigned long long *total;  // kCount / kCountPerWalk: += matches
    uint32_t *walk_count;       // kCountPerWalk: matches per walk
    const int64_t *walk_off;    // kPositions: output offset per walk
    int64_t *positions;         // kPositions
    int64_t cap;
};

// Orders this lane's LDS accesses against the other lanes' of the same wave:
// LDS executes one wave's instructions in order, so waiting for the lane's
// own outstanding LDS operations is enough; the clobber stops the compiler
// from moving memory accesses across.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// The kernels declare no static LDS, so dynamic LDS (and with it the table,
// placed first) starts at LDS address 0.  Reading the table through an
// absolute LDS address keeps the step's address one 24-bit multiply-add.
typedef __attribute__((address_space(3))) const uint8_t lds_u8;
__device__ __forceinline__ uint32_t table_step(uint32_t q, uint32_t c) {
    return *reinterpret_cast<lds_u8 *>(uintptr_t(__umul24(q, uint32_t(kRow)) + c));
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, int w) {
    return w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w;
}

// 16 bytes at text[a..a+15]; bytes at or past n read as 0 (a byte outside
// every pattern: it sends the automaton to q0 and never completes a match).
__device__ __forceinline__ uint4 load_unit_guarded(const uint8_t *text, int64_t n, int64_t a) {
    if (a + 16 <= n) return *reinterpret_cast<const uint4 *>(text + a);
    uint32_t w[4] = {0, 0, 0, 0};
    for (int i = 0; i < 16; ++i)
        if (a + i < n) w[i >> 2] |= uint32_t(text[a + i]) << (8 * (i & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Fetch round r of the wave's walks into registers: slot s, load j covers walk
// 64*s + 8*j + (lane>>3), 16-byte unit (lane & 7).
template <int K, bool GUARDED>
__device__ __forceinline__ void fetch_round(uint4 (&pf)[K][kUnits], const ScanParams &p,
                                            int64_t g0, int lane, int r) {
    const int lrow = lane >> 3, lunit = lane & 7;
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int j = 0; j < kUnits; ++j) {
            const int64_t g = g0 + s * kWave + j * 8 + lrow;
            const int64_t a = g * p.S + int64_t(r) * kLine + 16 * lunit;
            if (GUARDED)
                pf[s][j] = load_unit_guarded(p.text, p.n, a);
            else
                pf[s][j] = *reinterpret_cast<const uint4 *>(p.text + a);
        }
    }
}

// Registers -> LDS -> registers: afterwards t[s][u] holds bytes 16u..16u+15 of
// this round for the lane's own walk in slot s.  Units are XOR-swizzled by
// row so that both the writes and the transposed reads are bank-conflict free.
template <int K>
__device__ __forceinline__ void transpose_round(uint4 (&t)[K][kUnits], const uint4 (&pf)[K][kUnits],
                                                uint4 *xb, int lane) {
    const int lrow = lane >> 3, lunit = lane & 7;
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int j = 0; j < kUnits; ++j) xb[(j * 8 + lrow) * kUnits + (lunit ^ lrow)] = pf[s][j];
        wave_lds_sync();
#pragma unroll
        for (int u = 0; u < kUnits; ++u) t[s][u] = xb[lane * kUnits + (u ^ (lane & 7))];
        wave_lds_sync();
    }
}

__host__ __device__ inline int table_lds_bytes(int m) { return ((m + 1) * kRow + 15) & ~15; }

// Walk one 128-byte round.  G = kNoGuard: every byte counts; kWaveLimit: only
// bytes j < wlim (same for the whole wave); kLaneLimit: only j < llim[s].
template <int K, int MODE, int G>
__device__ __forceinline__ void walk_round(const uint4 (&t)[K][kUnits], uint32_t (&q)[K],
                                           const uint8_t *tab, uint32_t m, int wlim,
                                           const int (&llim)[K], uint32_t &acc,
                                           uint32_t (&cnt)[K], int64_t (&off)[K],
                                           const int64_t (&pos0)[K], const ScanParams &p) {
#pragma unroll
    for (int u = 0; u < kUnits; ++u) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = u * 16 + w * 4 + b;
                if (G == kWaveLimit && j >= wlim) continue;
#pragma unroll
                for (int s = 0; s < K; ++s) {
                    const uint32_t c = (word_of(t[s][u], w) >> (8 * b)) & 0xffu;
                    q[s] = table_step(q[s], c);
                    bool hit = q[s] == m;
                    if (G == kLaneLimit) hit = hit && (j < llim[s]);
                    if (MODE == kCount) {
                        acc += __popcll(__ballot(hit));
                    } else if (MODE == kCountPerWalk) {
                        cnt[s] += hit ? 1u : 0u;
                    } else {
                        if (hit) {
                            if (off[s] < p.cap) p.positions[off[s]] = pos0[s] + j - (m - 1);
                            ++off[s];
                        }
                    }
                }
            }
        }
    }
}

template <int K, int MODE>
__global__ __launch_bounds__(256) void k_scan(ScanParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    // table first (offset 0 keeps the step's address a single multiply-add),
    // then one transpose buffer per wave
    uint8_t *tab = smem;
    uint4 *xb = reinterpret_cast<uint4 *>(smem + table_lds_bytes(p.m) + wave * kXbufBytes);

    // table -> LDS, rows padded to kRow bytes
    {
        const uint32_t *tg = reinterpret_cast<const uint32_t *>(p.table);
        const int words = (p.m + 1) * (DFA_ALPHABET / 4);
        for (int i = threadIdx.x; i < words; i += blockDim.x)
            *reinterpret_cast<uint32_t *>(tab + (i >> 6) * kRow + 4 * (i & 63)) = tg[i];
    }
    __syncthreads();

    const int64_t g0 = (int64_t(blockIdx.x) * nwaves + wave) * (kWave * K);
    const uint32_t m = uint32_t(p.m);

    // per-lane walk bookkeeping
    int64_t walk_len[K], pos0[K], off[K];
    uint32_t q[K], cnt[K];
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
        walk_len[s] = len;
        pos0[s] = start;
        q[s] = 0;
        cnt[s] = 0;
        off[s] = 0;
        if (MODE == kPositions) {
            const bool has = g < p.nwalks && p.walk_count[g] != 0;
            if (has) off[s] = p.walk_off[g];
            any_work |= has;
        }
    }
    if (MODE == kPositions && __ballot(any_work) == 0) return;  // no match in this wave's spans

    // whole wave in bounds: every load of every round lies inside the text
    const int64_t glast = g0 + kWave * K - 1;
    const bool full = glast < p.nwalks && glast * p.S + int64_t(p.rounds) * kLine <= p.n;
    const int lastlen = int(p.S + p.m - 1 - int64_t(p.rounds - 1) * kLine);  // bytes walked in the last round

    uint4 pf[K][kUnits];
    uint4 t[K][kUnits];
    uint32_t acc = 0;
    int llim[K];

    if (full) {
#pragma unroll
        for (int s = 0; s < K; ++s) llim[s] = 0;
        fetch_round<K, false>(pf, p, g0, lane, 0);
        // every round but the last: all 128 bytes belong to the walk
        for (int r = 0; r + 1 < p.rounds; ++r) {
            transpose_round<K>(t, pf, xb, lane);
            fetch_round<K, false>(pf, p, g0, lane, r + 1);
            walk_round<K, MODE, kNoGuard>(t, q, tab, m, 0, llim, acc, cnt, off, pos0, p);
#pragma unroll
            for (int s = 0; s < K; ++s) pos0[s] += kLine;
        }
        // last round: the walk ends after `lastlen` bytes
        transpose_round<K>(t, pf, xb, lane);
        walk_round<K, MODE, kWaveLimit>(t, q, tab, m, lastlen, llim, acc, cnt, off, pos0, p);
    } else {
        fetch_round<K, true>(pf, p, g0, lane, 0);
        for (int r = 0; r < p.rounds; ++r) {
            transpose_round<K>(t, pf, xb, lane);
            if (r + 1 < p.rounds) fetch_round<K, true>(pf, p, g0, lane, r + 1);
#pragma unroll
            for (int s = 0; s < K; ++s) {
                const int64_t rem = walk_len[s] - int64_t(r) * kLine;
                llim[s] = rem <= 0 ? 0 : (rem >= kLine ? kLine : int(rem));
            }
            walk_round<K, MODE, kLaneLimit>(t, q, tab, m, 0, llim, acc, cnt, off, pos0, p);
#pragma unroll
            for (int s = 0; s < K; ++s) pos0[s] += kLine;
        }
    }

    if (MODE == kPositions) return;

    if (MODE == kCountPerWalk) {
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int64_t g = g0 + s * kWave + lane;
            if (g < p.nwalks) p.walk_count[g] = cnt[s];
            unsigned long long v = cnt[s];
            // wave sum of the per-lane counts
            for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d);
            acc += uint32_t(v);
        }
    }
    // workgroup sum in LDS (reusing this wave's transpose buffer), one atomic
    unsigned long long *red = reinterpret_cast<unsigned long long *>(smem + table_lds_bytes(p.m));
    __syncthreads();
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int w = 0; w < nwaves; ++w) sum += red[w];
        if (sum) atomicAdd(p.total, sum);
    }
}

// ---------------------------------------------------------------------------
// Small helper kernels: zero the count, prefix-sum the per-walk counts.
// ---------------------------------------------------------------------------

__global__ void k_zero_u64(unsigned long long *x) { *x = 0; }

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 16;
constexpr int kScanBlock = kScanThreads * kScanPerThread;

// exclusive scan over the block's threads (in place on `v`), returns the block total
__device__ unsigned long long block_exclusive_scan(unsigned long long &v) {
    __shared__ unsigned long long sh[kScanThreads];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        unsigned long long add = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const unsigned long long incl = sh[threadIdx.x];
    const unsigned long long total = sh[kScanThreads - 1];
    __syncthreads();
    v = incl - v;
    return total;
}

__global__ __launch_bounds__(kScanThreads) void k_walk_sums(const uint32_t *cnt, int64_t nw,
                                                            unsigned long long *part) {
    const int64_t base = int64_t(blockIdx.x) * kScanBlock + threadIdx.x * kScanPerThread;
    unsigned long long v = 0;
    for (int i = 0; i < kScanPerThread; ++i)
        if (base + i < nw) v += cnt[base + i];
    unsigned long long total = block_exclusive_scan(v);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// one block: exclusive scan of the nb block totals; total match count to *count
__global__ __launch_bounds__(kScanThreads) void k_scan_parts(unsigned long long *part, int64_t nb,
                                                             int64_t *count) {
    unsigned long long carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        unsigned long long v = i < nb ? part[i] : 0;
        unsigned long long tot = block_exclusive_scan(v);
        if (i < nb) part[i] = v + carry;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = int64_t(carry);
}

__global__ __launch_bounds__(kScanThreads) void k_walk_offsets(const uint32_t *cnt, int64_t nw,
                                                               const unsigned long long *part,
                                                               int64_t *off) {
    const int64_t base = int64_t(blockIdx.x) * kScanBlock + threadIdx.x * kScanPerThread;
    unsigned long long v = 0;
    for (int i = 0; i < kScanPerThread; ++i)
        if (base + i < nw) v += cnt[base + i];
    block_exclusive_scan(v);
    unsigned long long run = part[blockIdx.x] + v;
    for (int i = 0; i < kScanPerThread; ++i)
        if (base + i < nw) {
            off[base + i] = int64_t(run);
            run += cnt[base + i];
        }
}

// ---------------------------------------------------------------------------
// Host side: planning and the C ABI
// ---------------------------------------------------------------------------

struct Plan {
    int64_t S = 0;
    int K = 2;
    int wpg = 4;
    int rounds = 0;
    int64_t nwalks = 0;
    int64_t blocks = 0;
    size_t lds = 0;
};

template <int K, int MODE>
const void *scan_fn() {
    return reinterpret_cast<const void *>(&k_scan<K, MODE>);
}

const void *pick_scan(int K, int mode) {
    if (K == 1) {
        if (mode == kCount) return scan_fn<1, kCount>();
        if (mode == kCountPerWalk) return scan_fn<1, kCountPerWalk>();
        return scan_fn<1, kPositions>();
    }
    if (mode == kCount) return scan_fn<2, kCount>();
    if (mode == kCountPerWalk) return scan_fn<2, kCountPerWalk>();
    return scan_fn<2, kPositions>();
}

size_t scan_lds_bytes(int wpg, int m) {
    return size_t(wpg) * kXbufBytes + size_t(table_lds_bytes(m));
}

struct DevInfo {
    int cus = 0;
};

int device_cus() {
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    std::lock_guard<std::mutex> lk(mu);
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        cache[dev] = v;
    }
    return cache[dev];
}

int64_t min_span(const dfa_tune *t) {
    return (t && t->chain_bytes > 0) ? t->chain_bytes : dfa::kMinChainBytes;
}

bool check_tune(const dfa_tune *t) {
    if (!t) return true;
    if (t->chain_bytes < 0 || (t->chain_bytes % 16) != 0 || (t->chain_bytes > 0 && t->chain_bytes < 16)) {
        dfa::set_error("tune.chain_bytes=%lld must be a positive multiple of 16 (or 0)",
                       (long long)t->chain_bytes);
        return false;
    }
    if (t->chain_bytes > (int64_t(1) << 30)) {
        dfa::set_error("tune.chain_bytes=%lld too large", (long long)t->chain_bytes);
        return false;
    }
    if (t->waves_per_group < 0 || t->waves_per_group > 4) {
        dfa::set_error("tune.waves_per_group=%d outside [1, 4]", t->waves_per_group);
        return false;
    }
    if (t->chains_per_lane < 0 || t->chains_per_lane > 2) {
        dfa::set_error("tune.chains_per_lane=%d outside [1, 2]", t->chains_per_lane);
        return false;
    }
    for (int i = 0; i < 4; ++i)
        if (t->reserved[i]) {
            dfa::set_error("tune.reserved must be zero");
            return false;
        }
    return true;
}

// Upper bound on the number of walks for any plan of (n, tune): used to size
// the workspace without a device query.
int64_t max_walks(int64_t n, const dfa_tune *t) { return n > 0 ? dfa::ceil_div(n, min_span(t)) : 0; }

int64_t workspace_for(int64_t nw) {
    if (nw <= 0) return 0;
    const int64_t nb = dfa::ceil_div(nw, kScanBlock);
    return dfa::round_up(nw * 4, 256) + dfa::round_up(nw * 8, 256) + dfa::round_up(nb * 8, 256);
}

bool make_plan(int64_t n, int m, int mode, const dfa_tune *t, Plan &pl) {
    pl.K = (t && t->chains_per_lane) ? t->chains_per_lane : 2;
    pl.wpg = (t && t->waves_per_group) ? t->waves_per_group : 4;
    pl.lds = scan_lds_bytes(pl.wpg, m);
    if (t && t->chain_bytes > 0) {
        pl.S = t->chain_bytes;
    } else {
        // one resident wave per group of 64*K walks: size the spans so that the
        // whole text is covered by the walks that fit on the device at once
        int cus = device_cus();
        if (cus <= 0) {
            dfa::set_error("no HIP device");
            return false;
        }
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pick_scan(pl.K, mode), pl.wpg * kWave,
                                                         pl.lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        const int64_t resident = int64_t(cus) * per_cu * pl.wpg * kWave * pl.K;
        pl.S = dfa::round_up(dfa::ceil_div(n, resident), 16);
        if (pl.S < dfa::kMinChainBytes) pl.S = dfa::kMinChainBytes;
    }
    pl.rounds = int(dfa::ceil_div(pl.S + m - 1, kLine));
    pl.nwalks = n > 0 ? dfa::ceil_div(n, pl.S) : 0;
    const int64_t walks_per_block = int64_t(pl.wpg) * kWave * pl.K;
    pl.blocks = dfa::ceil_div(pl.nwalks, walks_per_block);
    return true;
}

bool hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    dfa::set_error("%s: %s", what, hipGetErrorString(e));
    return false;
}

int launch_scan(const Plan &pl, int mode, const ScanParams &sp, hipStream_t st) {
    const void *fn = pick_scan(pl.K, mode);
    static std::mutex mu;
    {
        std::lock_guard<std::mutex> lk(mu);
        // allow the largest table (m = 255) with the largest workgroup
        if (!hip_ok(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        int(scan_lds_bytes(4, DFA_MAX_M))),
                    "hipFuncSetAttribute"))
            return DFA_EHIP;
    }
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

    // workspace: per-walk counts | per-walk offsets | block partials
    uint8_t *ws = reinterpret_cast<uint8_t *>(workspace);
    const int64_t nw = pl.nwalks;
    const int64_t nb = dfa::ceil_div(nw, kScanBlock);
    uint32_t *wcnt = reinterpret_cast<uint32_t *>(ws);
    int64_t *woff = reinterpret_cast<int64_t *>(ws + dfa::round_up(nw * 4, 256));
    unsigned long long *part =
        reinterpret_cast<unsigned long long *>(ws + dfa::round_up(nw * 4, 256) + dfa::round_up(nw * 8, 256));

    sp.walk_count = wcnt;
    int rc = launch_scan(pl, kCountPerWalk, sp, st);
    if (rc != DFA_OK) return rc;
    hipLaunchKernelGGL(k_walk_sums, dim3(unsigned(nb)), dim3(kScanThreads), 0, st, wcnt, nw, part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kScanThreads), 0, st, part, nb, count);
    hipLaunchKernelGGL(k_walk_offsets, dim3(unsigned(nb)), dim3(kScanThreads), 0, st, wcnt, nw,
                       (const unsigned long long *)part, woff);
    if (!hip_ok(hipGetLastError(), "prefix-sum launch")) return DFA_EHIP;
    sp.walk_off = woff;
    sp.positions = positions;
    rc = launch_scan(pl, kPositions, sp, st);
    if (rc == DFA_OK) dfa::clear_error();
    return rc;
}
