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
// far back, so the text is cut into 64 KiB chunks and processed in three
// passes:
//   A  per chunk: its last line start (with whether that line is a header),
//      its header count, and its kept bytes -- those before its first line
//      start counted apart, as their line began in an earlier chunk;
//   B  one workgroup: the line each chunk starts in (the last line start of
//      all earlier chunks), hence its kept bytes, and the chunk's output and
//      record offsets (prefix sums);
//   C  per chunk again: the kept bytes written, compacted, at their offsets,
//      and the record starts.
// A line start s is carried as 2 s + (byte s is '>'), so that one prefix max
// over line starts gives both where the current line began and whether it is
// a header, with no load of that byte.  Within a chunk a workgroup of 256
// threads takes 4 KiB per round, 16 bytes per thread (four dword loads;
// consecutive threads read consecutive 16-byte pieces, and the byte before a
// wave's first piece comes with them); per round one block scan carries the
// line start (prefix max) and one the kept and header counts (prefix sums,
// packed in 64 bits).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dfa.h"
#include "dfa_internal.h"
#include "launch_util.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaveSize = 64;
constexpr int kPer = 16;                 // bytes per thread per round
constexpr int kRound = kThreads * kPer;  // bytes per round
constexpr int64_t kChunk = 64 * 1024;    // bytes per workgroup
constexpr int kPlanThreads = 1024;

struct ChunkSummary {
    int64_t last_ls;     // last line start in the chunk, as 2 s + header, or -1
    uint32_t pre;        // bytes before its first line start that a sequence line would keep
    uint32_t kept;       // kept bytes from its first line start on
    uint32_t headers;    // header lines starting in the chunk
    uint32_t pad;
};

struct ChunkPlan {
    int64_t ls_before;   // last line start before the chunk (2 s + header), or -1
    int64_t out_off;     // kept bytes before the chunk
    int64_t rec_off;     // records before the chunk
};

constexpr uint32_t kNl = '\n', kCr = '\r', kGt = '>';

__device__ __forceinline__ int64_t wave_incl_max(int64_t v) {
    const int lane = threadIdx.x & (kWaveSize - 1);
#pragma unroll
    for (int d = 1; d < kWaveSize; d <<= 1) {
        const int64_t u = __shfl_up(v, d);
        if (lane >= d) v = u > v ? u : v;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_incl_sum(unsigned long long v) {
    const int lane = threadIdx.x & (kWaveSize - 1);
#pragma unroll
    for (int d = 1; d < kWaveSize; d <<= 1) {
        const unsigned long long u = __shfl_up(v, d);
        if (lane >= d) v += u;
    }
    return v;
}

// exclusive prefix max over the block (any multiple of 64 threads up to
// 1024), seeded with `carry`; *all = block max (and carry)
__device__ __forceinline__ int64_t block_excl_max(int64_t v, int64_t carry, int64_t *sh, int64_t *all) {
    const int lane = threadIdx.x & (kWaveSize - 1), w = threadIdx.x / kWaveSize;
    const int nw = blockDim.x / kWaveSize;
    const int64_t inc = wave_incl_max(v);
    int64_t ex = __shfl_up(inc, 1);
    if (lane == 0) ex = -1;
    if (lane == kWaveSize - 1) sh[w] = inc;
    __syncthreads();
    int64_t before = carry, tot = carry;
    for (int i = 0; i < nw; ++i) {
        if (i < w) before = sh[i] > before ? sh[i] : before;
        tot = sh[i] > tot ? sh[i] : tot;
    }
    __syncthreads();
    *all = tot;
    return ex > before ? ex : before;
}

// exclusive prefix sum over the block (any multiple of 64 threads up to 1024);
// *all = block total
__device__ __forceinline__ unsigned long long block_excl_sum(unsigned long long v, unsigned long long *sh,
                                                             unsigned long long *all) {
    const int lane = threadIdx.x & (kWaveSize - 1), w = threadIdx.x / kWaveSize;
    const int nw = blockDim.x / kWaveSize;
    const unsigned long long inc = wave_incl_sum(v);
    if (lane == kWaveSize - 1) sh[w] = inc;
    __syncthreads();
    unsigned long long before = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) before += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *all = tot;
    return before + inc - v;
}

// The thread's kPer bytes of a round (positions p .. p+kPer-1; p is a multiple
// of 4, raw 4-byte aligned), bytes at or past n absent (value 0x100), and
// whether a line starts at each of them: at position 0, or after a '\n' (the
// byte before the piece comes from the previous lane, or from memory for a
// wave's first lane).
__device__ __forceinline__ uint32_t load_piece(const uint8_t *raw, int64_t n, int64_t p, uint32_t (&b)[kPer]) {
    const int lane = threadIdx.x & (kWaveSize - 1);
    const uint32_t mem_before = lane == 0 ? (p == 0 ? kNl : (p - 1 < n ? uint32_t(raw[p - 1]) : 0x100u)) : 0u;
    if (p + kPer <= n) {
#pragma unroll
        for (int q = 0; q < kPer / 4; ++q) {
            const uint32_t w = *reinterpret_cast<const uint32_t *>(raw + p + 4 * q);
#pragma unroll
            for (int j = 0; j < 4; ++j) b[4 * q + j] = (w >> (8 * j)) & 0xffu;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kPer; ++j) b[j] = p + j < n ? raw[p + j] : 0x100u;
    }
    uint32_t before = uint32_t(__shfl_up(int(b[kPer - 1]), 1));
    if (lane == 0) before = mem_before;
    uint32_t starts = 0;  // bit j: a line starts at p + j
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const uint32_t prev = j ? b[j - 1] : before;
        if (prev == kNl && b[j] <= 0xffu) starts |= 1u << j;
    }
    return starts;
}

// The last line start among the piece's bytes (2 s + header), or -1.
__device__ __forceinline__ int64_t last_start(int64_t p, const uint32_t (&b)[kPer], uint32_t starts) {
    if (!starts) return -1;
    const int j = 31 - __clz(starts);
    int64_t v = -1;
#pragma unroll
    for (int k = 0; k < kPer; ++k)
        if (k == j) v = 2 * (p + k) + (b[k] == kGt ? 1 : 0);
    return v;
}

// Pass A
__global__ __launch_bounds__(kThreads) void k_fasta_summary(const uint8_t *raw, int64_t n, ChunkSummary *sum) {
    __shared__ int64_t shm[kThreads / kWaveSize];
    __shared__ unsigned long long shs[kThreads / kWaveSize];
    const int64_t c0 = int64_t(blockIdx.x) * kChunk;
    const int64_t c1 = c0 + kChunk < n ? c0 + kChunk : n;
    int64_t carry = -1;  // last line start inside the chunk so far
    unsigned long long pre = 0, kept = 0, headers = 0;
    for (int64_t r0 = c0; r0 < c1; r0 += kRound) {
        const int64_t p = r0 + kPer * int64_t(threadIdx.x);
        uint32_t b[kPer];
        const uint32_t starts = load_piece(raw, c1, p, b);
        int64_t all;
        int64_t cur = block_excl_max(last_start(p, b, starts), carry, shm, &all);
        carry = all;
        // pre, kept and header counts of the thread, packed 21 bits apart (each < 2^21)
        unsigned long long packed = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t x = b[j];
            if (x > 0xffu) continue;
            if ((starts >> j) & 1u) {
                cur = 2 * (p + j) + (x == kGt ? 1 : 0);
                if (x == kGt) ++packed;
            }
            if (x == kNl || x == kCr) continue;
            if (cur < 0)
                packed += 1ull << 42;
            else if (!(cur & 1))
                packed += 1ull << 21;
        }
        unsigned long long t;
        block_excl_sum(packed, shs, &t);
        pre += t >> 42;
        kept += (t >> 21) & 0x1fffffu;
        headers += t & 0x1fffffu;
    }
    if (threadIdx.x == 0) {
        ChunkSummary s;
        s.last_ls = carry;
        s.pre = uint32_t(pre);
        s.kept = uint32_t(kept);
        s.headers = uint32_t(headers);
        s.pad = 0;
        sum[blockIdx.x] = s;
    }
}

// Pass B: one workgroup of kPlanThreads, each thread a run of consecutive
// chunks: the last line start before each chunk (prefix max), then its kept
// bytes and the output and record offsets (prefix sums).
__global__ __launch_bounds__(kPlanThreads) void k_fasta_plan(const ChunkSummary *sum, int64_t nchunks,
                                                             ChunkPlan *plan, int64_t *totals) {
    __shared__ int64_t shm[kPlanThreads / kWaveSize];
    __shared__ unsigned long long shs[kPlanThreads / kWaveSize];
    const int64_t per = (nchunks + kPlanThreads - 1) / kPlanThreads;
    const int64_t i0 = int64_t(threadIdx.x) * per, i1 = i0 + per < nchunks ? i0 + per : nchunks;
    int64_t run_max = -1;
    for (int64_t c = i0; c < i1; ++c) run_max = sum[c].last_ls > run_max ? sum[c].last_ls : run_max;
    int64_t all;
    const int64_t before0 = block_excl_max(run_max, -1, shm, &all);
    // the kept bytes and records of the run
    unsigned long long kept = 0, recs = 0;
    int64_t before = before0;
    for (int64_t c = i0; c < i1; ++c) {
        const ChunkSummary s = sum[c];
        kept += (before >= 0 && (before & 1) ? 0ull : s.pre) + s.kept;
        recs += s.headers;
        before = s.last_ls > before ? s.last_ls : before;
    }
    unsigned long long tk, tr;
    unsigned long long out = block_excl_sum(kept, shs, &tk);
    unsigned long long rec = block_excl_sum(recs, shs, &tr);
    before = before0;
    for (int64_t c = i0; c < i1; ++c) {
        const ChunkSummary s = sum[c];
        ChunkPlan cp;
        cp.ls_before = before;
        cp.out_off = int64_t(out);
        cp.rec_off = int64_t(rec);
        plan[c] = cp;
        out += (before >= 0 && (before & 1) ? 0ull : s.pre) + s.kept;
        rec += s.headers;
        before = s.last_ls > before ? s.last_ls : before;
    }
    if (threadIdx.x == 0) {
        totals[0] = int64_t(tk);
        totals[1] = int64_t(tr);
    }
}

// Pass C
__global__ __launch_bounds__(kThreads) void k_fasta_write(const uint8_t *raw, int64_t n, const ChunkPlan *plan,
                                                          uint8_t *out, int64_t *rec_start, int64_t rec_cap) {
    __shared__ int64_t shm[kThreads / kWaveSize];
    __shared__ unsigned long long shs[kThreads / kWaveSize];
    const int64_t c0 = int64_t(blockIdx.x) * kChunk;
    const int64_t c1 = c0 + kChunk < n ? c0 + kChunk : n;
    const ChunkPlan cp = plan[blockIdx.x];
    int64_t carry = cp.ls_before;
    int64_t o = cp.out_off;
    int64_t rec = cp.rec_off;
    for (int64_t r0 = c0; r0 < c1; r0 += kRound) {
        const int64_t p = r0 + kPer * int64_t(threadIdx.x);
        uint32_t b[kPer];
        const uint32_t starts = load_piece(raw, c1, p, b);
        int64_t all;
        const int64_t cur0 = block_excl_max(last_start(p, b, starts), carry, shm, &all);
        carry = all;
        // kept bytes and header starts of the thread, packed as (kept << 32) | headers
        int64_t cur = cur0;
        unsigned long long packed = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t x = b[j];
            if (x > 0xffu) continue;
            if ((starts >> j) & 1u) {
                cur = 2 * (p + j) + (x == kGt ? 1 : 0);
                if (x == kGt) ++packed;
            }
            if (x != kNl && x != kCr && !(cur & 1)) packed += 1ull << 32;
        }
        unsigned long long tot;
        const unsigned long long ex = block_excl_sum(packed, shs, &tot);
        int64_t w = o + int64_t(ex >> 32);
        int64_t h = rec + int64_t(ex & 0xffffffffu);
        cur = cur0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t x = b[j];
            if (x > 0xffu) continue;
            if ((starts >> j) & 1u) {
                cur = 2 * (p + j) + (x == kGt ? 1 : 0);
                if (x == kGt) {
                    if (h < rec_cap) rec_start[h] = w;
                    ++h;
                }
            }
            if (x != kNl && x != kCr && !(cur & 1)) out[w++] = uint8_t(x - 'a' < 26u ? x - 0x20u : x);
        }
        o += int64_t(tot >> 32);
        rec += int64_t(tot & 0xffffffffu);
    }
}

using dfa::hip_ok;

int64_t nchunks_of(int64_t n) { return n > 0 ? dfa::ceil_div(n, kChunk) : 0; }

}  // namespace

extern "C" int64_t dfa_fasta_workspace_bytes(int64_t n) {
    if (n < 0) {
        dfa::set_error("dfa_fasta_workspace_bytes: n < 0");
        return DFA_EINVAL;
    }
    const int64_t c = nchunks_of(n);
    return dfa::round_up(c * int64_t(sizeof(ChunkSummary)), 256) + dfa::round_up(c * int64_t(sizeof(ChunkPlan)), 256);
}

extern "C" int dfa_fasta_normalize(const uint8_t *raw, int64_t n, uint8_t *out, int64_t *rec_start, int64_t rec_cap,
                                   int64_t *totals, void *workspace, int64_t workspace_bytes, void *stream) {
    if (n < 0 || (n > 0 && (!raw || !out)) || !totals || rec_cap < 0 || (rec_cap > 0 && !rec_start)) {
        dfa::set_error("dfa_fasta_normalize: null argument or negative size");
        return DFA_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(raw) & 3) || (reinterpret_cast<uintptr_t>(totals) & 7) ||
        (reinterpret_cast<uintptr_t>(rec_start) & 7)) {
        dfa::set_error("dfa_fasta_normalize: raw must be 4-byte, totals and rec_start 8-byte aligned");
        return DFA_EINVAL;
    }
    const int64_t need = dfa_fasta_workspace_bytes(n);
    if (need > 0 && (!workspace || workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255))) {
        dfa::set_error("dfa_fasta_normalize: workspace of %lld bytes (256-aligned) needed, got %lld", (long long)need,
                       (long long)workspace_bytes);
        return DFA_ENOSPACE;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t c = nchunks_of(n);
    if (c > 0x7fffffff) {
        dfa::set_error("dfa_fasta_normalize: text too large");
        return DFA_EINVAL;
    }
    uint8_t *ws = reinterpret_cast<uint8_t *>(workspace);
    ChunkSummary *sum = reinterpret_cast<ChunkSummary *>(ws);
    ChunkPlan *plan = reinterpret_cast<ChunkPlan *>(ws + dfa::round_up(c * int64_t(sizeof(ChunkSummary)), 256));
    if (c > 0) hipLaunchKernelGGL(k_fasta_summary, dim3(unsigned(c)), dim3(kThreads), 0, st, raw, n, sum);
    hipLaunchKernelGGL(k_fasta_plan, dim3(1), dim3(kPlanThreads), 0, st, (const ChunkSummary *)sum, c, plan, totals);
    if (c > 0)
        hipLaunchKernelGGL(k_fasta_write, dim3(unsigned(c)), dim3(kThreads), 0, st, raw, n, (const ChunkPlan *)plan,
                           out, rec_start, rec_cap);
    if (!hip_ok(hipGetLastError(), "fasta launch")) return DFA_EHIP;
    dfa::clear_error();
    return DFA_OK;
}
