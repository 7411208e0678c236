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
//   A  per chunk: its last newline, its header starts, and its kept bytes --
//      those before its first newline counted apart, as their line may have
//      started in an earlier chunk;
//   B  one workgroup: the line each chunk starts in (the last newline of all
//      earlier chunks), hence its kept bytes, and the chunk's output and
//      record offsets (prefix sums);
//   C  per chunk again: the kept bytes written, compacted, at their offsets,
//      and the record starts.
// Within a chunk a workgroup of 256 threads takes 1 KiB per round, 4 bytes
// per thread (one coalesced dword load); block scans carry the last newline
// (prefix max) and the kept and header counts (prefix sums) across threads.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dfa.h"
#include "dfa_internal.h"
#include "launch_util.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaveSize = 64;
constexpr int kRound = kThreads * 4;  // bytes per round
constexpr int64_t kChunk = 64 * 1024;  // bytes per workgroup

struct ChunkSummary {
    int64_t last_nl;     // position of the chunk's last '\n', or -1
    uint32_t pre;        // bytes before its first '\n' that would be kept in a sequence line
    uint32_t kept;       // kept bytes after its first '\n'
    uint32_t headers;    // header lines starting in the chunk
    uint32_t pad;
};

struct ChunkPlan {
    int64_t nl_before;   // last '\n' before the chunk, or -1
    int64_t out_off;     // kept bytes before the chunk
    int64_t rec_off;     // records before the chunk
};

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

// exclusive prefix max over the block, seeded with `carry`; *all = block max (and carry)
__device__ __forceinline__ int64_t block_excl_max(int64_t v, int64_t carry, int64_t *sh, int64_t *all) {
    const int lane = threadIdx.x & (kWaveSize - 1), w = threadIdx.x / kWaveSize;
    const int64_t inc = wave_incl_max(v);
    int64_t ex = __shfl_up(inc, 1);
    if (lane == 0) ex = -1;
    if (lane == kWaveSize - 1) sh[w] = inc;
    __syncthreads();
    int64_t before = carry, tot = carry;
#pragma unroll
    for (int i = 0; i < kThreads / kWaveSize; ++i) {
        if (i < w) before = sh[i] > before ? sh[i] : before;
        tot = sh[i] > tot ? sh[i] : tot;
    }
    __syncthreads();
    *all = tot;
    return ex > before ? ex : before;
}

// exclusive prefix sum over the block; *all = block total
__device__ __forceinline__ unsigned long long block_excl_sum(unsigned long long v, unsigned long long *sh,
                                                             unsigned long long *all) {
    const int lane = threadIdx.x & (kWaveSize - 1), w = threadIdx.x / kWaveSize;
    const unsigned long long inc = wave_incl_sum(v);
    if (lane == kWaveSize - 1) sh[w] = inc;
    __syncthreads();
    unsigned long long before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kThreads / kWaveSize; ++i) {
        if (i < w) before += sh[i];
        tot += sh[i];
    }
    __syncthreads();
    *all = tot;
    return before + inc - v;
}

// The thread's 4 bytes of a round (positions p .. p+3); bytes at or past n are
// absent (value 0x100).
__device__ __forceinline__ void load4(const uint8_t *raw, int64_t n, int64_t p, uint32_t (&b)[4]) {
    if (p + 4 <= n) {
        const uint32_t w = *reinterpret_cast<const uint32_t *>(raw + p);
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = (w >> (8 * j)) & 0xffu;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = p + j < n ? raw[p + j] : 0x100u;
    }
}

constexpr uint32_t kNl = '\n', kCr = '\r', kGt = '>';

// Is the byte before position p a newline (or p the start of the text)?
__device__ __forceinline__ bool line_starts_at(const uint8_t *raw, int64_t p, const uint32_t (&b)[4], int j) {
    if (j > 0) return b[j - 1] == kNl;
    return p == 0 || raw[p - 1] == kNl;
}

// Pass A
__global__ __launch_bounds__(kThreads) void k_fasta_summary(const uint8_t *raw, int64_t n, ChunkSummary *sum) {
    __shared__ int64_t shm[kThreads / kWaveSize];
    __shared__ unsigned long long shs[kThreads / kWaveSize];
    const int64_t c0 = int64_t(blockIdx.x) * kChunk;
    const int64_t c1 = c0 + kChunk < n ? c0 + kChunk : n;
    int64_t carry_nl = -1;  // last '\n' inside the chunk so far
    unsigned long long pre = 0, kept = 0, headers = 0;
    for (int64_t r0 = c0; r0 < c1; r0 += kRound) {
        const int64_t p = r0 + 4 * int64_t(threadIdx.x);
        uint32_t b[4];
        load4(raw, c1, p, b);
        int64_t mine = -1;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (b[j] == kNl) mine = p + j;
        int64_t all;
        int64_t nl = block_excl_max(mine, carry_nl, shm, &all);
        carry_nl = all;
        // the line state at the thread's first byte, when its line starts inside the chunk
        bool hdr = nl >= 0 && nl + 1 < c1 && raw[nl + 1] == kGt;
        unsigned long long my_pre = 0, my_kept = 0, my_hdr = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t x = b[j];
            if (x > 0xffu) continue;
            if (x == kGt && line_starts_at(raw, p + j, b, j)) ++my_hdr;
            if (x == kNl) {
                nl = p + j;
                hdr = j + 1 < 4 ? b[j + 1] == kGt : (p + 4 < c1 && raw[p + 4] == kGt);
                continue;
            }
            if (x == kCr) continue;
            if (nl < 0)
                ++my_pre;
            else if (!hdr)
                ++my_kept;
        }
        unsigned long long t;
        block_excl_sum(my_pre, shs, &t);
        pre += t;
        block_excl_sum(my_kept, shs, &t);
        kept += t;
        block_excl_sum(my_hdr, shs, &t);
        headers += t;
    }
    if (threadIdx.x == 0) {
        ChunkSummary s;
        s.last_nl = carry_nl;
        s.pre = uint32_t(pre);
        s.kept = uint32_t(kept);
        s.headers = uint32_t(headers);
        s.pad = 0;
        sum[blockIdx.x] = s;
    }
}

// Pass B: one workgroup over all chunks
__global__ __launch_bounds__(kThreads) void k_fasta_plan(const uint8_t *raw, int64_t n, const ChunkSummary *sum,
                                                         int64_t nchunks, ChunkPlan *plan, int64_t *totals) {
    __shared__ int64_t shm[kThreads / kWaveSize];
    __shared__ unsigned long long shs[kThreads / kWaveSize];
    int64_t carry_nl = -1;
    unsigned long long out = 0, rec = 0;
    for (int64_t base = 0; base < nchunks; base += kThreads) {
        const int64_t c = base + threadIdx.x;
        const bool ok = c < nchunks;
        const ChunkSummary s = ok ? sum[c] : ChunkSummary{-1, 0, 0, 0, 0};
        int64_t all;
        const int64_t before = block_excl_max(s.last_nl, carry_nl, shm, &all);
        carry_nl = all;
        // the line the chunk starts in begins right after `before`
        const int64_t ls = before + 1;
        const bool hdr = ok && ls < n && raw[ls] == kGt;
        const unsigned long long kept = ok ? (hdr ? 0ull : s.pre) + s.kept : 0ull;
        unsigned long long tk, th;
        const unsigned long long ok_off = block_excl_sum(kept, shs, &tk);
        const unsigned long long rec_off = block_excl_sum(ok ? s.headers : 0u, shs, &th);
        if (ok) {
            ChunkPlan cp;
            cp.nl_before = before;
            cp.out_off = int64_t(out + ok_off);
            cp.rec_off = int64_t(rec + rec_off);
            plan[c] = cp;
        }
        out += tk;
        rec += th;
    }
    if (threadIdx.x == 0) {
        totals[0] = int64_t(out);
        totals[1] = int64_t(rec);
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
    int64_t carry_nl = cp.nl_before;
    int64_t o = cp.out_off;
    int64_t rec = cp.rec_off;
    for (int64_t r0 = c0; r0 < c1; r0 += kRound) {
        const int64_t p = r0 + 4 * int64_t(threadIdx.x);
        uint32_t b[4];
        load4(raw, c1, p, b);
        int64_t mine = -1;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (b[j] == kNl) mine = p + j;
        int64_t all;
        int64_t nl = block_excl_max(mine, carry_nl, shm, &all);
        carry_nl = all;
        const bool hdr0 = nl + 1 < n && raw[nl + 1] == kGt;
        // kept bytes and header starts of the thread, packed as (kept << 32) | headers
        bool hdr = hdr0;
        unsigned long long packed = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t x = b[j];
            if (x > 0xffu) continue;
            if (x == kGt && line_starts_at(raw, p + j, b, j)) ++packed;
            if (x == kNl) {
                hdr = j + 1 < 4 ? b[j + 1] == kGt : (p + 4 < n && raw[p + 4] == kGt);
                continue;
            }
            if (x != kCr && !hdr) packed += 1ull << 32;
        }
        unsigned long long tot;
        const unsigned long long ex = block_excl_sum(packed, shs, &tot);
        int64_t w = o + int64_t(ex >> 32);
        int64_t h = rec + int64_t(ex & 0xffffffffu);
        hdr = hdr0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t x = b[j];
            if (x > 0xffu) continue;
            if (x == kGt && line_starts_at(raw, p + j, b, j)) {
                if (h < rec_cap) rec_start[h] = w;
                ++h;
            }
            if (x == kNl) {
                hdr = j + 1 < 4 ? b[j + 1] == kGt : (p + 4 < n && raw[p + 4] == kGt);
                continue;
            }
            if (x != kCr && !hdr) out[w++] = uint8_t(x - 'a' < 26u ? x - 0x20u : x);
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
    hipLaunchKernelGGL(k_fasta_plan, dim3(1), dim3(kThreads), 0, st, raw, n, (const ChunkSummary *)sum, c, plan,
                       totals);
    if (c > 0)
        hipLaunchKernelGGL(k_fasta_write, dim3(unsigned(c)), dim3(kThreads), 0, st, raw, n, (const ChunkPlan *)plan,
                           out, rec_start, rec_cap);
    if (!hip_ok(hipGetLastError(), "fasta launch")) return DFA_EHIP;
    dfa::clear_error();
    return DFA_OK;
}
