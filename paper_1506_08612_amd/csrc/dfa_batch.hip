// Batched automaton scans for gfx950: many patterns over many texts in one
// launch.
//
// Texts are segments of one buffer; every (segment, pattern) pair asks for the
// number of occurrences of the pattern inside the segment (a match never spans
// two segments).  The paper's multi-pattern automaton merges equal-length
// patterns and notes that the m-1 overlap of Algorithm 1 is only exact for
// equal lengths (Sec. III.A); here every pattern keeps its own single-pattern
// automaton and its own overlap m_i - 1, which is exact for any mix of
// lengths.
//
// Work decomposition.  The host packs the patterns of each segment into
// groups whose tables fit one LDS row space (at most 256 rows of 256 columns;
// a table's entries are shifted by its first row so that a state is directly
// a row number).  A work item is (one tile of a segment, one group).  Each
// workgroup stages its group's tables in LDS and the tile's text once, and
// every lane walks its own span of the tile with all automata of the group
// interleaved: the automata share the text bytes (one fetch, one transpose)
// and give every lane several independent dependent chains to overlap.  Each
// automaton reads m_i - 1 bytes past the lane's span, clipped at the segment
// end.  Counts are kept per automaton with wave ballots and added to the
// pair's counter with one atomic per workgroup and automaton.
//
// Items are ordered so that consecutive items on the same XCD (workgroups are
// dealt to the 8 XCDs in turn) process the same tile with different groups,
// which keeps the tile in that XCD's L2 while its groups are walked.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "dfa.h"
#include "dfa_internal.h"
#include "launch_util.h"
#include "walk_common.h"

namespace {

using namespace dfa_dev;

constexpr int kLine = 128;          // bytes of every walk fetched per round
constexpr int kMaxRows = 256;       // rows of one group's shared row space (states fit a byte)
constexpr int kNullRow = kMaxRows - 1;  // self-looping row of the padding automata; never final
constexpr int kMaxGroup = 16;       // automata per group, at most
constexpr int kXcds = 8;            // workgroups are dealt to the XCDs in turn
constexpr int64_t kMinSpan = 256;   // shortest walk span the planner uses
constexpr int64_t kMaxSpan = 2048;  // longest

struct DevDfa {
    int64_t table_off;  // byte offset of the (m+1) x 256 table in the tables buffer
    int32_t m;
    int32_t base_row;   // first row of this automaton in the group's row space
    int32_t pair;       // output counter, or -1
    int32_t pad;
};

struct DevGroup {
    int32_t ndfa;  // real automata; slots ndfa.. are padding that sits in kNullRow
    int32_t rows;  // rows used
    int32_t minm, maxm;
    DevDfa dfa[kMaxGroup];
};

struct DevItem {
    int64_t tile_start;  // first byte of the tile (= start of its first walk)
    int64_t own_end;     // match starts owned by the tile end here
    int64_t seg_end;     // no automaton reads past the end of its segment
    int32_t group;
    int32_t span;        // walk span S of this item (multiple of 16)
};

struct BatchParams {
    const uint8_t *text;
    int64_t n;
    const uint8_t *tables;
    const DevGroup *groups;
    const DevItem *items;
    unsigned long long *counts;
};

// Walk 16 bytes with all G automata (padding automata included: a uniform
// branch per automaton would cut the unrolled steps into blocks and lose the
// overlap of the G independent table reads).  Byte b of word w is byte
// jb + 4w + b of the walk; with GUARD only bytes below the automaton's own
// length count.
template <int G, bool GUARD>
__device__ __forceinline__ void walk_unit_multi(const v4u &t, uint32_t (&q)[G], const uint32_t (&fin)[G],
                                                const uint32_t (&len)[G], uint32_t jb, uint32_t (&acc)[G]) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t c = (t[w] >> (8 * b)) & 0xffu;
            // all G table reads of this byte go out before the first count, so
            // G reads are in flight at once
#pragma unroll
            for (int d = 0; d < G; ++d) q[d] = table_step(q[d], c);
            __builtin_amdgcn_sched_barrier(0);  // keep the reads grouped ahead of the counts
#pragma unroll
            for (int d = 0; d < G; ++d) {
                bool hit = q[d] == fin[d];
                if (GUARD) hit = hit && (jb + uint32_t(4 * w + b) < len[d]);
                add_hits(acc[d], hit);
            }
        }
    }
}

template <int G>
__global__ __launch_bounds__(512) void k_batch(BatchParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const DevItem it = p.items[blockIdx.x];
    const DevGroup &gr = p.groups[it.group];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    const int nwaves = blockDim.x / kWave;
    const int ndfa = __builtin_amdgcn_readfirstlane(gr.ndfa);
    const int tab_bytes = table_lds_rows_bytes(kMaxRows);
    v4u *xb = reinterpret_cast<v4u *>(smem + tab_bytes + wave * (kWave * kLine));

    // the group's tables -> LDS: row base_row + q holds state q, and every entry
    // is shifted by base_row so that the next state is directly a row number
    for (int d = 0; d < ndfa; ++d) {
        const DevDfa dd = gr.dfa[d];
        const uint32_t *tg = reinterpret_cast<const uint32_t *>(p.tables + dd.table_off);
        const uint32_t add = uint32_t(dd.base_row) * 0x01010101u;  // no byte carries: entries + base <= 255
        const int words = (dd.m + 1) * (DFA_ALPHABET / 4);
        for (int i = threadIdx.x; i < words; i += blockDim.x)
            *reinterpret_cast<uint32_t *>(smem + (dd.base_row + (i >> 6)) * kRow + 4 * (i & 63)) = tg[i] + add;
    }
    for (int i = threadIdx.x; i < DFA_ALPHABET / 4; i += blockDim.x)  // padding: every byte stays in kNullRow
        *reinterpret_cast<uint32_t *>(smem + kNullRow * kRow + 4 * i) = uint32_t(kNullRow) * 0x01010101u;
    __syncthreads();

    uint32_t q[G], fin[G], len[G], acc[G];
    const int64_t S = it.span;
    const int64_t wbase = it.tile_start + int64_t(wave) * kWave * S;  // the wave's first walk
    const int64_t wstart = wbase + int64_t(lane) * S;
    int64_t own = it.own_end - wstart;
    own = own < 0 ? 0 : (own > S ? S : own);
#pragma unroll
    for (int d = 0; d < G; ++d) {
        const bool real = d < ndfa;
        const int m = real ? gr.dfa[d].m : 1;
        const int base = real ? gr.dfa[d].base_row : kNullRow;
        q[d] = uint32_t(base);
        fin[d] = real ? uint32_t(base + m) : 0x100u;  // no row is 0x100
        int64_t L = 0;
        if (own > 0) {
            L = own + m - 1;
            if (wstart + L > it.seg_end) L = it.seg_end - wstart;
        }
        len[d] = uint32_t(L);
        acc[d] = 0;
    }
    const int maxm = __builtin_amdgcn_readfirstlane(gr.maxm);
    const int minm = __builtin_amdgcn_readfirstlane(gr.minm);
    const int rounds = int((S + maxm - 1 + kLine - 1) / kLine);
    const uint32_t lane_off = uint32_t(lane / Geo<kLine>::U) * uint32_t(S) + 16u * uint32_t(lane % Geo<kLine>::U);

    // every walk of the wave full (own span S, overlap inside the segment) and
    // every load inside the text
    const int64_t wlast = wbase + int64_t(kWave - 1) * S;
    const bool full = wlast + S <= it.own_end && wlast + S + maxm - 1 <= it.seg_end &&
                      wlast + int64_t(rounds) * kLine <= p.n;
    const int safe = int(S) + minm - 1;  // bytes that count for every automaton of a full walk

    v4u pf[1][Geo<kLine>::U];
    if (full) {
        fetch_round<1, kLine, false>(pf, p.text, p.n, wbase, S, lane_off, 0);
        for (int r = 0; r < rounds; ++r) {
            stage_round<1, kLine>(pf, xb, lane);
            if (r + 1 < rounds) fetch_round<1, kLine, false>(pf, p.text, p.n, wbase, S, lane_off, r + 1);
            v4u cur = unit_of<kLine>(xb, 0, lane, 0), nxt = cur;
            for (int u = 0; u < Geo<kLine>::U; ++u) {
                if (u + 1 < Geo<kLine>::U) nxt = unit_of<kLine>(xb, 0, lane, u + 1);
                const int jb = r * kLine + 16 * u;
                if (jb + 16 <= safe)
                    walk_unit_multi<G, false>(cur, q, fin, len, uint32_t(jb), acc);
                else if (jb < int(S) + maxm - 1)
                    walk_unit_multi<G, true>(cur, q, fin, len, uint32_t(jb), acc);
                cur = nxt;
            }
        }
    } else {
        fetch_round<1, kLine, true>(pf, p.text, p.n, wbase, S, lane_off, 0);
        for (int r = 0; r < rounds; ++r) {
            stage_round<1, kLine>(pf, xb, lane);
            if (r + 1 < rounds) fetch_round<1, kLine, true>(pf, p.text, p.n, wbase, S, lane_off, r + 1);
            v4u cur = unit_of<kLine>(xb, 0, lane, 0), nxt = cur;
            for (int u = 0; u < Geo<kLine>::U; ++u) {
                if (u + 1 < Geo<kLine>::U) nxt = unit_of<kLine>(xb, 0, lane, u + 1);
                walk_unit_multi<G, true>(cur, q, fin, len, uint32_t(r * kLine + 16 * u), acc);
                cur = nxt;
            }
        }
    }

    // per automaton: sum the waves in LDS (reusing the transpose buffers), one atomic
    __syncthreads();
    uint32_t *red = reinterpret_cast<uint32_t *>(smem + tab_bytes);
    if (lane == 0) {
#pragma unroll
        for (int d = 0; d < G; ++d) red[d * nwaves + wave] = acc[d];
    }
    __syncthreads();
    if (int(threadIdx.x) < ndfa) {
        const int d = threadIdx.x;
        unsigned long long sum = 0;
        for (int w = 0; w < nwaves; ++w) sum += red[d * nwaves + w];
        const int pair = gr.dfa[d].pair;
        if (sum && pair >= 0) atomicAdd(p.counts + pair, sum);
    }
}

__global__ void k_zero_counts(unsigned long long *c, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        c[i] = 0;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

const void *batch_fn(int G) {
    if (G == 2) return reinterpret_cast<const void *>(&k_batch<2>);
    if (G == 4) return reinterpret_cast<const void *>(&k_batch<4>);
    if (G == 8) return reinterpret_cast<const void *>(&k_batch<8>);
    if (G == 16) return reinterpret_cast<const void *>(&k_batch<16>);
    return nullptr;
}

size_t batch_lds_bytes(int waves) {
    return size_t(table_lds_rows_bytes(kMaxRows)) + size_t(waves) * kWave * kLine;
}

using dfa::hip_ok;

struct HostPlan {
    std::vector<DevGroup> groups;
    std::vector<DevItem> items;
    int G = 8;
    int waves = 8;
    int64_t text_bytes = 0;    // bytes of text the segments span
    int64_t tables_bytes = 0;  // bytes of the tables buffer the referenced tables span
};

int plan_batch(const int64_t *seg_off, int32_t nseg, const int64_t *table_off, const int32_t *m,
               int32_t npat, const int32_t *pair_seg, const int32_t *pair_pat, int64_t npairs,
               const dfa_tune *t, HostPlan &hp) {
    if (nseg < 0 || npat < 0 || npairs < 0 || (nseg > 0 && !seg_off) ||
        (npat > 0 && (!table_off || !m)) || (npairs > 0 && (!pair_seg || !pair_pat))) {
        dfa::set_error("dfa_batch: bad counts or null arrays");
        return DFA_EINVAL;
    }
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
        if (t->dfas_per_group && t->dfas_per_group != 2 && t->dfas_per_group != 4 && t->dfas_per_group != 8 &&
            t->dfas_per_group != 16) {
            dfa::set_error("tune.dfas_per_group=%d must be 2, 4, 8 or 16 (or 0)", t->dfas_per_group);
            return DFA_EINVAL;
        }
        if (t->waves_per_group < 0 || t->waves_per_group > 8) {
            dfa::set_error("tune.waves_per_group=%d outside [1, 8]", t->waves_per_group);
            return DFA_EINVAL;
        }
        if (t->chain_bytes < 0 || t->chain_bytes % 16 || (t->chain_bytes && (t->chain_bytes < 16 || t->chain_bytes > (1 << 20)))) {
            dfa::set_error("tune.chain_bytes=%lld must be a multiple of 16 in [16, 2^20] (or 0)",
                           (long long)t->chain_bytes);
            return DFA_EINVAL;
        }
    }
    hp.G = (t && t->dfas_per_group) ? t->dfas_per_group : 4;
    hp.waves = (t && t->waves_per_group) ? t->waves_per_group : 8;
    const int64_t fixed_span = t ? t->chain_bytes : 0;
    for (int32_t s = 0; s <= nseg - 1; ++s)
        if (seg_off[s + 1] < seg_off[s] || seg_off[s] < 0) {
            dfa::set_error("dfa_batch: seg_off must be nondecreasing and >= 0");
            return DFA_EINVAL;
        }
    hp.text_bytes = nseg > 0 ? seg_off[nseg] : 0;
    for (int32_t j = 0; j < npat; ++j) {
        // one row of the 256-row space is the padding automata's, so m <= 254
        if (m[j] < 1 || m[j] > kNullRow - 1 || table_off[j] < 0 || (table_off[j] & 3)) {
            dfa::set_error("dfa_batch: pattern %d: m=%d (batched scans take 1..%d) or table_off=%lld "
                           "(4-byte aligned) invalid", j, m[j], kNullRow - 1, (long long)table_off[j]);
            return DFA_EINVAL;
        }
    }
    // pairs of each segment
    std::vector<std::vector<int64_t>> by_seg(size_t(std::max(nseg, 0)));
    for (int64_t k = 0; k < npairs; ++k) {
        if (pair_seg[k] < 0 || pair_seg[k] >= nseg || pair_pat[k] < 0 || pair_pat[k] >= npat) {
            dfa::set_error("dfa_batch: pair %lld refers to segment %d / pattern %d out of range", (long long)k,
                           pair_seg[k], pair_pat[k]);
            return DFA_EINVAL;
        }
        by_seg[size_t(pair_seg[k])].push_back(k);
        const int64_t end = table_off[pair_pat[k]] + int64_t(m[pair_pat[k]] + 1) * DFA_ALPHABET;
        if (end > hp.tables_bytes) hp.tables_bytes = end;
    }
    // segments in decreasing length: the longest work is dispatched first
    std::vector<int32_t> order;
    for (int32_t s = 0; s < nseg; ++s)
        if (!by_seg[size_t(s)].empty()) order.push_back(s);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return seg_off[a + 1] - seg_off[a] > seg_off[b + 1] - seg_off[b];
    });
    const int64_t walks_per_tile = int64_t(hp.waves) * kWave;
    for (int32_t s : order) {
        const int64_t lo = seg_off[s], hi = seg_off[s + 1];
        const int64_t len = hi - lo;
        if (len <= 0) continue;
        // groups: pack this segment's pairs, longest patterns first, up to G
        // automata and kMaxRows rows each
        std::vector<int64_t> ks = by_seg[size_t(s)];
        std::stable_sort(ks.begin(), ks.end(), [&](int64_t a, int64_t b) { return m[pair_pat[a]] > m[pair_pat[b]]; });
        const size_t g_first = hp.groups.size();
        DevGroup cur{};
        auto flush = [&]() {
            if (cur.ndfa > 0) hp.groups.push_back(cur);
            cur = DevGroup{};
        };
        for (int64_t k : ks) {
            const int mm = m[pair_pat[k]];
            if (cur.ndfa == hp.G || cur.rows + mm + 1 > kNullRow) flush();
            DevDfa &d = cur.dfa[cur.ndfa++];
            d.table_off = table_off[pair_pat[k]];
            d.m = mm;
            d.base_row = cur.rows;
            d.pair = int32_t(k);
            cur.rows += mm + 1;
            cur.maxm = std::max(cur.maxm, mm);
            cur.minm = cur.minm ? std::min(cur.minm, mm) : mm;
        }
        flush();
        const int64_t ng = int64_t(hp.groups.size() - g_first);
        // walk span: long segments get the longest span, short ones just enough
        // to spread one tile over all lanes
        int64_t S = fixed_span;
        if (!S) {
            S = dfa::round_up(dfa::ceil_div(len, walks_per_tile), 16);
            S = std::min(std::max(S, kMinSpan), kMaxSpan);
        }
        const int64_t tile = S * walks_per_tile;
        const int64_t ntiles = dfa::ceil_div(len, tile);
        // (tile, group) items; within a block of kXcds tiles the tile index is the
        // fastest, so that item i and i + kXcds (same XCD) share a tile
        for (int64_t tb = 0; tb < ntiles; tb += kXcds) {
            const int64_t nt = std::min<int64_t>(kXcds, ntiles - tb);
            for (int64_t g = 0; g < ng; ++g)
                for (int64_t ti = 0; ti < nt; ++ti) {
                    DevItem it{};
                    it.tile_start = lo + (tb + ti) * tile;
                    it.own_end = std::min(hi, it.tile_start + tile);
                    it.seg_end = hi;
                    it.group = int32_t(g_first + g);
                    it.span = int32_t(S);
                    hp.items.push_back(it);
                }
        }
    }
    if (hp.items.size() > size_t(0x7fffffff)) {
        dfa::set_error("dfa_batch: too many work items");
        return DFA_EINVAL;
    }
    return DFA_OK;
}

int64_t plan_bytes(const HostPlan &hp) {
    return dfa::round_up(int64_t(hp.groups.size() * sizeof(DevGroup)), 256) +
           dfa::round_up(int64_t(hp.items.size() * sizeof(DevItem)), 256);
}

}  // namespace

extern "C" int dfa_batch_prepare(const int64_t *seg_off, int32_t nseg, const int64_t *table_off,
                                 const int32_t *m, int32_t npat, const int32_t *pair_seg,
                                 const int32_t *pair_pat, int64_t npairs, void *workspace,
                                 int64_t workspace_bytes, const dfa_tune *tune, dfa_batch_plan *plan,
                                 void *stream) {
    if (!plan) {
        dfa::set_error("dfa_batch_prepare: null plan");
        return DFA_EINVAL;
    }
    HostPlan hp;
    int rc = plan_batch(seg_off, nseg, table_off, m, npat, pair_seg, pair_pat, npairs, tune, hp);
    if (rc != DFA_OK) return rc;
    std::memset(plan, 0, sizeof(*plan));
    plan->nitems = int64_t(hp.items.size());
    plan->ngroups = int64_t(hp.groups.size());
    plan->npairs = npairs;
    plan->text_bytes = hp.text_bytes;
    plan->tables_bytes = hp.tables_bytes;
    plan->dfas_per_group = hp.G;
    plan->waves_per_group = hp.waves;
    plan->workspace_bytes = plan_bytes(hp);
    if (!workspace) {
        dfa::clear_error();
        return DFA_OK;  // size query
    }
    if (workspace_bytes < plan->workspace_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        dfa::set_error("dfa_batch_prepare: workspace of %lld bytes (256-aligned) needed, got %lld",
                       (long long)plan->workspace_bytes, (long long)workspace_bytes);
        return DFA_ENOSPACE;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    uint8_t *ws = reinterpret_cast<uint8_t *>(workspace);
    const int64_t gbytes = dfa::round_up(int64_t(hp.groups.size() * sizeof(DevGroup)), 256);
    // pageable sources: the copies return once the host data has been consumed
    if (!hp.groups.empty() &&
        !hip_ok(hipMemcpyAsync(ws, hp.groups.data(), hp.groups.size() * sizeof(DevGroup), hipMemcpyHostToDevice, st),
                "plan upload"))
        return DFA_EHIP;
    if (!hp.items.empty() &&
        !hip_ok(hipMemcpyAsync(ws + gbytes, hp.items.data(), hp.items.size() * sizeof(DevItem), hipMemcpyHostToDevice,
                               st),
                "plan upload"))
        return DFA_EHIP;
    // the host arrays above are freed on return: make sure the copies are done
    if (!hip_ok(hipStreamSynchronize(st), "plan upload")) return DFA_EHIP;
    plan->items_offset = gbytes;
    dfa::clear_error();
    return DFA_OK;
}

extern "C" int dfa_batch_run(const uint8_t *text, int64_t n, const uint8_t *tables, int64_t tables_bytes,
                             const void *workspace, const dfa_batch_plan *plan, int64_t *counts, void *stream) {
    if (!plan || n < 0 || (!text && n > 0) || (plan->npairs > 0 && !counts) ||
        (plan->nitems > 0 && (!workspace || !tables))) {
        dfa::set_error("dfa_batch_run: null argument or n < 0");
        return DFA_EINVAL;
    }
    if (plan->tables_bytes > tables_bytes) {
        dfa::set_error("dfa_batch_run: the plan's tables span %lld bytes, buffer has %lld",
                       (long long)plan->tables_bytes, (long long)tables_bytes);
        return DFA_EINVAL;
    }
    if (plan->text_bytes > n) {
        dfa::set_error("dfa_batch_run: segments span %lld bytes, text has %lld", (long long)plan->text_bytes,
                       (long long)n);
        return DFA_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(text) & 15) || (reinterpret_cast<uintptr_t>(tables) & 3) ||
        (reinterpret_cast<uintptr_t>(counts) & 7)) {
        dfa::set_error("dfa_batch_run: text must be 16-byte, tables 4-byte, counts 8-byte aligned");
        return DFA_EINVAL;
    }
    const void *fn = batch_fn(plan->dfas_per_group);
    if (!fn || plan->waves_per_group < 1 || plan->waves_per_group > 8) {
        dfa::set_error("dfa_batch_run: plan not made by dfa_batch_prepare");
        return DFA_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (plan->npairs > 0) {
        const int64_t want = dfa::ceil_div(plan->npairs, 256);
        hipLaunchKernelGGL(k_zero_counts, dim3(unsigned(std::min<int64_t>(want, 4096))), dim3(256), 0, st,
                           reinterpret_cast<unsigned long long *>(counts), plan->npairs);
        if (!hip_ok(hipGetLastError(), "k_zero_counts launch")) return DFA_EHIP;
    }
    if (plan->nitems == 0) {
        dfa::clear_error();
        return DFA_OK;
    }
    if (!dfa::allow_lds(fn, int(batch_lds_bytes(8)))) return DFA_EHIP;
    const uint8_t *ws = reinterpret_cast<const uint8_t *>(workspace);
    BatchParams bp{};
    bp.text = text;
    bp.n = n;
    bp.tables = tables;
    bp.groups = reinterpret_cast<const DevGroup *>(ws);
    bp.items = reinterpret_cast<const DevItem *>(ws + plan->items_offset);
    bp.counts = reinterpret_cast<unsigned long long *>(counts);
    void *args[] = {&bp};
    if (!hip_ok(hipLaunchKernel(fn, dim3(unsigned(plan->nitems)), dim3(plan->waves_per_group * kWave), args,
                                batch_lds_bytes(plan->waves_per_group), st),
                "k_batch launch"))
        return DFA_EHIP;
    dfa::clear_error();
    return DFA_OK;
}

extern "C" int dfa_count_batch(const uint8_t *text, int64_t n, const int64_t *seg_off, int32_t nseg,
                               const uint8_t *tables, int64_t tables_bytes, const int64_t *table_off,
                               const int32_t *m, int32_t npat,
                               const int32_t *pair_seg, const int32_t *pair_pat, int64_t npairs, int64_t *counts,
                               void *workspace, int64_t workspace_bytes, const dfa_tune *tune, void *stream) {
    dfa_batch_plan plan;
    int rc = dfa_batch_prepare(seg_off, nseg, table_off, m, npat, pair_seg, pair_pat, npairs, workspace,
                               workspace_bytes, tune, &plan, stream);
    if (rc != DFA_OK) return rc;
    if (!workspace && plan.workspace_bytes > 0) {
        dfa::set_error("dfa_count_batch: workspace of %lld bytes needed", (long long)plan.workspace_bytes);
        return DFA_ENOSPACE;
    }
    return dfa_batch_run(text, n, tables, tables_bytes, workspace, &plan, counts, stream);
}
