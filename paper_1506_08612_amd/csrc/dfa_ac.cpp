// Host construction of the merged multi-pattern automaton and its C entry
// point dfa_ac_build.
//
// Construction (Sec. "Implementation Aspects", Fig. 4).  The patterns are put
// in a trie; a breadth-first pass gives every state its failure state (the
// state of the longest proper suffix of its prefix that is also a prefix) and
// folds the failure links into the transitions, so that every (state, byte)
// has exactly one next state and a scan never follows a failure link.  A state
// reports its own patterns and those of its failure state.  Renumbering puts
// the states that report nothing first and the reporting ("final") states
// last, both in breadth-first order.

#include <algorithm>
#include <cstring>
#include <deque>
#include <vector>

#include "ac_build.h"
#include "dfa.h"
#include "dfa_internal.h"

namespace dfa {

namespace {

void make_classes(const std::vector<const uint8_t *> &pats, const std::vector<int32_t> &lens, AcAutomaton &a) {
    bool used[256] = {};
    for (size_t i = 0; i < pats.size(); ++i)
        for (int32_t j = 0; j < lens[i]; ++j) used[pats[i][j]] = true;
    a.ncls = 1;
    for (int b = 0; b < 256; ++b) a.cls[b] = used[b] ? uint8_t(a.ncls++) : 0;
}

}  // namespace

int64_t ac_count_states(const std::vector<const uint8_t *> &pats, const std::vector<int32_t> &lens) {
    // distinct prefixes = trie nodes: sort the patterns and count, for each, the
    // bytes past its longest common prefix with its predecessor
    std::vector<size_t> order(pats.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        const int32_t n = std::min(lens[a], lens[b]);
        const int c = std::memcmp(pats[a], pats[b], size_t(n));
        return c ? c < 0 : lens[a] < lens[b];
    });
    int64_t states = 1;
    for (size_t k = 0; k < order.size(); ++k) {
        const size_t i = order[k];
        int32_t common = 0;
        if (k > 0) {
            const size_t p = order[k - 1];
            const int32_t n = std::min(lens[i], lens[p]);
            while (common < n && pats[i][common] == pats[p][common]) ++common;
        }
        states += lens[i] - common;
    }
    return states;
}

bool ac_build(const std::vector<const uint8_t *> &pats, const std::vector<int32_t> &lens, int64_t max_states,
              AcAutomaton &a) {
    make_classes(pats, lens, a);
    const int C = a.ncls;
    // trie
    std::vector<int32_t> go(size_t(C), -1);
    std::vector<int32_t> depth(1, 0);
    std::vector<std::vector<int32_t>> own(1);
    for (size_t i = 0; i < pats.size(); ++i) {
        int32_t s = 0;
        for (int32_t j = 0; j < lens[i]; ++j) {
            const int k = a.cls[pats[i][j]];
            int32_t &c = go[size_t(s) * C + k];
            if (c < 0) {
                if (int64_t(depth.size()) >= max_states) return false;
                c = int32_t(depth.size());
                depth.push_back(depth[size_t(s)] + 1);
                own.emplace_back();
                go.resize(go.size() + size_t(C), -1);
            }
            s = go[size_t(s) * C + k];
        }
        own[size_t(s)].push_back(int32_t(i));
    }
    const int32_t N = int32_t(depth.size());
    // breadth-first: failure states and the folded transitions
    std::vector<int32_t> fail(static_cast<size_t>(N), 0), delta(static_cast<size_t>(N) * C, 0), bfs;
    bfs.reserve(size_t(N));
    std::deque<int32_t> queue;
    bfs.push_back(0);
    for (int k = 0; k < C; ++k) {
        const int32_t c = go[size_t(k)];
        if (c >= 0) {
            fail[size_t(c)] = 0;
            delta[size_t(k)] = c;
            queue.push_back(c);
        }
    }
    while (!queue.empty()) {
        const int32_t s = queue.front();
        queue.pop_front();
        bfs.push_back(s);
        for (int k = 0; k < C; ++k) {
            const int32_t c = go[size_t(s) * C + k];
            const int32_t via_fail = delta[size_t(fail[size_t(s)]) * C + k];
            if (c >= 0) {
                fail[size_t(c)] = via_fail;
                delta[size_t(s) * C + k] = c;
                queue.push_back(c);
            } else {
                delta[size_t(s) * C + k] = via_fail;
            }
        }
    }
    // outputs: own patterns, then the failure state's (computed earlier in bfs order)
    std::vector<std::vector<int32_t>> out(static_cast<size_t>(N));
    for (int32_t s : bfs) {
        out[size_t(s)] = own[size_t(s)];
        if (s != 0) {
            const auto &f = out[size_t(fail[size_t(s)])];
            out[size_t(s)].insert(out[size_t(s)].end(), f.begin(), f.end());
        }
    }
    // renumber: non-reporting states first, then reporting ones, each in bfs order
    std::vector<int32_t> id(size_t(N), -1);
    int32_t next_id = 0;
    for (int32_t s : bfs)
        if (out[size_t(s)].empty()) id[size_t(s)] = next_id++;
    a.first_final = next_id;
    for (int32_t s : bfs)
        if (!out[size_t(s)].empty()) id[size_t(s)] = next_id++;
    a.nstates = N;
    a.next.assign(size_t(N) * C, 0);
    a.depth.assign(size_t(N), 0);
    std::vector<int32_t> by_id(static_cast<size_t>(N));
    for (int32_t s = 0; s < N; ++s) by_id[size_t(id[size_t(s)])] = s;
    for (int32_t q = 0; q < N; ++q) {
        const int32_t s = by_id[size_t(q)];
        a.depth[size_t(q)] = depth[size_t(s)];
        for (int k = 0; k < C; ++k) a.next[size_t(q) * C + k] = id[size_t(delta[size_t(s) * C + k])];
    }
    a.out_off.assign(size_t(N - a.first_final) + 1, 0);
    a.out_pat.clear();
    for (int32_t q = a.first_final; q < N; ++q) {
        const auto &o = out[size_t(by_id[size_t(q)])];
        a.out_pat.insert(a.out_pat.end(), o.begin(), o.end());
        a.out_off[size_t(q - a.first_final) + 1] = int32_t(a.out_pat.size());
    }
    return true;
}

}  // namespace dfa

extern "C" int64_t dfa_ac_build(const uint8_t *patterns, const int64_t *pat_off, const int32_t *pat_len, int32_t npat,
                                uint16_t *table, int64_t max_states, int32_t *first_final, int32_t *out_off,
                                int32_t *out_pat, int64_t out_cap, int64_t *n_out) {
    if (npat < 1 || !patterns || !pat_off || !pat_len) {
        dfa::set_error("dfa_ac_build: need at least one pattern and non-null arrays");
        return DFA_EINVAL;
    }
    std::vector<const uint8_t *> pats(static_cast<size_t>(npat));
    std::vector<int32_t> lens(static_cast<size_t>(npat));
    for (int32_t i = 0; i < npat; ++i) {
        if (pat_len[i] < 1 || pat_len[i] > DFA_MAX_M || pat_off[i] < 0) {
            dfa::set_error("dfa_ac_build: pattern %d has length %d (1..%d) or offset %lld", i, pat_len[i], DFA_MAX_M,
                           (long long)pat_off[i]);
            return DFA_EINVAL;
        }
        pats[size_t(i)] = patterns + pat_off[i];
        lens[size_t(i)] = pat_len[i];
    }
    dfa::AcAutomaton a;
    if (!dfa::ac_build(pats, lens, DFA_AC_MAX_STATES, a)) {
        dfa::set_error("dfa_ac_build: the patterns need more than %d states", DFA_AC_MAX_STATES);
        return DFA_EINVAL;
    }
    if (first_final) *first_final = a.first_final;
    if (n_out) *n_out = int64_t(a.out_pat.size());
    if (table) {
        if (max_states < a.nstates) {
            dfa::set_error("dfa_ac_build: %d states, table has room for %lld", a.nstates, (long long)max_states);
            return DFA_ENOSPACE;
        }
        for (int32_t q = 0; q < a.nstates; ++q)
            for (int b = 0; b < DFA_ALPHABET; ++b)
                table[size_t(q) * DFA_ALPHABET + b] = uint16_t(a.next[size_t(q) * a.ncls + a.cls[b]]);
    }
    if (out_off) {
        for (size_t i = 0; i < a.out_off.size(); ++i) out_off[i] = a.out_off[i];
    }
    if (out_pat) {
        if (out_cap < int64_t(a.out_pat.size())) {
            dfa::set_error("dfa_ac_build: %zu outputs, room for %lld", a.out_pat.size(), (long long)out_cap);
            return DFA_ENOSPACE;
        }
        std::copy(a.out_pat.begin(), a.out_pat.end(), out_pat);
    }
    dfa::clear_error();
    return a.nstates;
}
