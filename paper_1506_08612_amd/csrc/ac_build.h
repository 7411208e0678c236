// Host construction of the merged multi-pattern automaton (the paper's
// improved Aho-Corasick automaton, Sec. "Implementation Aspects", Fig. 4):
// one state per distinct prefix of the patterns, a transition for every byte
// with the failure links folded in, and the states that report a pattern
// numbered last so that "is final" is one comparison.
#pragma once

#include <cstdint>
#include <vector>

namespace dfa {

struct AcAutomaton {
    // byte classes: every byte that occurs in some pattern is a class of its
    // own (1..ncls-1, in increasing byte order); all other bytes are class 0,
    // on which every state returns to the start state
    int ncls = 0;
    uint8_t cls[256] = {};
    int32_t nstates = 0;
    int32_t first_final = 0;     // states >= first_final report at least one pattern
    std::vector<int32_t> next;   // nstates x ncls: next state per class
    std::vector<int32_t> depth;  // prefix length of each state
    // reported patterns of each final state f (indices into the pattern list
    // given to the builder): out_pat[out_off[f - first_final] .. out_off[f - first_final + 1])
    std::vector<int32_t> out_off;
    std::vector<int32_t> out_pat;
};

// Patterns are pats[i] (lens[i] >= 1 bytes).  Builds over the byte classes of
// exactly these patterns.  Returns false if more than max_states states would
// be needed.
bool ac_build(const std::vector<const uint8_t *> &pats, const std::vector<int32_t> &lens, int64_t max_states,
              AcAutomaton &out);

// Number of distinct nonempty prefixes of the patterns plus one (the states
// ac_build would make), without building transitions.
int64_t ac_count_states(const std::vector<const uint8_t *> &pats, const std::vector<int32_t> &lens);

}  // namespace dfa
