// Degenerate patterns: IUPAC nucleotide codes, optionally with the reverse
// complement strand, expanded into the set of plain k-mers they match.
//
// The paper's pattern table (Table 3) pairs every 8-mer with its reverse
// complement and lets one position take one of three bases.  Written with
// IUPAC codes such a pattern is one string; its matches are the start
// positions where one of its expansions (or of its reverse complement's)
// occurs.  All expansions have the same length, so no two of them match at
// the same start, and the count of a degenerate pattern is the sum of the
// counts of its distinct expansions -- which the merged multi-pattern scan
// computes in one pass when every expansion's pair adds into the pattern's
// counter.

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "dfa.h"
#include "dfa_internal.h"

namespace {

// bases of a code as a bit set: A=1, C=2, G=4, T=8; 0 for a byte that is not a code
int code_bases(uint8_t c) {
    switch (c) {
        case 'A': return 1;
        case 'C': return 2;
        case 'G': return 4;
        case 'T': return 8;
        case 'R': return 5;
        case 'Y': return 10;
        case 'S': return 6;
        case 'W': return 9;
        case 'K': return 12;
        case 'M': return 3;
        case 'B': return 14;
        case 'D': return 13;
        case 'H': return 11;
        case 'V': return 7;
        case 'N': return 15;
        default: return 0;
    }
}

const char kBase[4] = {'A', 'C', 'G', 'T'};

// complement of a base set: A<->T, C<->G (bit 0 <-> bit 3, bit 1 <-> bit 2)
int complement_bases(int b) { return ((b & 1) << 3) | ((b & 8) >> 3) | ((b & 2) << 1) | ((b & 4) >> 1); }

void expand(const std::vector<int> &sets, std::vector<std::string> &out) {
    const size_t m = sets.size();
    std::string cur(m, 'A');
    // odometer over the choices of every position
    std::vector<int> choice(m, 0);
    std::vector<std::vector<char>> opts(m);
    for (size_t j = 0; j < m; ++j)
        for (int b = 0; b < 4; ++b)
            if (sets[j] & (1 << b)) opts[j].push_back(kBase[b]);
    while (true) {
        for (size_t j = 0; j < m; ++j) cur[j] = opts[j][size_t(choice[j])];
        out.push_back(cur);
        size_t j = m;
        while (j > 0) {
            --j;
            if (++choice[j] < int(opts[j].size())) break;
            choice[j] = 0;
            if (j == 0) return;
        }
        if (m == 0) return;
    }
}

}  // namespace

extern "C" int64_t dfa_degenerate_expand(const uint8_t *code, int32_t m, int32_t both_strands, uint8_t *out,
                                         int64_t out_cap) {
    if (!code || m < 1 || m > DFA_MAX_M) {
        dfa::set_error("dfa_degenerate_expand: m=%d outside [1, %d] or null code", m, DFA_MAX_M);
        return DFA_EINVAL;
    }
    std::vector<int> sets(static_cast<size_t>(m)), rc(static_cast<size_t>(m));
    double total = 1.0;
    for (int32_t j = 0; j < m; ++j) {
        const int b = code_bases(code[j]);
        if (!b) {
            dfa::set_error("dfa_degenerate_expand: byte %d at %d is not an IUPAC nucleotide code", int(code[j]), j);
            return DFA_EINVAL;
        }
        sets[size_t(j)] = b;
        rc[size_t(m - 1 - j)] = complement_bases(b);
        total *= __builtin_popcount(unsigned(b));
    }
    if (total * (both_strands ? 2 : 1) > double(DFA_DEGENERATE_MAX_KMERS)) {
        dfa::set_error("dfa_degenerate_expand: more than %d expansions", DFA_DEGENERATE_MAX_KMERS);
        return DFA_EINVAL;
    }
    std::vector<std::string> kmers;
    expand(sets, kmers);
    if (both_strands) expand(rc, kmers);
    std::sort(kmers.begin(), kmers.end());
    kmers.erase(std::unique(kmers.begin(), kmers.end()), kmers.end());
    const int64_t k = int64_t(kmers.size());
    if (out) {
        if (out_cap < k) {
            dfa::set_error("dfa_degenerate_expand: %lld k-mers, room for %lld", (long long)k, (long long)out_cap);
            return DFA_ENOSPACE;
        }
        for (int64_t i = 0; i < k; ++i) std::memcpy(out + i * m, kmers[size_t(i)].data(), size_t(m));
    }
    dfa::clear_error();
    return k;
}
