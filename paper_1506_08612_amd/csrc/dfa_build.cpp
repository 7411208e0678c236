// Host-side automaton construction and error reporting for libdfa.
//
// The single-pattern automaton is the failure-free Aho-Corasick automaton of
// Sec. III.B restricted to one pattern: every (state, byte) pair has an
// explicit successor, so each text byte costs exactly one table lookup.  It is
// stored as the sparse state transition table of Sec. III.B: one column per
// byte value (256), bytes that lead nowhere go to q0, and the final state is
// numbered last (state m), so the final-state test is q == m.
//
// Construction keeps a "shadow" state X: the state the automaton is in after
// reading P[1..q-1].  Row q equals row X except that the byte P[q] advances
// to q+1; afterwards X moves on by P[q].  Row m is row X for X = the state of
// P[1..m-1], the longest proper border of P, which is what lets the walk find
// overlapping occurrences.  O(256 m) time.

#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "dfa.h"
#include "dfa_internal.h"

namespace dfa {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

}  // namespace dfa

extern "C" const char *dfa_last_error(void) { return dfa::g_err; }

extern "C" const char *dfa_version(void) { return "libdfa 0.1 gfx950"; }

extern "C" int64_t dfa_table_bytes(int32_t m) {
    if (m < 1 || m > DFA_MAX_M) {
        dfa::set_error("dfa_table_bytes: m=%d outside [1, %d]", m, DFA_MAX_M);
        return DFA_EINVAL;
    }
    return int64_t(m + 1) * DFA_ALPHABET;
}

extern "C" int dfa_build(const uint8_t *pattern, int32_t m, uint8_t *table) {
    if (!pattern || !table) {
        dfa::set_error("dfa_build: null pointer");
        return DFA_EINVAL;
    }
    if (m < 1 || m > DFA_MAX_M) {
        dfa::set_error("dfa_build: m=%d outside [1, %d]", m, DFA_MAX_M);
        return DFA_EINVAL;
    }
    std::memset(table, 0, size_t(m + 1) * DFA_ALPHABET);
    table[pattern[0]] = 1;
    int x = 0;
    for (int q = 1; q <= m; ++q) {
        std::memcpy(table + size_t(q) * DFA_ALPHABET, table + size_t(x) * DFA_ALPHABET,
                    DFA_ALPHABET);
        if (q < m) {
            table[size_t(q) * DFA_ALPHABET + pattern[q]] = uint8_t(q + 1);
            x = table[size_t(x) * DFA_ALPHABET + pattern[q]];
        }
    }
    dfa::clear_error();
    return DFA_OK;
}
