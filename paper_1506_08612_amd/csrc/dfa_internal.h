// Internal helpers shared by the host and HIP translation units of libdfa.
#pragma once

#include <cstdint>

namespace dfa {

// thread-local error message returned by dfa_last_error()
void set_error(const char *fmt, ...);
void clear_error();

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

}  // namespace dfa
