// Device-side building blocks shared by the automaton scan kernels of libdfa
// (gfx950): the LDS table layout and step, the wave-level match count, and
// the coalesced fetch + LDS transpose that gives every lane consecutive bytes
// of its own walk.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dfa.h"

namespace dfa_dev {

constexpr int kRow = DFA_ALPHABET + 24;  // LDS bytes per table row (256 columns + bank padding)
constexpr int kWave = 64;

// 16 text bytes as a native 4 x u32 register vector
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Geometry of one round: every walk receives LINE consecutive bytes (U units
// of 16 bytes); one wave-wide 16-byte load covers 64/U walks.  The round is
// transposed through a wave-private LDS buffer of 64 rows of LINE bytes per
// walk slot, then walked one 16-byte unit at a time straight from LDS.
template <int LINE>
struct Geo {
    static constexpr int U = LINE / 16;     // units per walk per round
    static constexpr int kPer = kWave / U;  // walks per wave load
    // XOR swizzle of the unit index by buffer row: any 8 consecutive lanes
    // reading the same unit index hit 8 different 16-byte bank groups
    __device__ static __forceinline__ int swz(int row) { return (row / (8 / U)) % U; }
};

__host__ __device__ inline int table_lds_rows_bytes(int rows) { return (rows * kRow + 15) & ~15; }

// Orders this lane's LDS accesses against the other lanes' of the same wave:
// LDS executes one wave's instructions in order, so waiting for the lane's
// own outstanding LDS operations is enough; the clobber stops the compiler
// from moving memory accesses across.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// The kernels declare no static LDS, so dynamic LDS (and with it the tables,
// placed first) starts at LDS address 0.  Reading a table through an absolute
// LDS address keeps the step's address one 24-bit multiply-add.  `q` is a row
// number: the row of state q of a table whose rows start at row `base` is
// base + q, and entries hold row numbers.
typedef __attribute__((address_space(3))) const uint8_t lds_u8;
__device__ __forceinline__ uint32_t table_step(uint32_t q, uint32_t c) {
    return *reinterpret_cast<lds_u8 *>(uintptr_t(__umul24(q, uint32_t(kRow)) + c));
}

// acc += number of lanes of the wave with `hit` set: one compare into a lane
// mask, then a scalar bit count and add.  Written out so that the running
// sum stays one scalar register (the compiler otherwise parks every step's
// partial count in a register of its own).
__device__ __forceinline__ void add_hits(uint32_t &acc, bool hit) {
    const unsigned long long mask = __ballot(hit);
    uint32_t tmp;
    uint32_t a = __builtin_amdgcn_readfirstlane(acc);  // the count is wave-uniform
    asm("s_bcnt1_i32_b64 %1, %2\n\ts_add_u32 %0, %0, %1" : "+s"(a), "=&s"(tmp) : "s"(mask) : "scc");
    acc = a;
}

// Sixteen automaton steps over one 16-byte unit, counting visits of the final
// state, for the in-bounds count-only walk.  Each step computes the next LDS
// address and issues the byte read first; the next text byte is extracted and
// the previous state tested against the final state while the read is in
// flight, so the dependent chain per byte is one multiply-add and one LDS read.
// The read is waited for inside the same block.  States alternate between two
// registers (the test reads the older one while the read fills the other); the
// unit ends with the state in `q`, all sixteen states tested.
__device__ __forceinline__ void walk16_count(uint32_t &q, const v4u &t, uint32_t &acc, uint32_t m) {
    uint32_t qb, a, c, tmp;
    unsigned long long mk;
    uint32_t s = __builtin_amdgcn_readfirstlane(acc);
    asm(
        "v_bfe_u32 %[c], %[w0], 0, 8\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w0], 8, 8\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w0], 16, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w0], 24, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 0, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 8, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 16, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 24, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 0, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 8, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 16, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 24, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 0, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 8, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 16, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 24, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "s_bcnt1_i32_b64 %[t], %[mk]\n\t"
        "s_add_u32 %[acc], %[acc], %[t]\n\t"
        : [q] "+v"(q), [qb] "=&v"(qb), [a] "=&v"(a), [c] "=&v"(c), [mk] "=&s"(mk), [t] "=&s"(tmp), [acc] "+s"(s)
        : [w0] "v"(t.x), [w1] "v"(t.y), [w2] "v"(t.z), [w3] "v"(t.w), [m] "s"(m), [row] "s"(uint32_t(kRow))
        : "scc");
    acc = s;
}

// The same sixteen steps, recording which of them reached the final state:
// `hm` gets one bit per byte, the first byte in bit 15 and the last in bit 0
// (each step doubles hm and adds the step's compare result as a carry), so a
// lane's matches in the unit end at bytes 15 - (set bit positions).
__device__ __forceinline__ void walk16_hits(uint32_t &q, const v4u &t, uint32_t &hm, uint32_t m) {
    uint32_t qb, a, c;
    unsigned long long mk, co;
    asm(
        "v_mov_b32 %[hm], 0\n\t"
        "v_bfe_u32 %[c], %[w0], 0, 8\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w0], 8, 8\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w0], 16, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w0], 24, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 0, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 8, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 16, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 24, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 0, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 8, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 16, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 24, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 0, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 8, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 16, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 24, 8\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[qb]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_cmp_eq_u32_e64 %[mk], %[m], %[q]\n\t"
        "v_addc_co_u32_e64 %[hm], %[co], %[hm], %[hm], %[mk]\n\t"
        : [q] "+v"(q), [qb] "=&v"(qb), [a] "=&v"(a), [c] "=&v"(c), [hm] "=&v"(hm), [mk] "=&s"(mk), [co] "=&s"(co)
        : [w0] "v"(t.x), [w1] "v"(t.y), [w2] "v"(t.z), [w3] "v"(t.w), [m] "s"(m), [row] "s"(uint32_t(kRow)));
}

// The same sixteen steps over a MARKED table: entry 2 q + f for the state q
// reached, f = 1 iff q is final, with row e at e x kRow holding state e / 2's
// transitions (each row stored twice), so the walk's register holds entries.
// One funnel shift per byte moves the entry's low bit into `hm`: byte i of the
// unit ends in bit i (the first byte in bit 0).  No compare is needed.
__device__ __forceinline__ void walk16_marks(uint32_t &q, const v4u &t, uint32_t &hm) {
    uint32_t qb, a, c;
    hm = 0;  // shifted out: only the 16 bits the steps insert are kept
    asm(
        "v_bfe_u32 %[c], %[w0], 0, 8\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w0], 8, 8\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w0], 16, 8\n\t"
        "v_alignbit_b32 %[hm], %[qb], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w0], 24, 8\n\t"
        "v_alignbit_b32 %[hm], %[q], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 0, 8\n\t"
        "v_alignbit_b32 %[hm], %[qb], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 8, 8\n\t"
        "v_alignbit_b32 %[hm], %[q], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 16, 8\n\t"
        "v_alignbit_b32 %[hm], %[qb], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w1], 24, 8\n\t"
        "v_alignbit_b32 %[hm], %[q], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 0, 8\n\t"
        "v_alignbit_b32 %[hm], %[qb], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 8, 8\n\t"
        "v_alignbit_b32 %[hm], %[q], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 16, 8\n\t"
        "v_alignbit_b32 %[hm], %[qb], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w2], 24, 8\n\t"
        "v_alignbit_b32 %[hm], %[q], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 0, 8\n\t"
        "v_alignbit_b32 %[hm], %[qb], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 8, 8\n\t"
        "v_alignbit_b32 %[hm], %[q], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 16, 8\n\t"
        "v_alignbit_b32 %[hm], %[qb], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[q], %[row], %[c]\n\t"
        "ds_read_u8 %[qb], %[a]\n\t"
        "v_bfe_u32 %[c], %[w3], 24, 8\n\t"
        "v_alignbit_b32 %[hm], %[q], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_mad_u32_u24 %[a], %[qb], %[row], %[c]\n\t"
        "ds_read_u8 %[q], %[a]\n\t"
        "v_alignbit_b32 %[hm], %[qb], %[hm], 1\n\t"
        "s_waitcnt lgkmcnt(0)\n\t"
        "v_alignbit_b32 %[hm], %[q], %[hm], 1\n\t"
        : [q] "+v"(q), [qb] "=&v"(qb), [a] "=&v"(a), [c] "=&v"(c), [hm] "+v"(hm)
        : [w0] "v"(t.x), [w1] "v"(t.y), [w2] "v"(t.z), [w3] "v"(t.w), [row] "s"(uint32_t(kRow)));
    hm >>= 16;
}

// 16 bytes at text[a..a+15]; bytes at or past n read as 0 (a byte outside
// every pattern: it sends the automaton to q0 and never completes a match).
__device__ __forceinline__ v4u load_unit_guarded(const uint8_t *text, int64_t n, int64_t a) {
    if (a + 16 <= n) return *reinterpret_cast<const v4u *>(text + a);
    v4u v = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (a + i < n) v[i >> 2] |= uint32_t(text[a + i]) << (8 * (i & 3));
    return v;
}

// Fetch round r of a wave's walks into registers.  The wave's walk w of slot
// s starts at byte wbase + (64 s + w) S.  Load j of slot s covers the walks
// 64 s + j kPer + lane/U (unit lane % U of each): U lanes read one LINE-byte
// piece, so every load is made of whole, aligned pieces.  `lane_off` is
// (lane / U) * S + 16 (lane % U).
template <int K, int LINE, bool GUARDED>
__device__ __forceinline__ void fetch_round(v4u (&pf)[K][Geo<LINE>::U], const uint8_t *text, int64_t n,
                                            int64_t wbase, int64_t S, uint32_t lane_off, int r) {
    using G = Geo<LINE>;
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int j = 0; j < G::U; ++j) {
            // wave-uniform base of this load, plus a 32-bit per-lane offset
            const int64_t ub = wbase + int64_t(s * kWave + j * G::kPer) * S + int64_t(r) * LINE;
            if (GUARDED)
                pf[s][j] = load_unit_guarded(text, n, ub + int64_t(lane_off));
            else
                pf[s][j] = *reinterpret_cast<const v4u *>(text + ub + lane_off);
        }
    }
}

// Registers -> LDS: slot s of the wave's round lands in rows 64 s .. 64 s + 63
// of the wave's buffer, one row of LINE bytes per walk.
template <int K, int LINE>
__device__ __forceinline__ void stage_round(const v4u (&pf)[K][Geo<LINE>::U], v4u *xb, int lane) {
    using G = Geo<LINE>;
    const int lrow = lane / G::U, lunit = lane % G::U;
    wave_lds_sync();  // the previous round's reads of this buffer are done
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int j = 0; j < G::U; ++j) {
            const int row = j * G::kPer + lrow;
            xb[(s * kWave + row) * G::U + (lunit ^ G::swz(row))] = pf[s][j];
        }
    }
    wave_lds_sync();
}

// Unit u (bytes 16u .. 16u + 15 of the round) of the lane's own walk in slot s.
template <int LINE>
__device__ __forceinline__ v4u unit_of(const v4u *xb, int s, int lane, int u) {
    using G = Geo<LINE>;
    return xb[(s * kWave + lane) * G::U + (u ^ G::swz(lane))];
}

// The first H units of the overlap of each of the lane's walks, taken right
// after round 0 is staged: the overlap of walk (slot s, lane l) is the start
// of walk (s, l + 1), row s * 64 + l + 1 of the wave's buffer (walk (s, l)
// starts at byte wb + (64 s + l) S).  The last walk
// of the wave (whose neighbour is another wave's) and units past the ones the
// buffer holds (`valid` < H only for spans shorter than a round) are loaded
// from memory, with u clamped to hu - 1 so that every address stays inside
// the overlap.
template <int K, int LINE, int H>
__device__ __forceinline__ void grab_halo(v4u (&h)[K][H], const v4u *xb, int lane, const uint8_t *text, int64_t wb,
                                          int64_t S, int hu, int valid) {
    using G = Geo<LINE>;
    const int last = hu > 0 ? hu - 1 : 0;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int rho = s * kWave + lane + 1;
        const bool in_buf = rho < K * kWave;
        const int rr = in_buf ? rho : K * kWave - 1;
        const int row = rr % kWave;
#pragma unroll
        for (int u = 0; u < H; ++u) {
            v4u v = xb[rr * G::U + (u ^ G::swz(row))];
            if (hu > 0 && (!in_buf || u >= valid))
                v = *reinterpret_cast<const v4u *>(text + wb + int64_t(s * kWave + lane + 1) * S +
                                                   16 * (u < last ? u : last));
            h[s][u] = v;
        }
    }
}

// Rounds r and r + 1 (r even) of 64-byte rounds, fetched as whole 128-byte
// lines (the walk's span is a multiple of 128 bytes and starts on a line):
// load i of slot s covers walks 64 s + 8 i + lane / 8, bytes 16 (lane % 8)
// .. + 15 of their line at 64 r, so lanes with lane % 8 < 4 hold round r and
// the others round r + 1 (unit lane % 4 of it).  Non-temporal loads: the text
// is read once, and whole-line non-temporal requests streamed faster than
// plain ones on gfx950 (half-line ones slower: the second half of the line
// then missed the cache).  Past the last round (r > rlast) the pair reads the
// text's first line instead (a cache hit whose values are never used).
// `pair_off` is (lane / 8) S + 16 (lane % 8).
template <int K>
__device__ __forceinline__ void fetch_pair(v4u (&pp)[K][8], const uint8_t *text, int64_t wb, int64_t S,
                                           uint32_t pair_off, int lane, int r, int rlast) {
    const bool real = r <= rlast;  // wave-uniform
    const uint32_t off = real ? pair_off : 16u * uint32_t(lane % 8);
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t ub = real ? wb + int64_t(s * kWave + 8 * i) * S + int64_t(r) * 64 : 0;
            pp[s][i] = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(text + ub + off));
        }
    }
}

// Round r (HALF 0) or r + 1 (HALF 1) of a fetched pair into the wave's
// buffer: the same rows and units as stage_round<K, 64>, written by the half
// of the lanes that holds that round.
template <int K, int HALF>
__device__ __forceinline__ void stage_pair(const v4u (&pp)[K][8], v4u *xb, int lane) {
    using G = Geo<64>;
    wave_lds_sync();  // the previous round's reads of this buffer are done
    if ((lane % 8) / 4 == HALF) {
        const int unit = lane % 4;
#pragma unroll
        for (int s = 0; s < K; ++s) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int row = 8 * i + lane / 8;
                xb[(s * kWave + row) * G::U + (unit ^ G::swz(row))] = pp[s][i];
            }
        }
    }
    wave_lds_sync();
}

// Round r of the wave's walks (in-bounds path): rounds before the last use the
// lane's own unit offset, the last one the clamped offset; r past the last
// round loads the text's first line (a cache hit whose values are never used).
template <int K, int LINE>
__device__ __forceinline__ void fetch_round_or_none(v4u (&pf)[K][Geo<LINE>::U], const uint8_t *text, int64_t wb,
                                                    int64_t S, uint32_t off, uint32_t off_last, uint32_t off_none,
                                                    int r, int rlast) {
    const bool real = r <= rlast;  // wave-uniform
    fetch_round<K, LINE, false>(pf, text, 0, real ? wb : 0, real ? S : 0,
                                r < rlast ? off : (real ? off_last : off_none), real ? r : 0);
}

}  // namespace dfa_dev
