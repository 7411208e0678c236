// LDS read rate of the device (measurement only).
//
// Every automaton step of the paper's scan is one table read at an address
// that depends on the state and the text byte (Alg. 1; the sparse transition
// table of Sec. III.B).  On gfx950 the tables live in LDS, so the rate at
// which LDS serves single-byte and two-byte reads at scattered addresses is
// the ceiling of every table-bound scan here (the merged multi-pattern scan
// above all).  This kernel measures that rate three ways (the C ABI's mode
// 0, 1 and 2 are scattered, dependent and conflict-free):
//
//   scattered    eight reads per lane and iteration at addresses that do not
//                depend on the values read (a lane's base plus fixed
//                offsets): the gather throughput at scattered addresses,
//                where lanes of a wave meet in the same bank;
//   conflict-free  the same, but lane l of each half-wave reads dword l of a
//                128-byte row, so that no two lanes of a half-wave share a
//                bank: the conflict-free read rate;
//   dependent    eight chains per lane, each read's address computed from the
//                previous value of its chain as an automaton step computes
//                the next row from the state (value x row + column), over
//                rows of 61 one-byte or of 5 two-byte entries (a class-
//                compressed automaton's row over A, C, G, T and the rest):
//                the rate a walk reaches when every lane has eight walks in
//                flight.  Row strides that are multiples of 128 bytes would
//                put every lane of a wave in one bank.
//
// The table is 16 KiB, every address is inside it by construction (values
// are row numbers: below 128 for the independent reads, below 256 or 1600 for
// the dependent ones), and the loaded values are kept alive by a store that
// only an impossible checksum would make.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dfa.h"
#include "dfa_internal.h"
#include "launch_util.h"

namespace {

constexpr int kProbeBytes = 16 * 1024;
constexpr int kProbeThreads = 512;
constexpr int kReadsPerIter = 8;
constexpr uint32_t kStride = 1022;   // bytes between a lane's independent reads (even)
constexpr uint32_t kAdvance = 2474;  // bytes a lane's base moves per iteration (even)
constexpr uint32_t kRow8 = 61;       // dependent reads: bytes per row of 1-byte entries (256 rows)
constexpr uint32_t kRow16 = 5;       // ... entries per row of 2-byte entries (1600 rows)
constexpr uint32_t kRows16 = 1600;

typedef __attribute__((address_space(3))) const uint8_t lds8;
typedef __attribute__((address_space(3))) const uint16_t lds16;

__device__ __forceinline__ uint32_t mix(uint32_t x) {  // a 32-bit integer hash (xorshift-multiply)
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

template <int WIDTH>
__device__ __forceinline__ uint32_t lds_read(uint32_t addr) {
    if (WIDTH == 1) return *reinterpret_cast<lds8 *>(uintptr_t(addr));
    return *reinterpret_cast<lds16 *>(uintptr_t(addr));
}

enum ProbeMode { kIndependent = 0, kDependent = 1, kLinear = 2 };

template <int WIDTH, int MODE>
__global__ __launch_bounds__(kProbeThreads) void k_lds_probe(int64_t iters, unsigned long long *sink) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (MODE == kDependent && WIDTH == 2) {
        // row numbers below 1600 (1600 rows of 5 entries: 16000 bytes)
        for (int i = threadIdx.x; i < kProbeBytes / 2; i += blockDim.x)
            reinterpret_cast<uint16_t *>(smem)[i] = uint16_t(mix(uint32_t(i) * 2654435761u + 12345u) % kRows16);
    } else {
        // values below 128 (independent reads), or any byte (row numbers of the
        // 256 one-byte rows of the dependent reads)
        const uint32_t keep = MODE == kDependent ? 0xffffffffu : WIDTH == 1 ? 0x7f7f7f7fu : 0x007f007fu;
        for (int i = threadIdx.x; i < kProbeBytes / 4; i += blockDim.x)
            reinterpret_cast<uint32_t *>(smem)[i] = mix(uint32_t(i) * 2654435761u + 12345u) & keep;
    }
    __syncthreads();
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    if (MODE == kLinear) {
        // lane l of a half-wave: byte 4 (l % 32) of a row; rows move by whole 128-byte
        // steps (base < 8 KiB, offsets 7 x 1024 at most: every address < 16 KiB)
        uint32_t base = 4u * (threadIdx.x & 31u) + (mix(tid >> 6) & 63u) * 128u;
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < kReadsPerIter; ++c) acc += lds_read<WIDTH>(base + uint32_t(c) * 1024u);
            base = (base + 19u * 128u) & uint32_t(kProbeBytes / 2 - 1);
        }
    } else if (MODE == kIndependent) {
        // base < 8 KiB, offsets <= 7 x 1022: every address < 16 KiB; even for 2-byte reads
        uint32_t base = mix(tid) & uint32_t(kProbeBytes / 2 - WIDTH);
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < kReadsPerIter; ++c) acc += lds_read<WIDTH>(base + uint32_t(c) * kStride);
            base = (base + kAdvance) & uint32_t(kProbeBytes / 2 - WIDTH);
        }
    } else {  // kDependent
        // 1-byte entries: row v < 256 of 61 bytes, column 7c < 61 (address < 15616);
        // 2-byte entries: row v < 1600 of 5, column c % 5 (address < 16000)
        uint32_t v[kReadsPerIter];
#pragma unroll
        for (int c = 0; c < kReadsPerIter; ++c) v[c] = mix(tid * kReadsPerIter + c) % (WIDTH == 1 ? 256u : kRows16);
        for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int c = 0; c < kReadsPerIter; ++c) {
                if (WIDTH == 1)
                    v[c] = lds_read<1>(__umul24(v[c], kRow8) + uint32_t(7 * c));
                else
                    v[c] = lds_read<2>(2u * (__umul24(v[c], kRow16) + uint32_t(c % 5)));
            }
        }
#pragma unroll
        for (int c = 0; c < kReadsPerIter; ++c) acc += v[c];
    }
    if (acc == 0xffffffffu) sink[0] = acc;  // never true (sums of eight values < 1600): keeps the reads
}

template <int WIDTH>
const void *probe_fn_w(int mode) {
    if (mode == kDependent) return reinterpret_cast<const void *>(&k_lds_probe<WIDTH, kDependent>);
    if (mode == kLinear) return reinterpret_cast<const void *>(&k_lds_probe<WIDTH, kLinear>);
    return reinterpret_cast<const void *>(&k_lds_probe<WIDTH, kIndependent>);
}

const void *probe_fn(int width, int mode) { return width == 1 ? probe_fn_w<1>(mode) : probe_fn_w<2>(mode); }

}  // namespace

extern "C" int64_t dfa_lds_probe(int32_t width, int32_t mode, int32_t blocks, int64_t iters,
                                 unsigned long long *sink, void *stream) {
    if ((width != 1 && width != 2) || mode < 0 || mode > 2 || blocks < 1 || blocks > (1 << 20) ||
        iters < 1 || iters > (int64_t(1) << 24) || !sink || (reinterpret_cast<uintptr_t>(sink) & 7)) {
        dfa::set_error("dfa_lds_probe: bad arguments");
        return DFA_EINVAL;
    }
    const void *fn = probe_fn(width, mode);
    if (!dfa::allow_lds(fn, kProbeBytes)) return DFA_EHIP;
    int64_t it = iters;
    void *args[] = {&it, &sink};
    if (!dfa::hip_ok(hipLaunchKernel(fn, dim3(unsigned(blocks)), dim3(kProbeThreads), args, kProbeBytes,
                                     reinterpret_cast<hipStream_t>(stream)),
                     "k_lds_probe launch"))
        return DFA_EHIP;
    dfa::clear_error();
    return int64_t(blocks) * kProbeThreads * iters * kReadsPerIter;
}
