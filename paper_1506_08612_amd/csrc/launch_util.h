// Host-side launch helpers shared by the HIP translation units of libdfa.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <set>
#include <utility>

#include "dfa_internal.h"

namespace dfa {

inline bool hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    set_error("%s: %s", what, hipGetErrorString(e));
    return false;
}

// Raise a kernel's dynamic-LDS limit once per (device, kernel), so that later
// calls -- including calls made while a stream is being captured into a
// graph -- only enqueue launches.  The scan kernels read their tables at
// absolute LDS addresses counted from 0, where dynamic LDS starts only when
// the kernel has no static LDS (a device-library call such as a workgroup
// vote can bring some in): such a kernel is refused here.
inline bool allow_lds(const void *fn, int bytes) {
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> done;
    int dev = 0;
    if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return false;
    std::lock_guard<std::mutex> lk(mu);
    if (done.count({dev, fn})) return true;
    hipFuncAttributes a{};
    if (!hip_ok(hipFuncGetAttributes(&a, fn), "hipFuncGetAttributes")) return false;
    if (a.sharedSizeBytes != 0) {
        set_error("kernel has %zu bytes of static LDS: its table would not start at LDS address 0",
                  size_t(a.sharedSizeBytes));
        return false;
    }
    if (!hip_ok(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes), "hipFuncSetAttribute"))
        return false;
    done.insert({dev, fn});
    return true;
}

}  // namespace dfa
