// XCD-aware block order shared by the kernels: MI355X has 8 XCDs, each with
// its own L2, and hardware block b of a launch runs on XCD b % 8.
#pragma once

#include <hip/hip_runtime.h>

namespace fvk {

// Logical index of hardware block b of nb: block b runs on XCD b % 8 as that
// XCD's (b / 8)-th block; XCDs 0 .. r-1 (r = nb % 8) get q + 1 = nb / 8 + 1
// consecutive logical indices, the others q -- a bijection for any nb.
__device__ __forceinline__ long xcd_remap(long b, long nb) {
    const long q = nb / 8, r = nb % 8, x = b % 8;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + b / 8;
}

}  // namespace fvk
