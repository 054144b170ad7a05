// Device helpers shared by the HIP kernels of libnfftgp.
#pragma once

#include <hip/hip_runtime.h>

namespace nfftgp {

// i / d for 0 <= i < 2^22 and d >= 1 by a float reciprocal and one
// correction step (exact in that range: the float quotient is off by less
// than one).
__device__ __forceinline__ int fdiv_small(int i, int d, float inv_d)
{
    int q = (int)((float)i * inv_d);
    const int r = i - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

// Device arrays reached through pointers stored in a descriptor: the compiler
// cannot tell such generic pointers from LDS ones, and loads through generic
// pointers are FLAT instructions, which also count in the LDS wait counter, so
// one global load in flight (a prefetch) turns every LDS wait into a full
// wait.  Kernels read these arrays through global-address-space pointers.
template <typename T>
using gmem = const __attribute__((address_space(1))) T;

// The dispatcher deals work-groups round-robin over the 8 XCDs (work-group b
// runs on XCD b % 8), and each XCD has its own L2.  Work lists are ordered in
// space (by tile), so giving every XCD one contiguous range of the list keeps
// the grid region a range reads inside one L2: the b-th work-group takes item
// xcd_item(b, n), a bijection of [0, n).
__device__ __forceinline__ int xcd_item(int b, int n)
{
    constexpr int X = 8;
    const int x = b % X, k = b / X;
    const int q = n / X, r = n % X;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace nfftgp
