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

}  // namespace nfftgp
