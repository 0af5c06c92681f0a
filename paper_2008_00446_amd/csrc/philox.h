// Counter-based Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11) for the constraint draw theta_i of the
// sampled convex program (Sec. 4.2).  Only output word 0 is needed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stba {

__device__ inline uint64_t philox4x64_10_word0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    return c0;
}

// Keep the link into the observation of camera `cam` of point `pt` at LM
// iteration `t` iff its 53-bit uniform is below `thr` = ceil(alpha * 2^53).
__device__ inline bool keep_link(uint64_t seed, uint64_t t, uint64_t pt, uint64_t cam, uint64_t thr) {
    const uint64_t x0 = philox4x64_10_word0(t, pt, cam, 0ull, seed, 0ull);
    return (x0 >> 11) < thr;
}

}  // namespace stba
