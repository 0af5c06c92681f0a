// Shared device/host definitions of the STBA gfx950 library (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "stba.h"

namespace stba {

constexpr int kNB = 32;            // Cholesky tile order (FP64)
// Per-observation record written by the point kernel for the Schur assembly:
// G = J_p R_s^-1 (2x3 row-major, R_s^T R_s = V*_s), M = I - J_p V*_s^-1 J_p^T
// (m00 m01 m11), r = f + J_p V*_s^-1 w'_s (2), so that Y = J_c^T G and
// W V*^-1 W'^T = J_c^T (G G'^T) J_c'.  FP64: [G pad M r pad] (16 doubles: G
// in the first 64 bytes, M and r in the second), the assembly reading J_c from
// the Jacobian itself; FP32: [J_c G M r pad] (32 floats), J_c copied in (FP32
// J_c rows are only 8-byte aligned).
template <typename T> constexpr int obs_rec_elems() { return sizeof(T) == 8 ? 16 : 32; }
inline size_t obs_rec_bytes(bool fp64) { return fp64 ? 16 * 8 : 32 * 4; }
constexpr int kSegRec = 16;        // per-segment record at the head observation: R^-1 (6), V*^-1 (6), V*^-1 w' (3)
constexpr int kSchurChunk = 512;   // observation pairs per Schur work item (16 rounds of 32 pair slots)
constexpr int kSchurPart = 100;    // doubles per partial sum: 81 block entries, 9 diag(U), 9 rhs, pad
constexpr int kVjpPart = 1792;     // observations per wavefront in the camera sums of J^T v (28 rounds of 64)
constexpr int kMaxCamsForClusters = 16384;   // cluster layout: every camera id and cluster count held in LDS
constexpr int kSgcMaxCams = 6144;          // graph clustering: cameras held in one workgroup's LDS (24 B each)

// Status words kept in the workspace (int32[16]).
enum StatusWord : int {
    kStSticky = 0,       // first device-side data error (STBA_EINVAL / STBA_EDATA)
    kStJacRan = 1,       // 1 if the residual/Jacobian kernel ran in this iteration
    kStPointBad = 2,     // a segment block V*_s failed to factorise
    kStCount = 16,
};

__host__ __device__ inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

__device__ inline void set_status(int32_t *w, int code) {
    atomicCAS(reinterpret_cast<int *>(w), 0, code);
}

// Thread t's sum of p[t], p[t + 256], .. in that order, eight loads in flight
// at a time (the same additions as a plain strided loop, so the same result).
__device__ inline double strided_sum_256(const double *__restrict__ p, int64_t count) {
    double s = 0.0;
    int64_t i = threadIdx.x;
    for (; i + 7 * 256 < count; i += 8 * 256) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[i + u * 256];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; i < count; i += 256) s += p[i];
    return s;
}

// Deterministic fixed-order sum over a 256-thread block (LDS tree).
__device__ inline double block_sum_256(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

}  // namespace stba
