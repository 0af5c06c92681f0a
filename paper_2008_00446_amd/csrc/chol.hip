// a5: independent dense solves S_k dc_k = b_k, one workgroup per cluster
// (Eq. 13: the decomposed reduced camera systems; the paper uses a dense LL^T
// per cluster).  Blocked right-looking Cholesky with 32 x 32 FP64 tiles:
//   (a) factor the diagonal tile in LDS and forward-solve its slice of b,
//   (b) triangular solve of the panel below it (one row per thread),
//   (c) trailing update A_ij -= L_ip L_jp^T with v_mfma_f64_16x16x4_f64,
// then the backward solve L^T x = y.  Matrices are column-major, padded to a
// multiple of 32 with an identity tail.
#include "kernels.h"

namespace stba {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// MFMA f64 16x16x4 register layout on gfx950 (checked on the device): operand
// A[i][k] (16 x 4) in lane i + 16 k, operand B[k][j] (4 x 16) in lane j + 16 k,
// result D[i][j] in lane j + 16 (i % 4), element i / 4.
__device__ inline void tile_update(double *A, int64_t Np, int64_t ri, int64_t cj, int64_t off, int lane) {
    const int lr = lane & 15, lk = lane >> 4;
    d4 acc[2][2];
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[R][C][v] = A[(ri + 16 * R + lr) + (cj + 16 * C + 4 * v + lk) * Np];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const int64_t col = (off + 4 * kk + lk) * Np;
        const double bi0 = A[ri + lr + col], bi1 = A[ri + 16 + lr + col];
        const double aj0 = -A[cj + lr + col], aj1 = -A[cj + 16 + lr + col];
        // D[i][j] = sum_k L_j[16C + i][k] L_i[16R + j][k] = (L_i L_j^T)[16R + j][16C + i];
        // this lane holds i = 4 v + lk, j = lr
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj0, bi0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj1, bi0, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj0, bi1, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj1, bi1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) A[(ri + 16 * R + lr) + (cj + 16 * C + 4 * v + lk) * Np] = acc[R][C][v];
}

__global__ __launch_bounds__(256) void k_chol(int32_t l, const int32_t *__restrict__ cl_n,
                                              const int32_t *__restrict__ cl_Np, const int64_t *__restrict__ S_off,
                                              const int32_t *__restrict__ cl_start,
                                              const int32_t *__restrict__ cl_cams, double *__restrict__ S,
                                              const double *__restrict__ b, double *__restrict__ dcam,
                                              int32_t *__restrict__ cl_status, int32_t max_Np) {
    extern __shared__ double smem[];
    double(*T)[kNB + 1] = reinterpret_cast<double(*)[kNB + 1]>(smem);
    double *x = smem + kNB * (kNB + 1);
    double *red = x + max_Np;
    __shared__ int bad;
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nk = cl_n[k];
    if (nk == 0) {
        if (tid == 0) cl_status[k] = STBA_OK;
        return;
    }
    const int64_t Np = cl_Np[k];
    const int N = 9 * nk;
    const int nt = (int)(Np / kNB);
    double *A = S + S_off[k];
    const int c0 = cl_start[k];
    for (int i = tid; i < Np; i += 256) x[i] = (i < N) ? b[9 * (int64_t)cl_cams[c0 + i / 9] + i % 9] : 0.0;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int p = 0; p < nt; ++p) {
        const int64_t off = (int64_t)p * kNB;
        // (a) diagonal tile
        for (int e = tid; e < kNB * kNB; e += 256) {
            const int i = e & (kNB - 1), j = e / kNB;
            T[i][j] = A[(off + i) + (off + j) * Np];
        }
        __syncthreads();
        for (int kk = 0; kk < kNB; ++kk) {
            if (tid == 0) {
                double d = T[kk][kk];
                if (!(d > 0.0) || !isfinite(d)) {
                    bad = 1;
                    d = 1.0;
                }
                const double s = sqrt(d);
                T[kk][kk] = s;
                x[off + kk] /= s;
            }
            __syncthreads();
            if (tid > kk && tid < kNB) T[tid][kk] /= T[kk][kk];
            __syncthreads();
            for (int e = tid; e < kNB * kNB; e += 256) {
                const int i = e & (kNB - 1), j = e / kNB;
                if (j > kk && i >= j) T[i][j] -= T[i][kk] * T[j][kk];
            }
            if (tid > kk && tid < kNB) x[off + tid] -= T[tid][kk] * x[off + kk];
            __syncthreads();
        }
        for (int e = tid; e < kNB * kNB; e += 256) {
            const int i = e & (kNB - 1), j = e / kNB;
            if (i >= j) A[(off + i) + (off + j) * Np] = T[i][j];
        }
        // (b) panel below: X L_pp^T = A_panel, one row per thread
        for (int64_t row = off + kNB + tid; row < Np; row += 256) {
            double rv[kNB];
#pragma unroll
            for (int kk = 0; kk < kNB; ++kk) rv[kk] = A[row + (off + kk) * Np];
#pragma unroll
            for (int kk = 0; kk < kNB; ++kk) {
                double s = rv[kk];
#pragma unroll
                for (int k2 = 0; k2 < kk; ++k2) s -= rv[k2] * T[kk][k2];
                rv[kk] = s / T[kk][kk];
            }
            double s = 0.0;
#pragma unroll
            for (int kk = 0; kk < kNB; ++kk) {
                A[row + (off + kk) * Np] = rv[kk];
                s += rv[kk] * x[off + kk];
            }
            x[row] -= s;
        }
        __syncthreads();
        // (c) trailing update of the lower tiles (ti >= tj > p)
        const int nrem = nt - p - 1;
        const int ntiles = nrem * (nrem + 1) / 2;
        for (int tt = wave; tt < ntiles; tt += 4) {
            int a = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
            while ((a + 1) * (a + 2) / 2 <= tt) ++a;
            while (a * (a + 1) / 2 > tt) --a;
            const int bcol = tt - a * (a + 1) / 2;
            tile_update(A, Np, (int64_t)(p + 1 + a) * kNB, (int64_t)(p + 1 + bcol) * kNB, off, lane);
        }
        __syncthreads();
    }
    // backward solve L^T x = y
    for (int p = nt - 1; p >= 0; --p) {
        const int64_t off = (int64_t)p * kNB;
        {
            const int kk = tid >> 3, g = tid & 7;
            double s = 0.0;
            for (int64_t row = off + kNB + g; row < Np; row += 8) s += A[row + (off + kk) * Np] * x[row];
            red[g * kNB + kk] = s;
        }
        for (int e = tid; e < kNB * kNB; e += 256) {
            const int i = e & (kNB - 1), j = e / kNB;
            T[i][j] = A[(off + i) + (off + j) * Np];
        }
        __syncthreads();
        if (tid < kNB) {
            double s = 0.0;
#pragma unroll
            for (int g = 0; g < 8; ++g) s += red[g * kNB + tid];
            x[off + tid] -= s;
        }
        __syncthreads();
        for (int kk = kNB - 1; kk >= 0; --kk) {
            if (tid == 0) x[off + kk] /= T[kk][kk];
            __syncthreads();
            if (tid < kk) x[off + tid] -= T[kk][tid] * x[off + kk];
            __syncthreads();
        }
    }
    for (int i = tid; i < N; i += 256) dcam[9 * (int64_t)cl_cams[c0 + i / 9] + i % 9] = x[i];
    if (tid == 0) cl_status[k] = bad ? STBA_ENOTPD : STBA_OK;
}

}  // namespace

hipError_t launch_chol(int32_t l, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                       const int32_t *cl_start, const int32_t *cl_cams, double *S, const double *b, double *dcam,
                       int32_t *cl_status, int32_t max_Np, hipStream_t st) {
    const size_t shmem = sizeof(double) * ((size_t)kNB * (kNB + 1) + (size_t)max_Np + 8 * kNB);
    k_chol<<<(unsigned)l, 256, shmem, st>>>(l, cl_n, cl_Np, S_off, cl_start, cl_cams, S, b, dcam, cl_status,
                                            max_Np);
    return hipGetLastError();
}

}  // namespace stba
