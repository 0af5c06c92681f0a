// a5: independent dense solves S_k dc_k = b_k, one workgroup per cluster
// (Eq. 13: the decomposed reduced camera systems; the paper uses a dense LL^T
// per cluster).  Blocked right-looking Cholesky with 32 x 32 FP64 tiles and the
// forward substitution carried along:
//   (a) one wavefront factors and inverts the diagonal tile in registers
//       (W = L_pp^-1, kept in LDS and transposed in the unused upper triangle)
//       and forward-solves its slice of the right-hand side,
//   (b) the panel below is X = A_ip W^T, an MFMA product per 32-row tile, and
//       the right-hand side is updated with it,
//   (c) trailing update A_ij -= L_ip L_jp^T of the lower tiles with
//       v_mfma_f64_16x16x4_f64; the next panel's column is updated first so
//       that its diagonal tile is factored while the other waves finish (c);
// then the backward solve L^T x = y with the stored W^T.  Matrices are
// column-major, padded to a multiple of 32 with an identity tail.
#include "kernels.h"

namespace stba {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kCholThreads = 512;
constexpr int kCholWaves = kCholThreads / 64;

__device__ inline double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Diagonal tile (rows/cols off..off+31), one wavefront, registers only.  Lane r
// owns row r (lanes 32..63 mirror rows 0..31).  L = chol(A_pp) right-looking with
// the pivot column broadcast by v_readlane; entries above the diagonal hold
// don't-care values, so the updates carry no predicate.  Then W = L^-1, lane c
// computing column c by forward substitution with L[rr][k] read from lane rr.
// Writes L to the lower triangle of A, W^T to its strict upper triangle, W to
// LDS, and replaces x_p by y_p = W x_p.  Returns true if a pivot failed.
__device__ __attribute__((noinline)) bool diag_factor_invert(double *A, int64_t Np, int64_t off, int lane, double (*Wi)[kNB + 1],
                                          double *x) {
    const int r = lane & (kNB - 1);
    double a[kNB];
#pragma unroll
    for (int j = 0; j < kNB; ++j) a[j] = A[(off + r) + (off + j) * Np];
    bool bad = false;
    int rq = r;
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
        // make the lane index opaque per step so the lane-mask compares of all 32
        // steps are not hoisted into SGPRs at once
        asm volatile("" : "+v"(rq));
        double d = readlane_d(a[k], k);
        if (!(d > 0.0) || !isfinite(d)) {
            bad = true;
            d = 1.0;
        }
        const double s = sqrt(d);
        const double is = 1.0 / s;
        a[k] = (rq == k) ? s : ((rq > k) ? a[k] * is : 0.0);
        // readlane results live in SGPRs: consume them in chunks of 8 so that at
        // most 16 SGPRs are live at a time (scheduling barriers stop hoisting)
#pragma unroll
        for (int j = k + 1; j < kNB; ++j) {
            a[j] = fma(-a[k], readlane_d(a[k], j), a[j]);
            if (((j - k) & 7) == 0) __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    const int c = r;
    double w[kNB];
    int cq = c;
#pragma unroll
    for (int rr = 0; rr < kNB; ++rr) {
        asm volatile("" : "+v"(cq));
        double s0 = (cq == rr) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < rr; ++k) {
            if (k & 1) s1 = fma(-readlane_d(a[k], rr), w[k], s1);
            else s0 = fma(-readlane_d(a[k], rr), w[k], s0);
            if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
        w[rr] = (s0 + s1) / readlane_d(a[rr], rr);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (lane < kNB) {
#pragma unroll
        for (int j = 0; j < kNB; ++j) {
            if (j <= r) A[(off + r) + (off + j) * Np] = a[j];   // L (lower, with diagonal)
            else A[(off + r) + (off + j) * Np] = w[j];           // W^T: W[j][r] at (row r, column j)
            Wi[j][c] = w[j];
        }
    }
    __syncwarp();
    double y = 0.0;
#pragma unroll 8
    for (int j = 0; j < kNB; ++j) y = fma(Wi[c][j], x[off + j], y);
    __syncwarp();
    if (lane < kNB) x[off + c] = y;
    return bad;
}

// MFMA f64 16x16x4 register layout on gfx950 (checked on the device): operand
// A[i][k] (16 x 4) in lane i + 16 k, operand B[k][j] (4 x 16) in lane j + 16 k,
// result D[i][j] in lane j + 16 (i % 4), element i / 4.  With the first operand
// taken from the column tile and the second from the row tile, D[i][j] is the
// output element (row 16R + j, column 16C + i), so stores are row-contiguous.

// Panel tile: X = A_ip W^T in place (rows ri..ri+31, columns off..off+31), and
// x_i -= X y_p for the right-hand side.
__device__ inline void tile_trsm(double *A, int64_t Np, int64_t ri, int64_t off, int lane,
                                 const double (*Wi)[kNB + 1], const double *y, double *x) {
    const int lr = lane & 15, lk = lane >> 4;
    double bop[2][8];
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) bop[R][kk] = A[(ri + 16 * R + lr) + (off + 4 * kk + lk) * Np];
    d4 acc[2][2];
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C) acc[R][C] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const double a0 = Wi[lr][4 * kk + lk], a1 = Wi[16 + lr][4 * kk + lk];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bop[0][kk], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bop[0][kk], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bop[1][kk], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bop[1][kk], acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int R = 0; R < 2; ++R) {
        double s = 0.0;
#pragma unroll
        for (int C = 0; C < 2; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                A[(ri + 16 * R + lr) + (off + 16 * C + 4 * v + lk) * Np] = acc[R][C][v];
                s = fma(acc[R][C][v], y[16 * C + 4 * v + lk], s);
            }
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        if (lk == 0) x[ri + 16 * R + lr] -= s;
    }
}

// Trailing tile: A_ij -= L_ip L_jp^T (rows ri.., columns cj.., panel columns off..).
__device__ inline void tile_update(double *A, int64_t Np, int64_t ri, int64_t cj, int64_t off, int lane) {
    const int lr = lane & 15, lk = lane >> 4;
    double bi[2][8], aj[2][8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const int64_t col = (off + 4 * kk + lk) * Np;
        bi[0][kk] = A[ri + lr + col];
        bi[1][kk] = A[ri + 16 + lr + col];
        aj[0][kk] = -A[cj + lr + col];
        aj[1][kk] = -A[cj + 16 + lr + col];
    }
    d4 acc[2][2];
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[R][C][v] = A[(ri + 16 * R + lr) + (cj + 16 * C + 4 * v + lk) * Np];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj[0][kk], bi[0][kk], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj[1][kk], bi[0][kk], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj[0][kk], bi[1][kk], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aj[1][kk], bi[1][kk], acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) A[(ri + 16 * R + lr) + (cj + 16 * C + 4 * v + lk) * Np] = acc[R][C][v];
}

__global__ __launch_bounds__(kCholThreads) void k_chol(int32_t l, const int32_t *__restrict__ cl_n,
                                                       const int32_t *__restrict__ cl_Np,
                                                       const int64_t *__restrict__ S_off,
                                                       const int32_t *__restrict__ cl_start,
                                                       const int32_t *__restrict__ cl_cams, double *__restrict__ S,
                                                       const double *__restrict__ b, double *__restrict__ dcam,
                                                       int32_t *__restrict__ cl_status, int32_t max_Np) {
    extern __shared__ double smem[];
    double(*Wi)[kNB + 1] = reinterpret_cast<double(*)[kNB + 1]>(smem);
    double *x = smem + kNB * (kNB + 1);
    double *red = x + max_Np;             // kCholThreads
    double *zb = red + kCholThreads;      // kNB
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
    for (int i = tid; i < Np; i += kCholThreads) x[i] = (i < N) ? b[9 * (int64_t)cl_cams[c0 + i / 9] + i % 9] : 0.0;
    if (tid == 0) bad = 0;
    __syncthreads();
    // Look-ahead schedule: after panel p is solved, the tiles of column p + 1 are
    // updated first; then wave 0 factors diagonal tile p + 1 while the other
    // waves finish the trailing update of step p.
    if (wave == 0) {
        const bool fb = diag_factor_invert(A, Np, 0, lane, Wi, x);
        if (fb && lane == 0) bad = 1;
    }
    __syncthreads();
    for (int i = 1 + wave; i < nt; i += kCholWaves) tile_trsm(A, Np, (int64_t)i * kNB, 0, lane, Wi, x, x);
    __syncthreads();
    for (int p = 0; p + 1 < nt; ++p) {
        const int64_t off = (int64_t)p * kNB;
        const int q = p + 1;   // next panel
        // column q of the trailing matrix: tiles (i, q), i >= q
        for (int i = q + wave; i < nt; i += kCholWaves)
            tile_update(A, Np, (int64_t)i * kNB, (int64_t)q * kNB, off, lane);
        __syncthreads();
        if (wave == 0) {
            const bool fb = diag_factor_invert(A, Np, (int64_t)q * kNB, lane, Wi, x);
            if (fb && lane == 0) bad = 1;
        } else {
            // remaining trailing tiles (i, j), q < j <= i
            const int nrem = nt - q - 1;
            const int ntiles = nrem * (nrem + 1) / 2;
            for (int tt = wave - 1; tt < ntiles; tt += kCholWaves - 1) {
                int a = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
                while ((a + 1) * (a + 2) / 2 <= tt) ++a;
                while (a * (a + 1) / 2 > tt) --a;
                const int bcol = tt - a * (a + 1) / 2;
                tile_update(A, Np, (int64_t)(q + 1 + a) * kNB, (int64_t)(q + 1 + bcol) * kNB, off, lane);
            }
        }
        __syncthreads();
        const int64_t offq = (int64_t)q * kNB;
        for (int i = q + 1 + wave; i < nt; i += kCholWaves)
            tile_trsm(A, Np, (int64_t)i * kNB, offq, lane, Wi, x + offq, x);
        __syncthreads();
    }
    // backward solve L^T x = y: x_p = W_p^T (y_p - sum_{i > p} L_ip^T x_i)
    for (int p = nt - 1; p >= 0; --p) {
        const int64_t off = (int64_t)p * kNB;
        {
            constexpr int G = kCholThreads / kNB;
            const int c = tid / G, g = tid % G;
            double s = 0.0;
            for (int64_t row = off + kNB + g; row < Np; row += G) s = fma(A[row + (off + c) * Np], x[row], s);
            red[c * G + g] = s;
        }
        __syncthreads();
        if (tid < kNB) {
            constexpr int G = kCholThreads / kNB;
            double s = x[off + tid];
#pragma unroll
            for (int g = 0; g < G; ++g) s -= red[tid * G + g];
            zb[tid] = s;
        }
        __syncthreads();
        if (tid < kNB) {
            const int r = tid;
            double s = zb[r] / A[(off + r) + (off + r) * Np];
            for (int c = r + 1; c < kNB; ++c) s = fma(A[(off + r) + (off + c) * Np], zb[c], s);   // W[c][r]
            x[off + r] = s;
        }
        __syncthreads();
    }
    for (int i = tid; i < N; i += kCholThreads) dcam[9 * (int64_t)cl_cams[c0 + i / 9] + i % 9] = x[i];
    if (tid == 0) cl_status[k] = bad ? STBA_ENOTPD : STBA_OK;
}

}  // namespace

hipError_t launch_chol(int32_t l, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                       const int32_t *cl_start, const int32_t *cl_cams, double *S, const double *b, double *dcam,
                       int32_t *cl_status, int32_t max_Np, hipStream_t st) {
    const size_t shmem = sizeof(double) * ((size_t)kNB * (kNB + 1) + (size_t)max_Np + kCholThreads + kNB);
    k_chol<<<(unsigned)l, kCholThreads, shmem, st>>>(l, cl_n, cl_Np, S_off, cl_start, cl_cams, S, b, dcam, cl_status,
                                                     max_Np);
    return hipGetLastError();
}

}  // namespace stba
