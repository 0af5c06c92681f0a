// a5: independent dense solves S_k dc_k = b_k (Eq. 13: the decomposed reduced
// camera systems; the paper uses a dense LL^T per cluster), blocked Cholesky
// with 32 x 32 FP64 tiles.  Matrices are column-major, padded to a multiple of
// 32 with an identity tail.  Two forms:
//  - k_chol, one workgroup per cluster (many clusters), right-looking with the
//    forward substitution carried along:
//   (a) one wavefront factors and inverts the diagonal tile in registers
//       (W = L_pp^-1, kept in LDS and transposed in the unused upper triangle)
//       and forward-solves its slice of the right-hand side,
//   (b) the panel below is X = A_ip W^T, an MFMA product per 32-row tile, and
//       the right-hand side is updated with it,
//   (c) trailing update A_ij -= L_ip L_jp^T of the lower tiles with
//       v_mfma_f64_16x16x4_f64; the next panel's column is updated first so
//       that its diagonal tile is factored while the other waves finish (c);
//    then the backward solve L^T x = y with the stored W^T;
//  - k_chol_tiles, one wavefront per tile (few clusters): a dataflow over the
//    tiles with the substitutions in the same launch (described where it is
//    defined);
//  - k_chol_team, teams of wavefronts per cluster for maps with many clusters.
// k_sweep repeats both substitutions with a stored factor (the MIXED
// refinement step).
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

// 1 / sqrt(d) from v_rsq_f64 (about 24 correct bits) and one Newton step: relative error near
// 2^-47, below the rounding that a column of 32 or more products already
// carries; used on the diagonal chain of the tile factorisation, where every
// dependent operation costs about 32 cycles.
__device__ inline double rsqrt_once(double d) {
    const double h = 0.5 * d;
    const double y = __builtin_amdgcn_rsq(d);
    return fma(y, fma(-h * y, y, 0.5), y);
}

// 1 / sqrt(d): the hardware estimate and two Newton steps y += y (1/2 - d y^2 / 2),
// each of which squares the relative error; a shorter dependent chain than a
// correctly rounded square root followed by a division.
__device__ inline double rsqrt_refined(double d) {
    const double h = 0.5 * d;
    double y = __builtin_amdgcn_rsq(d);
    y = fma(y, fma(-h * y, y, 0.5), y);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}

// Diagonal tile (rows/cols off..off+31), one wavefront, right-looking.  Lane r
// holds row r of the tile in registers (lanes 32..63 mirror rows 0..31).  At
// step k the pivot comes from lane k (v_readlane); every lane scales its entry
// of column k and writes it to LDS, and all lanes read the column back (LDS
// operations of one wavefront complete in order) to update their row.  Entries
// above the diagonal are carried as don't-care values, so no update is
// predicated.  The inverse W = L^-1 is built in the same sweep from the same
// broadcast column: lane c holds column c of W, and at step k
//   W[k][c] /= L_kk,   W[r][c] -= L_rk W[k][c]  (r > k).
// Both store W^T in the upper triangle of the tile with its diagonal (so the
// diagonal holds 1 / L_rr).
// kTile = false: the tile is read from A; L goes to the strict lower triangle
//   and x_p (LDS) is replaced by y_p = W x_p.
// kTile = true: the tile is read from Ls (row-major); the stores are at device
//   scope and the lower triangle is left as it was (no reader needs it).
// Both leave W row-major in Wi.  Returns true if a pivot was not positive.
template <bool kTile>
__device__ __forceinline__ bool diag_factor_invert(double *A, int64_t Np, int64_t off, int lane,
                                                   double (*Ls)[kNB + 1], double (*Wi)[kNB + 1], double *col,
                                                   double *x) {
    const int r = lane & (kNB - 1);
    double a[kNB], w[kNB];
#pragma unroll
    for (int j = 0; j < kNB; ++j) {
        a[j] = kTile ? Ls[r][j] : A[(off + r) + (off + j) * Np];
        w[j] = (j == r) ? 1.0 : 0.0;
    }
    bool bad = false;
    // scheduling barriers keep each step's instructions together, so that the
    // unrolled steps are not interleaved into more live registers than exist
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
        double d = readlane_d(a[k], k);
        if (!(d > 0.0) || !isfinite(d)) {
            bad = true;
            d = 1.0;
        }
        const double is = rsqrt_refined(d);
        const double sd = d * is;
        a[k] = (r == k) ? sd : ((r > k) ? a[k] * is : 0.0);
        w[k] *= is;
        if (k + 1 < kNB) {
            col[r] = a[k];
#pragma unroll
            for (int j = k + 1; j < kNB; ++j) {
                const double lj = col[j];
                a[j] = fma(-a[k], lj, a[j]);
                w[j] = fma(-lj, w[k], w[j]);
            }
            // pin the updated rows here: otherwise the updates are sunk to the
            // next use of each entry and every column read stays live
#pragma unroll
            for (int j = k + 1; j < kNB; ++j) asm volatile("" : "+v"(a[j]), "+v"(w[j]));
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    const int c = r;
    if (lane < kNB) {
#pragma unroll
        for (int j = 0; j < kNB; ++j) {
            Wi[j][c] = w[j];
            if (kTile) {
                if (j >= r)
                    __hip_atomic_store(A + (off + r) + (off + j) * Np, w[j], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);   // W^T: W[j][r] at (row r, column j)
            } else {
                A[(off + r) + (off + j) * Np] = j < r ? a[j] : w[j];
            }
        }
    }
    __syncwarp();
    if (kTile) return bad;
    double y = 0.0;
#pragma unroll 8
    for (int j = 0; j < kNB; ++j) y = fma(Wi[c][j], x[off + j], y);
    __syncwarp();
    if (lane < kNB) x[off + c] = y;
    return bad;
}

// Raise *f = v after all earlier stores of the wavefront have completed.
__device__ inline void raise_flag(int32_t *f, int v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Diagonal tile of the tile-parallel factorisation, one wavefront: the tile
// comes in Ls (row-major).  Lanes 0..31 carry row r of the tile and become row
// r of L; lanes 32..63 carry column r of the identity and become column r of
// W = L^-1.  Both updates of a right-looking step have the form
// v_j -= v_k l_jk (row: l_rk l_jk; column of W: W[k][c] l_jk), so one
// instruction serves both halves.  At step k the pivot comes from lane k
// (v_readlane) and the scaled column l_.k goes through LDS.  At the end W goes
// row-major to Wl and W^T to the upper triangle of the tile in A (device scope,
// diagonal included, so it holds 1 / L_kk).
// Returns true if a pivot was not positive.
// panel_flag (nullable): raised a few pivots in, once the stores issued before
// the call have completed (the loop issues no other global memory operations).
__device__ __forceinline__ bool band_factor_invert(double *A, int64_t Np, int64_t off, int lane,
                                                   double (*Ls)[kNB + 1], double (*Wl)[kNB + 1],
                                                   double *col, int32_t *panel_flag) {
    const int r = lane & (kNB - 1);
    const bool wl = lane >= kNB;
    double v[kNB];
#pragma unroll
    for (int j = 0; j < kNB; ++j) v[j] = wl ? (j == r ? 1.0 : 0.0) : Ls[r][j];
    bool bad = false;
    int rq = r;
    // the pivot of the next step only needs lane k+1's own entries
    // (a_k+1,k+1 - l_k+1,k^2), so its reciprocal square root is computed while
    // the broadcast of column k through LDS is in flight
    double d = readlane_d(v[0], 0);
    if (!(d > 0.0) || !isfinite(d)) {
        bad = true;
        d = 1.0;
    }
    double is = rsqrt_once(d);
    // Software-pipelined steps.  Step k needs of step k-1's updates only those
    // of columns k and k+1 (its pivot and the next one); the others (columns
    // >= k+2) are issued in step k among the dependent operations of the next
    // pivot's reciprocal square root, whose latencies they fill.  The columns
    // of L alternate between the two halves of col, so step k reads column
    // k-1 again for them.
    double vkp = 0.0;   // this lane's entry of column k-1
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kNB; ++k) {
        // an opaque copy of the lane index per step: the lane compares are not
        // hoisted into masks for all 32 steps at once
        asm volatile("" : "+v"(rq));
        if (k == 4 && panel_flag != nullptr) raise_flag(panel_flag, 1);
        double *cc = col + (k & 1) * kNB;
        const double *cp = col + ((k + 1) & 1) * kNB;
        // one scaling for every lane: rows r > k get l_rk, lane k gets d / sqrt(d)
        // = L_kk, W lanes get W[k][c]; rows above k keep don't-care values that
        // only touch entries above the diagonal
        v[k] *= is;
        if (k + 1 < kNB) {
            if (!wl) cc[rq] = v[k];
            const double t = fma(-v[k], v[k], v[k + 1]);
            __builtin_amdgcn_sched_barrier(0);
            double lc[kNB], lp[kNB];
#pragma unroll
            for (int j = k + 1; j < kNB; ++j) lc[j] = cc[j];
            if (k >= 1) {
#pragma unroll
                for (int j = k + 2; j < kNB; ++j) lp[j] = cp[j];
            }
            __builtin_amdgcn_sched_barrier(0);
            // the next pivot (lane k+1's own entries only) while the column
            // reads are in flight, and step k-1's deferred updates: every lane
            // takes the reciprocal square root of its own t and lane k+1's is
            // broadcast, so the pivot check stays off this chain (a pivot that is
            // not positive yields NaN, and the tile reports it as failed)
            const double is_next = readlane_d(rsqrt_once(t), k + 1);
            const double dn = readlane_d(t, k + 1);
            bad |= !(dn > 0.0) || !isfinite(dn);
            if (k >= 1) {
#pragma unroll
                for (int j = k + 2; j < kNB; ++j) v[j] = fma(-vkp, lp[j], v[j]);
#pragma unroll
                for (int j = k + 2; j < kNB; ++j) asm volatile("" : "+v"(v[j]));   // not sunk to later steps
            }
            __builtin_amdgcn_sched_barrier(0);
            // the updates of columns k+1 and k+2 (the next step's pivot column
            // and its next pivot); the rest waits for the next step
            v[k + 1] = fma(-v[k], lc[k + 1], v[k + 1]);
            if (k + 2 < kNB) v[k + 2] = fma(-v[k], lc[k + 2], v[k + 2]);
            vkp = v[k];
            asm volatile("" : "+v"(v[k + 1]));
            if (k + 2 < kNB) asm volatile("" : "+v"(v[k + 2]));
            // computed within this step, not sunk to its use in the next one
            is = is_next;
            asm volatile("" : "+v"(is));
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    // W lane c now holds column c of W (v[k] = W[k][c], zero for k < c): W to
    // Wl (row-major) and W^T to row c of the tile in A, whose upper triangle
    // then holds W^T with the diagonal.  The zeros land in the lower triangle,
    // which no reader of a factored diagonal tile uses.
    if (wl) {
        double *dst = A + (off + rq) + off * Np;
#pragma unroll
        for (int k = 0; k < kNB; ++k) {
            Wl[k][rq] = v[k];
            __hip_atomic_store(dst + k * Np, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncwarp();
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

// Backward block solve with a factored S_k (L in the lower tiles, W_pp^T in the
// upper triangle of each diagonal tile, diagonal included), in place on x
// (LDS), by all kCholThreads threads; sums in a fixed order:
//   x_p = W_pp^T (x_p - sum_{i > p} L_ip^T x_i)
__device__ void block_backward(const double *A, int64_t Np, int nt, double *x, double *red, double *zb, int tid) {
    constexpr int G = kCholThreads / kNB;
    for (int p = nt - 1; p >= 0; --p) {
        const int64_t off = (int64_t)p * kNB;
        {
            const int c = tid / G, g = tid % G;
            double s = 0.0;
            for (int64_t row = off + kNB + g; row < Np; row += G) s = fma(A[row + (off + c) * Np], x[row], s);
            red[c * G + g] = s;
        }
        __syncthreads();
        if (tid < kNB) {
            double s = x[off + tid];
#pragma unroll
            for (int g = 0; g < G; ++g) s -= red[tid * G + g];
            zb[tid] = s;
        }
        __syncthreads();
        if (tid < kNB) {
            const int r = tid;
            double s = 0.0;
            for (int c = r; c < kNB; ++c) s = fma(A[(off + r) + (off + c) * Np], zb[c], s);   // W[c][r]
            x[off + r] = s;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kCholThreads) void k_chol(int32_t l, const int32_t *__restrict__ cl_n,
                                                       const int32_t *__restrict__ cl_Np,
                                                       const int64_t *__restrict__ S_off,
                                                       const int32_t *__restrict__ cl_start,
                                                       const int32_t *__restrict__ cl_cams, double *__restrict__ S,
                                                       const double *__restrict__ b, double *__restrict__ dcam,
                                                       int32_t *__restrict__ cl_status, int32_t max_Np,
                                                       const int32_t *skip) {
    // skip (nullable): 1 when the team form has already solved every cluster
    if (skip != nullptr && skip[0] == 1) return;
    extern __shared__ double smem[];
    double(*Wi)[kNB + 1] = reinterpret_cast<double(*)[kNB + 1]>(smem);
    double(*Ls)[kNB + 1] = reinterpret_cast<double(*)[kNB + 1]>(smem + kNB * (kNB + 1));
    double *col = smem + 2 * kNB * (kNB + 1);   // 2 kNB
    double *x = col + 2 * kNB;
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
        const bool fb = diag_factor_invert<false>(A, Np, 0, lane, Ls, Wi, col, x);
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
            const bool fb = diag_factor_invert<false>(A, Np, (int64_t)q * kNB, lane, Ls, Wi, col, x);
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
    // backward solve L^T x = y
    block_backward(A, Np, nt, x, red, zb, tid);
    for (int i = tid; i < N; i += kCholThreads) dcam[9 * (int64_t)cl_cams[c0 + i / 9] + i % 9] = x[i];
    if (tid == 0) cl_status[k] = bad ? STBA_ENOTPD : STBA_OK;
}

// ---------------------------------------------------------------------------
// Tile-parallel variant for maps with few clusters: the lower 32 x 32 tiles of
// every S_k are spread over wavefronts, so a cluster runs on up to ~T^2 / 2
// compute units instead of one.  One band wavefront per cluster runs the whole
// diagonal chain (panel (i, i-1), its update of (i, i), factor and inverse of
// (i, i)) with W kept in its LDS, so no hand-over between wavefronts lies on the
// critical path; row workers apply the other updates of tiles (i, i) and
// (i, i-1) ahead of time, and every other tile (i, j), j <= i - 2, has its own
// wavefront that keeps the tile in MFMA registers, applies A_ij -= L_ip L_jp^T
// for p < j as soon as tiles (i, p) and (j, p) are final, then solves the panel
// X = A_ij W_jj^T.  A tile handed to another wavefront (final, or partial for
// the band worker) is written with device-scope stores and a flag is raised
// after the stores have completed; readers poll the flag and read with
// device-scope loads.  No cache write-back or invalidation is needed, since a
// wavefront reads another's tile only after its flag.  Every dependency points
// to an earlier diagonal step, so with all wavefronts resident the dataflow
// cannot deadlock; every wait is still bounded, and a time-out raises a
// grid-wide abort word that ends all other waits (the cluster then reports
// STBA_EHIP).  The row workers then run the substitutions as chains over the
// blocks, each block vector handed on as soon as it is known:
//   forward   y_i = W_ii (b_i - sum_{j < i} L_ij y_j),
//   backward  x_i = W_ii^T (y_i - sum_{j > i} L_ji^T x_j),
// A block vector goes to the other row workers through memory: its entries
// start as kEmpty and a reader polls the 32 entries themselves, so a hand-over
// costs one store and the reader's next poll.  The last wavefront of a cluster
// to finish writes the cluster's status and returns its flag words and vector
// entries to their initial state for the next factorisation.
// ---------------------------------------------------------------------------
constexpr int kWaitPolls = 1 << 20;

__device__ inline double ld_dev(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_dev(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lane 0 polls *f until it is non-zero or the abort word is set; every lane gets
// the flag value (0: aborted or timed out).
__device__ inline int wait_flag(const int32_t *f, int32_t *abort_w) {
    int v = 0;
    if ((threadIdx.x & 63) == 0) {
        for (int it = 0; it < kWaitPolls; ++it) {
            // both loads in flight together: one round trip per poll
            v = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int a = __hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v != 0 || a != 0) break;
            __builtin_amdgcn_s_sleep(1);
        }
        if (v == 0) __hip_atomic_store(abort_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    v = __shfl(v, 0, 64);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return v;
}

// The entries of the block vectors that row workers hand to each other start
// as this signalling NaN.  Arithmetic never yields it (a NaN result is quiet),
// so an entry that differs from it has been published.
constexpr long long kEmpty = 0x7FF4535442410000ll;

// Every lane: entry (lane mod 32) of the 32-vector v once all 32 entries have
// been published by another wavefront.  Bounded like wait_flag; on time-out or
// abort it returns 0 and clears ok.
__device__ inline double wait_vec(const double *v, int32_t *abort_w, bool &ok) {
    const int lane = threadIdx.x & 63;
    const double *p = v + (lane & (kNB - 1));
    for (int it = 0; it < kWaitPolls; ++it) {
        // both loads in flight together: one round trip per poll
        const double x = ld_dev(p);
        const int a = __hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__ballot(__double_as_longlong(x) != kEmpty) == ~0ull) return x;
        if (a != 0) break;
        __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) __hip_atomic_store(abort_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok = false;
    return 0.0;
}


__device__ inline int tile_ix(int i, int j) { return i * (i + 1) / 2 + j; }

// Rows row0..row0+31 of the final panel p (columns off..off+31) as MFMA operands:
// v[R][kk] = L(row0 + 16 R + lr, off + 4 kk + lk).
__device__ inline void load_panel(const double *A, int64_t Np, int64_t row0, int64_t off, int lr, int lk,
                                  double (&v)[2][8]) {
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const int64_t col = (off + 4 * kk + lk) * Np;
        v[0][kk] = ld_dev(A + row0 + lr + col);
        v[1][kk] = ld_dev(A + row0 + 16 + lr + col);
    }
}

// acc -= Li Lj^T, acc[R][C][v] = tile(16 R + lr, 16 C + 4 v + lk), Li and Lj as from load_panel.
__device__ inline void mfma_downdate(d4 (&acc)[2][2], const double (&li)[2][8], const double (&lj)[2][8]) {
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(-lj[0][kk], li[0][kk], acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-lj[1][kk], li[0][kk], acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(-lj[0][kk], li[1][kk], acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-lj[1][kk], li[1][kk], acc[1][1], 0, 0, 0);
    }
}

// Panel solve X = T W^T for the tile T in acc, W = L_jj^-1 read from the final
// diagonal tile D (W[c][q] = D(q, c) for q <= c, else 0).
__device__ inline void panel_solve(const d4 (&acc)[2][2], const double *D, int64_t Np, int lr, int lk, d4 (&x)[2][2]) {
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C) x[R][C] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const int q = 4 * kk + lk;
        const double w0 = ld_dev(D + q + (int64_t)lr * Np);
        const double w1 = ld_dev(D + q + (int64_t)(16 + lr) * Np);
        const double a0 = q <= lr ? w0 : 0.0;
        const double a1 = q <= 16 + lr ? w1 : 0.0;
        // operand B: T(16 R + lr, q) = acc[R][kk / 4][kk % 4]
        x[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, acc[0][kk >> 2][kk & 3], x[0][0], 0, 0, 0);
        x[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, acc[0][kk >> 2][kk & 3], x[0][1], 0, 0, 0);
        x[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, acc[1][kk >> 2][kk & 3], x[1][0], 0, 0, 0);
        x[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, acc[1][kk >> 2][kk & 3], x[1][1], 0, 0, 0);
    }
}

__device__ inline void load_tile(const double *A, int64_t Np, int64_t ri, int64_t cj, int lr, int lk, d4 (&acc)[2][2]) {
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[R][C][v] = A[(ri + 16 * R + lr) + (cj + 16 * C + 4 * v + lk) * Np];
}

__device__ inline void store_tile_dev(double *A, int64_t Np, int64_t ri, int64_t cj, int lr, int lk,
                                      const d4 (&x)[2][2]) {
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v) st_dev(A + (ri + 16 * R + lr) + (cj + 16 * C + 4 * v + lk) * Np, x[R][C][v]);
}

// Broadcast the 32 values v (lane r holds entry r) through LDS.
__device__ inline void share32(double *zs, double v, int lane) {
    __syncwarp();
    if (lane < kNB) zs[lane] = v;
    __syncwarp();
}

// Panel solve X = T W^T with W = L_jj^-1 row-major in LDS (zero above the diagonal).
__device__ inline void panel_solve_lds(const d4 (&acc)[2][2], const double (*Wl)[kNB + 1], int lr, int lk,
                                       d4 (&x)[2][2]) {
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C) x[R][C] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const double a0 = Wl[lr][4 * kk + lk], a1 = Wl[16 + lr][4 * kk + lk];
        x[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, acc[0][kk >> 2][kk & 3], x[0][0], 0, 0, 0);
        x[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, acc[0][kk >> 2][kk & 3], x[0][1], 0, 0, 0);
        x[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, acc[1][kk >> 2][kk & 3], x[1][0], 0, 0, 0);
        x[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, acc[1][kk >> 2][kk & 3], x[1][1], 0, 0, 0);
    }
}

__device__ inline void load_tile_dev(const double *A, int64_t Np, int64_t ri, int64_t cj, int lr, int lk,
                                     d4 (&acc)[2][2]) {
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[R][C][v] = ld_dev(A + (ri + 16 * R + lr) + (cj + 16 * C + 4 * v + lk) * Np);
}

// Row-worker chains.  Lane (r, h) = (lane mod 32, lane / 32) holds entry r of
// a block vector and columns hc = 16 h .. 16 h + 15 of a tile, so a 32 x 32
// block product is two 16-term partial sums per entry, added across the halves.

// t[m] = A(r0, c0 + m): along a row (the lanes of a half read 32 consecutive
// rows of one column at a time).  kDev: device-scope loads (tiles written by
// other wavefronts of this kernel).
template <bool kDev>
__device__ inline void ld_row16(const double *A, int64_t Np, int64_t r0, int64_t c0, double (&t)[16]) {
#pragma unroll
    for (int m = 0; m < 16; ++m) t[m] = kDev ? ld_dev(A + r0 + (c0 + m) * Np) : A[r0 + (c0 + m) * Np];
}

// t[m] = A(r0 + m, c0): 16 consecutive entries down a column
template <bool kDev>
__device__ inline void ld_col16(const double *A, int64_t Np, int64_t r0, int64_t c0, double (&t)[16]) {
#pragma unroll
    for (int m = 0; m < 16; ++m) t[m] = kDev ? ld_dev(A + r0 + m + c0 * Np) : A[r0 + m + c0 * Np];
}

// sum_m t[m] z[m] in a fixed order (four partial sums)
__device__ inline double dot16(const double (&t)[16], const double *z) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < 16; ++m) a[m & 3] = fma(t[m], z[m], a[m & 3]);
    return (a[0] + a[1]) + (a[2] + a[3]);
}

// the two halves' partial sums of entry r (the same value in lanes r and r + 32)
__device__ inline double halves(double s) { return s + __shfl_xor(s, 32, 64); }

// W_ii = L_ii^-1 from the final diagonal tile D (W^T in its upper triangle,
// diagonal included), zero outside the triangle, for the forward product
// y_r = sum_{q <= r} W[r][q] z_q, W[r][q] = D(q, r), or the backward one
// x_r = sum_{q >= r} W[q][r] z_q, W[q][r] = D(r, q).
template <bool kFwd>
__device__ inline void ld_w16(const double *A, int64_t Np, int64_t ri, int r, int hc, double (&w)[16]) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int q = hc + m;
        const double v = kFwd ? ld_dev(A + ri + q + (ri + r) * Np) : ld_dev(A + ri + r + (ri + q) * Np);
        w[m] = (kFwd ? q <= r : q >= r) ? v : 0.0;
    }
}

__device__ inline void publish(double *v, double x, int lane) {
    if (lane < kNB) st_dev(v + lane, x);
}

// Backward chain, block i: v_i = W_ii^T (rhs - sum_{j > i} L_ji^T v_j),
// published to v; every tile is final; w from ld_w16<false>.
__device__ __forceinline__ double bwd_chain(const double *A, int64_t Np, int T, int i, int r, int hc, double rhs,
                                            const double (&w)[16], double *v, double *zs, int lane,
                                            int32_t *abort_w, bool &ok) {
    const int64_t ri = (int64_t)i * kNB;
    double s = 0.0;
    if (i + 1 < T) {
        double t[16];
        ld_col16<true>(A, Np, (int64_t)(T - 1) * kNB + hc, ri + r, t);
        for (int j = T - 1; j > i + 1; --j) {
            double tn[16];
            ld_col16<true>(A, Np, (int64_t)(j - 1) * kNB + hc, ri + r, tn);
            share32(zs, wait_vec(v + (int64_t)j * kNB, abort_w, ok), lane);
            s += dot16(t, zs + hc);
#pragma unroll
            for (int m = 0; m < 16; ++m) t[m] = tn[m];
        }
        // the last term (the critical one) with no load in flight: global loads
        // complete in order, so one issued before the wait would delay it
        share32(zs, wait_vec(v + (int64_t)(i + 1) * kNB, abort_w, ok), lane);
        s += dot16(t, zs + hc);
    }
    share32(zs, rhs - halves(s), lane);
    const double x = halves(dot16(w, zs + hc));
    publish(v + ri, x, lane);
    return x;
}

// Wavefront roles per cluster (wave w of the cluster's wpc wavefronts):
//   w = 0, the band worker: the whole diagonal chain.  Step i takes the partial
//     tiles P_i,i-1 and P_ii (all updates but the last applied), solves the panel
//     L_i,i-1 = P_i,i-1 W_i-1^T with W_i-1 still in its LDS, applies
//     P_ii -= L_i,i-1 L_i,i-1^T from registers, and factors and inverts the
//     diagonal tile; no hand-over between wavefronts lies on this chain.
//   w = 1 + i, row worker i: applies A_ii -= L_ip L_ip^T and
//     A_i,i-1 -= L_ip L_i-1,p^T for p <= i - 2 as the panels become final,
//     publishes the partial tiles, then runs the chains of block i.
//   w > tmax, one wavefront per tile (i, j), j <= i - 2.
// Flags per cluster (fpc words): [tile (i, j) final at i (i + 1) / 2 + j]
// [partial tiles of row i at tt + i][error word at tt + tmax][finished
// wavefronts at tt + tmax + 1], tt = tmax (tmax + 1) / 2; diagonal tile flags
// are 1 (final) or 2 (final, pivot failed).  After the last cluster: the abort
// word, then the count of finished clusters.  Block vectors per cluster (yx):
// y and x, tmax blocks of 32 each.
constexpr int kVecSets = 2;

// One wavefront's part; false if one of its waits failed.
__device__ __forceinline__ bool chol_tiles_wave(int w, int k, int32_t tmax, int32_t fpc, const int32_t *cl_n,
                                                const int32_t *cl_Np, const int64_t *S_off, const int32_t *cl_start,
                                                const int32_t *cl_cams, double *S, const double *b, double *dcam,
                                                int32_t *flags, int32_t l, double *yx,
                                                double (*Wi)[kNB + 1], double (*Ls)[kNB + 1], double *zs) {
    const int lane = threadIdx.x;
    const int64_t Np = cl_Np[k];
    const int T = (int)(Np / kNB);
    if (T == 0) return true;
    const int tt = tmax * (tmax + 1) / 2;
    int32_t *fl = flags + (int64_t)k * fpc;
    int32_t *fl_part = fl + tt;
    int32_t *abort_w = flags + (int64_t)l * fpc;
    double *A = S + S_off[k];
    const int lr = lane & 15, lk = lane >> 4;
    bool ok = true;
    if (w > tmax) {
        // tile (i, j), j <= i - 2
        const int g = w - 1 - tmax;
        int i2 = (int)((sqrt(8.0 * g + 1.0) - 1.0) * 0.5);
        while ((i2 + 1) * (i2 + 2) / 2 <= g) ++i2;
        while (i2 * (i2 + 1) / 2 > g) --i2;
        const int j = g - i2 * (i2 + 1) / 2;
        const int i = i2 + 2;
        if (i >= T) return true;
        const int64_t ri = (int64_t)i * kNB, cj = (int64_t)j * kNB;
        d4 acc[2][2];
        load_tile(A, Np, ri, cj, lr, lk, acc);
        for (int p = 0; p < j; ++p) {
            ok &= wait_flag(fl + tile_ix(i, p), abort_w) != 0;
            ok &= wait_flag(fl + tile_ix(j, p), abort_w) != 0;
            double li[2][8], lj[2][8];
            load_panel(A, Np, ri, (int64_t)p * kNB, lr, lk, li);
            load_panel(A, Np, cj, (int64_t)p * kNB, lr, lk, lj);
            mfma_downdate(acc, li, lj);
        }
        ok &= wait_flag(fl + tile_ix(j, j), abort_w) != 0;
        d4 x[2][2];
        panel_solve(acc, A + cj + cj * Np, Np, lr, lk, x);
        store_tile_dev(A, Np, ri, cj, lr, lk, x);
        raise_flag(fl + tile_ix(i, j), 1);
        return ok;
    }
    if (w == 0) {
        // band worker: the critical path, ahead of the other wavefronts on its SIMD
        __builtin_amdgcn_s_setprio(3);
        for (int i = 0; i < T; ++i) {
            const int64_t ri = (int64_t)i * kNB;
            d4 accD[2][2], accP[2][2];
            // rows 0 and 1 have no earlier panels: their tiles are the assembled ones
            if (i >= 2) ok &= wait_flag(fl_part + i, abort_w) != 0;
            load_tile_dev(A, Np, ri, ri, lr, lk, accD);
            if (i >= 1) load_tile_dev(A, Np, ri, ri - kNB, lr, lk, accP);
            if (i >= 1) {
                d4 x[2][2];
                panel_solve_lds(accP, Wi, lr, lk, x);
                store_tile_dev(A, Np, ri, ri - kNB, lr, lk, x);
                double li[2][8];
#pragma unroll
                for (int R = 0; R < 2; ++R)
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk) li[R][kk] = x[R][kk >> 2][kk & 3];
                mfma_downdate(accD, li, li);
            }
            __syncwarp();   // the previous step's W has been read
#pragma unroll
            for (int R = 0; R < 2; ++R)
#pragma unroll
                for (int C = 0; C < 2; ++C)
#pragma unroll
                    for (int v = 0; v < 4; ++v) Ls[16 * R + lr][16 * C + 4 * v + lk] = accD[R][C][v];
            __syncwarp();
            // the panel's flag is raised inside, once its stores have completed
            const bool bad = band_factor_invert(A, Np, ri, lane, Ls, Wi, zs, i >= 1 ? fl + tile_ix(i, i - 1) : nullptr);
            raise_flag(fl + tile_ix(i, i), bad ? 2 : 1);
        }
        return ok;
    }
    // row worker i
    const int i = w - 1;
    if (i >= T) return true;
    const int64_t ri = (int64_t)i * kNB;
    if (i >= 2) {   // rows 0 and 1 have no updates before the band worker's
        d4 accD[2][2], accP[2][2];
        load_tile(A, Np, ri, ri, lr, lk, accD);
        load_tile(A, Np, ri, ri - kNB, lr, lk, accP);
        for (int p = 0; p + 1 < i; ++p) {
            ok &= wait_flag(fl + tile_ix(i, p), abort_w) != 0;
            ok &= wait_flag(fl + tile_ix(i - 1, p), abort_w) != 0;
            double li[2][8], lj[2][8];
            load_panel(A, Np, ri, (int64_t)p * kNB, lr, lk, li);
            load_panel(A, Np, ri - kNB, (int64_t)p * kNB, lr, lk, lj);
            mfma_downdate(accP, li, lj);
            mfma_downdate(accD, li, li);
        }
        store_tile_dev(A, Np, ri, ri, lr, lk, accD);
        store_tile_dev(A, Np, ri, ri - kNB, lr, lk, accP);
        raise_flag(fl_part + i, 1);
    }
    const int r = lane & (kNB - 1);
    const int hc = 16 * (lane >> 5);
    const int N = 9 * cl_n[k];
    const int c0 = cl_start[k];
    const int64_t vs = (int64_t)tmax * kNB;
    double *yv = yx + (int64_t)k * kVecSets * vs;
    double *xv = yv + vs;
    const int64_t row = ri + r;
    const int64_t drow = row < N ? 9 * (int64_t)cl_cams[c0 + row / 9] + row % 9 : 0;
    const double bi = row < N ? b[drow] : 0.0;
    // forward: y_i = W_ii (b_i - sum_{j < i} L_ij y_j).  Tiles (i, j), j <= i - 2,
    // were awaited above; tile (i, i - 1) is the band worker's panel.
    double s = 0.0;
    for (int j = 0; j < i; ++j) {
        if (j == i - 1) ok &= wait_flag(fl + tile_ix(i, i - 1), abort_w) != 0;
        double t[16];
        ld_row16<true>(A, Np, row, (int64_t)j * kNB + hc, t);
        share32(zs, wait_vec(yv + (int64_t)j * kNB, abort_w, ok), lane);
        s += dot16(t, zs + hc);
    }
    ok &= wait_flag(fl + tile_ix(i, i), abort_w) != 0;
    double y;
    {
        double wf[16];
        ld_w16<true>(A, Np, ri, r, hc, wf);
        share32(zs, bi - halves(s), lane);
        y = halves(dot16(wf, zs + hc));
    }
    publish(yv + ri, y, lane);
    // backward: x_i = W_ii^T (y_i - sum_{j > i} L_ji^T x_j); the last diagonal
    // tile is final only after every other tile
    ok &= wait_flag(fl + tile_ix(T - 1, T - 1), abort_w) != 0;
    double wb[16];
    ld_w16<false>(A, Np, ri, r, hc, wb);
    const double x = bwd_chain(A, Np, T, i, r, hc, y, wb, xv, zs, lane, abort_w, ok);
    if (lane < kNB && row < N) dcam[drow] = x;
    return ok;
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_chol_tiles(
    int32_t wpc, int32_t tmax, int32_t fpc, const int32_t *__restrict__ cl_n, const int32_t *__restrict__ cl_Np,
    const int64_t *__restrict__ S_off, const int32_t *__restrict__ cl_start, const int32_t *__restrict__ cl_cams,
    double *__restrict__ S, const double *__restrict__ b, double *__restrict__ dcam, int32_t *__restrict__ cl_status,
    int32_t *flags, int32_t l, double *yx, int32_t xcd_major) {
    __shared__ double Wi[kNB][kNB + 1];
    __shared__ double Ls[kNB][kNB + 1];
    __shared__ __align__(16) double zs[2 * kNB];
    const int lane = threadIdx.x;
    // xcd_major: workgroups go to the 8 XCDs in turn (block b to XCD b mod 8), so
    // cluster k is given the blocks of XCD k mod 8 and its hand-overs stay within
    // one XCD; the grid is padded to 8 ceil(l / 8) wpc blocks and the spare ones
    // belong to no cluster.  Otherwise cluster k has blocks k wpc .. k wpc + wpc - 1.
    int k, w;
    if (xcd_major) {
        const unsigned sl = blockIdx.x >> 3;
        const int rk = (int)(sl / (unsigned)wpc);
        w = (int)(sl - (unsigned)rk * (unsigned)wpc);
        k = (int)(blockIdx.x & 7u) + 8 * rk;
        if (k >= l) return;
    } else {
        k = (int)(blockIdx.x / (unsigned)wpc);
        w = (int)(blockIdx.x - (unsigned)k * (unsigned)wpc);
    }
    const bool ok = chol_tiles_wave(w, k, tmax, fpc, cl_n, cl_Np, S_off, cl_start, cl_cams, S, b, dcam, flags, l, yx,
                                    Wi, Ls, zs);
    // every wavefront of the grid ends here
    const int tt = tmax * (tmax + 1) / 2;
    int32_t *fl = flags + (int64_t)k * fpc;
    int32_t *fl_err = fl + tt + tmax;
    int32_t *fl_cnt = fl_err + 1;
    int32_t *abort_w = flags + (int64_t)l * fpc;
    if (!ok && lane == 0) __hip_atomic_store(fl_err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);   // this wavefront's stores have completed
    int last = 0;
    if (lane == 0)
        last = __hip_atomic_fetch_add(fl_cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == wpc - 1;
    if (__shfl(last, 0, 64) == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // the last wavefront of cluster k: status, then the initial state
    const int T = (int)(cl_Np[k] / kNB);
    if (lane == 0) {
        bool anybad = false;
        for (int p = 0; p < T; ++p)
            anybad |= __hip_atomic_load(fl + tile_ix(p, p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 2;
        const bool failed = __hip_atomic_load(fl_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                            __hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        cl_status[k] = failed ? STBA_EHIP : (anybad ? STBA_ENOTPD : STBA_OK);
    }
    for (int q = lane; q < fpc - 1; q += 64) fl[q] = 0;
    const int64_t nv = (int64_t)kVecSets * tmax * kNB;
    double *vec = yx + (int64_t)k * nv;
    for (int64_t q = lane; q < nv; q += 64) vec[q] = __longlong_as_double(kEmpty);
    __builtin_amdgcn_s_waitcnt(0);
    if (lane == 0) {
        __hip_atomic_store(fl_cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the last cluster clears the abort word and the cluster count
        if (__hip_atomic_fetch_add(abort_w + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == l - 1) {
            __hip_atomic_store(abort_w, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(abort_w + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// Triangular sweeps with the factors of S_k (L in the lower tiles, W_pp^T in
// the upper triangle of diagonal tile p, diagonal included), one 1024-thread
// workgroup per cluster, right-looking: once block p of the solution is known,
// the right-hand sides of all remaining blocks are updated at once.
//   forward:  y_p = W_pp z_p,   z_i -= L_ip y_p   (i > p)
//   backward: x_p = W_pp^T z_p, z_j -= L_pj^T x_p (j < p)
// One workgroup alone pulls at most about 80 GB/s, so the sweep is bound by
// streaming the factor (T (T + 1) / 2 tiles of 8 KB) through the CU.  The tiles
// flow through a ring of kRing LDS slots in the order the sweep uses them
// (step s: the diagonal tile, then the panel of step s), moved by load-to-LDS
// instructions: wavefront w owns slot w, keeps one tile in flight and loads the
// tile kRing further on as soon as the previous one has been used, so about
// 128 KB stay in flight.  The tiles are used in segments of at most kSeg
// tiles of one step: wait for the segment's tiles, the diagonal block (first
// segment of a step), then the segment's panel updates, each output a dot
// product of 32 shared by four lanes.
// Column col of a tile occupies 256 bytes of its slot, its 16-byte part q (rows
// 2q, 2q + 1) at position (q + col) mod 16: the 32 lanes that read one row of 32
// columns, or 32 rows of one column, meet at most two to a bank.
// Used for the MIXED refinement step after any of the factorisations:
// dcam += backward(forward(r)) with the residual r in camera order.
// ---------------------------------------------------------------------------
constexpr int kSwThreads = 1024;
constexpr int kRing = kSwThreads / 64;             // one slot per wavefront
constexpr int kSeg = 8;
constexpr int kTileBytes = kNB * kNB * 8;
constexpr size_t kSwStaticLds = (size_t)kRing * kTileBytes + kNB * 8;

// element (row, col) of a tile in its ring slot
__device__ inline int sw_at(int row, int col) { return col * 256 + ((((row >> 1) + col) & 15) << 4) + ((row & 1) << 3); }

// tile t of the sweep sequence (the forward steps, then the backward ones):
// block row a, block column b, step, index k in the step
__device__ inline void sw_tile(int t, int T, int *a, int *b, bool *fwd) {
    const int n = T * (T + 1) / 2;
    *fwd = t < n;
    if (t >= n) t -= n;
    int s = 0, off = 0;
    while (off + (T - s) <= t) {
        off += T - s;
        ++s;
    }
    const int k = t - off;
    if (*fwd) {            // step s: W_ss, then L_{s+k, s}
        *a = k == 0 ? s : s + k;
        *b = s;
    } else {               // step s (block p = T-1-s): W_pp, then L_{p, k-1}
        const int p = T - 1 - s;
        *a = p;
        *b = k == 0 ? p : k - 1;
    }
}

// wavefront-uniform: issue the eight 1 KB load-to-LDS instructions of tile t
__device__ inline void sw_issue(const double *A, int64_t Np, int T, int t, char *slot, int lane) {
    int a, b;
    bool fwd;
    sw_tile(t, T, &a, &b, &fwd);
    const int sl = lane & 15;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int col = 4 * i + (lane >> 4);
        const int q = (sl - col) & 15;   // part stored at position sl of column col
        const double *src = A + (int64_t)a * kNB + 2 * q + ((int64_t)b * kNB + col) * Np;
        __builtin_amdgcn_global_load_lds((const void *)src,
                                         (void __attribute__((address_space(3))) *)(slot + i * 1024), 16, 0, 0);
    }
}

// The diagonal block of a step: 32 outputs, one lane each (all 32 terms, four
// partial sums), into xb.
template <bool kFwd>
__device__ __forceinline__ void sw_diag(const char *d, const double *z, double *xb, int p, int tid) {
    if (tid >= kNB) return;
    int r = tid;
    asm volatile("" : "+v"(r));   // opaque: the 32 addresses below are not hoisted out of the step loop
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {   // two halves of 16 terms: the registers of a 1024-thread block are few
        double dv[16], zv[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {   // forward: W[r][c] = D(c, r); backward: W[c][r] = D(r, c)
            const int c = 16 * h + m;
            dv[m] = *reinterpret_cast<const double *>(d + (kFwd ? sw_at(c, r) : sw_at(r, c)));
            zv[m] = z[p * kNB + c];
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int c = 16 * h + m;
            const bool in = kFwd ? c <= r : c >= r;   // y_r = sum_{c <= r} W[r][c] z_c; x_r = sum_{c >= r} W[c][r] z_c
            acc[m & 3] = fma(in ? dv[m] : 0.0, zv[m], acc[m & 3]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    xb[r] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// The panel tiles [kb, k1) of the step whose diagonal block is p (tile index k
// >= 1 in the step): 8 tiles x 32 outputs x 4 lanes (8 of the 32 terms each).
template <bool kFwd>
__device__ __forceinline__ void sw_panel(const char *ring, double *z, const double *xb, int p, int kb, int k1, int t0,
                                         int tid) {
    int lt = tid;
    asm volatile("" : "+v"(lt));   // opaque, as in sw_diag
    const int g = lt >> 7, e = (lt >> 2) & 31, qq = lt & 3;
    const int kk = kb + g;
    double acc = 0.0;
    const bool act = kk < k1;
    if (act) {
        const char *d = ring + (((t0 + kk) % kRing) * kTileBytes);
        double lv[8], xv[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int c = 8 * qq + m;
            // forward, tile L_{p+kk, p}: z_{p+kk}[e] -= sum_c L(e, c) y_p[c];
            // backward, tile L_{p, kk-1}: z_{kk-1}[e] -= sum_c L(c, e) x_p[c]
            lv[m] = *reinterpret_cast<const double *>(d + (kFwd ? sw_at(e, c) : sw_at(c, e)));
            xv[m] = xb[c];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) acc = fma(lv[m], xv[m], acc);
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (act && qq == 0) z[(kFwd ? p + kk : kk - 1) * kNB + e] -= acc;
}

__global__ __launch_bounds__(kSwThreads) void k_sweep(const int32_t *__restrict__ cl_n,
                                                      const int32_t *__restrict__ cl_Np,
                                                      const int64_t *__restrict__ S_off,
                                                      const int32_t *__restrict__ cl_start,
                                                      const int32_t *__restrict__ cl_cams,
                                                      const double *__restrict__ S,
                                                      const double *__restrict__ rhs, double *__restrict__ dcam) {
    __shared__ __align__(16) char ring[kRing * kTileBytes];
    __shared__ double xb[kNB];
    extern __shared__ double z[];   // Np
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int nk = cl_n[k];
    if (nk == 0) return;
    const int64_t Np = cl_Np[k];
    const int N = 9 * nk;
    const int T = (int)(Np / kNB);
    const double *A = S + S_off[k];
    const int c0 = cl_start[k];
    const int ntiles = T * (T + 1);
    char *slot = ring + w * kTileBytes;
    int mine = w;   // the tile this wavefront has in flight (or has landed)
    if (mine < ntiles) sw_issue(A, Np, T, mine, slot, lane);
    for (int i = tid; i < Np; i += kSwThreads)
        z[i] = i < N ? rhs[9 * (int64_t)cl_cams[c0 + i / 9] + i % 9] : 0.0;
    // segments: (sweep, step s, tiles [k0, k1) of the step).  One barrier between
    // segments: it publishes the previous segment's results and its end of use of
    // the ring slots, and (after the owners' waits) the landing of this one's tiles.
    int t0 = 0, pa = 0, pb = 0;   // the previous segment's tiles [pa, pb)
    for (int sweep = 0; sweep < 2; ++sweep) {
        const bool fwd = sweep == 0;
        for (int s = 0; s < T; ++s) {
            const int cnt = T - s;
            const int p = fwd ? s : T - 1 - s;   // the diagonal block of the step
            for (int k0 = 0; k0 < cnt; k0 += kSeg) {
                const int k1 = min(cnt, k0 + kSeg);
                const int ta = t0 + k0, tb = t0 + k1;
                if (mine >= ta && mine < tb) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): my tile landed
                __syncthreads();
                asm volatile("" ::"v"(ring) : "memory");
                if (mine >= pa && mine < pb) {   // my previous tile is used: load the one kRing further
                    mine += kRing;
                    if (mine < ntiles) sw_issue(A, Np, T, mine, slot, lane);
                }
                if (k0 == 0) {
                    const char *dg = ring + ((t0 % kRing) * kTileBytes);
                    if (fwd) sw_diag<true>(dg, z, xb, p, tid);
                    else sw_diag<false>(dg, z, xb, p, tid);
                    __syncthreads();
                    if (tid >= kSwThreads - kNB) z[p * kNB + tid - (kSwThreads - kNB)] = xb[tid - (kSwThreads - kNB)];
                }
                const int kb = k0 == 0 ? 1 : k0;
                if (fwd) sw_panel<true>(ring, z, xb, p, kb, k1, t0, tid);
                else sw_panel<false>(ring, z, xb, p, kb, k1, t0, tid);
                pa = ta;
                pb = tb;
            }
            t0 += cnt;
        }
    }
    __syncthreads();
    for (int i = tid; i < N; i += kSwThreads) {
        double *d = dcam + 9 * (int64_t)cl_cams[c0 + i / 9] + i % 9;
        *d += z[i];
    }
}


// ---------------------------------------------------------------------------
// Team factorisation for maps with many clusters (when one wavefront per tile
// of every cluster would not be resident at once).  One launch of G
// one-wavefront workgroups; every wavefront works out its cluster and role
// from the clusters' padded orders (the same arithmetic in every wavefront):
// cluster k gets a band wavefront and W_k workers, W_k proportional to T_k^3
// (its share of the factorisation's work), at least one when there are tiles
// below the first subdiagonal.  The tiles stay in memory; every hand-over
// goes through device-scope stores, flags raised after the stores complete,
// and device-scope loads.
//   band: the diagonal chain as in the tile-parallel form (partial tiles P_ii
//     and P_i,i-1 -> panel L_i,i-1 with W_i-1 in LDS, last update of the
//     diagonal tile, factor and inverse) with the forward substitution folded
//     in: y_i = W_ii (b_i - sum_{j <= i-2} c_ij - L_i,i-1 y_i-1), where the
//     workers publish c_ij = L_ij y_j; after the last diagonal tile the
//     backward substitution x_i = W_ii^T (y_i - sum_{j >= i+2} d_ji -
//     L_i+1,i^T x_i+1) with d_ji = L_ji^T x_j from the workers.
//   workers: own a share of the tasks (round robin over the task list in
//     column order): R(i), 2 <= i < T, applies A_ii -= L_ip L_ip^T and
//     A_i,i-1 -= L_ip L_i-1,p^T for p <= i - 2 and publishes the partial tiles;
//     F(i, j), j <= i - 2, applies A_ij -= L_ip L_jp^T for p < j, solves the
//     panel L_ij = A_ij W_jj^T, then publishes c_ij and, once x_i is known,
//     d_ij.  A worker never waits on one task: each pass checks every pending
//     task's inputs at once (one flag load per lane) and advances the ready
//     ones, applying all the consecutive updates whose panels are final in one
//     visit of the tile.
// Flags of cluster k start at 2 S_off[k] / 1024 + 8 k: F(i, j) final at
// i (i + 1) / 2 + j (2 on a failed pivot of a diagonal tile), then per block
// row the partial tiles, y_i and x_i published, then the error word and the
// count of finished wavefronts.  Block vectors (c, d per tile, y, x per block
// row) start at S_off[k] / 32 in their buffers and hold kEmpty between uses.
// ---------------------------------------------------------------------------
constexpr int kTeamLook = 4;   // updates a worker checks ahead per task and pass

struct TeamBufs {
    int32_t *flags;      // cluster flag words, then the abort word and the finished-cluster count
    int64_t abort_at;    // index of the abort word
    double *cv, *dv, *yv, *xv;
};

__device__ inline int64_t team_fbase(const int64_t *S_off, int k) { return 2 * (S_off[k] >> 10) + 8 * (int64_t)k; }
__device__ inline int64_t team_vbase(const int64_t *S_off, int k) { return S_off[k] >> 5; }

// Non-blocking flag test (lane-local).
__device__ inline bool flag_set(const int32_t *f) {
    return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__host__ __device__ inline int team_ntasks(int T) { return T < 3 ? 0 : (T - 2) + (T - 1) * (T - 2) / 2; }

// Task g of a cluster with T block rows, column-major groups: column j holds
// R(j + 2) and then F(j + 2 .. T - 1, j).  Packed as kind << 30 | i << 15 | j
// (kind 0: F, 1: R, whose j field is i - 1).
__device__ inline int32_t team_task(int g, int T) {
    int j = 0;
    while (true) {
        const int n = T - 1 - j;   // tasks of column j
        if (g < n) break;
        g -= n;
        ++j;
    }
    if (g == 0) return (1 << 30) | ((j + 2) << 15) | (j + 1);
    return ((j + 1 + g) << 15) | j;
}

// Tasks of worker w0 (0 .. W - 1) of a team with W workers: every W-th task
// of the list, from task w0.
__device__ inline int team_own(int T, int W, int w0) {
    const int nt = team_ntasks(T);
    return w0 < nt ? (nt - w0 + W - 1) / W : 0;
}

// This wavefront's cluster k, its index r in the team (0: band) and the
// number of workers W (every wavefront computes the same layout).
// Empty clusters get no wavefront; n_act receives the number of the others.
// False for a spare wavefront, and for every wavefront when the teams would
// not fit in G (fits = false).
__device__ inline bool team_role(int wave, int G, int l, const int32_t *cl_Np, int &k_out, int &r_out, int &W_out,
                                 int &n_act, bool &fits) {
    const int lane = threadIdx.x & 63;
    int64_t sw = 0;
    int n3 = 0, n1 = 0;
    for (int k = lane; k < l; k += 64) {
        const int T = cl_Np[k] / kNB;
        if (T >= 1) ++n1;
        if (T >= 3) {
            sw += (int64_t)T * T * T;
            ++n3;
        }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        sw += __shfl_xor(sw, d, 64);
        n3 += __shfl_xor(n3, d, 64);
        n1 += __shfl_xor(n1, d, 64);
    }
    n_act = n1;
    const int64_t wtot = (int64_t)G - 2 * (int64_t)n1 - n3;
    fits = wtot >= 0;
    if (!fits) return false;
    int64_t base = 0;
    for (int c0 = 0; c0 < l; c0 += 64) {
        const int k = c0 + lane;
        int64_t size = 0, W = 0;
        if (k < l) {
            const int T = cl_Np[k] / kNB;
            if (T >= 3) {
                W = sw > 0 ? wtot * ((int64_t)T * T * T) / sw : 0;
                if (W < 1) W = 1;
                if (W > team_ntasks(T)) W = team_ntasks(T);
            }
            size = T >= 1 ? 2 + W : 0;
        }
        int64_t inc = size;   // inclusive scan over the 64 clusters of this chunk
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t n = __shfl_up(inc, d, 64);
            if (lane >= d) inc += n;
        }
        const int64_t start = base + inc - size;
        const unsigned long long hit = __ballot(k < l && wave >= start && wave < start + size);
        if (hit) {
            const int src = __ffsll(hit) - 1;
            k_out = c0 + src;
            r_out = wave - __shfl((int)start, src, 64);
            W_out = __shfl((int)W, src, 64);
            return true;
        }
        base += __shfl((int)inc, 63, 64);
    }
    return false;
}

// y[r] = sum_c M[r][c] z[c] over a 32 x 32 row-major LDS matrix, lanes (r, half);
// the sum of both halves lands in lanes r and r + 32.
__device__ inline double lds_matvec(const double (*M)[kNB + 1], const double *z, int lane) {
    const int r = lane & (kNB - 1), hc = 16 * (lane >> 5);
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < 16; ++m) a[m & 3] = fma(M[r][hc + m], z[hc + m], a[m & 3]);
    return halves((a[0] + a[1]) + (a[2] + a[3]));
}

// Sum of cnt published 32-vectors at base + 32 slot(q), q = 0 .. cnt - 1, entry
// (lane mod 32) in every lane, each returned to kEmpty after use.  Sixteen
// vectors per round trip (half h of the wavefront loads q = h, h + 2, ...);
// an entry still kEmpty is polled again (bounded).  The order of the sum is
// fixed: each half adds its vectors in increasing q, then the two halves.
template <class Slot>
__device__ inline double take_sum(double *base, int cnt, Slot slot, int32_t *abort_w, bool &ok) {
    const int lane = threadIdx.x & 63, r = lane & (kNB - 1), h = lane >> 5;
    double acc = 0.0;
    for (int q0 = 0; q0 < cnt; q0 += 16) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + 2 * u + h;
            v[u] = q < cnt ? ld_dev(base + 32 * (int64_t)slot(q) + r) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + 2 * u + h;
            double *p = base + 32 * (int64_t)slot(q < cnt ? q : 0) + r;
            for (int it = 0; it < kWaitPolls; ++it) {
                const bool empty = q < cnt && __double_as_longlong(v[u]) == kEmpty;
                if (__ballot(empty) == 0ull) break;
                const int a = __hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (a != 0 || it + 1 == kWaitPolls) {
                    if (lane == 0) __hip_atomic_store(abort_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = false;
                    v[u] = 0.0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                if (empty) v[u] = ld_dev(p);
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + 2 * u + h;
            if (q < cnt) {
                acc += v[u];
                st_dev(base + 32 * (int64_t)slot(q) + r, __longlong_as_double(kEmpty));
            }
        }
    }
    return acc + __shfl_xor(acc, 32, 64);
}

// The band wavefront of cluster k: the diagonal chain, then the backward
// substitution.
__device__ __forceinline__ bool team_band(int k, const int64_t *S_off, const int32_t *cl_n, const int32_t *cl_Np,
                                          const int32_t *cl_start, const int32_t *cl_cams, double *S, double *dcam,
                                          const TeamBufs &tb, double (*Wi)[kNB + 1], double (*Ls)[kNB + 1],
                                          double *zs) {
    const int lane = threadIdx.x;
    const int64_t Np = cl_Np[k];
    const int T = (int)(Np / kNB);
    if (T == 0) return true;
    const int tt = T * (T + 1) / 2;
    int32_t *fl = tb.flags + team_fbase(S_off, k);
    int32_t *fl_part = fl + tt, *fl_y = fl_part + T, *fl_x = fl_y + T;
    int32_t *abort_w = tb.flags + tb.abort_at;
    const int64_t vb = team_vbase(S_off, k);
    double *dv = tb.dv + vb, *yv = tb.yv + vb, *xv = tb.xv + vb;
    double *A = S + S_off[k];
    const int lr = lane & 15, lk = lane >> 4;
    const int r = lane & (kNB - 1), hc = 16 * (lane >> 5);
    const int N = 9 * cl_n[k];
    const int c0 = cl_start[k];
    bool ok = true;
    __builtin_amdgcn_s_setprio(3);
    for (int i = 0; i < T; ++i) {
        const int64_t ri = (int64_t)i * kNB;
        d4 accD[2][2], accP[2][2];
        if (i >= 2) ok &= wait_flag(fl_part + i, abort_w) != 0;
        load_tile_dev(A, Np, ri, ri, lr, lk, accD);
        if (i >= 1) {
            load_tile_dev(A, Np, ri, ri - kNB, lr, lk, accP);
            d4 x[2][2];
            panel_solve_lds(accP, Wi, lr, lk, x);
            store_tile_dev(A, Np, ri, ri - kNB, lr, lk, x);
            double li[2][8];
#pragma unroll
            for (int R = 0; R < 2; ++R)
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) li[R][kk] = x[R][kk >> 2][kk & 3];
            mfma_downdate(accD, li, li);
        }
        __syncwarp();   // the previous step's W has been read
#pragma unroll
        for (int R = 0; R < 2; ++R)
#pragma unroll
            for (int C = 0; C < 2; ++C)
#pragma unroll
                for (int v = 0; v < 4; ++v) Ls[16 * R + lr][16 * C + 4 * v + lk] = accD[R][C][v];
        __syncwarp();
        const bool bad = band_factor_invert(A, Np, ri, lane, Ls, Wi, zs, i >= 1 ? fl + tile_ix(i, i - 1) : nullptr);
        raise_flag(fl + tile_ix(i, i), bad ? 2 : 1);
    }
    // backward substitution once the forward one is complete; W_T-1 is still
    // in Wi (row-major W): x_T-1 = W^T y_T-1
    ok &= wait_flag(fl_y + (T - 1), abort_w) != 0;
    double x;
    {
        share32(zs, ld_dev(yv + (int64_t)(T - 1) * kNB + r), lane);
        double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < 16; ++m) a[m & 3] = fma(Wi[hc + m][r], zs[hc + m], a[m & 3]);
        x = halves((a[0] + a[1]) + (a[2] + a[3]));
    }
    double x2 = 0.0;   // x_i+2
    for (int i = T - 1; i >= 0; --i) {
        const int64_t ri = (int64_t)i * kNB;
        if (i < T - 1) {
            // x_i = W_ii^T (y_i - L_i+1,i^T x_i+1 - L_i+2,i^T x_i+2 - sum_{j >= i+3} d_ji):
            // the two nearest terms here, the others from the workers (published
            // at least three steps ago); every load is issued before the sums
            double t1[16], t2[16], w[16];
            ld_col16<true>(A, Np, ri + kNB + hc, ri + r, t1);   // column r of L_i+1,i, rows hc..hc+15
            if (i + 2 < T) ld_col16<true>(A, Np, ri + 2 * kNB + hc, ri + r, t2);
            ld_w16<false>(A, Np, ri, r, hc, w);
            const double yi = ld_dev(yv + ri + r);
            const double dsum =
                take_sum(dv, i + 3 < T ? T - i - 3 : 0, [&](int q) { return tile_ix(i + 3 + q, i); }, abort_w, ok);
            __syncwarp();
            if (lane < kNB) {
                zs[lane] = x;            // x_i+1
                zs[kNB + lane] = x2;     // x_i+2
            }
            __syncwarp();
            double z = yi - halves(dot16(t1, zs + hc));
            if (i + 2 < T) z -= halves(dot16(t2, zs + kNB + hc));
            z -= dsum;
            x2 = x;
            share32(zs, z, lane);
            x = halves(dot16(w, zs + hc));
        }
        publish(xv + ri, x, lane);
        raise_flag(fl_x + i, 1);
        const int64_t row = ri + r;
        if (lane < kNB && row < N) dcam[9 * (int64_t)cl_cams[c0 + row / 9] + row % 9] = x;
    }
    return ok;
}

// The forward substitution of cluster k, one wavefront behind the band:
// y_i = W_ii (b_i - L_i,i-1 y_i-1 - sum_{j <= i-2} c_ij) once tile (i, i) is
// final, published with its flag.
__device__ __forceinline__ bool team_forward(int k, const int64_t *S_off, const int32_t *cl_n, const int32_t *cl_Np,
                                             const int32_t *cl_start, const int32_t *cl_cams, const double *S,
                                             const double *b, const TeamBufs &tb, double *zs, double *ys) {
    const int lane = threadIdx.x;
    const int64_t Np = cl_Np[k];
    const int T = (int)(Np / kNB);
    if (T == 0) return true;
    const int tt = T * (T + 1) / 2;
    int32_t *fl = tb.flags + team_fbase(S_off, k);
    int32_t *fl_y = fl + tt + T;
    int32_t *abort_w = tb.flags + tb.abort_at;
    const int64_t vb = team_vbase(S_off, k);
    double *cv = tb.cv + vb, *yv = tb.yv + vb;
    const double *A = S + S_off[k];
    const int r = lane & (kNB - 1), hc = 16 * (lane >> 5);
    const int N = 9 * cl_n[k];
    const int c0 = cl_start[k];
    bool ok = true;
    for (int i = 0; i < T; ++i) {
        const int64_t ri = (int64_t)i * kNB;
        const int64_t row = ri + r;
        const double bi = row < N ? b[9 * (int64_t)cl_cams[c0 + row / 9] + row % 9] : 0.0;
        const double csum = take_sum(cv, i >= 2 ? i - 1 : 0, [&](int q) { return tile_ix(i, q); }, abort_w, ok);
        ok &= wait_flag(fl + tile_ix(i, i), abort_w) != 0;   // also orders tile (i, i - 1)
        double w[16];
        ld_w16<true>(A, Np, ri, r, hc, w);
        double z = bi - csum;
        if (i >= 1) {
            double t[16];
            ld_row16<true>(A, Np, row, ri - kNB + hc, t);
            z -= halves(dot16(t, ys + hc));   // L_i,i-1 y_i-1
        }
        share32(zs, z, lane);
        const double y = halves(dot16(w, zs + hc));
        __syncwarp();
        if (lane < kNB) ys[lane] = y;
        __syncwarp();
        publish(yv + ri, y, lane);
        raise_flag(fl_y + i, 1);
    }
    return ok;
}

// Worker r (1 <= r <= W) of cluster k.  tasks / st: LDS lists of this
// wavefront's tasks and their states (phase << 16 | next update).
__device__ __forceinline__ bool team_worker(int k, int r, int W, const int64_t *S_off, const int32_t *cl_Np, double *S,
                                            const TeamBufs &tb, int32_t *tasks, int32_t *st, int32_t *rdy,
                                            double *zs) {
    const int lane = threadIdx.x;
    const int64_t Np = cl_Np[k];
    const int T = (int)(Np / kNB);
    const int w0 = r - 1;
    const int own = team_own(T, W, w0);
    if (own == 0) return true;
    const int tt = T * (T + 1) / 2;
    int32_t *fl = tb.flags + team_fbase(S_off, k);
    int32_t *fl_part = fl + tt, *fl_y = fl_part + T, *fl_x = fl_y + T;
    int32_t *abort_w = tb.flags + tb.abort_at;
    const int64_t vb = team_vbase(S_off, k);
    double *cv = tb.cv + vb, *dv = tb.dv + vb, *yv = tb.yv + vb, *xv = tb.xv + vb;
    double *A = S + S_off[k];
    const int lr = lane & 15, lk = lane >> 4;
    const int rr = lane & (kNB - 1), hc = 16 * (lane >> 5);
    for (int s = lane; s < own; s += 64) {
        const int32_t tk = team_task(w0 + W * s, T);
        tasks[s] = tk;
        // a panel of the first block column has no updates: it starts at its solve
        st[s] = ((tk >> 30) == 0 && (tk & 0x7FFF) == 0) ? (1 << 16) : 0;
    }
    __syncwarp();
    int left = own, idle = 0;
    while (left > 0) {
        // readiness of every pending task, one lane per task: rdy = number of
        // consecutive updates ready (phase 0) or 1 (other phases), 0 if none
        for (int s = lane; s < own; s += 64) {
            const int32_t tk = tasks[s], sv = st[s];
            const int ph = sv >> 16, pn = sv & 0xFFFF;
            const int i = (tk >> 15) & 0x7FFF, j = tk & 0x7FFF;
            const bool isR = (tk >> 30) != 0;
            int n = 0;
            if (ph == 0) {
                const int lim = isR ? i - 1 : j;   // updates p < lim
                const int i2 = isR ? i - 1 : j;
#pragma unroll
                for (int q = 0; q < kTeamLook; ++q) {
                    const int p = pn + q;
                    if (p >= lim || n < q) break;
                    if (flag_set(fl + tile_ix(i, p)) && flag_set(fl + tile_ix(i2, p))) n = q + 1;
                }
                // a tile far from the diagonal is visited once several updates
                // are ready (each visit loads and stores the tile), the
                // partial tiles and the tiles next to the band at once
                if (!isR && i - j >= 3 && n < min(kTeamLook, lim - pn)) n = 0;
            } else if (ph == 1) {
                n = flag_set(fl + tile_ix(j, j)) ? 1 : 0;
            } else if (ph == 2) {
                n = flag_set(fl_y + j) ? 1 : 0;
            } else if (ph == 3) {
                n = flag_set(fl_x + i) ? 1 : 0;
            }
            rdy[s] = n;
        }
        __syncwarp();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        bool progress = false;
        for (int s = 0; s < own; ++s) {
            const int cnt = rdy[s];
            if (cnt == 0) continue;   // inputs not ready, or done
            const int32_t tk = tasks[s], sv = st[s];
            const int i = (tk >> 15) & 0x7FFF, j = tk & 0x7FFF;
            const bool isR = (tk >> 30) != 0;
            int ph = sv >> 16, pn = sv & 0xFFFF;
            const int64_t ri = (int64_t)i * kNB, cj = (int64_t)j * kNB;
            progress = true;
            if (isR) {
                // R(i): tiles (i, i) and (i, i - 1), updates p = pn .. pn + cnt - 1 (<= i - 2)
                d4 accD[2][2], accP[2][2];
                load_tile_dev(A, Np, ri, ri, lr, lk, accD);
                load_tile_dev(A, Np, ri, ri - kNB, lr, lk, accP);
                for (int q = 0; q < cnt; ++q) {
                    const int64_t off = (int64_t)(pn + q) * kNB;
                    double li[2][8], lj[2][8];
                    load_panel(A, Np, ri, off, lr, lk, li);
                    load_panel(A, Np, ri - kNB, off, lr, lk, lj);
                    mfma_downdate(accP, li, lj);
                    mfma_downdate(accD, li, li);
                }
                store_tile_dev(A, Np, ri, ri, lr, lk, accD);
                store_tile_dev(A, Np, ri, ri - kNB, lr, lk, accP);
                pn += cnt;
                if (pn >= i - 1) {
                    raise_flag(fl_part + i, 1);
                    ph = 4;
                    --left;
                }
            } else if (ph == 0) {
                d4 acc[2][2];
                load_tile_dev(A, Np, ri, cj, lr, lk, acc);
                for (int q = 0; q < cnt; ++q) {
                    const int64_t off = (int64_t)(pn + q) * kNB;
                    double li[2][8], lj[2][8];
                    load_panel(A, Np, ri, off, lr, lk, li);
                    load_panel(A, Np, cj, off, lr, lk, lj);
                    mfma_downdate(acc, li, lj);
                }
                pn += cnt;
                bool solved = false;
                if (pn == j) {
                    ph = 1;
                    // the diagonal tile may already be final: solve in this visit
                    int fin = 0;
                    if (lane == 0) fin = flag_set(fl + tile_ix(j, j)) ? 1 : 0;
                    if (__shfl(fin, 0, 64)) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                        d4 x[2][2];
                        panel_solve(acc, A + cj + cj * Np, Np, lr, lk, x);
                        store_tile_dev(A, Np, ri, cj, lr, lk, x);
                        raise_flag(fl + tile_ix(i, j), 1);
                        ph = 2;
                        solved = true;
                    }
                }
                if (!solved) store_tile_dev(A, Np, ri, cj, lr, lk, acc);
            } else if (ph == 1) {
                d4 acc[2][2], x[2][2];
                load_tile_dev(A, Np, ri, cj, lr, lk, acc);
                panel_solve(acc, A + cj + cj * Np, Np, lr, lk, x);
                store_tile_dev(A, Np, ri, cj, lr, lk, x);
                raise_flag(fl + tile_ix(i, j), 1);
                ph = 2;
            } else if (ph == 2) {
                // c_ij = L_ij y_j
                double t[16];
                ld_row16<true>(A, Np, ri + rr, cj + hc, t);
                share32(zs, ld_dev(yv + cj + rr), lane);
                const double c = halves(dot16(t, zs + hc));
                publish(cv + 32 * (int64_t)tile_ix(i, j), c, lane);
                // the band takes L_ij^T x_i itself for the two nearest blocks
                if (i - j >= 3) {
                    ph = 3;
                } else {
                    ph = 4;
                    --left;
                }
            } else if (ph == 3) {
                // d_ij = L_ij^T x_i: column rr of the tile, rows hc .. hc + 15
                double t[16];
                ld_col16<true>(A, Np, ri + hc, cj + rr, t);
                share32(zs, ld_dev(xv + ri + rr), lane);
                const double d = halves(dot16(t, zs + hc));
                publish(dv + 32 * (int64_t)tile_ix(i, j), d, lane);
                ph = 4;
                --left;
            }
            __syncwarp();
            if (lane == 0) st[s] = (ph << 16) | pn;
            __syncwarp();
        }
        if (!progress) {
            if (++idle >= kWaitPolls) {
                if (lane == 0) __hip_atomic_store(abort_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            int a = 0;
            if (lane == 0) a = __hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__shfl(a, 0, 64)) return false;
            __builtin_amdgcn_s_sleep(1);
        } else {
            idle = 0;
        }
    }
    return true;
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_chol_team(
    int32_t G, int32_t l, const int32_t *__restrict__ cl_n, const int32_t *__restrict__ cl_Np,
    const int64_t *__restrict__ S_off, const int32_t *__restrict__ cl_start, const int32_t *__restrict__ cl_cams,
    double *__restrict__ S, const double *__restrict__ b, double *__restrict__ dcam, int32_t *__restrict__ cl_status,
    TeamBufs tb) {
    // dynamic LDS, team_lds_bytes(): the band's W, staged tile, column and y,
    // or a worker's column buffer and task lists
    extern __shared__ __align__(16) double team_lds[];
    double *zs = team_lds;                      // 2 kNB
    double *ys = zs + 2 * kNB;                  // kNB
    double(*Wi)[kNB + 1] = reinterpret_cast<double(*)[kNB + 1]>(ys + kNB);
    double(*Ls)[kNB + 1] = Wi + kNB;
    int32_t *lists = reinterpret_cast<int32_t *>(ys + kNB);
    const int lane = threadIdx.x;
    int k = 0, r = 0, W = 0, n_act = 0;
    bool fits = false;
    const bool found = team_role((int)blockIdx.x, G, l, cl_Np, k, r, W, n_act, fits);
    if (blockIdx.x == 0) {
        // the empty clusters' status, and whether the workgroup form must still run
        for (int q = lane; q < l; q += 64)
            if (cl_Np[q] == 0) cl_status[q] = STBA_OK;
        if (lane == 0) tb.flags[tb.abort_at + 2] = fits ? 1 : 0;
    }
    if (!found) return;   // spare wavefront, or the teams do not fit
    bool ok;
    if (r == 0)
        ok = team_band(k, S_off, cl_n, cl_Np, cl_start, cl_cams, S, dcam, tb, Wi, Ls, zs);
    else if (r == 1)
        ok = team_forward(k, S_off, cl_n, cl_Np, cl_start, cl_cams, S, b, tb, zs, ys);
    else {
        // list capacity: the most tasks any worker of this team owns (at most
        // all of them, which the launch's LDS holds for the largest cluster)
        const int T = cl_Np[k] / kNB;
        const int cap = team_own(T, W, 0);
        ok = team_worker(k, r - 1, W, S_off, cl_Np, S, tb, lists, lists + cap, lists + 2 * cap, zs);
    }
    // every wavefront of the team ends here; the last one writes the status
    // and returns the cluster's flags and vectors to their initial state
    const int T = cl_Np[k] / kNB;
    const int tt = T * (T + 1) / 2;
    int32_t *fl = tb.flags + team_fbase(S_off, k);
    int32_t *fl_err = fl + tt + 3 * T;
    int32_t *fl_cnt = fl_err + 1;
    int32_t *abort_w = tb.flags + tb.abort_at;
    if (!ok && lane == 0) __hip_atomic_store(fl_err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    int last = 0;
    if (lane == 0) last = __hip_atomic_fetch_add(fl_cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == W + 1;
    if (__shfl(last, 0, 64) == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    bool failed = false;
    if (lane == 0) {
        bool anybad = false;
        for (int p = 0; p < T; ++p)
            anybad |= __hip_atomic_load(fl + tile_ix(p, p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 2;
        failed = __hip_atomic_load(fl_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                 __hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        cl_status[k] = failed ? STBA_EHIP : (anybad ? STBA_ENOTPD : STBA_OK);
    }
    failed = __shfl((int)failed, 0, 64) != 0;
    for (int q = lane; q < tt + 3 * T + 1; q += 64) fl[q] = 0;
    const int64_t vb = team_vbase(S_off, k);
    for (int q = lane; q < T * kNB; q += 64) {
        tb.yv[vb + q] = __longlong_as_double(kEmpty);
        tb.xv[vb + q] = __longlong_as_double(kEmpty);
    }
    if (failed)   // after an abort the tile vectors may still hold values
        for (int64_t q = lane; q < (int64_t)tt * kNB; q += 64) {
            tb.cv[vb + q] = __longlong_as_double(kEmpty);
            tb.dv[vb + q] = __longlong_as_double(kEmpty);
        }
    __builtin_amdgcn_s_waitcnt(0);
    if (lane == 0) {
        __hip_atomic_store(fl_cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__hip_atomic_fetch_add(abort_w + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == n_act - 1) {
            __hip_atomic_store(abort_w, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(abort_w + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Dynamic LDS of k_chol_team for clusters of at most max_Np: the band's part,
// or a worker's lists for the most tasks one wavefront can own (one worker).
size_t team_lds_bytes(int32_t max_Np) {
    const int T = max_Np / kNB;
    const size_t band = sizeof(double) * (3 * kNB + 2 * kNB * (kNB + 1));
    const size_t worker = sizeof(double) * 3 * kNB + 12 * (size_t)team_ntasks(T);
    return band > worker ? band : worker;
}

// The initial state of the tile-parallel factorisation's flag words (zero)
// and block vectors (kEmpty).
__global__ void k_init_chol_sync(int32_t *flags, int64_t nf, double *yx, int64_t nv) {
    const int64_t n = nf > nv ? nf : nv;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < nf) flags[i] = 0;
        if (i < nv) yx[i] = __longlong_as_double(kEmpty);
    }
}

}  // namespace

// Wavefronts of k_chol_tiles that the current device holds at once (its
// dataflow waits need every wavefront of the grid resident); 0 if the query
// fails.  Asked on every call (no cached state), so a change of the current
// device is seen.
int64_t chol_tile_resident() {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_chol_tiles), 64, 0) !=
        hipSuccess)
        return 0;
    return (int64_t)cus * per_cu;
}

// Wavefronts of k_chol_team the current device holds at once with the LDS a
// cluster of order max_Np needs; 0 if the query fails.
int64_t chol_team_resident(int32_t max_Np) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_chol_team), 64,
                                                     team_lds_bytes(max_Np)) != hipSuccess)
        return 0;
    return (int64_t)cus * per_cu;
}

int chol_tile_layout(int32_t l, int32_t max_Np, int32_t *wpc, int32_t *tmax, int32_t *fpc, int32_t *xcd_major) {
    const int32_t tm = max_Np / kNB;
    if (tm < 1) return 0;
    const int64_t waves = 1 + (int64_t)tm + (int64_t)(tm - 1) * (tm - 2) / 2;   // band, rows, tiles
    if ((int64_t)l * waves > kCholTileWaves) return 0;
    // every wave must be resident at once (they wait on each other); keep a
    // sixteenth of the capacity in reserve
    if (16 * (int64_t)l * waves > 15 * chol_tile_resident()) return 0;
    const int64_t words = (int64_t)tm * (tm + 1) / 2 + tm + 2;
    if ((int64_t)l * words + 2 > chol_flag_words() || (int64_t)l * kVecSets * tm * kNB > chol_yx_doubles()) return 0;
    *tmax = tm;
    *wpc = (int32_t)waves;
    *fpc = (int32_t)words;
    // whole clusters per XCD when one XCD's share of the resident capacity (with
    // a quarter in reserve) holds ceil(l / 8) clusters
    *xcd_major = 4 * (((int64_t)l + 7) / 8) * waves <= 3 * (chol_tile_resident() / 8) ? 1 : 0;
    return 1;
}

int chol_form_fits(int32_t form, int32_t l, int32_t max_Np, bool l_on_device, const CholTeam *team) {
    if (form == STBA_CHOL_WORKGROUP) return 1;
    if (form == STBA_CHOL_TILES) {
        int32_t wpc, tmax, fpc, xcd;
        return !l_on_device && chol_tile_layout(l, max_Np, &wpc, &tmax, &fpc, &xcd);
    }
    if (form == STBA_CHOL_TEAM) {
        if (team == nullptr || team->flags == nullptr || max_Np > kTeamMaxNp) return 0;
        const int64_t G = 15 * chol_team_resident(max_Np) / 16;
        return G >= 3 * (int64_t)l || (l_on_device && G >= 3);
    }
    return 0;
}

hipError_t launch_chol(int32_t l, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                       const int32_t *cl_start, const int32_t *cl_cams, double *S, const double *b, double *dcam,
                       int32_t *cl_status, int32_t max_Np, int32_t *flags, double *yx, const CholTeam *team,
                       hipStream_t st) {
    int32_t wpc = 0, tmax = 0, fpc = 0, xcd = 0;
    const int32_t form = team != nullptr ? team->form : STBA_CHOL_AUTO;
    if (form == STBA_CHOL_WORKGROUP) goto workgroup_path;
    // with the number of clusters on the device the tile grid cannot be sized
    if (team != nullptr && (form == STBA_CHOL_TEAM || team->l_on_device)) goto team_path;
    if (flags && yx && chol_tile_layout(l, max_Np, &wpc, &tmax, &fpc, &xcd)) {
        // the flag words are zero and the vector entries kEmpty here: set when the
        // workspace was prepared and again at the end of every factorisation
        const int64_t blocks = xcd ? 8 * (((int64_t)l + 7) / 8) * wpc : (int64_t)l * wpc;
        k_chol_tiles<<<(unsigned)blocks, 64, 0, st>>>(wpc, tmax, fpc, cl_n, cl_Np, S_off, cl_start, cl_cams, S, b,
                                                     dcam, cl_status, flags, l, yx, xcd);
        return hipGetLastError();
    }
team_path:
    if (team != nullptr && team->flags != nullptr && max_Np <= kTeamMaxNp) {
        // every wavefront of a team waits on the others: all must be resident,
        // with a sixteenth of the capacity in reserve; a band, a forward wavefront
        // and a worker per cluster
        // With the number of clusters on the device the team form is tried
        // first and the workgroup form runs after it only if the teams did not
        // fit (a word the team launch writes).
        const int64_t G = 15 * chol_team_resident(max_Np) / 16;
        if (G >= 3 * (int64_t)l || (team->l_on_device && G >= 3)) {
            TeamBufs tb;
            tb.flags = team->flags;
            tb.abort_at = team->abort_at;
            tb.cv = team->vec;
            tb.dv = team->vec + team->vec_len;
            tb.yv = team->vec + 2 * team->vec_len;
            tb.xv = team->vec + 3 * team->vec_len;
            k_chol_team<<<(unsigned)G, 64, team_lds_bytes(max_Np), st>>>((int32_t)G, l, cl_n, cl_Np, S_off, cl_start,
                                                                         cl_cams, S, b, dcam, cl_status, tb);
            if (team->l_on_device) {
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
                const size_t shmem = sizeof(double) * (2 * (size_t)kNB * (kNB + 1) + 2 * kNB + (size_t)max_Np +
                                                       kCholThreads + kNB);
                k_chol<<<(unsigned)l, kCholThreads, shmem, st>>>(l, cl_n, cl_Np, S_off, cl_start, cl_cams, S, b, dcam,
                                                                 cl_status, max_Np, team->flags + team->abort_at + 2);
            }
            return hipGetLastError();
        }
    }
workgroup_path:
    const size_t shmem = sizeof(double) * (2 * (size_t)kNB * (kNB + 1) + 2 * kNB + (size_t)max_Np + kCholThreads + kNB);
    k_chol<<<(unsigned)l, kCholThreads, shmem, st>>>(l, cl_n, cl_Np, S_off, cl_start, cl_cams, S, b, dcam, cl_status,
                                                     max_Np, nullptr);
    return hipGetLastError();
}

hipError_t launch_clear_chol_flags(int32_t *flags, double *yx, const CholTeam *team, hipStream_t st) {
    const int64_t nf = chol_flag_words(), nv = chol_yx_doubles();
    k_init_chol_sync<<<(unsigned)(((nf > nv ? nf : nv) + 255) / 256), 256, 0, st>>>(flags, nf, yx, nv);
    if (team != nullptr && team->flags != nullptr) {
        const int64_t tf = team->abort_at + 3, tv = 4 * team->vec_len;
        int64_t blocks = ((tf > tv ? tf : tv) + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        k_init_chol_sync<<<(unsigned)blocks, 256, 0, st>>>(team->flags, tf, team->vec, tv);
    }
    return hipGetLastError();
}

hipError_t launch_sweep(int32_t l, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                        const int32_t *cl_start, const int32_t *cl_cams, const double *S, const double *r,
                        double *dcam, int32_t max_Np, hipStream_t st) {
    if (kSwStaticLds + sizeof(double) * (size_t)max_Np > 160 * 1024) return hipErrorInvalidConfiguration;
    k_sweep<<<(unsigned)l, kSwThreads, sizeof(double) * (size_t)max_Np, st>>>(cl_n, cl_Np, S_off, cl_start, cl_cams,
                                                                               S, r, dcam);
    return hipGetLastError();
}

}  // namespace stba
