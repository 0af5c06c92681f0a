// The inexact alternative to the cluster Cholesky (App. A, Table 3): each
// split reduced camera system S_k dc_k = b_k solved by conjugate gradient with
// the camera-block Jacobi preconditioner M = blockdiag(S_ii), from dc = 0 until
// ||r|| <= tol ||b|| or a cap on the iterations.
//
// One 512-thread workgroup per cluster; the five vectors (x, r, z, p, q) live in
// LDS.  The product S p visits only the 9 x 9 blocks of camera pairs that the
// plan links (per-camera lists of linked cameras in LDS, built from the plan's
// block list), so an iteration costs O(r') in the sampled camera connections,
// reading the lower triangle of the assembled S_k (the upper blocks as
// transposes of the stored lower ones).  Thread t owns rows t, t + 512, ...;
// every sum runs in a fixed order (per-thread rows, a wave butterfly, the waves
// in order), so results do not depend on scheduling.
#include "kernels.h"

namespace stba {
namespace {

constexpr int kPcgThreads = 512;
constexpr int kPcgWaves = kPcgThreads / 64;

__global__ __launch_bounds__(256) void k_cluster_of(const int32_t *cl_start, const int32_t *cl_cams, int32_t *clus) {
    const int k = blockIdx.x;
    for (int j = cl_start[k] + threadIdx.x; j < cl_start[k + 1]; j += blockDim.x) clus[cl_cams[j]] = k;
}

// Sum over the workgroup in a fixed order; every thread gets the result.
__device__ inline double wg_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kPcgWaves; ++w) s += red[w];
    __syncthreads();
    return s;
}

__device__ inline bool has_block(const uint32_t *bits, int n, int a, int c) {
    const int e = a * n + c;
    return (bits[e >> 5] >> (e & 31)) & 1u;
}

// One 9-entry product of row i of block (a, c) with p_c (column-major A, lower
// triangle stored, leading dimension Np): S_ac itself when c < a, the transpose
// of the stored S_ca when c > a, the symmetric diagonal block when c == a.
__device__ inline double block_row_dot(const double *A, int64_t Np, int a, int c, int i, const double *p) {
    const int64_t row = 9 * (int64_t)a + i;
    const double *pc = p + 9 * c;
    double v[9];
    if (c < a) {
        const double *col = A + 9 * (int64_t)c * Np + row;
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = col[j * Np];
    } else if (c > a) {
        const double *col = A + row * Np + 9 * (int64_t)c;
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = col[j];
    } else {
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int64_t rr = 9 * (int64_t)a + (i > j ? i : j), cc = 9 * (int64_t)a + (i > j ? j : i);
            v[j] = A[cc * Np + rr];
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 9; ++j) acc += v[j] * pc[j];
    return acc;
}

// (S p)_row for row = 9 a + i over camera a's linked cameras nbr[0..deg) (in
// ascending order), four blocks' loads in flight at a time; the partial sums are
// added in neighbour order.
__device__ inline double spmv_row(const double *A, int64_t Np, const int16_t *nbr, int deg, int a, int i,
                                  const double *p) {
    double acc = 0.0;
    int t = 0;
    for (; t + 4 <= deg; t += 4) {
        const double s0 = block_row_dot(A, Np, a, nbr[t], i, p);
        const double s1 = block_row_dot(A, Np, a, nbr[t + 1], i, p);
        const double s2 = block_row_dot(A, Np, a, nbr[t + 2], i, p);
        const double s3 = block_row_dot(A, Np, a, nbr[t + 3], i, p);
        acc += s0;
        acc += s1;
        acc += s2;
        acc += s3;
    }
    for (; t < deg; ++t) acc += block_row_dot(A, Np, a, nbr[t], i, p);
    return acc;
}

// z_row = (M^-1 r)_row with the inverse camera block of the row's camera.
__device__ inline double precond_row(const double *Mi, int a, int i, const double *r) {
    const double *m = Mi + 81 * (int64_t)a + 9 * i;
    const double *ra = r + 9 * a;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 9; ++j) s += m[j] * ra[j];
    return s;
}

__global__ __launch_bounds__(kPcgThreads) void k_pcg(
    const int32_t *__restrict__ clus, const int32_t *__restrict__ cl_n, const int32_t *__restrict__ cl_Np,
    const int64_t *__restrict__ S_off, const int32_t *__restrict__ cl_start, const int32_t *__restrict__ cl_cams,
    const int32_t *__restrict__ cam_local, const int64_t *__restrict__ n_blocks, const int2 *__restrict__ blk_key,
    const double *__restrict__ S, const double *__restrict__ b, double *__restrict__ dcam, double *__restrict__ Minv,
    int32_t max_np, int32_t max_n, int32_t max_iters, double tol, int32_t *__restrict__ iters_out,
    double *__restrict__ resid_out, int32_t *__restrict__ cl_status) {
    extern __shared__ double lds[];
    const int k = blockIdx.x, tid = threadIdx.x;
    const int n = cl_n[k], N = 9 * n;
    const int64_t Np = cl_Np[k];
    const double *A = S + S_off[k];
    const int c0 = cl_start[k];
    double *Mi = Minv + 81 * (int64_t)c0;
    double *x = lds, *r = x + max_np, *z = r + max_np, *p = z + max_np, *q = p + max_np;
    double *red = q + max_np;
    int32_t *flag = reinterpret_cast<int32_t *>(red + kPcgWaves);
    uint32_t *bits = reinterpret_cast<uint32_t *>(flag + 2);
    const int words = (n * n + 31) / 32;
    int32_t *nbr_off = reinterpret_cast<int32_t *>(bits + ((max_n * max_n + 31) / 32));   // [max_n + 1]
    int16_t *nbr = reinterpret_cast<int16_t *>(nbr_off + max_n + 1);                      // [max_n^2]

    // camera pairs of this cluster that the plan links (and every diagonal)
    for (int w = tid; w < words; w += kPcgThreads) bits[w] = 0u;
    if (tid == 0) flag[0] = 0;
    __syncthreads();
    const int64_t nb = n_blocks[0];
    for (int64_t e = tid; e < nb; e += kPcgThreads) {
        const int2 key = blk_key[e];
        if (clus[key.x] != k || clus[key.y] != k) continue;
        const int a = cam_local[key.x], c = cam_local[key.y];
        if (a >= n || c >= n) continue;   // a map rejected at the layout has n = 0
        atomicOr(&bits[(a * n + c) >> 5], 1u << ((a * n + c) & 31));
        atomicOr(&bits[(c * n + a) >> 5], 1u << ((c * n + a) & 31));
    }
    // the inverse camera blocks: Cholesky L of S_aa, W = L^-1, M^-1 = W^T W
    for (int a = tid; a < n; a += kPcgThreads) {
        const int e = a * n + a;
        atomicOr(&bits[e >> 5], 1u << (e & 31));
        double L[9][9];
        bool ok = true;
        for (int j = 0; j < 9; ++j) {
            for (int i = j; i < 9; ++i) {
                double v = A[(9 * (int64_t)a + j) * Np + 9 * a + i];
                for (int t = 0; t < j; ++t) v -= L[i][t] * L[j][t];
                if (i == j) {
                    ok = ok && v > 0.0 && isfinite(v);
                    L[j][j] = sqrt(v > 0.0 ? v : 1.0);
                } else {
                    L[i][j] = v / L[j][j];
                }
            }
        }
        double W[9][9];
        for (int j = 0; j < 9; ++j) {
            W[j][j] = 1.0 / L[j][j];
            for (int i = j + 1; i < 9; ++i) {
                double s = 0.0;
                for (int t = j; t < i; ++t) s += L[i][t] * W[t][j];
                W[i][j] = -s / L[i][i];
            }
        }
        for (int i = 0; i < 9; ++i)
            for (int j = 0; j < 9; ++j) {
                double s = 0.0;
                for (int t = (i > j ? i : j); t < 9; ++t) s += W[t][i] * W[t][j];
                Mi[81 * (int64_t)a + 9 * i + j] = s;
            }
        if (!ok) atomicOr(flag, 1);
    }
    __syncthreads();
    // neighbour lists: counts, offsets by a scan in camera order, ascending lists
    for (int a = tid; a < n; a += kPcgThreads) {
        int cnt = 0;
        for (int c = 0; c < n; ++c) cnt += has_block(bits, n, a, c) ? 1 : 0;
        nbr_off[a + 1] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
        nbr_off[0] = 0;
        for (int a = 0; a < n; ++a) nbr_off[a + 1] += nbr_off[a];
    }
    __syncthreads();
    for (int a = tid; a < n; a += kPcgThreads) {
        int o = nbr_off[a];
        for (int c = 0; c < n; ++c)
            if (has_block(bits, n, a, c)) nbr[o++] = (int16_t)c;
    }
    for (int row = tid; row < N; row += kPcgThreads) {
        x[row] = 0.0;
        r[row] = b[9 * (int64_t)cl_cams[c0 + row / 9] + row % 9];
    }
    __syncthreads();
    int status = flag[0] ? STBA_ENOTPD : STBA_OK;
    int it = 0;
    double bn = 0.0, rn = 0.0;
    if (status == STBA_OK) {
        double rz_p = 0.0, bb_p = 0.0;
        for (int row = tid; row < N; row += kPcgThreads) {
            const double zz = precond_row(Mi, row / 9, row % 9, r);
            z[row] = zz;
            p[row] = zz;
            rz_p += r[row] * zz;
            bb_p += r[row] * r[row];
        }
        double rz = wg_sum(rz_p, red);
        bn = sqrt(wg_sum(bb_p, red));
        rn = bn;
        while (bn > 0.0 && it < max_iters) {
            // p is complete (the sums above end with a barrier)
            double pq_p = 0.0;
            for (int row = tid; row < N; row += kPcgThreads) {
                const int a = row / 9;
                const double qq = spmv_row(A, Np, nbr + nbr_off[a], nbr_off[a + 1] - nbr_off[a], a, row % 9, p);
                q[row] = qq;
                pq_p += p[row] * qq;
            }
            const double pq = wg_sum(pq_p, red);
            if (!(pq > 0.0)) {
                status = STBA_ENOTPD;
                break;
            }
            const double alpha = rz / pq;
            double rr_p = 0.0;
            for (int row = tid; row < N; row += kPcgThreads) {
                x[row] += alpha * p[row];
                r[row] -= alpha * q[row];
                rr_p += r[row] * r[row];
            }
            rn = sqrt(wg_sum(rr_p, red));
            ++it;
            if (rn <= tol * bn) break;
            double rz_n = 0.0;
            for (int row = tid; row < N; row += kPcgThreads) {
                const double zz = precond_row(Mi, row / 9, row % 9, r);
                z[row] = zz;
                rz_n += r[row] * zz;
            }
            const double rz_new = wg_sum(rz_n, red);
            const double beta = rz_new / rz;
            rz = rz_new;
            for (int row = tid; row < N; row += kPcgThreads) p[row] = z[row] + beta * p[row];
            __syncthreads();
        }
    }
    for (int row = tid; row < N; row += kPcgThreads)
        dcam[9 * (int64_t)cl_cams[c0 + row / 9] + row % 9] = status == STBA_OK ? x[row] : 0.0;
    if (tid == 0) {
        iters_out[k] = it;
        resid_out[k] = bn > 0.0 ? rn / bn : 0.0;
        cl_status[k] = status;
    }
}

}  // namespace

size_t pcg_lds_bytes(int32_t max_np, int32_t max_n) {
    return sizeof(double) * (5 * (size_t)max_np + kPcgWaves) + 2 * sizeof(int32_t) +
           sizeof(uint32_t) * (((size_t)max_n * max_n + 31) / 32) + sizeof(int32_t) * ((size_t)max_n + 1) +
           sizeof(int16_t) * (size_t)max_n * max_n;
}

hipError_t launch_pcg(int32_t l, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                      const int32_t *cl_start, const int32_t *cl_cams, const int32_t *cam_local,
                      const int64_t *n_blocks, const int2 *blk_key, const double *S, const double *b, double *dcam,
                      int32_t *clus, double *Minv, int32_t max_np, int32_t max_n, int32_t max_iters, double tol,
                      int32_t *iters_out, double *resid_out, int32_t *cl_status, hipStream_t st) {
    const size_t shmem = pcg_lds_bytes(max_np, max_n);
    if (shmem > 160 * 1024) return hipErrorInvalidConfiguration;
    k_cluster_of<<<(unsigned)l, 256, 0, st>>>(cl_start, cl_cams, clus);
    k_pcg<<<(unsigned)l, kPcgThreads, shmem, st>>>(clus, cl_n, cl_Np, S_off, cl_start, cl_cams, cam_local, n_blocks,
                                                   blk_key, S, b, dcam, Minv, max_np, max_n, max_iters, tol, iters_out,
                                                   resid_out, cl_status);
    return hipGetLastError();
}

}  // namespace stba
