// Set-up of the static plan: validation of the visibility graph (Sec. 3) and the
// list of same-point observation pairs grouped by camera pair, i.e. the
// sparsity of E C^-1 E^T in the reduced camera matrix (Eq. 5).  Runs once per
// problem; the per-iteration kernels only read what it builds.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "kernels.h"

namespace stba {

namespace {

__device__ inline int64_t lower_bound_i32(const int32_t *a, int64_t len, int32_t key) {
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// scratch[0] += sum v(v+1)/2, scratch[1] = max v, scratch[2] |= error bits
__global__ __launch_bounds__(256) void k_analyze_points(int32_t n, int64_t q, const int32_t *obs_pt,
                                                        unsigned long long *scratch) {
    __shared__ double sh[256];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t pairs = 0;
    if (j < n) {
        const int64_t lo = lower_bound_i32(obs_pt, q, (int32_t)j);
        const int64_t hi = lower_bound_i32(obs_pt, q, (int32_t)(j + 1));
        const int64_t v = hi - lo;
        pairs = v * (v + 1) / 2;
        if (v == 0) atomicOr(&scratch[2], 1ull);
        atomicMax(&scratch[1], (unsigned long long)v);
    }
    // exact in double below 2^53 pairs per block
    const double s = block_sum_256((double)pairs, sh);
    if (threadIdx.x == 0) atomicAdd(&scratch[0], (unsigned long long)s);
}

__global__ __launch_bounds__(256) void k_analyze_obs(int32_t m, int32_t n, int64_t q, const int32_t *obs_cam,
                                                     const int32_t *obs_pt, unsigned long long *scratch) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= q) return;
    const int32_t c = obs_cam[o], j = obs_pt[o];
    if (c < 0 || c >= m || j < 0 || j >= n) { atomicOr(&scratch[2], 2ull); return; }
    if (o > 0) {
        const int32_t c0 = obs_cam[o - 1], j0 = obs_pt[o - 1];
        if (!(j0 < j || (j0 == j && c0 < c))) atomicOr(&scratch[2], 4ull);
    }
}

__global__ __launch_bounds__(256) void k_point_offsets(int32_t n, int64_t q, const int32_t *obs_pt,
                                                       int64_t *pt_off, int64_t *pair_cnt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > n) return;
    const int64_t lo = lower_bound_i32(obs_pt, q, (int32_t)j);
    pt_off[j] = lo;
    if (j < n) {
        const int64_t v = lower_bound_i32(obs_pt, q, (int32_t)(j + 1)) - lo;
        pair_cnt[j] = v * (v + 1) / 2;
    }
}

// All pairs (a, b), b <= a, of one point's observations; a has the larger camera.
__global__ __launch_bounds__(256) void k_gen_pairs(int32_t n, int32_t m, const int32_t *obs_cam,
                                                   const int64_t *pt_off, const int64_t *pair_off,
                                                   uint64_t *keys, uint64_t *vals) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int64_t out = pair_off[j];
    const int64_t p0 = pt_off[j], p1 = pt_off[j + 1];
    for (int64_t a = p0; a < p1; ++a) {
        const uint64_t ca = (uint64_t)obs_cam[a];
        for (int64_t b = p0; b <= a; ++b) {
            keys[out] = ca * (uint64_t)m + (uint64_t)obs_cam[b];
            vals[out] = ((uint64_t)a << 32) | (uint64_t)b;
            ++out;
        }
    }
}

__global__ __launch_bounds__(256) void k_head_flags(int64_t np, const uint64_t *keys, int64_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_scatter_heads(int64_t np, int32_t m, const uint64_t *keys,
                                                       const int64_t *flags, const int64_t *blk_of,
                                                       int2 *blk_key, int64_t *blk_start, int64_t *n_blocks,
                                                       int64_t *diag_blk) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    if (flags[i]) {
        const int64_t k = blk_of[i];
        const int32_t r = (int32_t)(keys[i] / (uint64_t)m), c = (int32_t)(keys[i] % (uint64_t)m);
        blk_key[k] = make_int2(r, c);
        blk_start[k] = i;
        if (r == c) diag_blk[r] = k;
    }
    if (i == np - 1) {
        const int64_t nb = blk_of[i] + flags[i];
        n_blocks[0] = nb;
        blk_start[nb] = np;
    }
}

// chunks of each block for the Schur assembly (zero past the last block)
__global__ __launch_bounds__(256) void k_block_chunks(int64_t cap, const int64_t *n_blocks, const int64_t *blk_start,
                                                      int64_t *nch) {
    const int64_t nb = n_blocks[0];
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= cap; b += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = 0;
        if (b < nb) {
            const int64_t len = blk_start[b + 1] - blk_start[b];
            c = (len + kSchurChunk - 1) / kSchurChunk;
        }
        nch[b] = c;
    }
}

// block index of every chunk
__global__ __launch_bounds__(256) void k_chunk_blk(const int64_t *n_blocks, const int64_t *blk_chunk_off,
                                                   int32_t *chunk_blk) {
    const int64_t nb = n_blocks[0];
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t c = blk_chunk_off[b]; c < blk_chunk_off[b + 1]; ++c) chunk_blk[c] = (int32_t)b;
    }
}

__global__ void k_total_chunks(const int64_t *n_blocks, const int64_t *blk_chunk_off, int64_t *n_chunks) {
    n_chunks[0] = blk_chunk_off[n_blocks[0]];
}

// Exclusive scan of one value per camera by one workgroup of 1024 threads:
// returns the sum of the values of the cameras before this thread's, the
// round's total in `total`.  Every thread of the workgroup calls it.
__device__ inline int64_t block_scan_excl(int64_t s, int64_t *wsum, int64_t &total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t inc = s;   // inclusive scan within the wavefront, then over the 16 wavefronts
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int64_t before = 0;
    total = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wv) before += wsum[w];
        total += wsum[w];
    }
    __syncthreads();   // wsum is rewritten by the next call
    return before + inc - s;
}

// Camera parts of the J^T v camera sums: camera r's diagonal-block list of
// len_r observations in ceil(len_r / kVjpPart) parts (one for a camera with
// none); part_off by an exclusive scan over the cameras in order, part_off[m]
// the total (at most m + q / kVjpPart); obs_off the exclusive scan of len_r
// (obs_off[m] = q).  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_vjp_parts(int32_t m, const int64_t *diag_blk, const int64_t *blk_start,
                                                    int64_t *part_off, int32_t *part_cam, int64_t cap,
                                                    int64_t *obs_off) {
    __shared__ int64_t wsum[16];
    int64_t carry = 0, carry_o = 0;
    for (int32_t base = 0; base < m; base += 1024) {
        const int32_t r = base + (int32_t)threadIdx.x;
        int64_t s = 0, len = 0;
        if (r < m) {
            const int64_t kb = diag_blk[r];
            len = kb >= 0 ? blk_start[kb + 1] - blk_start[kb] : 0;
            s = len > 0 ? (len + kVjpPart - 1) / kVjpPart : 1;
        }
        int64_t total = 0, total_o = 0;
        const int64_t first = carry + block_scan_excl(s, wsum, total);
        const int64_t first_o = carry_o + block_scan_excl(len, wsum, total_o);
        if (r < m) {
            part_off[r] = first;
            obs_off[r] = first_o;
            for (int64_t i = 0; i < s; ++i)
                if (first + i < cap) part_cam[first + i] = r;
        }
        carry += total;
        carry_o += total_o;
    }
    if (threadIdx.x == 0) {
        part_off[m] = carry < cap ? carry : cap;
        obs_off[m] = carry_o;
    }
}

// (observation, point) of camera r's diagonal-block pairs in list order at
// oj[obs_off[r] ..]: one wavefront per camera.  Without duplicated
// observations (which stba_analyze reports) there are q entries; past q
// nothing is written.
__global__ __launch_bounds__(256) void k_vjp_oj(int32_t m, int64_t q, const int64_t *diag_blk,
                                                const int64_t *blk_start, const uint64_t *pairs,
                                                const int32_t *obs_pt, const int64_t *obs_off, int2 *oj) {
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= m) return;
    const int64_t kb = diag_blk[r];
    if (kb < 0) return;
    const int64_t p0 = blk_start[kb], d0 = obs_off[r];
    int64_t len = blk_start[kb + 1] - p0;
    if (d0 + len > q) len = q > d0 ? q - d0 : 0;
    for (int64_t t = threadIdx.x & 63; t < len; t += 64) {
        const int32_t o = (int32_t)(pairs[p0 + t] >> 32);
        oj[d0 + t] = make_int2(o, obs_pt[o]);
    }
}

__global__ void k_fill_i64(int64_t *a, int64_t len, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) a[i] = v;
}

inline unsigned key_bits(int32_t m) {
    const uint64_t maxkey = (uint64_t)m * (uint64_t)m;
    unsigned bits = 1;
    while (bits < 64 && (1ull << bits) < maxkey) ++bits;
    return bits;
}

inline unsigned grid_for(int64_t count, int bs = 256) { return (unsigned)((count + bs - 1) / bs); }

}  // namespace

hipError_t launch_analyze(const stba_problem &p, int64_t *d_scratch, hipStream_t st) {
    auto *s = reinterpret_cast<unsigned long long *>(d_scratch);
    k_fill_i64<<<1, 64, 0, st>>>(d_scratch, 4, 0);
    k_analyze_obs<<<grid_for(p.q), 256, 0, st>>>(p.m, p.n, p.q, p.obs_cam, p.obs_pt, s);
    k_analyze_points<<<grid_for(p.n), 256, 0, st>>>(p.n, p.q, p.obs_pt, s);
    return hipGetLastError();
}

size_t prepare_tmp_bytes(int64_t n_pairs, int32_t m, hipStream_t st) {
    size_t a = 0, b = 0;
    (void)rocprim::radix_sort_pairs((void *)nullptr, a, (uint64_t *)nullptr, (uint64_t *)nullptr, (uint64_t *)nullptr,
                              (uint64_t *)nullptr, (size_t)n_pairs, 0u, key_bits(m), st);
    // the scans run over n points and n_pairs pairs; n <= n_pairs
    (void)rocprim::exclusive_scan((void *)nullptr, b, (int64_t *)nullptr, (int64_t *)nullptr, (int64_t)0,
                            (size_t)n_pairs + 1, rocprim::plus<int64_t>(), st);
    return a > b ? a : b;
}

hipError_t launch_prepare(const stba_problem &p, int64_t np, const PrepBufs &b, int32_t *status, hipStream_t st) {
    (void)status;
    hipError_t e;
    k_point_offsets<<<grid_for((int64_t)p.n + 1), 256, 0, st>>>(p.n, p.q, p.obs_pt, b.pt_off, b.scratch_a);
    size_t tb = b.tmp_bytes;
    e = rocprim::exclusive_scan(b.tmp, tb, b.scratch_a, b.pair_off, (int64_t)0, (size_t)p.n,
                                rocprim::plus<int64_t>(), st);
    if (e != hipSuccess) return e;
    k_gen_pairs<<<grid_for(p.n), 256, 0, st>>>(p.n, p.m, p.obs_cam, b.pt_off, b.pair_off, b.keys_in, b.vals_in);
    tb = b.tmp_bytes;
    e = rocprim::radix_sort_pairs(b.tmp, tb, b.keys_in, b.keys_out, b.vals_in, b.pairs, (size_t)np, 0u,
                                  key_bits(p.m), st);
    if (e != hipSuccess) return e;
    k_head_flags<<<grid_for(np), 256, 0, st>>>(np, b.keys_out, b.scratch_a);
    tb = b.tmp_bytes;
    e = rocprim::exclusive_scan(b.tmp, tb, b.scratch_a, b.blk_of, (int64_t)0, (size_t)np,
                                rocprim::plus<int64_t>(), st);
    if (e != hipSuccess) return e;
    k_fill_i64<<<grid_for(p.m), 256, 0, st>>>(b.diag_blk, p.m, -1);
    k_scatter_heads<<<grid_for(np), 256, 0, st>>>(np, p.m, b.keys_out, b.scratch_a, b.blk_of, b.blk_key,
                                                  b.blk_start, b.n_blocks, b.diag_blk);
    // Schur work items: chunk counts into the (now free) sort buffer, exclusive scan, chunk -> block
    int64_t *nch = reinterpret_cast<int64_t *>(b.keys_in);
    k_block_chunks<<<grid_for(b.blk_cap + 1), 256, 0, st>>>(b.blk_cap, b.n_blocks, b.blk_start, nch);
    tb = b.tmp_bytes;
    e = rocprim::exclusive_scan(b.tmp, tb, nch, b.blk_chunk_off, (int64_t)0, (size_t)b.blk_cap + 1,
                                rocprim::plus<int64_t>(), st);
    if (e != hipSuccess) return e;
    k_chunk_blk<<<grid_for(b.blk_cap), 256, 0, st>>>(b.n_blocks, b.blk_chunk_off, b.chunk_blk);
    k_total_chunks<<<1, 1, 0, st>>>(b.n_blocks, b.blk_chunk_off, b.n_chunks);
    k_vjp_parts<<<1, 1024, 0, st>>>(p.m, b.diag_blk, b.blk_start, b.vjp_part_off, b.vjp_part_cam, b.vjp_part_cap,
                                    b.vjp_obs_off);
    k_vjp_oj<<<grid_for(p.m, 4), 256, 0, st>>>(p.m, p.q, b.diag_blk, b.blk_start, b.pairs, p.obs_pt, b.vjp_obs_off,
                                               b.vjp_oj);
    return hipGetLastError();
}

}  // namespace stba
