// Per-iteration kernels of one STBA LM iteration (Alg. 1) on gfx950, except the
// cluster Cholesky (chol.hip).  Every kernel reads its sizes and the LM state
// from device memory so an iteration can be captured in a HIP graph.
#include "camera.h"
#include "kernels.h"
#include "philox.h"

namespace stba {

namespace {

inline unsigned grid_for(int64_t count, int bs = 256) { return (unsigned)((count + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// cluster layout: cameras grouped by cluster (ascending id inside a cluster),
// per-cluster sizes, padded orders and offsets of S_k (Eq. 13).
// As the first kernel of an iteration it also clears the status words.
// ---------------------------------------------------------------------------
// Exclusive scan over the block (at most 1024 threads, whole wavefronts): wave
// scans by shuffles, then a scan of the wave totals.  *total gets the sum.
template <typename V>
__device__ inline V block_exclusive_scan(V v, V *wsum, V *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    V inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const V n = __shfl_up(inc, d, 64);
        if (lane >= d) inc += n;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        V x = lane < nw ? wsum[lane] : (V)0;
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) {
            const V n = __shfl_up(x, d, 64);
            if (lane >= d) x += n;
        }
        if (lane < nw) wsum[lane] = x;
    }
    __syncthreads();
    const V base = w > 0 ? wsum[w - 1] : (V)0;
    *total = wsum[nw - 1];
    __syncthreads();   // wsum may be reused by the next scan
    return base + inc - v;
}

// The same layout for m <= 1024 cameras without sorting: one thread per camera
// and per cluster (l <= m), per-cluster counts in LDS, the position of a camera
// in its cluster = the number of lower-numbered cameras of that cluster.
__global__ __launch_bounds__(1024) void k_clusters_small(const int32_t *cam_cluster, int32_t m, int32_t l,
                                                         const int32_t *l_dev, int32_t gamma_max, int32_t *cl_n,
                                                         int32_t *cl_Np, int32_t *cl_start, int32_t *cl_cams,
                                                         int32_t *cam_local, int64_t *S_off, int32_t *cl_status,
                                                         int32_t *status) {
    __shared__ __align__(16) int32_t cl[1024];
    __shared__ int32_t cnt[1024];
    __shared__ int32_t ws32[16];
    __shared__ int64_t ws64[16];
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t < kStCount) status[t] = 0;
    if (t == 0) bad = 0;
    // ids are checked against the device count when there is one (clusters up to l stay empty)
    const int32_t lv = l_dev != nullptr ? l_dev[0] : l;
    const int32_t lid = (lv >= 1 && lv <= l) ? lv : 0;
    if (t < l) cl_status[t] = STBA_OK;
    int32_t k = -1;
    if (t < m) {
        k = cam_cluster[t];
        if (k < 0 || k >= lid) {
            bad = 1;
            k = -1;
        }
    }
    cl[t] = k;
    cnt[t] = 0;
    __syncthreads();
    if (k >= 0) atomicAdd(&cnt[k], 1);
    // four ids per LDS read, several reads in flight (entries past m hold -1)
    int32_t rank = 0;
    const int4 *cl4 = reinterpret_cast<const int4 *>(cl);
#pragma unroll 8
    for (int j4 = 0; j4 < (m + 3) / 4; ++j4) {
        const int4 v = cl4[j4];
        const int j = 4 * j4;
        rank += (j < t && v.x == k) + (j + 1 < t && v.y == k) + (j + 2 < t && v.z == k) + (j + 3 < t && v.w == k);
    }
    __syncthreads();
    const int32_t nk = t < l ? cnt[t] : 0;
    if (nk > gamma_max) bad = 2;
    int32_t tot32;
    const int32_t start = block_exclusive_scan<int32_t>(nk, ws32, &tot32);   // barriers publish bad
    const bool ok = bad == 0;
    const int32_t n_out = ok ? nk : 0;
    const int32_t np_out = ok ? (int32_t)round_up(9 * (int64_t)nk, kNB) : 0;
    if (t < l) {
        cl_n[t] = n_out;
        cl_Np[t] = np_out;
        cl_start[t] = start;
        cnt[t] = start;   // now the first slot of cluster t
    }
    if (t == 0) cl_start[l] = tot32;
    if (!ok && t == 0) set_status(status + kStSticky, STBA_EINVAL);
    __syncthreads();
    if (k >= 0) {
        cl_cams[cnt[k] + rank] = t;
        cam_local[t] = rank;
    }
    int64_t tot64;
    const int64_t off = block_exclusive_scan<int64_t>(t < l ? (int64_t)np_out * np_out : 0, ws64, &tot64);
    if (t < l) S_off[t] = off;
    if (t == 0) S_off[l] = tot64;
}

// The same layout for any m (up to kMaxCamsForClusters): ceil(m / 256)
// workgroups.  Every workgroup counts the cameras of each cluster over all
// cameras and over those before its own chunk of 256 (the lanes of a
// wavefront that share a cluster add their number at once), scans the counts
// (the same result in each workgroup), then one wavefront ranks the chunk's
// cameras in four rounds of 64 by the same ballots, so each camera's position
// is its cluster's start plus the number of lower-numbered cameras of that
// cluster.  Workgroup 0 alone clears the status words and writes the
// per-cluster arrays and S_off, so a bad map is reported after the clearing.
constexpr int kClusterLargeThreads = 256;
__global__ __launch_bounds__(kClusterLargeThreads) void k_clusters_large(
    const int32_t *cam_cluster, int32_t m, int32_t l, const int32_t *l_dev, int32_t gamma_max, int32_t *cl_n,
    int32_t *cl_Np, int32_t *cl_start, int32_t *cl_cams, int32_t *cam_local, int64_t *S_off, int32_t *cl_status,
    int32_t *status) {
    extern __shared__ __align__(16) int32_t dyn[];
    int32_t *cnt = dyn;          // [l] cameras per cluster, then the first slot of each cluster
    int32_t *base = dyn + l;     // [l] cameras of each cluster before this workgroup's chunk
    __shared__ int32_t ws32[16];
    __shared__ int64_t ws64[16];
    __shared__ int bad;
    const int t = threadIdx.x, lane = t & 63;
    const bool lead = blockIdx.x == 0;
    const int32_t chunk0 = (int32_t)blockIdx.x * kClusterLargeThreads;
    if (lead && t < kStCount) status[t] = 0;
    if (t == 0) bad = 0;
    // ids are checked against the device count when there is one (clusters up to l stay empty)
    const int32_t lv = l_dev != nullptr ? l_dev[0] : l;
    const int32_t lid = (lv >= 1 && lv <= l) ? lv : 0;
    for (int i = t; i < l; i += kClusterLargeThreads) {
        cnt[i] = 0;
        base[i] = 0;
        if (lead) cl_status[i] = STBA_OK;
    }
    __syncthreads();
    bool bad_id = false;
    for (int i0 = t - lane; i0 < m; i0 += kClusterLargeThreads) {   // wavefront-uniform
        const int i = i0 + lane;
        int32_t k = i < m ? cam_cluster[i] : -1;
        if (i < m && (k < 0 || k >= lid)) {
            bad_id = true;
            k = -1;
        }
        unsigned long long todo = __ballot(k >= 0);
        while (todo) {
            const int ld = __ffsll(todo) - 1;
            const int32_t key = __shfl(k, ld, 64);
            const unsigned long long same = __ballot(k == key);
            if (lane == ld) {
                atomicAdd(&cnt[key], __popcll(same));
                if (i0 < chunk0) atomicAdd(&base[key], __popcll(same));
            }
            todo &= ~same;
        }
    }
    if (bad_id) bad = 1;
    __syncthreads();
    // each thread scans a contiguous chunk of clusters
    const int chunk = (l + kClusterLargeThreads - 1) / kClusterLargeThreads;
    const int k0 = min(l, t * chunk), k1 = min(l, k0 + chunk);
    int32_t loc = 0;
    for (int k = k0; k < k1; ++k) {
        loc += cnt[k];
        if (cnt[k] > gamma_max) bad = 2;
    }
    int32_t tot32;
    int32_t run = block_exclusive_scan<int32_t>(loc, ws32, &tot32);   // its barriers publish bad
    const bool ok = bad == 0;
    int64_t loc2 = 0;
    for (int k = k0; k < k1; ++k) {
        const int32_t nk = cnt[k];
        const int32_t np_out = ok ? (int32_t)round_up(9 * (int64_t)nk, kNB) : 0;
        if (lead) {
            cl_n[k] = ok ? nk : 0;
            cl_Np[k] = np_out;
            cl_start[k] = run;
        }
        loc2 += (int64_t)np_out * np_out;
        cnt[k] = run;
        run += nk;
    }
    if (lead && t == 0) {
        cl_start[l] = tot32;
        if (!ok) set_status(status + kStSticky, STBA_EINVAL);
    }
    int64_t tot64;
    int64_t off = block_exclusive_scan<int64_t>(loc2, ws64, &tot64);   // its barriers publish the cnt writes
    if (lead) {
        for (int k = k0; k < k1; ++k) {
            S_off[k] = off;
            const int32_t nk = (k + 1 < l ? cnt[k + 1] : tot32) - cnt[k];
            const int64_t np = ok ? round_up(9 * (int64_t)nk, kNB) : 0;
            off += np * np;
        }
        if (t == 0) S_off[l] = tot64;
    }
    // ranks of this chunk's cameras, 64 at a time in camera order
    if (t < 64) {
        for (int sub = 0; sub < kClusterLargeThreads / 64; ++sub) {
            const int i = chunk0 + 64 * sub + lane;
            int32_t k = i < m ? cam_cluster[i] : -1;
            if (k >= lid) k = -1;
            unsigned long long todo = __ballot(k >= 0);
            while (todo) {
                const int ld = __ffsll(todo) - 1;
                const int32_t key = __shfl(k, ld, 64);
                const unsigned long long same = __ballot(k == key);
                if (k == key) {
                    const int32_t rank = base[key] + __popcll(same & ((1ull << lane) - 1ull));
                    cl_cams[cnt[key] + rank] = i;
                    cam_local[i] = rank;
                }
                __syncwarp();
                if (lane == ld) base[key] += __popcll(same);
                __syncwarp();
                todo &= ~same;
            }
        }
    }
}

__global__ void k_reset_status(int32_t *status) {
    if (threadIdx.x < kStCount) status[threadIdx.x] = 0;
}

__global__ void k_lm_init(stba_lm_state *st, double lambda0, double lambda_corr) {
    st->lambda = lambda0;
    st->lambda_corr = lambda_corr;
    st->F = 0.0;
    st->F_new = __builtin_nan("");
    st->accepted = 0;
    st->status = 0;
    st->need_jac = 1;
    st->have_F = 0;
    st->last_status = 0;
    st->pad0 = 0;
    st->n_jac = 0;
    st->n_rcs = 0;
    st->n_accept = 0;
    st->lambda_min = 0.0;
}

// ---------------------------------------------------------------------------
// a1: residuals and Jacobian blocks, one thread per observation (Sec. 3).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_rj(int64_t q, const double *__restrict__ cam, const double *__restrict__ pt,
                                            const int32_t *__restrict__ oc, const int32_t *__restrict__ op,
                                            const double *__restrict__ uv, T *__restrict__ f, T *__restrict__ Jc,
                                            T *__restrict__ Jp, double *__restrict__ partials,
                                            const int32_t *need_jac, int32_t *jac_ran, ZeroS z, double huber) {
    // the blocks go out through LDS half a workgroup at a time (128
    // observations, 24.6 KB in FP64), so that more workgroups fit on a CU
    __shared__ double sh[256];
    __shared__ T sJc[128 * 18];
    __shared__ T sJp[128 * 6];
    if (z.S != nullptr) {
        // S and b of this iteration start from zero (the grid runs even when the
        // Jacobian is kept)
        int64_t total = z.S_off[z.l];
        if (total > z.S_cap) total = z.S_cap;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) z.S[i] = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < z.nb; i += stride) z.b[i] = 0.0;
    }
    if (need_jac != nullptr && need_jac[0] == 0) return;
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double sq = 0.0;
    T bc[18], bp[6];
    if (o < q) {
        const int32_t i = oc[o], j = op[o];
        double c[9], X[3];
#pragma unroll
        for (int k = 0; k < 9; ++k) c[k] = cam[9 * (int64_t)i + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) X[k] = pt[3 * (int64_t)j + k];
        double pix[2], jc[2][9], jp[2][3];
        camera_project_jac(c, X, pix, jc, jp);
        const double f0 = pix[0] - uv[2 * o], f1 = pix[1] - uv[2 * o + 1];
        const double s2 = f0 * f0 + f1 * f1;
        sq = huber_rho(s2, huber);
        const double rw = huber_root_weight(s2, huber);   // 1 for the squared loss
        f[2 * o] = (T)(rw * f0);
        f[2 * o + 1] = (T)(rw * f1);
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int k = 0; k < 9; ++k) bc[9 * r + k] = (T)(rw * jc[r][k]);
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) bp[3 * r + k] = (T)(rw * jp[r][k]);
    }
    // the block's J_c and J_p rows are contiguous in memory: each half is
    // written back with consecutive lanes on consecutive elements
    const int tl = threadIdx.x;
    for (int h = 0; h < 2; ++h) {
        const int lo = 128 * h;
        if (o < q && tl >= lo && tl < lo + 128) {
            const int u = tl - lo;
#pragma unroll
            for (int k = 0; k < 18; ++k) sJc[18 * u + k] = bc[k];
#pragma unroll
            for (int k = 0; k < 6; ++k) sJp[6 * u + k] = bp[k];
        }
        const int64_t ob = (int64_t)blockIdx.x * blockDim.x + lo;
        const int64_t left = q - ob;
        const int nv = left <= 0 ? 0 : (int)min((int64_t)128, left);   // observations of this half
        __syncthreads();
        // every LDS read of the half first, then the stores (256 threads: at
        // most 9 elements of J_c and 3 of J_p each)
        if (Jc != nullptr) {
            T v[9];
#pragma unroll
            for (int u = 0; u < 9; ++u) v[u] = tl + 256 * u < 18 * nv ? sJc[tl + 256 * u] : (T)0;
#pragma unroll
            for (int u = 0; u < 9; ++u)
                if (tl + 256 * u < 18 * nv) Jc[18 * ob + tl + 256 * u] = v[u];
        }
        if (Jp != nullptr) {
            T v[3];
#pragma unroll
            for (int u = 0; u < 3; ++u) v[u] = tl + 256 * u < 6 * nv ? sJp[tl + 256 * u] : (T)0;
#pragma unroll
            for (int u = 0; u < 3; ++u)
                if (tl + 256 * u < 6 * nv) Jp[6 * ob + tl + 256 * u] = v[u];
        }
        __syncthreads();   // the next half reuses sJc, sJp
    }
    if (partials != nullptr) {
        const double s = block_sum_256(sq, sh);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
    if (jac_ran != nullptr && blockIdx.x == 0 && threadIdx.x == 0) jac_ran[0] = 1;
}

// Residuals alone (no Jacobian requested, nothing to clear): the pixel only,
// with the same weighting and cost partials as k_rj.
template <typename T>
__global__ __launch_bounds__(256) void k_resid_only(int64_t q, const double *__restrict__ cam,
                                                    const double *__restrict__ pt, const int32_t *__restrict__ oc,
                                                    const int32_t *__restrict__ op, const double *__restrict__ uv,
                                                    T *__restrict__ f, double *__restrict__ partials, double huber) {
    __shared__ double sh[256];
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double sq = 0.0;
    if (o < q) {
        const int32_t i = oc[o], j = op[o];
        double c[9], X[3];
#pragma unroll
        for (int k = 0; k < 9; ++k) c[k] = cam[9 * (int64_t)i + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) X[k] = pt[3 * (int64_t)j + k];
        double pix[2];
        camera_project(c, X, pix);
        const double f0 = pix[0] - uv[2 * o], f1 = pix[1] - uv[2 * o + 1];
        const double s2 = f0 * f0 + f1 * f1;
        sq = huber_rho(s2, huber);
        const double rw = huber_root_weight(s2, huber);
        f[2 * o] = (T)(rw * f0);
        f[2 * o + 1] = (T)(rw * f1);
    }
    if (partials != nullptr) {
        const double sum = block_sum_256(sq, sh);
        if (threadIdx.x == 0) partials[blockIdx.x] = sum;
    }
}

// Fixed-order sum of per-block partials (one 256-thread block).
__global__ __launch_bounds__(256) void k_sum_partials(const double *partials, int64_t count, double *out) {
    __shared__ double sh[256];
    const double s = block_sum_256(strided_sum_256(partials, count), sh);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void k_set_damping(double *slot, double lambda, double lambda_corr) {
    slot[0] = lambda;
    slot[1] = lambda_corr;
}

// ---------------------------------------------------------------------------
// 3x3 symmetric positive definite helpers (upper Cholesky V = R^T R)
// packed symmetric order: 00 01 02 11 12 22
// ---------------------------------------------------------------------------
struct Chol3 {
    double R00, R01, R02, R11, R12, R22;   // R
    double I00, I01, I02, I11, I12, I22;   // R^-1 (upper)
    bool ok;
};

__device__ inline Chol3 chol3(const double V[6]) {
    Chol3 c;
    c.ok = true;
    double d = V[0];
    if (!(d > 0.0)) { c.ok = false; d = 1.0; }
    c.R00 = sqrt(d);
    c.R01 = V[1] / c.R00;
    c.R02 = V[2] / c.R00;
    d = V[3] - c.R01 * c.R01;
    if (!(d > 0.0)) { c.ok = false; d = 1.0; }
    c.R11 = sqrt(d);
    c.R12 = (V[4] - c.R01 * c.R02) / c.R11;
    d = V[5] - c.R02 * c.R02 - c.R12 * c.R12;
    if (!(d > 0.0)) { c.ok = false; d = 1.0; }
    c.R22 = sqrt(d);
    c.I00 = 1.0 / c.R00;
    c.I11 = 1.0 / c.R11;
    c.I22 = 1.0 / c.R22;
    c.I01 = -c.R01 * c.I00 * c.I11;
    c.I12 = -c.R12 * c.I11 * c.I22;
    c.I02 = -(c.R01 * c.I12 + c.R02 * c.I22) * c.I00;
    return c;
}

// V^-1 = R^-1 R^-T, packed
__device__ inline void chol3_inverse(const Chol3 &c, double Vi[6]) {
    Vi[0] = c.I00 * c.I00 + c.I01 * c.I01 + c.I02 * c.I02;
    Vi[1] = c.I01 * c.I11 + c.I02 * c.I12;
    Vi[2] = c.I02 * c.I22;
    Vi[3] = c.I11 * c.I11 + c.I12 * c.I12;
    Vi[4] = c.I12 * c.I22;
    Vi[5] = c.I22 * c.I22;
}

__device__ inline void sym3_mul(const double S[6], const double x[3], double y[3]) {
    y[0] = S[0] * x[0] + S[1] * x[1] + S[2] * x[2];
    y[1] = S[1] * x[0] + S[3] * x[1] + S[4] * x[2];
    y[2] = S[2] * x[0] + S[4] * x[1] + S[5] * x[2];
}

template <typename T>
__device__ inline void load_jp(const T *Jp, int64_t o, double jp[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) jp[k] = (double)Jp[6 * o + k];
}

// FP64 residual and Jacobian rows of observation o (camera part cp of
// camera_pre, point j) at x, weighted as the residual kernel weights them
// (Huber when huber > 0): f [2], jc [2][9] row-major as J_c is stored, jp
// [2][3] as J_p.
__device__ inline void obs_fj64(const double cp[kCamPre], const double *__restrict__ pt,
                                const double *__restrict__ uv, double huber, int32_t j, int64_t o, double f[2],
                                double jc[18], double jp[6]) {
    const double X[3] = {pt[3 * (int64_t)j], pt[3 * (int64_t)j + 1], pt[3 * (int64_t)j + 2]};
    double pix[2], a[2][9], b[2][3];
    project_jac_pre(cp, X, pix, a, b);
    const double f0 = pix[0] - uv[2 * o], f1 = pix[1] - uv[2 * o + 1];
    const double rw = huber_root_weight(f0 * f0 + f1 * f1, huber);
    f[0] = rw * f0;
    f[1] = rw * f1;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int k = 0; k < 9; ++k) jc[9 * r + k] = rw * a[r][k];
#pragma unroll
        for (int k = 0; k < 3; ++k) jp[3 * r + k] = rw * b[r][k];
    }
}

// the same from camera i's parameters (9 loads; forming the camera part again
// costs less than gathering it from memory per observation)
__device__ inline void obs_fj64(const double *__restrict__ cam, const double *__restrict__ pt,
                                const double *__restrict__ uv, double huber, int32_t i, int32_t j, int64_t o,
                                double f[2], double jc[18], double jp[6]) {
    double c[9], cp[kCamPre];
#pragma unroll
    for (int k = 0; k < 9; ++k) c[k] = cam[9 * (int64_t)i + k];
    camera_pre(c, cp);
    obs_fj64(cp, pt, uv, huber, j, o, f, jc, jp);
}

// ---------------------------------------------------------------------------
// a0 + a2 + a3: per point, the sampled segments (point splitting and binding,
// Sec. 4.1-4.2), segment blocks V_s = sum J_p^T J_p and w'_s = -sum J_p^T f,
// the steepest-descent correction when lambda >= lambda_corr (Sec. 4.3), and
// the per-observation record used by the Schur assembly:
//   Y_o = W_o R_s^-1 (W_o = J_c,o^T J_p,o, R_s^T R_s = V*_s), so that
//   W_o V*_s^-1 W_o'^T = Y_o Y_o'^T (Eq. 10),
//   M_o = I - J_p,o V*_s^-1 J_p,o^T and r_o = f_o + J_p,o V*_s^-1 w'_s, so that
//   S_ii = sum J_c^T M J_c + lambda diag(U_i) and b_i = -sum J_c^T r.
// Also the physical damped V*_j^-1 and w_j for the point update (Eq. 15).
// One thread per point.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_points(int32_t n, const int64_t *__restrict__ pt_off,
                                               const int32_t *__restrict__ obs_cam,
                                               const int32_t *__restrict__ cam_cluster, const T *__restrict__ f,
                                               const T *__restrict__ Jp, Damp dm,
                                               uint64_t seed, uint64_t t, uint64_t thr, int32_t *__restrict__ seg_head,
                                               double *__restrict__ seg_rec, double *__restrict__ Vinv,
                                               double *__restrict__ wph, int32_t *status) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double *lp = dm.at_pt(j);
    const double lam = lp[0];
    const bool corr = lam >= lp[1];
    const int64_t p0 = pt_off[j], p1 = pt_off[j + 1];
    // segment heads: the chain of a cluster follows camera order, which is storage order
    for (int64_t a = p0; a < p1; ++a) {
        const int32_t ca = obs_cam[a];
        const int32_t ka = cam_cluster[ca];
        int64_t pred = -1;
        for (int64_t b = a - 1; b >= p0; --b) {
            if (cam_cluster[obs_cam[b]] == ka) {
                pred = b;
                break;
            }
        }
        int32_t h = (int32_t)a;
        if (pred >= 0 && keep_link(seed, t, (uint64_t)j, (uint64_t)ca, thr)) h = seg_head[pred];
        seg_head[a] = h;
    }
    // physical blocks
    double V[6] = {0, 0, 0, 0, 0, 0}, w[3] = {0, 0, 0};
    for (int64_t a = p0; a < p1; ++a) {
        double jp[6];
        load_jp(Jp, a, jp);
        const double f0 = (double)f[2 * a], f1 = (double)f[2 * a + 1];
        V[0] += jp[0] * jp[0] + jp[3] * jp[3];
        V[1] += jp[0] * jp[1] + jp[3] * jp[4];
        V[2] += jp[0] * jp[2] + jp[3] * jp[5];
        V[3] += jp[1] * jp[1] + jp[4] * jp[4];
        V[4] += jp[1] * jp[2] + jp[4] * jp[5];
        V[5] += jp[2] * jp[2] + jp[5] * jp[5];
        w[0] -= jp[0] * f0 + jp[3] * f1;
        w[1] -= jp[1] * f0 + jp[4] * f1;
        w[2] -= jp[2] * f0 + jp[5] * f1;
    }
    bool ok = true;
    {
        double Vd[6] = {V[0] * (1.0 + lam), V[1], V[2], V[3] * (1.0 + lam), V[4], V[5] * (1.0 + lam)};
        const Chol3 c = chol3(Vd);
        ok &= c.ok;
        double Vi[6];
        chol3_inverse(c, Vi);
#pragma unroll
        for (int k = 0; k < 6; ++k) Vinv[6 * j + k] = Vi[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) wph[3 * j + k] = w[k];
    }
    for (int64_t h = p0; h < p1; ++h) {
        if (seg_head[h] != (int32_t)h) continue;
        double Vs[6] = {0, 0, 0, 0, 0, 0}, ws[3] = {0, 0, 0};
        for (int64_t a = h; a < p1; ++a) {
            if (seg_head[a] != (int32_t)h) continue;
            double jp[6];
            load_jp(Jp, a, jp);
            const double f0 = (double)f[2 * a], f1 = (double)f[2 * a + 1];
            Vs[0] += jp[0] * jp[0] + jp[3] * jp[3];
            Vs[1] += jp[0] * jp[1] + jp[3] * jp[4];
            Vs[2] += jp[0] * jp[2] + jp[3] * jp[5];
            Vs[3] += jp[1] * jp[1] + jp[4] * jp[4];
            Vs[4] += jp[1] * jp[2] + jp[4] * jp[5];
            Vs[5] += jp[2] * jp[2] + jp[5] * jp[5];
            ws[0] -= jp[0] * f0 + jp[3] * f1;
            ws[1] -= jp[1] * f0 + jp[4] * f1;
            ws[2] -= jp[2] * f0 + jp[5] * f1;
        }
        if (corr) {
            // g'_s = h_s (sum_s g_s) / (sum_s h_s), h_s = (1 + lambda) diag(V_s);
            // sum_s g_s = w_j and sum_s diag(V_s) = diag(V_j)
            ws[0] = Vs[0] * w[0] / V[0];
            ws[1] = Vs[3] * w[1] / V[3];
            ws[2] = Vs[5] * w[2] / V[5];
        }
        const double Vd[6] = {Vs[0] * (1.0 + lam), Vs[1], Vs[2], Vs[3] * (1.0 + lam), Vs[4], Vs[5] * (1.0 + lam)};
        const Chol3 c = chol3(Vd);
        ok &= c.ok;
        double Vi[6];
        chol3_inverse(c, Vi);
        double u[3];
        sym3_mul(Vi, ws, u);   // V*_s^-1 w'_s
        double *rec = seg_rec + (int64_t)kSegRec * h;
        rec[0] = c.I00;
        rec[1] = c.I01;
        rec[2] = c.I02;
        rec[3] = c.I11;
        rec[4] = c.I12;
        rec[5] = c.I22;
#pragma unroll
        for (int k = 0; k < 6; ++k) rec[6 + k] = Vi[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) rec[12 + k] = u[k];
    }
    if (!ok) set_status(status + kStPointBad, STBA_ENOTPD);
}

// The assembly record of observation a (layout at obs_rec_elems): G = J_p R^-1
// with R^-1 = I (upper, I00 I01 I02 I11 I12 I22), M = I - J_p V*^-1 J_p^T and
// r = f + J_p u, u = V*^-1 w'; jc is read only for FP32.  FP64: G (0..5), pad,
// M (8..10), r (11, 12), pad, 128 bytes; FP32: J_c (0..17), G, M, r, pad.
template <typename T>
__device__ inline void write_obs_rec(T *__restrict__ obsd, int64_t a, const double jc[18], const double jp[6],
                                     const Chol3 &c, const double Vi[6], const double u[3], double f0, double f1) {
    T *rec = obsd + (int64_t)obs_rec_elems<T>() * a;
    constexpr int kG = sizeof(T) == 8 ? 0 : 18;   // where G starts
    // where M and r start: in FP64 at the record's second 64 bytes, so that the
    // assembly's reads of G and of M, r each touch one 64-byte segment
    constexpr int kM = sizeof(T) == 8 ? 8 : kG + 6;
    if (sizeof(T) != 8) {
#pragma unroll
        for (int k = 0; k < 18; ++k) rec[k] = (T)jc[k];
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const double p0 = jp[3 * r], p1 = jp[3 * r + 1], p2 = jp[3 * r + 2];
        rec[kG + 3 * r + 0] = (T)(p0 * c.I00);
        rec[kG + 3 * r + 1] = (T)(p0 * c.I01 + p1 * c.I11);
        rec[kG + 3 * r + 2] = (T)(p0 * c.I02 + p1 * c.I12 + p2 * c.I22);
    }
    double G0[3], G1[3];
    const double r0v[3] = {jp[0], jp[1], jp[2]}, r1v[3] = {jp[3], jp[4], jp[5]};
    sym3_mul(Vi, r0v, G0);
    sym3_mul(Vi, r1v, G1);
    rec[kM + 0] = (T)(1.0 - (G0[0] * jp[0] + G0[1] * jp[1] + G0[2] * jp[2]));
    rec[kM + 1] = (T)(-(G0[0] * jp[3] + G0[1] * jp[4] + G0[2] * jp[5]));
    rec[kM + 2] = (T)(1.0 - (G1[0] * jp[3] + G1[1] * jp[4] + G1[2] * jp[5]));
    rec[kM + 3] = (T)(f0 + jp[0] * u[0] + jp[1] * u[1] + jp[2] * u[2]);
    rec[kM + 4] = (T)(f1 + jp[3] * u[0] + jp[4] * u[1] + jp[5] * u[2]);
#pragma unroll
    for (int k = kG + 6; k < kM; ++k) rec[k] = (T)0;
#pragma unroll
    for (int k = kM + 5; k < obs_rec_elems<T>(); ++k) rec[k] = (T)0;
}

// Per observation of segment s, the assembly record (see write_obs_rec) from
// the segment record of k_points.  One thread per observation.
template <typename T>
__global__ __launch_bounds__(256) void k_obs_rec(int64_t q, const int32_t *__restrict__ seg_head,
                                                 const double *__restrict__ seg_rec, const T *__restrict__ f,
                                                 const T *__restrict__ Jc, const T *__restrict__ Jp,
                                                 T *__restrict__ obsd) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= q) return;
    const double *sr = seg_rec + (int64_t)kSegRec * seg_head[a];
    Chol3 c;
    c.I00 = sr[0];
    c.I01 = sr[1];
    c.I02 = sr[2];
    c.I11 = sr[3];
    c.I12 = sr[4];
    c.I22 = sr[5];
    double Vi[6], u[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) Vi[k] = sr[6 + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = sr[12 + k];
    double jp[6], jc[18];
    load_jp(Jp, a, jp);
    if (sizeof(T) != 8) {
#pragma unroll
        for (int k = 0; k < 18; ++k) jc[k] = (double)Jc[18 * a + k];
    }
    write_obs_rec<T>(obsd, a, jc, jp, c, Vi, u, (double)f[2 * a], (double)f[2 * a + 1]);
}

// ---------------------------------------------------------------------------
// The same work as k_points + k_obs_rec with one lane per observation: wavefront
// g takes the points whose first observation lies in [G g, G (g + 1)), which
// spans at most G - 1 + max_track <= 64 observations.  Each lane finds its chain
// predecessor (the nearest earlier observation of its point in the same
// cluster) by shuffles, draws its link, and the segment heads follow by pointer
// jumping.  The point's and the segment's blocks are summed from LDS in
// observation order (the order k_points uses), every lane factors its
// segment's V*_s (3x3, in registers) and writes its own record.
// ---------------------------------------------------------------------------
constexpr int kPtWaves = 4;

template <typename T>
__global__ __launch_bounds__(64 * kPtWaves) void k_points_obs(
    int64_t ngroups, const int32_t *__restrict__ grp_first, const int64_t *__restrict__ pt_off,
    const int32_t *__restrict__ obs_pt, const int32_t *__restrict__ obs_cam, const int32_t *__restrict__ cam_cluster,
    const T *__restrict__ f, const T *__restrict__ Jc, const T *__restrict__ Jp, Damp dm,
    uint64_t seed, uint64_t t, uint64_t thr, int32_t *__restrict__ seg_head, T *__restrict__ obsd,
    double *__restrict__ Vinv, double *__restrict__ wph, int32_t *status) {
    // per wavefront: J_p^T J_p (6) and -J_p^T f (3) of each lane, later the
    // wavefront's assembly records on their way out
    constexpr int kRecB = 64 * obs_rec_elems<T>() * (int)sizeof(T);
    constexpr int kBufB = kRecB > 9 * 64 * 8 ? kRecB : 9 * 64 * 8;
    __shared__ __align__(16) char sBuf[kPtWaves][kBufB];
    __shared__ int32_t sHead[kPtWaves][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    double(&sVw)[9][64] = *reinterpret_cast<double(*)[9][64]>(sBuf[wv]);
    const int64_t g = (int64_t)blockIdx.x * kPtWaves + wv;
    if (g >= ngroups) return;
    // every window of G observations inside [0, q) holds a point start (G > max_track);
    // only the last window can be empty, and then the group before it runs to n
    const int32_t pa = grp_first[g];
    int32_t pb = grp_first[g + 1];
    if (pb < 0) pb = grp_first[ngroups];
    if (pa < 0 || pb < pa) return;
    const int64_t o0 = pt_off[pa], o1 = pt_off[pb];
    if (o1 - o0 > 64) {   // the plan does not fit this data (inconsistent max_track)
        if (lane == 0) set_status(status + kStSticky, STBA_EDATA);
        return;
    }
    const int cnt = (int)(o1 - o0);
    const bool act = lane < cnt;
    const int64_t a = o0 + (act ? lane : 0);
    // every per-observation input requested at once (one round trip), the
    // camera's cluster after it
    const int32_t j = obs_pt[a];
    const int32_t cam = obs_cam[a];
    double jp[6];
    load_jp(Jp, a, jp);
    const double f0 = (double)f[2 * a], f1 = (double)f[2 * a + 1];
    // J_c goes into the record only in FP32 (the FP64 assembly reads it from Jc)
    double jc[18];
    if (sizeof(T) != 8) {
#pragma unroll
        for (int k = 0; k < 18; ++k) jc[k] = (double)Jc[18 * a + k];
    }
    const double *lp = dm.at_pt(j);
    const double lam = lp[0];
    const bool corr = lam >= lp[1];
    const int32_t cl = act ? cam_cluster[cam] : -1;
    // my point's lanes [first, last): observations are sorted by point and the
    // group starts at a point, so the point starts are where obs_pt changes
    const int32_t jprev = __shfl(j, lane > 0 ? lane - 1 : 0, 64);
    const uint64_t starts = __ballot(act && (lane == 0 || j != jprev));
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    const uint64_t after = starts & ~upto & (cnt >= 64 ? ~0ull : ((1ull << cnt) - 1));
    const int first = act ? 63 - __builtin_clzll(starts & upto) : lane;
    const int last = act ? (after != 0 ? __builtin_ctzll(after) : cnt) : lane + 1;
    double c[9];
    c[0] = jp[0] * jp[0] + jp[3] * jp[3];
    c[1] = jp[0] * jp[1] + jp[3] * jp[4];
    c[2] = jp[0] * jp[2] + jp[3] * jp[5];
    c[3] = jp[1] * jp[1] + jp[4] * jp[4];
    c[4] = jp[1] * jp[2] + jp[4] * jp[5];
    c[5] = jp[2] * jp[2] + jp[5] * jp[5];
    c[6] = -(jp[0] * f0 + jp[3] * f1);
    c[7] = -(jp[1] * f0 + jp[4] * f1);
    c[8] = -(jp[2] * f0 + jp[5] * f1);
#pragma unroll
    for (int k = 0; k < 9; ++k) sVw[k][lane] = act ? c[k] : 0.0;
    // chain predecessor: nearest earlier lane of the same point in the same
    // cluster; the search ends as soon as no lane has one left to look at (the
    // longest track of the group, not 63 steps), four distances per round with
    // their exchanges in flight together
    int pred = -1;
    for (int d0 = 1; d0 < 64; d0 += 4) {
        int32_t clo[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int src = lane - d0 - u;
            clo[u] = __shfl(cl, src < 0 ? 0 : src, 64);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int src = lane - d0 - u;
            if (pred < 0 && src >= first && clo[u] == cl) pred = src;
        }
        if (__ballot(pred < 0 && lane - d0 - 4 >= first) == 0) break;
    }
    int head = lane;
    if (act && pred >= 0 && keep_link(seed, t, (uint64_t)j, (uint64_t)cam, thr)) head = pred;
    // pointer jumping: chains are at most 64 long
#pragma unroll
    for (int it = 0; it < 6; ++it) head = __shfl(head, head, 64);
    sHead[wv][lane] = head;
    __syncwarp();
    // point sums (V_j, w_j) and segment sums (V_s, w'_s) in observation order
    double V[6] = {0, 0, 0, 0, 0, 0}, w[3] = {0, 0, 0}, Vs[6] = {0, 0, 0, 0, 0, 0}, ws[3] = {0, 0, 0};
    for (int b = first; b < last; ++b) {
        const bool mine = sHead[wv][b] == head;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double x = sVw[k][b];
            V[k] += x;
            if (mine) Vs[k] += x;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double x = sVw[6 + k][b];
            w[k] += x;
            if (mine) ws[k] += x;
        }
    }
    __syncwarp();   // every read of sVw is done before the records overwrite it
    bool ok = true;
    if (act) {
        if (lane == first) {
            double Vd[6] = {V[0] * (1.0 + lam), V[1], V[2], V[3] * (1.0 + lam), V[4], V[5] * (1.0 + lam)};
            const Chol3 cj = chol3(Vd);
            ok &= cj.ok;
            double Vi[6];
            chol3_inverse(cj, Vi);
#pragma unroll
            for (int k = 0; k < 6; ++k) Vinv[6 * (int64_t)j + k] = Vi[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) wph[3 * (int64_t)j + k] = w[k];
        }
        if (corr) {
            // g'_s = h_s (sum_s g_s) / (sum_s h_s), h_s = (1 + lambda) diag(V_s);
            // sum_s g_s = w_j and sum_s diag(V_s) = diag(V_j)
            ws[0] = Vs[0] * w[0] / V[0];
            ws[1] = Vs[3] * w[1] / V[3];
            ws[2] = Vs[5] * w[2] / V[5];
        }
        const double Vd[6] = {Vs[0] * (1.0 + lam), Vs[1], Vs[2], Vs[3] * (1.0 + lam), Vs[4], Vs[5] * (1.0 + lam)};
        const Chol3 cs = chol3(Vd);
        ok &= cs.ok;
        double Vi[6], u[3];
        chol3_inverse(cs, Vi);
        sym3_mul(Vi, ws, u);   // V*_s^-1 w'_s
        seg_head[a] = (int32_t)(o0 + head);
        write_obs_rec<T>(reinterpret_cast<T *>(sBuf[wv]), lane, jc, jp, cs, Vi, u, f0, f1);
    }
    __syncwarp();
    // the group's records are contiguous in memory: consecutive lanes store
    // consecutive elements
    constexpr int E = obs_rec_elems<T>();
    const T *srec = reinterpret_cast<const T *>(sBuf[wv]);
#pragma unroll 4
    for (int i = lane; i < cnt * E; i += 64) obsd[o0 * E + i] = srec[i];
    if (!ok) set_status(status + kStPointBad, STBA_ENOTPD);
}

// first point of every group of k_points_obs: group g holds the points whose
// first observation lies in [G g, G (g + 1))
__global__ void k_point_groups(int32_t n, const int64_t *__restrict__ pt_off, int32_t G, int64_t ngroups,
                               int32_t *__restrict__ grp_first) {
    const int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jj < n) {
        const int64_t gg = pt_off[jj] / G;
        if (jj == 0 || pt_off[jj - 1] / G != gg) grp_first[gg] = (int32_t)jj;
    }
    if (jj == 0) grp_first[ngroups] = n;
}

// zero S (all clusters) and b
__global__ __launch_bounds__(256) void k_zero_S(double *S, double *b, int32_t m, const int64_t *S_off, int32_t l,
                                                int64_t S_cap) {
    int64_t total = S_off[l];
    if (total > S_cap) total = S_cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) S[i] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 9 * (int64_t)m; i += stride) b[i] = 0.0;
}

// ---------------------------------------------------------------------------
// a4: Schur assembly.  Every camera pair (r, c), r >= c, of the static pair list
// is cut into chunks of kSchurChunk observation pairs; one wavefront takes one
// chunk.  Lane (s, h): s in 0..31 is the pair slot (every 32nd pair of the
// chunk), h picks rows 0..4 or 5..8 of the 9x9 block, so each lane holds its
// rows in registers and every observation record is read once per pair.
// Off-diagonal blocks S_rc = -sum Y_u Y_w^T over pairs in the same segment
// (Eq. 10); diagonal blocks S_rr = sum J_c^T M J_c + lambda diag(U_r) and
// b_r = -sum J_c^T r (Eq. 13).  Blocks of cameras in different clusters are
// dropped (S' is cluster-diagonal).  The 32 slots are summed by a butterfly
// (bit-identical in every lane).  A block of one chunk is written directly; a
// block of several chunks stores one partial sum per chunk and k_schur_reduce
// adds them in chunk order, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void schur_butterfly(T (&acc)[5][9], T (&du)[5], T (&rb)[5], bool diag) {
#pragma unroll
    for (int d = 2; d < 64; d <<= 1) {
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            // one row in flight at a time: the exchanged copies would otherwise
            // double the accumulator registers
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[i][k] += __shfl_xor(acc[i][k], d, 64);
        }
        if (diag) {
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                du[i] += __shfl_xor(du[i], d, 64);
                rb[i] += __shfl_xor(rb[i], d, 64);
            }
        }
    }
}

// Staging of one wavefront's work in LDS.  A batch is 32 pairs.  An
// observation's inputs form a virtual record of 32 elements: J_c (0..17, 2x9
// row-major), G = J_p R^-1 (18..23), M (24..26), r (27, 28), pad; in FP64
// J_c comes from the Jacobian and the rest from the assembly record, in FP32
// the record holds all of it (obs_rec_elems).  Batches move from memory
// straight into LDS by load-to-LDS instructions in 16-byte parts, whole cache
// lines per instruction, no registers holding them in flight.
template <typename T> struct SchurShape {
    static constexpr int kPart = 16 / (int)sizeof(T);      // elements per 16-byte part (2 | 4)
    static constexpr int kLanesRec = 32 / kPart;             // parts of a virtual record (16 | 8)
    static constexpr int kRecStep = 64 / kLanesRec;          // records per load instruction
    static constexpr int kLoads = 64 / kRecStep;             // loads per lane for 64 records
    static constexpr int kOffParts = 24 / kPart;             // parts of J_c and G (an off-diagonal pair's use)
    static constexpr int kDiagParts = 28 / kPart + 1;        // parts up to r (a diagonal pair's use)
    static constexpr int kStage = 256;                       // pairs compacted at a time
    // part p of observation o's virtual record (FP32: the assembly record is
    // the virtual record; FP64 batches use the grouped layout below)
    __device__ static const T *src(const T *, const T *obsd, int64_t o, int p) {
        static_assert(sizeof(T) == 4, "FP64 batches are staged in the grouped layout");
        return obsd + (int64_t)obs_rec_elems<T>() * o + kPart * p;
    }
    // Batches: the 32 u records (side 0), then the 32 w (side 1) of an
    // off-diagonal batch, or the 32 records of a diagonal one (side 0).  Load
    // instruction i fills its own block of 64 x 16 bytes (lane j writes bytes
    // [16 j, 16 j + 16)) record by record: lanes kLanesRec q .. kLanesRec q +
    // kLanesRec - 1 take the parts of one record, so every four lanes read 64
    // contiguous bytes (the address unit serves them as one access instead of
    // four).  Instruction i of a side holds the records of slots i, i + kNI, ..,
    // so the four slots that eight consecutive lanes read together sit in
    // blocks kBlk bytes apart, on four different bank groups.
    static constexpr int kNI = 32 / kRecStep;                // load instructions per side
    static constexpr int kBlk = 1024 + 64;
    static constexpr int kDmaBytes = kLoads * kBlk;
    __device__ static int row_at(int R) {
        const int s = R & 31;
        return ((R >> 5) * kNI + s % kNI) * kBlk + (s / kNI) * kLanesRec * 16;
    }
    __device__ static constexpr int elem_at(int k) { return (k / kPart) * 16 + (k % kPart) * (int)sizeof(T); }
    // diagonal batches: side 0 only, kDiagParts parts per record (lanes past
    // them repeat the last one into the pad)
    static constexpr int kDLoads = kNI;
    static constexpr int kDBytes = kDLoads * kBlk;
    // FP64 batches use a layout of their own: the 12 parts a pair uses (J_c:
    // parts 0..8 from the Jacobian; G, or M and r in a diagonal batch: parts
    // 9..11 from the assembly record) of the 64 (32) records in 6 groups of
    // two parts.  Group t
    // holds parts 2t and 2t + 1 of every record, 32 bytes per record in record
    // order, so in a load instruction (one group, one side) two consecutive
    // lanes take one record and each lane keeps its record for all six groups:
    // two record indices and a few address operations per lane and batch.
    // Groups are kGS bytes apart (2 KB and one part): element k + 4 of a J_c
    // row lies exactly one group after element k (two parts on), so the lanes
    // of rows 4..8 read at a fixed distance from those of rows 0..4 and on
    // other banks.
    static constexpr int kGS = 2048 + 16;
    static constexpr int kOff64Bytes = 5 * kGS + 2048;
    // part of element k: J_c 0..8; G (18..23, off-diagonal batches) or M and r
    // (24..28, diagonal batches) 9..11
    __device__ static constexpr int part64(int k) { return k < 18 ? k / 2 : (k < 24 ? 9 + (k - 18) / 2 : 9 + (k - 24) / 2); }
    __device__ static constexpr int off64(int k) {   // element k of a record, record 0
        return (part64(k) / 2) * kGS + (part64(k) % 2) * 16 + (k % 2) * 8;
    }
};

// One off-diagonal pair of a lane's batch slot: rows e0..e0 + 4 of
// J_c,u^T (G_u G_w^T) J_c,w added to acc.  eu(k) / ew(k) read element k of
// the u / w virtual record (G at 18..23), eue(k) element k of J_c,u moved on
// to row e0.
template <typename T, typename EU, typename EUE, typename EW>
__device__ __forceinline__ void schur_pair(const EU &eu, const EUE &eue, const EW &ew, T (&acc)[5][9]) {
    // m = G_u G_w^T (2 x 2)
    T m[2][2];
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2)
            m[a2][b2] = fma(eu(18 + 3 * a2 + 2), ew(18 + 3 * b2 + 2),
                            fma(eu(18 + 3 * a2 + 1), ew(18 + 3 * b2 + 1), eu(18 + 3 * a2) * ew(18 + 3 * b2)));
    // rows e of J_c,u^T m, then one column of J_c,w at a time
    T p0[5], p1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const T je0 = eue(i), je1 = eue(9 + i);
        p0[i] = fma(je1, m[1][0], je0 * m[0][0]);
        p1[i] = fma(je1, m[1][1], je0 * m[0][1]);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const T j0 = ew(k), j1 = ew(9 + k);
#pragma unroll
        for (int i = 0; i < 5; ++i) acc[i][k] = fma(p1[i], j1, fma(p0[i], j0, acc[i][k]));
    }
}

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_schur(SchurChunks ch, const int2 *__restrict__ blk_key,
                                               const int64_t *__restrict__ blk_start,
                                               const uint64_t *__restrict__ pairs,
                                               const int32_t *__restrict__ cam_cluster, int32_t l,
                                               const int32_t *__restrict__ cam_local,
                                               const int32_t *__restrict__ cl_Np, const int64_t *__restrict__ S_off,
                                               const int32_t *__restrict__ seg_head, const T *__restrict__ Jc,
                                               const T *__restrict__ obsd, Damp dm,
                                               double *__restrict__ S, double *__restrict__ b) {
    using Sh = SchurShape<T>;
    constexpr int kOffB = sizeof(T) == 8 ? Sh::kOff64Bytes : Sh::kDmaBytes;
    constexpr int kBuf = kOffB > Sh::kDBytes ? kOffB : Sh::kDBytes;
    __shared__ int2 s_pairs[4][Sh::kStage];
    __shared__ __align__(16) char s_rec[4][kBuf];
    const int wv = threadIdx.x >> 6;
    int2 *sp = s_pairs[wv];
    char *sb = s_rec[wv];
    const int64_t nc = ch.n_chunks[0];
    // Workgroups go to the 8 XCDs in turn (block b to XCD b mod 8), and each XCD
    // has its own L2.  XCD x takes the contiguous eighth [x nc / 8, (x + 1) nc / 8)
    // of the items (chunks in camera-pair order), so the blocks of one camera row,
    // which read that camera's records again, run on one XCD at about the same time.
    const unsigned x = blockIdx.x & 7u;
    const int64_t nwg_x = ((int64_t)gridDim.x - (int64_t)x + 7) / 8;   // workgroups on XCD x
    const int64_t lo = (int64_t)x * nc / 8, hi = ((int64_t)x + 1) * nc / 8;
    const int64_t wstride = nwg_x * 4;
    for (int64_t item = lo + (int64_t)(blockIdx.x >> 3) * 4 + wv; item < hi; item += wstride) {
        const int32_t bk = ch.chunk_blk[item];
        const int2 key = blk_key[bk];
        const int32_t r = key.x, c = key.y;
        const int32_t kr = cam_cluster[r];
        if (kr < 0 || kr >= l || cam_cluster[c] != kr) continue;
        const int64_t Np = cl_Np[kr];
        if (Np == 0) continue;   // the map was rejected by the cluster layout
        const double lam = dm.at_cam(r)[0];
        const int64_t c0 = ch.blk_chunk_off[bk];
        const int64_t nch = ch.blk_chunk_off[bk + 1] - c0;
        const int64_t s0 = blk_start[bk] + (item - c0) * kSchurChunk;
        const int32_t len = (int32_t)min((int64_t)kSchurChunk, blk_start[bk + 1] - s0);   // >= 1
        const bool diag = r == c;
        // an opaque copy of the lane index per item: the lane-dependent addresses of
        // the two paths below are derived inside them instead of being hoisted out
        // of the item loop, where both sets would hold registers at once
        int lane = threadIdx.x & 63;
        asm volatile("" : "+v"(lane));
        const int slot = lane >> 1;
        // rows e0..e0 + 4: 0..4 and 4..8 (row 4 of the upper half is dropped), so
        // both halves start on a whole 16-byte part of a record
        const int e0 = 4 * (lane & 1);
        const int i0 = lane & 1;   // first row a half writes
        T acc[5][9], du[5], rb[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            du[i] = rb[i] = (T)0;
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[i][k] = (T)0;
        }
        for (int h0 = 0; h0 < len; h0 += Sh::kStage) {
            // the pairs of one segment among the next kStage, in pair order,
            // compacted into LDS (the others fill the tail in reverse); all pair
            // entries, then all segment heads, are requested before any is used
            const int hl = min(Sh::kStage, len - h0);
            constexpr int kRounds = Sh::kStage / 64;
            uint64_t pr[kRounds];
#pragma unroll
            for (int i = 0; i < kRounds; ++i) pr[i] = pairs[s0 + h0 + min(i * 64 + lane, hl - 1)];
            int32_t hu[kRounds], hw[kRounds];
#pragma unroll
            for (int i = 0; i < kRounds; ++i) hu[i] = hw[i] = 0;
            if (!diag && !ch.all_links) {
#pragma unroll
                for (int i = 0; i < kRounds; ++i) {
                    hu[i] = seg_head[(int64_t)(pr[i] >> 32)];
                    hw[i] = seg_head[(int64_t)(pr[i] & 0xFFFFFFFFull)];
                }
            }
            __builtin_amdgcn_wave_barrier();   // earlier reads of sp are done
            int32_t npv = 0, nskip = 0;
#pragma unroll
            for (int i = 0; i < kRounds; ++i) {
                const bool ok = i * 64 + lane < hl && hu[i] == hw[i];
                const uint64_t mask = __ballot(ok);
                const uint64_t mk = ok ? mask : ~mask;
                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                const int pos = ok ? npv + rank : Sh::kStage - 1 - (nskip + rank);
                sp[pos] = make_int2((int32_t)(pr[i] >> 32), (int32_t)(pr[i] & 0xFFFFFFFFull));
                npv += __popcll(mask);
                nskip += 64 - __popcll(mask);
            }
            __builtin_amdgcn_wave_barrier();
            const int nbat = (npv + 31) >> 5;
            int pl = lane;   // again opaque: nothing of a path is hoisted out of the stage loop
            asm volatile("" : "+v"(pl));
            if (diag) {
                // pairs (a, a): J_c^T M J_c, diag(J_c^T J_c), J_c^T r
                const int dq = pl / Sh::kLanesRec, dp = min(pl % Sh::kLanesRec, Sh::kDiagParts - 1);
                auto fetch = [&](int bt) {
                    if constexpr (sizeof(T) == 8) {
                        // the grouped layout, one side: J_c (parts 0..8), then M and r
                        // (parts 4..6 of the assembly record) as parts 9..11; all slots of
                        // sp hold pairs of this item
                        int ln = pl;
                        asm volatile("" : "+v"(ln));
                        const int jh = ln & 1, jr = ln >> 1;
                        const uint32_t o = (uint32_t)reinterpret_cast<const int *>(sp)[2 * (bt * 32 + jr)];
                        const char *a = reinterpret_cast<const char *>(Jc) + (uint64_t)o * 144u + 16 * jh;
                        const char *g = reinterpret_cast<const char *>(obsd) + (uint64_t)o * 128u;
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            __builtin_amdgcn_global_load_lds((const void *)(a + 32 * t),
                                                             (void __attribute__((address_space(3))) *)(sb + t * Sh::kGS),
                                                             16, 0, 0);
                        __builtin_amdgcn_global_load_lds((const void *)(jh ? g + 64 : a + 128),
                                                         (void __attribute__((address_space(3))) *)(sb + 4 * Sh::kGS),
                                                         16, 0, 0);
                        __builtin_amdgcn_global_load_lds((const void *)(g + 80 + 16 * jh),
                                                         (void __attribute__((address_space(3))) *)(sb + 5 * Sh::kGS),
                                                         16, 0, 0);
                    } else {
                        int64_t a[Sh::kDLoads];
#pragma unroll
                        for (int i = 0; i < Sh::kDLoads; ++i) a[i] = sp[min(bt * 32 + dq * Sh::kNI + i, npv - 1)].x;
#pragma unroll
                        for (int i = 0; i < Sh::kDLoads; ++i)
                            __builtin_amdgcn_global_load_lds((const void *)Sh::src(Jc, obsd, a[i], dp),
                                                             (void __attribute__((address_space(3))) *)(sb + i * Sh::kBlk),
                                                             16, 0, 0);
                    }
                };
                // element k of the lane's record, and of its J_c moved on to row e0
                auto eoff = [](int k) { return sizeof(T) == 8 ? Sh::off64(k) : Sh::elem_at(k); };
                const char *dd = sizeof(T) == 8 ? sb + 32 * (pl >> 1) : sb + Sh::row_at(pl >> 1);
                const char *de = sizeof(T) == 8 ? dd + (e0 / 4) * Sh::kGS : dd + Sh::elem_at(e0);
                auto d = [&](int k) -> T { return *reinterpret_cast<const T *>(dd + eoff(k)); };
                auto dr = [&](int k) -> T { return *reinterpret_cast<const T *>(de + eoff(k)); };
                for (int bt = 0; bt < nbat; ++bt) {
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the previous batch has been read
                    asm volatile("" ::: "memory");
                    fetch(bt);
                    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the batch is in LDS
                    asm volatile("" ::"v"(sb) : "memory");
                    if (bt * 32 + slot < npv) {
                        const T m00 = d(24), m01 = d(25), m11 = d(26), r0 = d(27), r1 = d(28);
                        // rows e of J_c^T M, then one column of J_c at a time
                        T p0[5], p1[5];
#pragma unroll
                        for (int i = 0; i < 5; ++i) {
                            const T je0 = dr(i), je1 = dr(9 + i);
                            p0[i] = fma(je1, m01, je0 * m00);
                            p1[i] = fma(je1, m11, je0 * m01);
                            du[i] = fma(je1, je1, fma(je0, je0, du[i]));
                            rb[i] = fma(je1, r1, fma(je0, r0, rb[i]));
                        }
#pragma unroll
                        for (int k = 0; k < 9; ++k) {
                            const T j0 = d(k), j1 = d(9 + k);
#pragma unroll
                            for (int i = 0; i < 5; ++i) acc[i][k] = fma(p1[i], j1, fma(p0[i], j0, acc[i][k]));
                        }
                    }
                }
            } else if constexpr (sizeof(T) == 8) {
                // off-diagonal pairs (u, w), FP64: S_rc -= J_c,u^T (G_u G_w^T) J_c,w as
                // below, batches in the grouped layout.  Every slot of sp holds a pair
                // of this item (the compaction writes all kStage of them), so the
                // records of slots past npv are valid ones that no lane uses.
                const int *spi = reinterpret_cast<const int *>(sp);
                auto fetch = [&](int bt) {
                    // lane (slot jr, part jh of each group); an opaque copy of the lane
                    // index, so that nothing of it is held across batches
                    int ln = pl;
                    asm volatile("" : "+v"(ln));
                    const int jh = ln & 1, jr = ln >> 1;
                    uint32_t o[2];
#pragma unroll
                    for (int b2 = 0; b2 < 2; ++b2) o[b2] = (uint32_t)spi[2 * (bt * 32 + jr) + b2];
#pragma unroll
                    for (int b2 = 0; b2 < 2; ++b2) {
                        const char *a = reinterpret_cast<const char *>(Jc) + (uint64_t)o[b2] * 144u + 16 * jh;
                        const char *g = reinterpret_cast<const char *>(obsd) + (uint64_t)o[b2] * 128u;
                        char *dst = sb + 1024 * b2;
#pragma unroll
                        for (int t = 0; t < 4; ++t)   // parts 0..7 of J_c
                            __builtin_amdgcn_global_load_lds((const void *)(a + 32 * t),
                                                             (void __attribute__((address_space(3))) *)(dst + t * Sh::kGS),
                                                             16, 0, 0);
                        // part 8 (the last of J_c) and part 9 (the first of G), then G's 10, 11
                        __builtin_amdgcn_global_load_lds((const void *)(jh ? g : a + 128),
                                                         (void __attribute__((address_space(3))) *)(dst + 4 * Sh::kGS),
                                                         16, 0, 0);
                        __builtin_amdgcn_global_load_lds((const void *)(g + 16 + 16 * jh),
                                                         (void __attribute__((address_space(3))) *)(dst + 5 * Sh::kGS),
                                                         16, 0, 0);
                    }
                };
                const char *ju = sb + 32 * (pl >> 1), *jw = sb + 32 * (32 + (pl >> 1));
                const char *jue = ju + (e0 / 4) * Sh::kGS;   // rows e0.. of J_c,u: 4 elements on
                auto eu = [&](int k) -> T { return *reinterpret_cast<const T *>(ju + Sh::off64(k)); };
                auto eue = [&](int k) -> T { return *reinterpret_cast<const T *>(jue + Sh::off64(k)); };
                auto ew = [&](int k) -> T { return *reinterpret_cast<const T *>(jw + Sh::off64(k)); };
                for (int bt = 0; bt < nbat; ++bt) {
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the previous batch has been read
                    asm volatile("" ::: "memory");
                    fetch(bt);
                    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the batch is in LDS
                    asm volatile("" ::"v"(sb) : "memory");
                    if (bt * 32 + slot < npv) schur_pair(eu, eue, ew, acc);
                }
            } else {
                // off-diagonal pairs (u, w): S_rc -= Y_u Y_w^T = J_c,u^T (G_u G_w^T) J_c,w.
                // Records 0..31 of a batch are the u, 32..63 the w.
                const int yr = pl / Sh::kLanesRec, yp = pl % Sh::kLanesRec;
                const bool ypart = yp < Sh::kOffParts;   // the lanes of M and r move nothing
                auto fetch = [&](int bt) {
                    // every record index first, then the loads
                    int64_t o[Sh::kLoads];
#pragma unroll
                    for (int i = 0; i < Sh::kNI; ++i) {
                        const int2 uw = sp[min(bt * 32 + yr * Sh::kNI + i, npv - 1)];
                        o[i] = uw.x;
                        o[Sh::kNI + i] = uw.y;
                    }
#pragma unroll
                    for (int i = 0; i < Sh::kLoads; ++i)
                        if (ypart)
                            __builtin_amdgcn_global_load_lds((const void *)Sh::src(Jc, obsd, o[i], yp),
                                                             (void __attribute__((address_space(3))) *)(sb + i * Sh::kBlk),
                                                             16, 0, 0);
                };
                const char *ru = sb + Sh::row_at(pl >> 1);
                const char *rue = ru + Sh::elem_at(e0);   // J_c,u from row e0 (a whole number of parts)
                const char *rw = sb + Sh::row_at(32 + (pl >> 1));
                auto eu = [&](int k) -> T { return *reinterpret_cast<const T *>(ru + Sh::elem_at(k)); };
                auto eue = [&](int k) -> T { return *reinterpret_cast<const T *>(rue + Sh::elem_at(k)); };
                auto ew = [&](int k) -> T { return *reinterpret_cast<const T *>(rw + Sh::elem_at(k)); };
                for (int bt = 0; bt < nbat; ++bt) {
                    // the previous batch has been read before the next one lands
                    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
                    asm volatile("" ::: "memory");
                    fetch(bt);
                    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the batch is in LDS
                    asm volatile("" ::"v"(sb) : "memory");
                    if (bt * 32 + slot < npv) schur_pair(eu, eue, ew, acc);
                }
            }
        }
        schur_butterfly<T>(acc, du, rb, diag);
        // slot k < 9 of each half holds column k of its rows
        T col[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            col[i] = acc[i][0];
#pragma unroll
            for (int k = 1; k < 9; ++k)
                if (slot == k) col[i] = acc[i][k];
        }
        if (slot >= 9) continue;
        if (nch == 1) {
            const int64_t at0 = S_off[kr] + 9 * (int64_t)cam_local[r] + (9 * (int64_t)cam_local[c] + slot) * Np;
            double *colp = S + at0;
            for (int i = i0; i < 5; ++i) {
                const int e = e0 + i;
                double v = (double)col[i];
                if (diag) {
                    if (e == slot) v += lam * (double)du[i];
                } else {
                    v = -v;
                }
                colp[e] = v;
            }
            if (diag && slot == 0)
                for (int i = i0; i < 5; ++i) b[9 * (int64_t)r + e0 + i] = -(double)rb[i];
        } else {
            double *mine = ch.part + item * kSchurPart;
            for (int i = i0; i < 5; ++i) mine[9 * (e0 + i) + slot] = (double)col[i];
            if (diag && slot == 0)
                for (int i = i0; i < 5; ++i) {
                    mine[81 + e0 + i] = (double)du[i];
                    mine[90 + e0 + i] = (double)rb[i];
                }
        }
    }
}

// Blocks of several chunks: 81 threads per block add the partial sums in chunk
// order and write the block (and b_r for a diagonal block).  The same grid puts
// ones on the diagonal of the padded tail of every S_k (rows 9 n_k .. Np - 1).
__global__ __launch_bounds__(128) void k_schur_reduce(SchurChunks ch, const int64_t *__restrict__ n_blocks_p,
                                                      const int2 *__restrict__ blk_key,
                                                      const int32_t *__restrict__ cam_cluster, int32_t l,
                                                      const int32_t *__restrict__ cam_local,
                                                      const int32_t *__restrict__ cl_n,
                                                      const int32_t *__restrict__ cl_Np,
                                                      const int64_t *__restrict__ S_off,
                                                      Damp dm, double *__restrict__ S,
                                                      double *__restrict__ b) {
    const int64_t nb = n_blocks_p[0];
    const int t = threadIdx.x;
    for (int32_t k = blockIdx.x; k < l; k += gridDim.x) {
        const int64_t Np = cl_Np[k];
        double *A = S + S_off[k];
        for (int64_t i = 9 * (int64_t)cl_n[k] + t; i < Np; i += blockDim.x) A[i + i * Np] = 1.0;
    }
    for (int64_t bk = blockIdx.x; bk < nb; bk += gridDim.x) {
        const int64_t c0 = ch.blk_chunk_off[bk];
        const int64_t nch = ch.blk_chunk_off[bk + 1] - c0;
        if (nch < 2) continue;
        const int2 key = blk_key[bk];
        const int32_t r = key.x, c = key.y;
        const int32_t kr = cam_cluster[r];
        if (kr < 0 || kr >= l || cam_cluster[c] != kr) continue;
        const int64_t Np = cl_Np[kr];
        if (Np == 0) continue;
        const bool diag = r == c;
        if (t >= 90 || (!diag && t >= 81)) continue;
        const double lam = dm.at_cam(r)[0];
        const double *q = ch.part + c0 * kSchurPart;
        if (t < 81) {
            const int e = t / 9, k = t - 9 * (t / 9);
            double v = 0.0, dv = 0.0;
            for (int64_t j = 0; j < nch; ++j) v += q[j * kSchurPart + t];
            if (diag && e == k) {
                for (int64_t j = 0; j < nch; ++j) dv += q[j * kSchurPart + 81 + e];
                v += lam * dv;
            }
            const int64_t at0 = S_off[kr] + 9 * cam_local[r] + e + (9 * (int64_t)cam_local[c] + k) * Np;
            S[at0] = diag ? v : -v;
        } else {
            const int e = t - 81;
            double v = 0.0;
            for (int64_t j = 0; j < nch; ++j) v += q[j * kSchurPart + 90 + e];
            b[9 * (int64_t)r + e] = -v;
        }
    }
}

// ---------------------------------------------------------------------------
// a6: point update with the physical blocks (Eq. 15):
//   dp_j = V*_j^-1 (w_j - sum_o J_p,o^T J_c,o dc_{i_o}).  One thread per point.
// ---------------------------------------------------------------------------
// kFp64J: J_c, J_p formed in FP64 at x (X: cam, pt, uv, huber) instead of
// read from Jc / Jp.
struct AtX {
    const double *cam, *pt, *uv;
    double huber;
};

template <typename T, bool kFp64J>
__global__ __launch_bounds__(256) void k_backsub(int32_t n, const int64_t *__restrict__ pt_off,
                                                 const int32_t *__restrict__ obs_cam, const T *__restrict__ Jc,
                                                 const T *__restrict__ Jp, const double *__restrict__ Vinv,
                                                 const double *__restrict__ wph, const double *__restrict__ dcam,
                                                 double *__restrict__ dpt, AtX X) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double g[3] = {wph[3 * j], wph[3 * j + 1], wph[3 * j + 2]};
    for (int64_t o = pt_off[j]; o < pt_off[j + 1]; ++o) {
        const double *dc = dcam + 9 * (int64_t)obs_cam[o];
        double jc[18], jp[6];
        if (kFp64J) {
            double f[2];
            obs_fj64(X.cam, X.pt, X.uv, X.huber, obs_cam[o], (int32_t)j, o, f, jc, jp);
        } else {
#pragma unroll
            for (int k = 0; k < 18; ++k) jc[k] = (double)Jc[18 * o + k];
#pragma unroll
            for (int k = 0; k < 6; ++k) jp[k] = (double)Jp[6 * o + k];
        }
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            t0 += jc[k] * dc[k];
            t1 += jc[9 + k] * dc[k];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] -= jp[k] * t0 + jp[3 + k] * t1;
    }
    double Vi[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) Vi[k] = Vinv[6 * j + k];
    double d[3];
    sym3_mul(Vi, g, d);
#pragma unroll
    for (int k = 0; k < 3; ++k) dpt[3 * j + k] = d[k];
}

// a6 with one lane per observation, in the groups of k_points_obs (whole points,
// at most 64 observations per wavefront): lane o forms J_p,o^T (J_c,o dc) of its
// camera, and the first lane of each point subtracts its point's terms from w_j
// in observation order (the order of k_backsub), then dp_j = V*_j^-1 (w_j - ...).
template <typename T, bool kFp64J>
__global__ __launch_bounds__(64 * kPtWaves) void k_backsub_obs(int64_t ngroups, const int32_t *__restrict__ grp_first,
                                                               const int64_t *__restrict__ pt_off,
                                                               const int32_t *__restrict__ obs_pt,
                                                               const int32_t *__restrict__ obs_cam,
                                                               const T *__restrict__ Jc, const T *__restrict__ Jp,
                                                               const double *__restrict__ Vinv,
                                                               const double *__restrict__ wph,
                                                               const double *__restrict__ dcam, double *__restrict__ dpt,
                                                               AtX X) {
    __shared__ double sT[kPtWaves][3][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * kPtWaves + wv;
    if (g >= ngroups) return;
    const int32_t pa = grp_first[g];
    int32_t pb = grp_first[g + 1];
    if (pb < 0) pb = grp_first[ngroups];
    if (pa < 0 || pb < pa) return;
    const int64_t o0 = pt_off[pa], o1 = pt_off[pb];
    if (o1 - o0 > 64) return;   // reported by k_points_obs
    const int cnt = (int)(o1 - o0);
    const bool act = lane < cnt;
    const int64_t a = o0 + (act ? lane : 0);
    const int32_t j = obs_pt[a];
    const int32_t cam = obs_cam[a];
    double jc[18], jp[6];
    if (kFp64J) {
        double f[2];
        obs_fj64(X.cam, X.pt, X.uv, X.huber, cam, j, a, f, jc, jp);
    } else {
#pragma unroll
        for (int k = 0; k < 18; ++k) jc[k] = (double)Jc[18 * a + k];
#pragma unroll
        for (int k = 0; k < 6; ++k) jp[k] = (double)Jp[6 * a + k];
    }
    const double *dc = dcam + 9 * (int64_t)cam;
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double d = dc[k];
        t0 += jc[k] * d;
        t1 += jc[9 + k] * d;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) sT[wv][k][lane] = act ? jp[k] * t0 + jp[3 + k] * t1 : 0.0;
    const int32_t jprev = __shfl(j, lane > 0 ? lane - 1 : 0, 64);
    const bool start = act && (lane == 0 || j != jprev);
    const uint64_t starts = __ballot(start);
    __syncwarp();
    if (!start) return;
    const uint64_t after = starts & (lane == 63 ? 0ull : ~((2ull << lane) - 1));
    const int last = after != 0 ? __builtin_ctzll(after) : cnt;
    double gv[3] = {wph[3 * (int64_t)j], wph[3 * (int64_t)j + 1], wph[3 * (int64_t)j + 2]};
    // (unrolled: reads in flight together, subtractions in order)
#pragma unroll 4
    for (int b = lane; b < last; ++b)
#pragma unroll
        for (int k = 0; k < 3; ++k) gv[k] -= sT[wv][k][b];
    double Vi[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) Vi[k] = Vinv[6 * (int64_t)j + k];
    double d[3];
    sym3_mul(Vi, gv, d);
#pragma unroll
    for (int k = 0; k < 3; ++k) dpt[3 * (int64_t)j + k] = d[k];
}

// Workgroups go to the 8 XCDs in turn (workgroup b to XCD b mod 8), each with
// its own L2.  Camera-major kernels with one wavefront per camera hand each XCD
// a contiguous range of cameras, so that what neighbouring cameras share (the
// points they see, those points' observations) is read through one L2:
// wavefront w of workgroup b (4 per workgroup, nb workgroups, nb a multiple of
// 8) takes camera 4 ((b mod 8) nb / 8 + b / 8) + w.
__device__ inline int64_t xcd_contiguous_item(unsigned b, unsigned nb, int w) {
    const unsigned per = nb >> 3;
    return 4 * ((int64_t)(b & 7u) * per + (b >> 3)) + w;
}
inline unsigned xcd_contiguous_grid(int64_t m) { return (grid_for(m, 4) + 7u) & ~7u; }

// The same hand-out for a count known only on the device: XCD x takes items
// [x per, (x + 1) per), per = ceil(count / 8), wavefront w of workgroup b the
// item x per + 4 (b / 8) + w; -1 past the count.  The grid is sized for a
// bound on the count (xcd_contiguous_grid(bound)).
__device__ inline int64_t xcd_split_item(unsigned b, int w, int64_t count) {
    const int64_t per = (count + 7) / 8;
    const int64_t u = 4 * (int64_t)(b >> 3) + w;
    const int64_t it = (int64_t)(b & 7u) * per + u;
    return (u < per && it < count) ? it : -1;
}

// Part `it` of the camera sums: its camera r, the pair range [p0, p1) of
// camera r's diagonal block it covers (empty for a camera without one), and
// the same entries' range [d0, d1) of the camera-major (observation, point)
// list (at most q entries; with obs_off null, left empty).
struct VjpPart {
    int64_t r, p0, p1, d0, d1;
    bool alone;   // the camera's only part
};
__device__ inline VjpPart vjp_part(int64_t it, const int64_t *part_off, const int32_t *part_cam,
                                   const int64_t *diag_blk, const int64_t *blk_start, const int64_t *obs_off,
                                   int64_t q_obs) {
    VjpPart q;
    q.r = part_cam[it];
    const int64_t first = part_off[q.r];
    q.alone = part_off[q.r + 1] - first == 1;
    const int64_t kb = diag_blk[q.r];
    q.p0 = q.p1 = q.d0 = q.d1 = 0;
    if (kb >= 0) {
        const int64_t end = blk_start[kb + 1];
        q.p0 = blk_start[kb] + (it - first) * kVjpPart;
        q.p1 = q.p0 + kVjpPart < end ? q.p0 + kVjpPart : end;
        if (obs_off != nullptr) {
            q.d0 = obs_off[q.r] + (q.p0 - blk_start[kb]);
            q.d1 = q.d0 + (q.p1 - q.p0);
            if (q.d1 > q_obs) q.d1 = q_obs;
            if (q.d0 > q.d1) q.d0 = q.d1;
        }
    }
    return q;
}


// ---------------------------------------------------------------------------
// MIXED: the residual of one FP64 refinement step of every cluster solve
// (Eq. 13), r = b - S x with the S and b of the FP64 method, taken from J
// recomputed in FP64 at x and never from the FP32-assembled S.  With the
// virtual-point blocks C_s = V_s + lambda diag(V_s), the point gradient w'_s
// (corrected when lambda >= lambda_corr, Sec. 4.3), B = U + lambda diag(U) and
// E the camera / virtual-point coupling (Eq. 10),
//   b - S x = (v - B x) - E C^-1 (w' - E^T x) = J_c^T e - lambda diag(U) x,
//   y_s = C_s^-1 (w'_s - sum_{o in s} J_p,o^T J_c,o x_{i_o}),
//   e_o = -(f_o + J_c,o x_{i_o} + J_p,o y_{s_o}),
// i.e. e is the linearised residual of the step with every virtual point at
// its own optimum y.  Part 1 (per point, segments from seg_head): y_s and e_o;
// the point's first lane also writes the FP64 V*_j^-1 and w_j that the point
// update (Eq. 15) then uses.  Part 2 (one wavefront per camera over the
// camera's observations, fixed order): r_i.
// ---------------------------------------------------------------------------
__device__ inline void refine_contrib(const double f[2], const double jc[18], const double jp[6], const double *dc,
                                      double &t0, double &t1, double cv[12]) {
    t0 = 0.0;
    t1 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        t0 += jc[k] * dc[k];
        t1 += jc[9 + k] * dc[k];
    }
    cv[0] = jp[0] * jp[0] + jp[3] * jp[3];
    cv[1] = jp[0] * jp[1] + jp[3] * jp[4];
    cv[2] = jp[0] * jp[2] + jp[3] * jp[5];
    cv[3] = jp[1] * jp[1] + jp[4] * jp[4];
    cv[4] = jp[1] * jp[2] + jp[4] * jp[5];
    cv[5] = jp[2] * jp[2] + jp[5] * jp[5];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cv[6 + k] = -(jp[k] * f[0] + jp[3 + k] * f[1]);   // -J_p^T f
        cv[9 + k] = jp[k] * t0 + jp[3 + k] * t1;          // J_p^T J_c x
    }
}

// y_s from the segment sums (Vs, ws, zs) and, for the correction, the point's (V, w)
__device__ inline void refine_segment_step(const double V[6], const double w[3], const double Vs[6],
                                           const double ws_in[3], const double zs[3], double lam, bool corr,
                                           double y[3]) {
    double ws[3] = {ws_in[0], ws_in[1], ws_in[2]};
    if (corr) {
        ws[0] = Vs[0] * w[0] / V[0];
        ws[1] = Vs[3] * w[1] / V[3];
        ws[2] = Vs[5] * w[2] / V[5];
    }
    const double Vd[6] = {Vs[0] * (1.0 + lam), Vs[1], Vs[2], Vs[3] * (1.0 + lam), Vs[4], Vs[5] * (1.0 + lam)};
    const Chol3 c = chol3(Vd);
    double Vi[6];
    chol3_inverse(c, Vi);
    const double g[3] = {ws[0] - zs[0], ws[1] - zs[1], ws[2] - zs[2]};
    sym3_mul(Vi, g, y);
}

__device__ inline void refine_point_blocks(const double V[6], const double w[3], double lam, double *Vinv_j,
                                           double *wph_j) {
    const double Vd[6] = {V[0] * (1.0 + lam), V[1], V[2], V[3] * (1.0 + lam), V[4], V[5] * (1.0 + lam)};
    const Chol3 c = chol3(Vd);
    double Vi[6];
    chol3_inverse(c, Vi);
#pragma unroll
    for (int k = 0; k < 6; ++k) Vinv_j[k] = Vi[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) wph_j[k] = w[k];
}

__device__ inline void refine_write_e(const double f[2], double t0, double t1, const double jp[6], const double y[3],
                                      double *e_o) {
    e_o[0] = -(f[0] + t0 + (jp[0] * y[0] + jp[1] * y[1] + jp[2] * y[2]));
    e_o[1] = -(f[1] + t1 + (jp[3] * y[0] + jp[4] * y[1] + jp[5] * y[2]));
}

// Part 1, one lane per observation in the groups of k_points_obs.
__global__ __launch_bounds__(64 * kPtWaves) void k_refine_obs(
    int64_t ngroups, const int32_t *__restrict__ grp_first, const int64_t *__restrict__ pt_off,
    const int32_t *__restrict__ obs_pt, const int32_t *__restrict__ obs_cam, const double *__restrict__ cam,
    const double *__restrict__ pt, const double *__restrict__ uv, double huber, const int32_t *__restrict__ seg_head,
    Damp dm, const double *__restrict__ dcam, double *__restrict__ e,
    double *__restrict__ Vinv, double *__restrict__ wph) {
    __shared__ double sV[kPtWaves][12][64];
    __shared__ int32_t sHead[kPtWaves][64];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * kPtWaves + wv;
    if (g >= ngroups) return;
    const int32_t pa = grp_first[g];
    int32_t pb = grp_first[g + 1];
    if (pb < 0) pb = grp_first[ngroups];
    if (pa < 0 || pb <= pa) return;
    const int64_t o0 = pt_off[pa], o1 = pt_off[pb];
    if (o1 - o0 > 64 || o1 <= o0) return;   // reported by k_points_obs
    const int cnt = (int)(o1 - o0);
    const bool act = lane < cnt;
    const int64_t a = o0 + (act ? lane : 0);
    const int32_t j = obs_pt[a];
    const int32_t ci = obs_cam[a];
    double f[2], jc[18], jp[6];
    obs_fj64(cam, pt, uv, huber, ci, j, a, f, jc, jp);
    double t0, t1, cv[12];
    refine_contrib(f, jc, jp, dcam + 9 * (int64_t)ci, t0, t1, cv);
#pragma unroll
    for (int k = 0; k < 12; ++k) sV[wv][k][lane] = act ? cv[k] : 0.0;
    // the segment's head is its first observation, in this point and so in this group
    int head = act ? (int)(seg_head[a] - o0) : lane;
    if (head < 0 || head > lane) head = lane;
    sHead[wv][lane] = head;
    const int32_t jprev = __shfl(j, lane > 0 ? lane - 1 : 0, 64);
    const uint64_t starts = __ballot(act && (lane == 0 || j != jprev));
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    const uint64_t after = starts & ~upto & (cnt >= 64 ? ~0ull : ((1ull << cnt) - 1));
    const int first = act ? 63 - __builtin_clzll(starts & upto) : lane;
    const int last = act ? (after != 0 ? __builtin_ctzll(after) : cnt) : lane + 1;
    __syncwarp();
    // point sums (V_j, w_j) and segment sums in observation order
    double V[6] = {0, 0, 0, 0, 0, 0}, w[3] = {0, 0, 0}, Vs[6] = {0, 0, 0, 0, 0, 0}, ws[3] = {0, 0, 0},
           zs[3] = {0, 0, 0};
    for (int b = first; b < last; ++b) {
        const bool mine = sHead[wv][b] == head;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double x = sV[wv][k][b];
            V[k] += x;
            if (mine) Vs[k] += x;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double x = sV[wv][6 + k][b];
            w[k] += x;
            if (mine) {
                ws[k] += x;
                zs[k] += sV[wv][9 + k][b];
            }
        }
    }
    if (!act) return;
    const double *lp = dm.at_pt(j);
    const double lam = lp[0];
    const bool corr = lam >= lp[1];
    if (lane == first) refine_point_blocks(V, w, lam, Vinv + 6 * (int64_t)j, wph + 3 * (int64_t)j);
    double y[3];
    refine_segment_step(V, w, Vs, ws, zs, lam, corr, y);
    refine_write_e(f, t0, t1, jp, y, e + 2 * a);
}

// Part 1, one thread per point (points too long for the groups); J recomputed
// on each pass over the point's observations.
__global__ __launch_bounds__(64) void k_refine_pt(int32_t n, const int64_t *__restrict__ pt_off,
                                                  const int32_t *__restrict__ obs_cam, const double *__restrict__ cam,
                                                  const double *__restrict__ pt, const double *__restrict__ uv,
                                                  double huber, const int32_t *__restrict__ seg_head,
                                                  Damp dm, const double *__restrict__ dcam,
                                                  double *__restrict__ e, double *__restrict__ Vinv,
                                                  double *__restrict__ wph) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double *lp = dm.at_pt(j);
    const double lam = lp[0];
    const bool corr = lam >= lp[1];
    const int64_t p0 = pt_off[j], p1 = pt_off[j + 1];
    double V[6] = {0, 0, 0, 0, 0, 0}, w[3] = {0, 0, 0};
    for (int64_t a = p0; a < p1; ++a) {
        double f[2], jc[18], jp[6], t0, t1, cv[12];
        const int32_t ci = obs_cam[a];
        obs_fj64(cam, pt, uv, huber, ci, (int32_t)j, a, f, jc, jp);
        refine_contrib(f, jc, jp, dcam + 9 * (int64_t)ci, t0, t1, cv);
#pragma unroll
        for (int k = 0; k < 6; ++k) V[k] += cv[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) w[k] += cv[6 + k];
    }
    refine_point_blocks(V, w, lam, Vinv + 6 * j, wph + 3 * j);
    for (int64_t h = p0; h < p1; ++h) {
        if (seg_head[h] != (int32_t)h) continue;
        double Vs[6] = {0, 0, 0, 0, 0, 0}, ws[3] = {0, 0, 0}, zs[3] = {0, 0, 0};
        for (int64_t a = h; a < p1; ++a) {
            if (seg_head[a] != (int32_t)h) continue;
            double f[2], jc[18], jp[6], t0, t1, cv[12];
            const int32_t ci = obs_cam[a];
            obs_fj64(cam, pt, uv, huber, ci, (int32_t)j, a, f, jc, jp);
            refine_contrib(f, jc, jp, dcam + 9 * (int64_t)ci, t0, t1, cv);
#pragma unroll
            for (int k = 0; k < 6; ++k) Vs[k] += cv[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ws[k] += cv[6 + k];
                zs[k] += cv[9 + k];
            }
        }
        double y[3];
        refine_segment_step(V, w, Vs, ws, zs, lam, corr, y);
        for (int64_t a = h; a < p1; ++a) {
            if (seg_head[a] != (int32_t)h) continue;
            double f[2], jc[18], jp[6], t0, t1, cv[12];
            const int32_t ci = obs_cam[a];
            obs_fj64(cam, pt, uv, huber, ci, (int32_t)j, a, f, jc, jp);
            refine_contrib(f, jc, jp, dcam + 9 * (int64_t)ci, t0, t1, cv);
            refine_write_e(f, t0, t1, jp, y, e + 2 * a);
        }
    }
}

// Part 2: r_i = sum_{o of camera i} J_c,o^T e_o - lambda diag(U_i) x_i, U_i =
// sum J_c,o^T J_c,o, over camera i's observations (its diagonal block's list)
// in the parts of the J^T v camera sums: one wavefront per part, the parts
// spread evenly over the XCDs, the camera's part of the projection formed
// once per wavefront and kept in LDS, the camera-major (observation, point)
// entries read two rounds ahead and the point, pixel and e gathers one round
// ahead; a fixed-order butterfly per part, a camera of one part writes r_i,
// the parts of the others are added in part order by k_refine_cam_sum.
__device__ inline void refine_cam_round(const double cp[kCamPre], const double X[3], double u0, double u1, double e0,
                                        double e1, double on, double huber, double (&acc)[9], double (&dg)[9]) {
    // obs_fj64's operations on the gathered values
    double pix[2], a[2][9], b[2][3];
    project_jac_pre(cp, X, pix, a, b);
    const double f0 = pix[0] - u0, f1 = pix[1] - u1;
    const double rw = huber_root_weight(f0 * f0 + f1 * f1, huber);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double j0 = rw * a[0][k], j1 = rw * a[1][k];
        acc[k] += j0 * e0 + j1 * e1;
        dg[k] += on * (j0 * j0 + j1 * j1);   // on = 0 for a lane past the part's end
    }
}

struct RefineRound {
    double X[3], u0, u1, e0, e1, on;
};
__device__ inline void refine_gather(int2 en, bool on, const double *__restrict__ pt, const double *__restrict__ uv,
                                     const double *__restrict__ e, RefineRound &g) {
    const int64_t o = en.x, j = en.y;
    g.X[0] = pt[3 * j];
    g.X[1] = pt[3 * j + 1];
    g.X[2] = pt[3 * j + 2];
    g.u0 = uv[2 * o];
    g.u1 = uv[2 * o + 1];
    g.e0 = on ? e[2 * o] : 0.0;   // a lane past the part's end adds zero
    g.e1 = on ? e[2 * o + 1] : 0.0;
    g.on = on ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void k_refine_cam(int32_t m, int64_t q_obs, const int64_t *__restrict__ part_off,
                                                    const int32_t *__restrict__ part_cam,
                                                    const int64_t *__restrict__ obs_off, const int2 *__restrict__ oj,
                                                    const double *__restrict__ cam, const double *__restrict__ pt,
                                                    const double *__restrict__ uv, double huber,
                                                    const int64_t *__restrict__ diag_blk,
                                                    const int64_t *__restrict__ blk_start, Damp dm,
                                                    const double *__restrict__ dcam, const double *__restrict__ e,
                                                    double *__restrict__ part_sum, double *__restrict__ r) {
    __shared__ double cps[4][kCamPre];
    const int lane = threadIdx.x & 63;
    const int64_t it = xcd_split_item(blockIdx.x, threadIdx.x >> 6, part_off[m]);
    if (it < 0) return;
    const VjpPart q = vjp_part(it, part_off, part_cam, diag_blk, blk_start, obs_off, q_obs);
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (q.d0 < q.d1) {
        double *cp = cps[threadIdx.x >> 6];
        {
            double c[9], cr[kCamPre];
#pragma unroll
            for (int k = 0; k < 9; ++k) c[k] = cam[9 * q.r + k];
            camera_pre(c, cr);
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < kCamPre; ++k) cp[k] = cr[k];
            }
            __syncwarp();
        }
        const int rounds = (int)((q.d1 - q.d0 + 63) / 64);
        auto entry = [&](int t) {
            const int64_t d = q.d0 + 64 * (int64_t)t + lane;
            return oj[d < q.d1 ? d : q.d0];
        };
        int2 e1 = rounds > 1 ? entry(1) : make_int2(0, 0);
        RefineRound g;
        refine_gather(entry(0), q.d0 + lane < q.d1, pt, uv, e, g);
        for (int t = 0; t < rounds; ++t) {
            int2 e2 = t + 2 < rounds ? entry(t + 2) : e1;
            asm volatile("" ::: "memory");   // cp is read from LDS in this round
            RefineRound gn = g;
            if (t + 1 < rounds) refine_gather(e1, q.d0 + 64 * (int64_t)(t + 1) + lane < q.d1, pt, uv, e, gn);
            refine_cam_round(cp, g.X, g.u0, g.u1, g.e0, g.e1, g.on, huber, acc, dg);
            g = gn;
            e1 = e2;
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            acc[k] += __shfl_xor(acc[k], d, 64);
            dg[k] += __shfl_xor(dg[k], d, 64);
        }
    double va = 0.0, vg = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        if (lane == k) {
            va = acc[k];
            vg = dg[k];
        }
    if (lane < 9) {
        if (q.alone) {
            const double lam = dm.at_cam(q.r)[0];
            r[9 * q.r + lane] = va - lam * vg * dcam[9 * q.r + lane];
        } else {
            part_sum[18 * it + lane] = va;
            part_sum[18 * it + 9 + lane] = vg;
        }
    }
}

// r of the cameras cut in several parts: their sums in part order.
__global__ __launch_bounds__(256) void k_refine_cam_sum(int32_t m, const int64_t *__restrict__ part_off,
                                                        const double *__restrict__ part_sum, Damp dm,
                                                        const double *__restrict__ dcam, double *__restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9 * (int64_t)m) return;
    const int64_t c = i / 9, k = i % 9;
    const int64_t a = part_off[c], b = part_off[c + 1];
    if (b - a < 2) return;
    double sa = 0.0, sg = 0.0;
    for (int64_t u = a; u < b; ++u) {
        sa += part_sum[18 * u + k];
        sg += part_sum[18 * u + 9 + k];
    }
    const double lam = dm.at_cam(c)[0];
    r[i] = sa - lam * sg * dcam[i];
}

// a7: cost at the candidate x + dx in FP64 (block partial sums).
__global__ __launch_bounds__(256) void k_cost_at(int64_t q, const double *__restrict__ cam,
                                                 const double *__restrict__ pt, const int32_t *__restrict__ oc,
                                                 const int32_t *__restrict__ op, const double *__restrict__ uv,
                                                 const double *__restrict__ dcam, const double *__restrict__ dpt,
                                                 double *__restrict__ partials, const stba_lm_state *st,
                                                 double *__restrict__ F_ref, double huber) {
    __shared__ double sh[256];
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // F(x) as it stands before the decision (and whether it is known yet), for
    // every block of k_accept_update
    if (F_ref != nullptr && o == 0) {
        F_ref[0] = st->F;
        F_ref[1] = st->have_F ? 1.0 : 0.0;
    }
    double sq = 0.0;
    if (o < q) {
        const int64_t i = oc[o], j = op[o];
        double c[9], X[3];
#pragma unroll
        for (int k = 0; k < 9; ++k) c[k] = cam[9 * i + k] + dcam[9 * i + k];
#pragma unroll
        for (int k = 0; k < 3; ++k) X[k] = pt[3 * j + k] + dpt[3 * j + k];
        double pix[2];
        camera_project(c, X, pix);
        const double f0 = pix[0] - uv[2 * o], f1 = pix[1] - uv[2 * o + 1];
        sq = huber_rho(f0 * f0 + f1 * f1, huber);
    }
    const double s = block_sum_256(sq, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// a7: accept iff F(x + dx) < F(x), the step is finite and every S_k factorised
// (Alg. 1); lambda /= 3 (not below lambda_min) on accept, *= 3 otherwise; x += dx on accept.  Every
// block sums the per-block partials in the same fixed order and compares with
// F(x): F_ref[0] (copied by k_cost_at) once the state holds it (F_ref[1] != 0),
// else the sum of the residual kernel's partials.  So all blocks take the same
// decision while block 0 rewrites the LM state.
__global__ __launch_bounds__(256) void k_accept_update(const double *rj_partials, const double *partials,
                                                       int64_t count, const double *F_ref,
                                                       const int32_t *cl_status, int32_t l, const int32_t *status,
                                                       stba_lm_state *st, int32_t m, int32_t n, double *cam,
                                                       double *pt, const double *dcam, const double *dpt) {
    __shared__ double sh[256];
    __shared__ int bad_pd, bad_hip;
    if (threadIdx.x == 0) bad_pd = bad_hip = 0;
    __syncthreads();
    double s = strided_sum_256(partials, count);
    for (int k = threadIdx.x; k < l; k += 256) {
        const int32_t c = cl_status[k];
        if (c == STBA_EHIP) bad_hip = 1;       // a factorisation wait timed out
        else if (c != STBA_OK) bad_pd = 1;
    }
    s = block_sum_256(s, sh);   // its barriers also publish bad_pd and bad_hip
    const double Fn = s;
    const bool have_F = F_ref[1] != 0.0;
    double F0 = F_ref[0];
    if (!have_F) {
        F0 = block_sum_256(strided_sum_256(rj_partials, count), sh);
    }
    const int32_t sticky = bad_hip ? STBA_EHIP : status[kStSticky];
    const bool pd = !bad_pd && status[kStPointBad] == 0;
    const bool fin = isfinite(Fn);
    const bool valid = pd && fin && sticky == 0;
    const bool acc = valid && (Fn < F0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->F = F0;
        st->have_F = 1;
        st->F_new = Fn;
        st->accepted = acc ? 1 : 0;
        st->lambda = acc ? fmax(st->lambda / 3.0, st->lambda_min) : st->lambda * 3.0;
        if (acc) st->F = Fn;
        st->need_jac = acc ? 1 : 0;
        st->n_rcs += 1;
        st->n_accept += acc ? 1 : 0;
        st->n_jac += status[kStJacRan] ? 1 : 0;
        st->last_status = bad_hip ? STBA_EHIP : (!pd ? STBA_ENOTPD : (!fin ? STBA_ENONFINITE : sticky));
        if (st->status == 0 && sticky != 0) st->status = sticky;
    }
    if (!acc) return;
    // x += dx, four elements per thread and round with all their loads issued
    // before any store
    const int64_t nc = 9 * (int64_t)m, total = nc + 3 * (int64_t)n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < total; i0 += 4 * stride) {
        double xv[4], dv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * stride;
            xv[u] = dv[u] = 0.0;
            if (i < nc) {
                xv[u] = cam[i];
                dv[u] = dcam[i];
            } else if (i < total) {
                xv[u] = pt[i - nc];
                dv[u] = dpt[i - nc];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + u * stride;
            if (i < nc) cam[i] = xv[u] + dv[u];
            else if (i < total) pt[i - nc] = xv[u] + dv[u];
        }
    }
}

// ---------------------------------------------------------------------------
// J^T v (differentiation of the residuals): the Jacobian is recomputed.
// Cameras: one wavefront per part of a camera's observations (at most
// kVjpPart of them, in list order; the parts spread evenly over the XCDs, a
// camera's parts next to each other), the camera's part of the projection
// formed once per lane; a camera of one part writes its sum, the parts of the
// others are added in part order by k_vjp_cam_sum.  Points: one thread per
// point; observed pixels: -v (its own pass: written from the point loops the
// stores scatter and cost more than a second read of v).
// ---------------------------------------------------------------------------

// The wavefront's nine sums (every lane holds all of them after the
// butterfly) to grad_cam, or to the part's slot of part_sum.
template <typename T>
__device__ inline void vjp_part_out(double (&acc)[9], const VjpPart &q, int64_t it, double *part_sum, T *grad_cam) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] += __shfl_xor(acc[k], d, 64);
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k)
        if (lane == k) g = acc[k];
    if (lane < 9) {
        if (q.alone)
            grad_cam[9 * q.r + lane] = (T)g;
        else
            part_sum[9 * it + lane] = g;
    }
}

// The gathers of one round of k_vjp_cam: the point and the cotangent of
// entry e, the cotangent zero for a lane past the part's end.
template <typename T>
struct VjpRound {
    double X[3], v0, v1;
};
template <typename T>
__device__ inline void vjp_gather(int2 e, bool on, const double *__restrict__ pt, const T *__restrict__ v,
                                  VjpRound<T> &g) {
    const int64_t o = e.x, j = e.y;
    g.X[0] = pt[3 * j];
    g.X[1] = pt[3 * j + 1];
    g.X[2] = pt[3 * j + 2];
    g.v0 = on ? (double)v[2 * o] : 0.0;
    g.v1 = on ? (double)v[2 * o + 1] : 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_vjp_cam(int32_t m, int64_t q_obs, const int64_t *__restrict__ part_off,
                                                 const int32_t *__restrict__ part_cam,
                                                 const int64_t *__restrict__ obs_off, const int2 *__restrict__ oj,
                                                 const double *__restrict__ cam, const double *__restrict__ pt,
                                                 const int64_t *__restrict__ diag_blk,
                                                 const int64_t *__restrict__ blk_start, const T *__restrict__ v,
                                                 double *__restrict__ part_sum, T *__restrict__ grad_cam) {
    // the camera's part of the projection in LDS (read in every round, not
    // held in 48 registers: the occupancy stays at four wavefronts)
    __shared__ double cps[4][kCamPre];
    const int lane = threadIdx.x & 63;
    const int64_t it = xcd_split_item(blockIdx.x, threadIdx.x >> 6, part_off[m]);
    if (it < 0) return;
    const VjpPart q = vjp_part(it, part_off, part_cam, diag_blk, blk_start, obs_off, q_obs);
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (q.d0 < q.d1) {
        double *cp = cps[threadIdx.x >> 6];
        {
            double c[9], cr[kCamPre];
#pragma unroll
            for (int k = 0; k < 9; ++k) c[k] = cam[9 * q.r + k];
            camera_pre(c, cr);
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < kCamPre; ++k) cp[k] = cr[k];
            }
            __syncwarp();
        }
        // Rounds of 64 entries in list order, lane l taking entry d0 + 64 t + l
        // in round t.  The list entries are read two rounds ahead and the
        // gathers they address one round ahead, so a round's arithmetic runs
        // while the next round's loads are in flight.  A lane past the end
        // reads the part's first entry and adds zero.
        const int rounds = (int)((q.d1 - q.d0 + 63) / 64);
        auto entry = [&](int t) {
            const int64_t d = q.d0 + 64 * (int64_t)t + lane;
            return oj[d < q.d1 ? d : q.d0];
        };
        int2 e1 = rounds > 1 ? entry(1) : make_int2(0, 0);
        VjpRound<T> g;
        vjp_gather(entry(0), q.d0 + lane < q.d1, pt, v, g);
        for (int t = 0; t < rounds; ++t) {
            int2 e2 = t + 2 < rounds ? entry(t + 2) : e1;
            asm volatile("" ::: "memory");   // cp is read from LDS in this round
            VjpRound<T> gn = g;
            if (t + 1 < rounds) vjp_gather(e1, q.d0 + 64 * (int64_t)(t + 1) + lane < q.d1, pt, v, gn);
            double pix[2], jc[2][9], jp[2][3];
            project_jac_pre(cp, g.X, pix, jc, jp);
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[k] += jc[0][k] * g.v0 + jc[1][k] * g.v1;
            g = gn;
            e1 = e2;
        }
    }
    vjp_part_out(acc, q, it, part_sum, grad_cam);
}

// grad_cam of the cameras cut in several parts: their part sums in part order.
template <typename T>
__global__ __launch_bounds__(256) void k_vjp_cam_sum(int32_t m, const int64_t *__restrict__ part_off,
                                                     const double *__restrict__ part_sum, T *__restrict__ grad_cam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9 * (int64_t)m) return;
    const int64_t r = i / 9, k = i % 9;
    const int64_t a = part_off[r], b = part_off[r + 1];
    if (b - a < 2) return;
    double s = 0.0;
    for (int64_t u = a; u < b; ++u) s += part_sum[9 * u + k];
    grad_cam[i] = (T)s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_vjp_pt(int32_t n, int64_t q, const double *__restrict__ cam,
                                                const double *__restrict__ pt, const int32_t *__restrict__ oc,
                                                const int64_t *__restrict__ pt_off, const T *__restrict__ v,
                                                T *__restrict__ grad_pt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double X[3] = {pt[3 * j], pt[3 * j + 1], pt[3 * j + 2]};
    double acc[3] = {0, 0, 0};
    for (int64_t o = pt_off[j]; o < pt_off[j + 1]; ++o) {
        double c[9];
        const int64_t i = oc[o];
#pragma unroll
        for (int k = 0; k < 9; ++k) c[k] = cam[9 * i + k];
        double pix[2], jc[2][9], jp[2][3];
        camera_project_jac(c, X, pix, jc, jp);
        const double v0 = (double)v[2 * o], v1 = (double)v[2 * o + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += jp[0][k] * v0 + jp[1][k] * v1;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) grad_pt[3 * j + k] = (T)acc[k];
}

// J^T v from the stored blocks (J_c, J_p as the residual kernel wrote them for
// this x): the same sums as k_vjp_cam / k_vjp_pt, in the same order, with each
// block read instead of recomputed.
template <typename T>
__global__ __launch_bounds__(256) void k_vjp_cam_stored(int32_t m, const int64_t *__restrict__ part_off,
                                                        const int32_t *__restrict__ part_cam,
                                                        const int64_t *__restrict__ diag_blk,
                                                        const int64_t *__restrict__ blk_start,
                                                        const uint64_t *__restrict__ pairs, const T *__restrict__ Jc,
                                                        const T *__restrict__ v, double *__restrict__ part_sum,
                                                        T *__restrict__ grad_cam) {
    const int lane = threadIdx.x & 63;
    const int64_t it = xcd_split_item(blockIdx.x, threadIdx.x >> 6, part_off[m]);
    if (it < 0) return;
    const VjpPart q = vjp_part(it, part_off, part_cam, diag_blk, blk_start, nullptr, 0);
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t p = q.p0 + lane; p < q.p1; p += 64) {
        const int64_t o = (int64_t)(pairs[p] >> 32);
        const T *jc = Jc + 18 * o;
        const double v0 = (double)v[2 * o], v1 = (double)v[2 * o + 1];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] += (double)jc[k] * v0 + (double)jc[9 + k] * v1;
    }
    vjp_part_out(acc, q, it, part_sum, grad_cam);
}

template <typename T>
__global__ __launch_bounds__(256) void k_vjp_pt_stored(int32_t n, const int64_t *__restrict__ pt_off,
                                                       const T *__restrict__ Jp, const T *__restrict__ v,
                                                       T *__restrict__ grad_pt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double acc[3] = {0, 0, 0};
    for (int64_t o = pt_off[j]; o < pt_off[j + 1]; ++o) {
        const T *jp = Jp + 6 * o;
        const double v0 = (double)v[2 * o], v1 = (double)v[2 * o + 1];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += (double)jp[k] * v0 + (double)jp[3 + k] * v1;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) grad_pt[3 * j + k] = (T)acc[k];
}

template <typename T>
__global__ __launch_bounds__(256) void k_neg(int64_t len, const T *v, T *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) out[i] = -v[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_reset_status(int32_t *status, hipStream_t st) {
    k_reset_status<<<1, 64, 0, st>>>(status);
    return hipGetLastError();
}

hipError_t launch_lm_init(stba_lm_state *s, double lambda0, double lambda_corr, hipStream_t st) {
    k_lm_init<<<1, 1, 0, st>>>(s, lambda0, lambda_corr);
    return hipGetLastError();
}

hipError_t launch_clusters(const int32_t *cam_cluster, int32_t m, int32_t l, const int32_t *l_dev, int32_t gamma_max,
                           int32_t *cl_n, int32_t *cl_Np, int32_t *cl_start, int32_t *cl_cams, int32_t *cam_local,
                           int64_t *S_off, int32_t *cl_status, int32_t *status, hipStream_t st) {
    if (m <= 1024) {
        k_clusters_small<<<1, (unsigned)round_up(m, 64), 0, st>>>(cam_cluster, m, l, l_dev, gamma_max, cl_n, cl_Np,
                                                                  cl_start, cl_cams, cam_local, S_off, cl_status,
                                                                  status);
        return hipGetLastError();
    }
    const size_t lds = sizeof(int32_t) * 2 * (size_t)l;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_clusters_large),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k_clusters_large<<<(unsigned)((m + kClusterLargeThreads - 1) / kClusterLargeThreads), kClusterLargeThreads, lds,
                       st>>>(cam_cluster, m, l, l_dev, gamma_max, cl_n, cl_Np, cl_start, cl_cams, cam_local, S_off,
                             cl_status, status);
    return hipGetLastError();
}

int64_t rj_blocks(int64_t q) { return (q + 255) / 256; }

template <typename T>
hipError_t launch_rj(const stba_problem &p, T *f, T *Jc, T *Jp, double *partials, const int32_t *need_jac,
                     int32_t *jac_ran, const ZeroS &z, hipStream_t st) {
    if (Jc == nullptr && Jp == nullptr && z.S == nullptr && need_jac == nullptr && jac_ran == nullptr) {
        k_resid_only<T><<<grid_for(p.q), 256, 0, st>>>(p.q, p.cam, p.pt, p.obs_cam, p.obs_pt, p.obs_uv, f, partials,
                                                       p.huber);
        return hipGetLastError();
    }
    k_rj<T><<<grid_for(p.q), 256, 0, st>>>(p.q, p.cam, p.pt, p.obs_cam, p.obs_pt, p.obs_uv, f, Jc, Jp, partials,
                                           need_jac, jac_ran, z, p.huber);
    return hipGetLastError();
}
template hipError_t launch_rj<double>(const stba_problem &, double *, double *, double *, double *,
                                      const int32_t *, int32_t *, const ZeroS &, hipStream_t);
template hipError_t launch_rj<float>(const stba_problem &, float *, float *, float *, double *, const int32_t *,
                                     int32_t *, const ZeroS &, hipStream_t);

hipError_t launch_sum_partials(const double *partials, int64_t count, double *out, hipStream_t st) {
    k_sum_partials<<<1, 256, 0, st>>>(partials, count, out);
    return hipGetLastError();
}

hipError_t launch_set_damping(double *slot, double lambda, double lambda_corr, hipStream_t st) {
    k_set_damping<<<1, 1, 0, st>>>(slot, lambda, lambda_corr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_points(const stba_problem &p, const int64_t *pt_off, const int32_t *cam_cluster, int32_t l,
                         const T *f, const T *Jc, const T *Jp, const Damp &dm, uint64_t seed, uint64_t t,
                         uint64_t thr, int32_t *seg_head, double *seg_rec, T *obsd, double *Vinv, double *wph,
                         int32_t *status, int32_t group_size, const int32_t *grp_first, hipStream_t st) {
    (void)l;
    if (group_size > 0) {
        const int64_t ng = (p.q + group_size - 1) / group_size;
        k_points_obs<T><<<(unsigned)((ng + kPtWaves - 1) / kPtWaves), 64 * kPtWaves, 0, st>>>(
            ng, grp_first, pt_off, p.obs_pt, p.obs_cam, cam_cluster, f, Jc, Jp, dm, seed, t, thr, seg_head, obsd,
            Vinv, wph, status);
        return hipGetLastError();
    }
    k_points<T><<<grid_for(p.n, 64), 64, 0, st>>>(p.n, pt_off, p.obs_cam, cam_cluster, f, Jp, dm, seed, t, thr,
                                                  seg_head, seg_rec, Vinv, wph, status);
    k_obs_rec<T><<<grid_for(p.q), 256, 0, st>>>(p.q, seg_head, seg_rec, f, Jc, Jp, obsd);
    return hipGetLastError();
}
template hipError_t launch_points<double>(const stba_problem &, const int64_t *, const int32_t *, int32_t,
                                          const double *, const double *, const double *, const Damp &, uint64_t,
                                          uint64_t, uint64_t, int32_t *, double *, double *, double *, double *,
                                          int32_t *, int32_t, const int32_t *, hipStream_t);
template hipError_t launch_points<float>(const stba_problem &, const int64_t *, const int32_t *, int32_t,
                                         const float *, const float *, const float *, const Damp &, uint64_t,
                                         uint64_t, uint64_t, int32_t *, double *, float *, double *, double *,
                                         int32_t *, int32_t, const int32_t *, hipStream_t);

__global__ void k_fill_i32(int32_t *a, int64_t len, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

hipError_t launch_point_groups(int32_t n, const int64_t *pt_off, int32_t group_size, int64_t ngroups,
                               int32_t *grp_first, hipStream_t st) {
    k_fill_i32<<<grid_for(ngroups + 1), 256, 0, st>>>(grp_first, ngroups + 1, -1);
    k_point_groups<<<grid_for(n), 256, 0, st>>>(n, pt_off, group_size, ngroups, grp_first);
    return hipGetLastError();
}

hipError_t launch_fill_S(double *S, double *b, int32_t m, const int64_t *S_off, int32_t l, int64_t S_cap,
                         hipStream_t st) {
    int64_t blocks = (S_cap + 1023) / 1024;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    k_zero_S<<<(unsigned)blocks, 256, 0, st>>>(S, b, m, S_off, l, S_cap);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_schur(const int64_t *n_blocks, int64_t n_blocks_cap, const SchurChunks &ch, const int2 *blk_key,
                        const int64_t *blk_start, const uint64_t *pairs, const int32_t *cam_cluster, int32_t l,
                        const int32_t *cam_local, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                        const int32_t *seg_head, const T *Jc, const T *obsd, const Damp &dm, double *S,
                        double *b, hipStream_t st) {
    int64_t wgs = (ch.chunk_cap + 3) / 4;
    if (wgs > 16384) wgs = 16384;
    if (ch.blocks > 0) wgs = ch.blocks;
    wgs = ((wgs < 8 ? 8 : wgs) + 7) / 8 * 8;   // every XCD gets its share of workgroups
    k_schur<T><<<(unsigned)wgs, 256, 0, st>>>(ch, blk_key, blk_start, pairs, cam_cluster, l, cam_local, cl_Np,
                                              S_off, seg_head, Jc, obsd, dm, S, b);
    int64_t rb = n_blocks_cap;
    if (rb > 8192) rb = 8192;
    if (rb < 1) rb = 1;
    k_schur_reduce<<<(unsigned)rb, 128, 0, st>>>(ch, n_blocks, blk_key, cam_cluster, l, cam_local, cl_n, cl_Np, S_off,
                                                 dm, S, b);
    return hipGetLastError();
}
template hipError_t launch_schur<double>(const int64_t *, int64_t, const SchurChunks &, const int2 *, const int64_t *,
                                         const uint64_t *, const int32_t *, int32_t, const int32_t *, const int32_t *,
                                         const int32_t *, const int64_t *, const int32_t *, const double *,
                                         const double *, const Damp &, double *, double *, hipStream_t);
template hipError_t launch_schur<float>(const int64_t *, int64_t, const SchurChunks &, const int2 *, const int64_t *,
                                        const uint64_t *, const int32_t *, int32_t, const int32_t *, const int32_t *,
                                        const int32_t *, const int64_t *, const int32_t *, const float *, const float *,
                                        const Damp &, double *, double *, hipStream_t);

template <typename T, bool kFp64J>
hipError_t backsub_as(const stba_problem &p, const int64_t *pt_off, const T *Jc, const T *Jp, const double *Vinv,
                      const double *wph, const double *dcam, double *dpt, int32_t group_size,
                      const int32_t *grp_first, hipStream_t st) {
    const AtX X{p.cam, p.pt, p.obs_uv, p.huber};
    if (group_size > 0) {
        const int64_t ng = (p.q + group_size - 1) / group_size;
        k_backsub_obs<T, kFp64J><<<(unsigned)((ng + kPtWaves - 1) / kPtWaves), 64 * kPtWaves, 0, st>>>(
            ng, grp_first, pt_off, p.obs_pt, p.obs_cam, Jc, Jp, Vinv, wph, dcam, dpt, X);
        return hipGetLastError();
    }
    k_backsub<T, kFp64J><<<grid_for(p.n), 256, 0, st>>>(p.n, pt_off, p.obs_cam, Jc, Jp, Vinv, wph, dcam, dpt, X);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_backsub(const stba_problem &p, const int64_t *pt_off, const T *Jc, const T *Jp,
                          const double *Vinv, const double *wph, const double *dcam, double *dpt,
                          int32_t group_size, const int32_t *grp_first, bool fp64_j, hipStream_t st) {
    if (fp64_j) return backsub_as<T, true>(p, pt_off, Jc, Jp, Vinv, wph, dcam, dpt, group_size, grp_first, st);
    return backsub_as<T, false>(p, pt_off, Jc, Jp, Vinv, wph, dcam, dpt, group_size, grp_first, st);
}
template hipError_t launch_backsub<double>(const stba_problem &, const int64_t *, const double *, const double *,
                                           const double *, const double *, const double *, double *, int32_t,
                                           const int32_t *, bool, hipStream_t);
template hipError_t launch_backsub<float>(const stba_problem &, const int64_t *, const float *, const float *,
                                          const double *, const double *, const double *, double *, int32_t,
                                          const int32_t *, bool, hipStream_t);

hipError_t launch_refine_residual(const stba_problem &p, const int64_t *pt_off, const int32_t *seg_head,
                                  int32_t group_size, const int32_t *grp_first, const Damp &dm,
                                  const double *dcam, double *e, double *Vinv, double *wph, const int64_t *diag_blk,
                                  const int64_t *blk_start, const VjpParts &parts, double *r, hipStream_t st) {
    if (group_size > 0) {
        const int64_t ng = (p.q + group_size - 1) / group_size;
        k_refine_obs<<<(unsigned)((ng + kPtWaves - 1) / kPtWaves), 64 * kPtWaves, 0, st>>>(
            ng, grp_first, pt_off, p.obs_pt, p.obs_cam, p.cam, p.pt, p.obs_uv, p.huber, seg_head, dm, dcam, e, Vinv,
            wph);
    } else {
        k_refine_pt<<<grid_for(p.n, 64), 64, 0, st>>>(p.n, pt_off, p.obs_cam, p.cam, p.pt, p.obs_uv, p.huber,
                                                      seg_head, dm, dcam, e, Vinv, wph);
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_refine_cam<<<xcd_contiguous_grid(parts.cap), 256, 0, st>>>(p.m, p.q, parts.off, parts.cam, parts.obs_off,
                                                                    parts.oj, p.cam, p.pt, p.obs_uv, p.huber,
                                                                    diag_blk, blk_start, dm, dcam, e, parts.sum, r);
    k_refine_cam_sum<<<grid_for(9 * (int64_t)p.m), 256, 0, st>>>(p.m, parts.off, parts.sum, dm, dcam, r);
    return hipGetLastError();
}

hipError_t launch_cost_at(const stba_problem &p, const double *dcam, const double *dpt, double *partials,
                          const stba_lm_state *s, double *F_ref, hipStream_t st) {
    k_cost_at<<<grid_for(p.q), 256, 0, st>>>(p.q, p.cam, p.pt, p.obs_cam, p.obs_pt, p.obs_uv, dcam, dpt, partials, s,
                                             F_ref, p.huber);
    return hipGetLastError();
}

hipError_t launch_accept_update(const stba_problem &p, const double *rj_partials, const double *partials,
                                int64_t count, const double *F_ref, const int32_t *cl_status, int32_t l,
                                const int32_t *status, stba_lm_state *s, const double *dcam, const double *dpt,
                                hipStream_t st) {
    // one block per CU at most: each one re-sums the candidate partials before
    // its share of x += dx
    unsigned blocks = grid_for(9 * (int64_t)p.m + 3 * (int64_t)p.n);
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    k_accept_update<<<blocks, 256, 0, st>>>(rj_partials, partials, count, F_ref, cl_status, l, status, s, p.m, p.n,
                                            p.cam, p.pt, dcam, dpt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Many problems in one LM step (Alg. 1 per problem): the problems are
// concatenated (cameras, points and observations in contiguous ranges, each
// point's observations and each cluster's cameras inside one problem) and
// every problem keeps its own damping, cost and accept decision.
// ---------------------------------------------------------------------------
// Cost of each problem at x (dcam = dpt = null) or at x + dx, one workgroup
// per problem over its observation range in a fixed order; also checks that
// every observation's camera and point belong to the range's problem.
__global__ __launch_bounds__(256) void k_cost_problems(int32_t n_prob, const int64_t *__restrict__ obs_off,
                                                       const double *__restrict__ cam, const double *__restrict__ pt,
                                                       const int32_t *__restrict__ oc, const int32_t *__restrict__ op,
                                                       const double *__restrict__ uv, const double *__restrict__ dcam,
                                                       const double *__restrict__ dpt, double huber,
                                                       const int32_t *__restrict__ prob_cam,
                                                       const int32_t *__restrict__ prob_pt, double *__restrict__ F,
                                                       int32_t *status) {
    __shared__ double sh[256];
    for (int32_t pb = blockIdx.x; pb < n_prob; pb += gridDim.x) {
        double s = 0.0;
        for (int64_t o = obs_off[pb] + threadIdx.x; o < obs_off[pb + 1]; o += 256) {
            const int64_t i = oc[o], j = op[o];
            if (prob_cam[i] != pb || prob_pt[j] != pb) set_status(status + kStSticky, STBA_EINVAL);
            double c[9], X[3];
#pragma unroll
            for (int k = 0; k < 9; ++k) c[k] = cam[9 * i + k] + (dcam ? dcam[9 * i + k] : 0.0);
#pragma unroll
            for (int k = 0; k < 3; ++k) X[k] = pt[3 * j + k] + (dpt ? dpt[3 * j + k] : 0.0);
            double pix[2];
            camera_project(c, X, pix);
            const double f0 = pix[0] - uv[2 * o], f1 = pix[1] - uv[2 * o + 1];
            s += huber_rho(f0 * f0 + f1 * f1, huber);
        }
        s = block_sum_256(s, sh);
        if (threadIdx.x == 0) F[pb] = s;
    }
}

// The problems whose clusters did not all factorise (bad[p] = 1: a non-PD S_k,
// 2: a factorisation wait that timed out); a cluster whose cameras span two
// problems is a data error.  bad is cleared by the caller.
__global__ __launch_bounds__(256) void k_batch_clusters(int32_t l, const int32_t *__restrict__ cl_start,
                                                        const int32_t *__restrict__ cl_cams,
                                                        const int32_t *__restrict__ cl_status,
                                                        const int32_t *__restrict__ prob_cam, int32_t *__restrict__ bad,
                                                        int32_t *status) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < l; k += gridDim.x * blockDim.x) {
        const int32_t a = cl_start[k], e = cl_start[k + 1];
        if (e <= a) continue;
        const int32_t pb = prob_cam[cl_cams[a]];
        for (int32_t u = a + 1; u < e; ++u)
            if (prob_cam[cl_cams[u]] != pb) set_status(status + kStSticky, STBA_EINVAL);
        const int32_t cs = cl_status[k];
        if (cs == STBA_EHIP) atomicMax(bad + pb, 2);
        else if (cs != STBA_OK) atomicMax(bad + pb, 1);
    }
}

// Per problem: accept iff F(x + dx) < F(x), finite, and every cluster of the
// problem factorised; the damping rule and counters of k_accept_update.  The
// point blocks' status and the sticky data error are shared by the batch.
__global__ __launch_bounds__(256) void k_batch_accept(int32_t n_prob, const double *__restrict__ F_x,
                                                      const double *__restrict__ F_c, const int32_t *__restrict__ bad,
                                                      const int32_t *status, stba_lm_state *states) {
    const int32_t pb = blockIdx.x * blockDim.x + threadIdx.x;
    if (pb >= n_prob) return;
    stba_lm_state *st = states + pb;
    const double F0 = F_x[pb], Fn = F_c[pb];
    const int32_t sticky = bad[pb] == 2 ? STBA_EHIP : status[kStSticky];
    const bool pd = bad[pb] == 0 && status[kStPointBad] == 0;
    const bool fin = isfinite(Fn);
    const bool acc = pd && fin && sticky == 0 && (Fn < F0);
    st->F = acc ? Fn : F0;
    st->have_F = 1;
    st->F_new = Fn;
    st->accepted = acc ? 1 : 0;
    st->lambda = acc ? fmax(st->lambda / 3.0, st->lambda_min) : st->lambda * 3.0;
    st->need_jac = acc ? 1 : 0;
    st->n_rcs += 1;
    st->n_accept += acc ? 1 : 0;
    st->n_jac += status[kStJacRan] ? 1 : 0;
    st->last_status = bad[pb] == 2 ? STBA_EHIP : (!pd ? STBA_ENOTPD : (!fin ? STBA_ENONFINITE : sticky));
    if (st->status == 0 && sticky != 0) st->status = sticky;
}

// x += dx for the cameras and points of the problems that accepted.
__global__ __launch_bounds__(256) void k_batch_apply(int32_t m, int32_t n, const int32_t *__restrict__ prob_cam,
                                                     const int32_t *__restrict__ prob_pt,
                                                     const stba_lm_state *__restrict__ states, double *cam,
                                                     double *pt, const double *__restrict__ dcam,
                                                     const double *__restrict__ dpt) {
    const int64_t nc = 9 * (int64_t)m, total = nc + 3 * (int64_t)n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        if (i < nc) {
            if (states[prob_cam[i / 9]].accepted) cam[i] += dcam[i];
        } else {
            const int64_t k = i - nc;
            if (states[prob_pt[k / 3]].accepted) pt[k] += dpt[k];
        }
    }
}

// flag = 1 if any problem of the batch needs f and J at its x.
__global__ __launch_bounds__(256) void k_batch_need_jac(int32_t n_prob, const stba_lm_state *__restrict__ states,
                                                        int32_t *flag) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int32_t pb = threadIdx.x; pb < n_prob; pb += blockDim.x)
        if (states[pb].need_jac) any = 1;
    __syncthreads();
    if (threadIdx.x == 0) flag[0] = any;
}

hipError_t launch_batch_need_jac(int32_t n_prob, const stba_lm_state *states, int32_t *flag, hipStream_t st) {
    k_batch_need_jac<<<1, 256, 0, st>>>(n_prob, states, flag);
    return hipGetLastError();
}

hipError_t launch_cost_problems(const stba_problem &p, int32_t n_prob, const int64_t *obs_off,
                                const int32_t *prob_cam, const int32_t *prob_pt, const double *dcam,
                                const double *dpt, double *F, int32_t *status, hipStream_t st) {
    const unsigned blocks = (unsigned)(n_prob < 4096 ? n_prob : 4096);
    k_cost_problems<<<blocks, 256, 0, st>>>(n_prob, obs_off, p.cam, p.pt, p.obs_cam, p.obs_pt, p.obs_uv, dcam, dpt,
                                            p.huber, prob_cam, prob_pt, F, status);
    return hipGetLastError();
}

hipError_t launch_batch_accept(const stba_problem &p, int32_t n_prob, int32_t l, const int32_t *cl_start,
                               const int32_t *cl_cams, const int32_t *cl_status, const int32_t *prob_cam,
                               const int32_t *prob_pt, const double *F_x, const double *F_c, int32_t *bad,
                               int32_t *status, stba_lm_state *states, const double *dcam, const double *dpt,
                               hipStream_t st) {
    k_fill_i32<<<grid_for(n_prob), 256, 0, st>>>(bad, n_prob, 0);
    k_batch_clusters<<<grid_for(l), 256, 0, st>>>(l, cl_start, cl_cams, cl_status, prob_cam, bad, status);
    k_batch_accept<<<grid_for(n_prob), 256, 0, st>>>(n_prob, F_x, F_c, bad, status, states);
    unsigned blocks = grid_for(9 * (int64_t)p.m + 3 * (int64_t)p.n);
    if (blocks > 2048) blocks = 2048;
    k_batch_apply<<<blocks, 256, 0, st>>>(p.m, p.n, prob_cam, prob_pt, states, p.cam, p.pt, dcam, dpt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_vjp(const stba_problem &p, const int64_t *pt_off, const int64_t *diag_blk, const int64_t *blk_start,
                      const uint64_t *pairs, const VjpParts &parts, const T *v, T *grad_cam, T *grad_pt, T *grad_uv,
                      hipStream_t st) {
    (void)pairs;
    k_vjp_cam<T><<<xcd_contiguous_grid(parts.cap), 256, 0, st>>>(p.m, p.q, parts.off, parts.cam, parts.obs_off,
                                                                 parts.oj, p.cam, p.pt, diag_blk, blk_start, v,
                                                                 parts.sum, grad_cam);
    k_vjp_cam_sum<T><<<grid_for(9 * (int64_t)p.m), 256, 0, st>>>(p.m, parts.off, parts.sum, grad_cam);
    k_vjp_pt<T><<<grid_for(p.n), 256, 0, st>>>(p.n, p.q, p.cam, p.pt, p.obs_cam, pt_off, v, grad_pt);
    k_neg<T><<<grid_for(2 * p.q), 256, 0, st>>>(2 * p.q, v, grad_uv);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_vjp_stored(const stba_problem &p, const int64_t *pt_off, const int64_t *diag_blk,
                             const int64_t *blk_start, const uint64_t *pairs, const VjpParts &parts, const T *v,
                             const T *Jc, const T *Jp, T *grad_cam, T *grad_pt, T *grad_uv, hipStream_t st) {
    k_vjp_cam_stored<T><<<xcd_contiguous_grid(parts.cap), 256, 0, st>>>(p.m, parts.off, parts.cam, diag_blk,
                                                                        blk_start, pairs, Jc, v, parts.sum, grad_cam);
    k_vjp_cam_sum<T><<<grid_for(9 * (int64_t)p.m), 256, 0, st>>>(p.m, parts.off, parts.sum, grad_cam);
    k_vjp_pt_stored<T><<<grid_for(p.n), 256, 0, st>>>(p.n, pt_off, Jp, v, grad_pt);
    k_neg<T><<<grid_for(2 * p.q), 256, 0, st>>>(2 * p.q, v, grad_uv);
    return hipGetLastError();
}
template hipError_t launch_vjp_stored<double>(const stba_problem &, const int64_t *, const int64_t *, const int64_t *,
                                              const uint64_t *, const VjpParts &, const double *, const double *,
                                              const double *, double *, double *, double *, hipStream_t);
template hipError_t launch_vjp_stored<float>(const stba_problem &, const int64_t *, const int64_t *, const int64_t *,
                                             const uint64_t *, const VjpParts &, const float *, const float *,
                                             const float *, float *, float *, float *, hipStream_t);
template hipError_t launch_vjp<double>(const stba_problem &, const int64_t *, const int64_t *, const int64_t *,
                                       const uint64_t *, const VjpParts &, const double *, double *, double *,
                                       double *, hipStream_t);
template hipError_t launch_vjp<float>(const stba_problem &, const int64_t *, const int64_t *, const int64_t *,
                                      const uint64_t *, const VjpParts &, const float *, float *, float *, float *,
                                      hipStream_t);

}  // namespace stba
