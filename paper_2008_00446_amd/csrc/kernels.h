// Launchers of the gfx950 kernels (internal header).  Each launcher enqueues on
// `st` and returns the launch status; shapes are checked by the caller.
#pragma once
#include "common.h"

namespace stba {

// --- set-up (prepare.hip) ---------------------------------------------------
hipError_t launch_analyze(const stba_problem &p, int64_t *d_scratch, hipStream_t st);
struct PrepBufs {
    int64_t *pt_off;      // [n+1] first observation of each point
    int64_t *pair_off;    // [n+1] first pair of each point (generation order)
    int64_t *scratch_a;   // [n_pairs] pair counts / head flags
    uint64_t *keys_in;    // [n_pairs] (row camera) * m + (column camera)
    uint64_t *keys_out;   // [n_pairs] sorted keys
    uint64_t *vals_in;    // [n_pairs] (row obs << 32) | column obs
    uint64_t *pairs;      // [n_pairs] sorted values: the pair list grouped by camera pair
    int64_t *blk_of;      // [n_pairs] block index of each sorted pair (exclusive scan of heads)
    int2 *blk_key;        // [n_pairs] (row camera, column camera) of each block (first n_blocks used)
    int64_t *blk_start;   // [n_pairs + 1] first pair of each block
    int64_t *n_blocks;    // [1]
    int64_t *diag_blk;    // [m] block index of camera pair (i, i)
    int64_t blk_cap;         // bound on the number of blocks: min(n_pairs, m (m + 1) / 2)
    int64_t *blk_chunk_off;  // [blk_cap + 1] first chunk of each block (chunks of kSchurChunk pairs)
    int32_t *chunk_blk;      // [chunk_cap] block of each chunk
    int64_t chunk_cap;       // blk_cap + n_pairs / kSchurChunk + 1
    int64_t *n_chunks;       // [1]
    // camera sums of J^T v: camera r's observations (its diagonal block) cut
    // into parts of at most kVjpPart, one wavefront each
    int64_t *vjp_part_off;   // [m + 1] first part of each camera; [m]: the number of parts
    int32_t *vjp_part_cam;   // [vjp_part_cap] camera of each part
    int64_t vjp_part_cap;    // m + n_pairs / kVjpPart + 1
    int64_t *vjp_obs_off;    // [m + 1] first entry of each camera in vjp_oj
    int2 *vjp_oj;            // [q] (observation, point) of each camera's observations, camera-major
    void *tmp;            // rocPRIM temporary storage
    size_t tmp_bytes;
};
size_t prepare_tmp_bytes(int64_t n_pairs, int32_t m, hipStream_t st);
hipError_t launch_prepare(const stba_problem &p, int64_t n_pairs, const PrepBufs &b, int32_t *status,
                          hipStream_t st);

// --- per iteration ----------------------------------------------------------
hipError_t launch_reset_status(int32_t *status, hipStream_t st);
hipError_t launch_lm_init(stba_lm_state *s, double lambda0, double lambda_corr, hipStream_t st);
// also clears the status words and sets every cluster's status (l of them) to
// STBA_OK; l_dev (nullable): the number of clusters on the device, l a bound
hipError_t launch_clusters(const int32_t *cam_cluster, int32_t m, int32_t l, const int32_t *l_dev, int32_t gamma_max,
                           int32_t *cl_n, int32_t *cl_Np, int32_t *cl_start, int32_t *cl_cams,
                           int32_t *cam_local, int64_t *S_off, int32_t *cl_status, int32_t *status, hipStream_t st);

// S (nullable): also zero S (the first min(S_off[l], S_cap) doubles) and b
// (nb doubles)
struct ZeroS {
    double *S = nullptr;
    const int64_t *S_off = nullptr;
    int32_t l = 0;
    int64_t S_cap = 0;
    double *b = nullptr;
    int64_t nb = 0;
};
template <typename T>
hipError_t launch_rj(const stba_problem &p, T *f, T *Jc, T *Jp, double *partials, const int32_t *need_jac,
                     int32_t *jac_ran, const ZeroS &z, hipStream_t st);
int64_t rj_blocks(int64_t q);

hipError_t launch_sum_partials(const double *partials, int64_t count, double *out, hipStream_t st);
hipError_t launch_set_damping(double *slot, double lambda, double lambda_corr, hipStream_t st);

// Damping of the step: lambda and lambda_corr of one problem (lam2[0], lam2[1]),
// or of each problem of a batch: problem p's pair at lam2 + stride p, where p
// is prob_cam[i] for camera i and prob_pt[j] for point j.
struct Damp {
    const double *lam2 = nullptr;
    const int32_t *prob_cam = nullptr, *prob_pt = nullptr;   // null: one problem
    int64_t stride = 0;
    Damp() = default;
    Damp(const double *l) : lam2(l) {}
    __device__ const double *at_cam(int64_t i) const { return prob_cam ? lam2 + stride * prob_cam[i] : lam2; }
    __device__ const double *at_pt(int64_t j) const { return prob_pt ? lam2 + stride * prob_pt[j] : lam2; }
};

// Segments, point blocks and per-observation records.  group_size > 0: one
// lane per observation (groups from launch_point_groups, max_track <= 32);
// otherwise one thread per point and one per observation (seg_rec staging).

template <typename T>
hipError_t launch_points(const stba_problem &p, const int64_t *pt_off, const int32_t *cam_cluster, int32_t l,
                         const T *f, const T *Jc, const T *Jp, const Damp &dm, uint64_t seed, uint64_t t,
                         uint64_t thr, int32_t *seg_head, double *seg_rec, T *obsd, double *Vinv, double *wph,
                         int32_t *status, int32_t group_size, const int32_t *grp_first, hipStream_t st);
// group g of the one-lane-per-observation path starts at grp_first[g]
// (ngroups + 1 entries); group_size = 65 - max_track
hipError_t launch_point_groups(int32_t n, const int64_t *pt_off, int32_t group_size, int64_t ngroups,
                               int32_t *grp_first, hipStream_t st);
inline int32_t point_group_size(int32_t max_track) { return max_track <= 32 ? 65 - max_track : 0; }

// zero S and b
hipError_t launch_fill_S(double *S, double *b, int32_t m, const int64_t *S_off, int32_t l, int64_t S_cap,
                         hipStream_t st);

struct SchurChunks {
    const int64_t *n_chunks;
    const int64_t *blk_chunk_off;
    const int32_t *chunk_blk;
    int64_t chunk_cap;
    double *part;          // partial sums, kSchurPart doubles per chunk
    int32_t blocks = 0;    // workgroups of k_schur (0: from the chunk count)
    int32_t all_links = 0;  // alpha = 1: every same-cluster link is kept, so the pairs of a block
                            // share their segment and the segment-head check is skipped
};
template <typename T>
hipError_t launch_schur(const int64_t *n_blocks, int64_t n_blocks_cap, const SchurChunks &ch, const int2 *blk_key,
                        const int64_t *blk_start, const uint64_t *pairs, const int32_t *cam_cluster, int32_t l,
                        const int32_t *cam_local, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                        const int32_t *seg_head, const T *Jc, const T *obsd, const Damp &dm, double *S,
                        double *b, hipStream_t st);

// Cluster solves.  With few clusters (l wavefront sets of T + (T-1)(T-2)/2,
// T = max_Np / 32, within kCholTileWaves and resident at once) and flags / yx
// given: one wavefront per tile (tile-parallel dataflow); otherwise one
// workgroup per cluster.  flags: chol_flag_words() int32; yx: chol_yx_doubles().
constexpr int kCholTileWaves = 2048;   // e.g. one cluster of up to 64 tile rows (Np <= 2048)
// per cluster T (T + 1) / 2 + T + 2 flag words <= 2.5 x its wavefronts, plus the
// abort word and the count of finished clusters
inline int64_t chol_flag_words() { return 4 * (int64_t)kCholTileWaves + 2; }
// per cluster 2 block vectors of T x 32 doubles (y, x), T <= its wavefronts
inline int64_t chol_yx_doubles() { return 2 * (int64_t)kCholTileWaves * kNB; }
int chol_tile_layout(int32_t l, int32_t max_Np, int32_t *wpc, int32_t *tmax, int32_t *fpc, int32_t *xcd_major);
// Buffers of the team factorisation (many clusters, tiles in memory): flag
// words (per cluster 2 T^2 + 8 from 2 S_off / 1024 + 8 k, then the abort word
// at abort_at and the finished-cluster count) and four block-vector buffers of
// vec_len doubles each (c, d per tile, y, x per block row, from S_off / 32).
// form: STBA_CHOL_* (a form that does not fit falls back to the built-in order).
struct CholTeam {
    int32_t *flags = nullptr;
    int64_t abort_at = 0;
    double *vec = nullptr;
    int64_t vec_len = 0;
    int32_t form = STBA_CHOL_AUTO;
    bool l_on_device = false;   // l is a bound: the number of clusters is known only on the device
};
constexpr int32_t kTeamMaxNp = 2048;
// ... then the abort word, the finished-cluster count and whether the teams ran
inline int64_t chol_team_flag_words(int64_t S_cap, int32_t m) { return 2 * (S_cap / 1024) + 8 * (int64_t)m + 3; }
inline int64_t chol_team_vec_len(int64_t S_cap) { return S_cap / 32; }
// the flag words and block vectors have to be in their initial state before the
// first factorisation; every tile-parallel or team factorisation leaves them so again
hipError_t launch_clear_chol_flags(int32_t *flags, double *yx, const CholTeam *team, hipStream_t st);
// whether launch_chol would run `form` itself (rather than fall back) for l clusters
int chol_form_fits(int32_t form, int32_t l, int32_t max_Np, bool l_on_device, const CholTeam *team);
// The factorisation leaves L in S's lower tiles and W_pp^T = (L_pp^-1)^T in the
// upper triangle of each diagonal tile.
hipError_t launch_chol(int32_t l, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                       const int32_t *cl_start, const int32_t *cl_cams, double *S, const double *b,
                       double *dcam, int32_t *cl_status, int32_t max_Np, int32_t *flags, double *yx,
                       const CholTeam *team, hipStream_t st);

// The camera parts of stba_prepare (vjp_part_off, vjp_part_cam, part_cap of
// them at most) and part_sum, 18 doubles per part (the camera sums of J^T v
// use 9), for the cameras cut in several; the camera-major observation list.
struct VjpParts {
    const int64_t *off;
    const int32_t *cam;
    int64_t cap;
    double *sum;
    const int64_t *obs_off;   // [m + 1] first entry of each camera in oj
    const int2 *oj;           // [q] (observation, point), camera-major in diagonal-block order
};

// MIXED refinement residual r = b - S x of the FP64 method's S and b, formed
// from J recomputed in FP64 at x (never from the FP32-assembled S): e [2 q]
// receives the linearised residuals, r [9 m] the residual in camera order;
// Vinv / wph are overwritten with the FP64 physical point blocks.
hipError_t launch_refine_residual(const stba_problem &p, const int64_t *pt_off, const int32_t *seg_head,
                                  int32_t group_size, const int32_t *grp_first, const Damp &dm,
                                  const double *dcam, double *e, double *Vinv, double *wph, const int64_t *diag_blk,
                                  const int64_t *blk_start, const VjpParts &parts, double *r, hipStream_t st);
// dcam += S^-1 r with the factors left in S by launch_chol (r in camera order)
hipError_t launch_sweep(int32_t l, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                        const int32_t *cl_start, const int32_t *cl_cams, const double *S, const double *r,
                        double *dcam, int32_t max_Np, hipStream_t st);

template <typename T>
// group_size > 0: one lane per observation in the groups of launch_points.
// fp64_j: J_c, J_p formed in FP64 at x instead of read from Jc / Jp.
hipError_t launch_backsub(const stba_problem &p, const int64_t *pt_off, const T *Jc, const T *Jp,
                          const double *Vinv, const double *wph, const double *dcam, double *dpt,
                          int32_t group_size, const int32_t *grp_first, bool fp64_j, hipStream_t st);

// F_ref (nullable, 2 doubles): receives s->F and s->have_F for launch_accept_update
hipError_t launch_cost_at(const stba_problem &p, const double *dcam, const double *dpt, double *partials,
                          const stba_lm_state *s, double *F_ref, hipStream_t st);

// rj_partials: the residual kernel's partials (F(x) while the state has none)
hipError_t launch_accept_update(const stba_problem &p, const double *rj_partials, const double *partials,
                                int64_t count, const double *F_ref, const int32_t *cl_status, int32_t l,
                                const int32_t *status, stba_lm_state *s, const double *dcam, const double *dpt,
                                hipStream_t st);

// Batched LM (many problems, one step): per-problem cost (at x when dcam and
// dpt are null), then the per-problem decisions and x += dx where accepted.
// bad: n_prob int32 of scratch.
hipError_t launch_batch_need_jac(int32_t n_prob, const stba_lm_state *states, int32_t *flag, hipStream_t st);
hipError_t launch_cost_problems(const stba_problem &p, int32_t n_prob, const int64_t *obs_off,
                                const int32_t *prob_cam, const int32_t *prob_pt, const double *dcam,
                                const double *dpt, double *F, int32_t *status, hipStream_t st);
hipError_t launch_batch_accept(const stba_problem &p, int32_t n_prob, int32_t l, const int32_t *cl_start,
                               const int32_t *cl_cams, const int32_t *cl_status, const int32_t *prob_cam,
                               const int32_t *prob_pt, const double *F_x, const double *F_c, int32_t *bad,
                               int32_t *status, stba_lm_state *states, const double *dcam, const double *dpt,
                               hipStream_t st);

template <typename T>
hipError_t launch_vjp(const stba_problem &p, const int64_t *pt_off, const int64_t *diag_blk,
                      const int64_t *blk_start, const uint64_t *pairs, const VjpParts &parts, const T *v,
                      T *grad_cam, T *grad_pt, T *grad_uv, hipStream_t st);
// The same products from stored blocks Jc [q][18], Jp [q][6] (precision T).
template <typename T>
hipError_t launch_vjp_stored(const stba_problem &p, const int64_t *pt_off, const int64_t *diag_blk,
                             const int64_t *blk_start, const uint64_t *pairs, const VjpParts &parts, const T *v,
                             const T *Jc, const T *Jp, T *grad_cam, T *grad_pt, T *grad_uv, hipStream_t st);

// --- camera clustering (sgc.hip) ---------------------------------------------
// One workgroup; Pg / Tg / Wg hold a pair label, clock and weight per block of
// the Schur plan (at least n_blocks each) when the graph has more than 4096 blocks.
hipError_t launch_sgc(int32_t m, const int64_t *n_blocks, const int2 *blk_key, const int64_t *blk_start,
                      int32_t gamma, double beta, uint64_t seed, uint64_t iter, uint32_t *Pg, double *Tg,
                      int32_t *Wg, int32_t *cam_cluster, int32_t *n_clusters, int32_t *status, hipStream_t st);

// --- inexact cluster solves (pcg.hip) ---------------------------------------
// Dynamic LDS of one cluster's conjugate-gradient workgroup (<= 160 KB required).
size_t pcg_lds_bytes(int32_t max_np, int32_t max_n);
// clus [m] and Minv [81 m] are scratch; iters_out, resid_out, cl_status [l].
hipError_t launch_pcg(int32_t l, const int32_t *cl_n, const int32_t *cl_Np, const int64_t *S_off,
                      const int32_t *cl_start, const int32_t *cl_cams, const int32_t *cam_local,
                      const int64_t *n_blocks, const int2 *blk_key, const double *S, const double *b, double *dcam,
                      int32_t *clus, double *Minv, int32_t max_np, int32_t max_n, int32_t max_iters, double tol,
                      int32_t *iters_out, double *resid_out, int32_t *cl_status, hipStream_t st);

}  // namespace stba
