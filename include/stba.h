/*
 * stba.h - C ABI of the MI355X (gfx950) hot path of Stochastic Bundle Adjustment.
 *
 * Method: L. Zhou et al., "Stochastic Bundle Adjustment for Efficient and Scalable
 * 3D Reconstruction", ECCV 2020 (arXiv 2008.00446).  One LM iteration of STBA
 * (Alg. 1) is: the camera clustering (Sec. 4.4, optionally drawn on the device),
 * residuals and Jacobian (Sec. 3), the sampled constraint set as
 * point segments (Sec. 4.1-4.2), the optional steepest-descent correction
 * (Sec. 4.3), one reduced camera system per camera cluster from the clustered
 * Schur complement S' = B - E' C'^-1 E'^T (Eq. 10, 13), independent dense
 * Cholesky solves per cluster (Eq. 13), the physical point update (Eq. 15) and
 * the accept/reject rule on the FP64 cost (Alg. 1).
 *
 * Conventions shared by every entry point
 *  - Pointers are DEVICE pointers unless the comment says (host).  The caller
 *    owns all memory; the library never allocates or frees and keeps no global
 *    state.  Everything it needs between calls lives in the caller's workspace
 *    (the one exception: the scratch of stba_residual_jacobian_static).
 *  - Calls that take a stream only enqueue work on it and return; they do not
 *    synchronise (stba_analyze is the one exception and says so).
 *  - Host-detectable argument errors return an error code before anything is
 *    enqueued.  Conditions only the device can see (bad ids, unsorted input,
 *    a cluster matrix that is not positive definite, non-finite values) are
 *    written to device status words and seen at the caller's next sync.
 *  - Camera parameters: 9 doubles (w0 w1 w2 t0 t1 t2 f k1 k2): rotation vector,
 *    translation, focal length, radial distortion.  A point X projects to
 *    P = R(w) X + t, (x, y) = (P_x, P_y)/P_z, r2 = x^2 + y^2,
 *    pixel = f (1 + k1 r2 + k2 r2^2)(x, y) (image-centred).  The residual is
 *    f_o = pixel - observed and the cost F = sum ||f_o||^2 (Sec. 3, no 1/2), or
 *    with the robust loss of stba_problem.huber F = sum rho(||f_o||^2).
 *  - Observations are sorted by (point, camera) with at most one observation
 *    per (camera, point); every point has at least one observation.
 *  - Per-observation Jacobian blocks are stored observation-major:
 *    f [q][2], Jc [q][2][9], Jp [q][2][3] (row-major inside an observation).
 *  - Every call after stba_prepare takes the same (dims, precision, ws, ws_bytes)
 *    that sized and prepared the workspace; the layout is derived from them.
 */
#ifndef STBA_H
#define STBA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* precision of residuals, Jacobians and Schur assembly */
#define STBA_FP64  0   /* everything in FP64 */
#define STBA_MIXED 1   /* f, J, Hessian blocks and Schur assembly in FP32 with FP32
                          accumulation; Cholesky, point update and cost in FP64,
                          and one FP64 refinement step of every cluster solve:
                          dc += S_k^-1 (b - S x) with b - S x formed from J
                          recomputed in FP64 at x (the FP64 method's S and b,
                          never the FP32-assembled S_k), the factor that of the
                          FP32-assembled S_k; the point update (Eq. 15) then
                          also takes J and its blocks in FP64 */
#define STBA_MIXED_NOREFINE 2  /* STBA_MIXED without the refinement step: the point
                          update with the FP32 J */

/* status codes (int32) */
#define STBA_OK          0
#define STBA_EINVAL     -1   /* bad argument (host) or bad id / size (device) */
#define STBA_ENOTPD     -2   /* a cluster matrix S_k is not positive definite */
#define STBA_ENONFINITE -3   /* NaN / Inf in a step or cost */
#define STBA_EWORKSPACE -4   /* workspace too small */
#define STBA_EHIP       -5   /* a HIP runtime call failed, or a wait inside a cluster factorisation
                                timed out (device) */
#define STBA_EDATA      -6   /* observations not sorted / duplicated / point unseen */

/* Bundle-adjustment problem: the visibility graph and x = [c; p] (Sec. 3). */
typedef struct stba_problem {
    int32_t m;                 /* cameras, >= 1 */
    int32_t n;                 /* points, >= 1 */
    int64_t q;                 /* observations, 1 <= q < 2^31 */
    double *cam;               /* [m][9] FP64 master copy; stba_lm_step updates it on accept */
    double *pt;                /* [n][3] FP64 master copy; stba_lm_step updates it on accept */
    const int32_t *obs_cam;    /* [q] camera of each observation */
    const int32_t *obs_pt;     /* [q] point of each observation, (obs_pt, obs_cam) increasing */
    const double *obs_uv;      /* [q][2] observed pixel, image-centred */
    double huber;              /* robust loss (Sec. 5.1): Huber scale a > 0 on each observation's
                                  error norm, rho(s) = s for s = ||f||^2 <= a^2, else 2 a sqrt(s) - a^2,
                                  applied by IRLS weights sqrt(rho'(s)) on f and J; 0: squared loss.
                                  Must be finite and >= 0. */
} stba_problem;

/* forms of the cluster factorisation (stba_dims.chol_form) */
#define STBA_CHOL_AUTO      0   /* the built-in choice: tiles when they fit, else teams, else workgroups */
#define STBA_CHOL_TILES     1   /* one wavefront per tile, all clusters' tiles resident at once */
#define STBA_CHOL_TEAM      2   /* per cluster a band, a forward and worker wavefronts, tiles in memory */
#define STBA_CHOL_WORKGROUP 3   /* one workgroup per cluster */

/* Data-dependent sizes, filled by stba_analyze (host struct), and the launch
 * settings stba_autotune chooses (stba_analyze sets them to 0, the built-in
 * choices; a caller may also set them). */
typedef struct stba_dims {
    int64_t n_pairs;           /* sum over points of v (v + 1) / 2, v = observations of the point */
    int32_t max_track;         /* largest v */
    int32_t gamma_max;         /* largest cluster (cameras) the workspace must hold */
    int32_t chol_form;         /* STBA_CHOL_*; a form that does not fit falls back to the built-in order */
    int32_t schur_blocks;      /* workgroups of the Schur assembly, 0 or 8..65536 */
} stba_dims;

/* One draw of the constraint sampler Theta(alpha) (Sec. 4.2). */
typedef struct stba_sample {
    const int32_t *cam_cluster; /* [m] cluster of each camera, values in [0, l) */
    int32_t l;                  /* number of clusters, 1 <= l <= m; with l_dev: an upper bound */
    int32_t pad0;
    double alpha;               /* confidence level in (0, 1]; 1 keeps every intra-cluster link */
    uint64_t seed;              /* Philox4x64-10 key word 0 */
    uint64_t iter;              /* LM iteration t, Philox counter word 0 */
    const int32_t *l_dev;       /* (device, nullable) the number of clusters, read on the device, so a
                                   map drawn on the device (stba_sample_clusters) needs no read-back:
                                   ids must lie in [0, *l_dev), 1 <= *l_dev <= l, and the launches are
                                   sized for the bound l (clusters *l_dev .. l - 1 are empty).  A value
                                   outside [1, l] rejects the step as an invalid map. */
} stba_sample;

/* Damping for the standalone assembly call (Eq. 1-4, Sec. 4.3). */
typedef struct stba_damping {
    double lambda;              /* LM damping, > 0 */
    double lambda_corr;         /* correction threshold: correct iff lambda >= lambda_corr (paper: 0.1) */
} stba_damping;

/* Device-resident LM state updated by stba_lm_step (Alg. 1). */
typedef struct stba_lm_state {
    double lambda;              /* current damping */
    double lambda_corr;         /* correction threshold */
    double F;                   /* cost at the current x (valid once have_F = 1) */
    double F_new;               /* cost at the last candidate x + dx (NaN if the step failed) */
    int32_t accepted;           /* 1 if the last step was accepted */
    int32_t status;             /* sticky: first device-side error (STBA_* code), 0 if none */
    int32_t need_jac;           /* 1 if f and J must be evaluated at the current x */
    int32_t have_F;             /* 1 once F holds the cost at x */
    int32_t last_status;        /* status of the last step only (0, STBA_ENOTPD, STBA_ENONFINITE, STBA_EHIP,
                                   or the sticky data error) */
    int32_t pad0;
    int64_t n_jac;              /* Jacobian evaluations */
    int64_t n_rcs;              /* RCS builds / solves */
    int64_t n_accept;           /* accepted steps */
    double lambda_min;          /* lower bound of lambda after an accepted step (0: none); stba_lm_init
                                   sets 0, a caller may overwrite it in place (the correction
                                   ablation of Sec. 5.4 keeps lambda >= 0.1) */
} stba_lm_state;

/* Views into the workspace written by stba_build_cluster_rcs (read-only for
 * the caller, valid until the workspace is reused).  All device pointers. */
typedef struct stba_rcs {
    const double *S;            /* concatenated cluster matrices, column-major, padded to Np_k */
    const int64_t *S_off;       /* [l+1] offset (doubles) of cluster k's matrix in S */
    const int32_t *cl_n;        /* [l] cameras in cluster k */
    const int32_t *cl_Np;       /* [l] padded order of S_k (multiple of 32, >= 9 cl_n[k]) */
    const int32_t *cl_start;    /* [l+1] offset of cluster k in cl_cams */
    const int32_t *cl_cams;     /* [m] cameras grouped by cluster, ascending id inside a cluster */
    const int32_t *cam_local;   /* [m] index of each camera inside its cluster */
    const double *b;            /* [m][9] right-hand side b' = v' - E' C'^-1 w' (Eq. 13) */
    const int32_t *seg_head;    /* [q] sampled segment of each observation, named by its first
                                   observation (smallest camera) - the bound virtual point */
    int32_t l;                  /* the sample's l (a bound when l_dev is set) */
    int32_t precision;
    const int32_t *l_dev;       /* the sample's l_dev (nullable) */
} stba_rcs;

/* ---- set-up ------------------------------------------------------------ */

/* Size of the device scratch buffer stba_analyze needs (bytes, host, pure). */
size_t stba_analyze_scratch_bytes(void);

/* Check the observation arrays and measure the data-dependent sizes (Sec. 3's
 * visibility graph).  SYNCHRONISES `stream`.  d_scratch: device buffer of at
 * least stba_analyze_scratch_bytes().  dims (host) receives n_pairs and
 * max_track; dims->gamma_max is left untouched.  Returns STBA_EDATA if the
 * observations are unsorted, duplicated, out of range or a point is unseen. */
int stba_analyze(const stba_problem *p, void *d_scratch, stba_dims *dims, hipStream_t stream);

/* Workspace bytes for a problem, its dims (dims->gamma_max = largest cluster
 * that will be passed) and a precision.  Host, pure; 0 on bad arguments. */
size_t stba_workspace_bytes(const stba_problem *p, const stba_dims *dims, int precision);

/* Build the static plan in the workspace: per-point offsets and the list of
 * observation pairs (same point) grouped by camera pair, which is the sparsity
 * of E C^-1 E^T (Eq. 5).  Must be called once before the per-iteration calls;
 * asynchronous.  ws must be 256-byte aligned. */
int stba_prepare(const stba_problem *p, const stba_dims *dims, int precision, void *ws,
                 size_t ws_bytes, hipStream_t stream);

/* ---- per-iteration calls (all asynchronous, graph-capturable) ---------- */

/* Residuals f and Jacobian blocks J_c, J_p of every observation (Sec. 3, Alg. 1).
 * precision selects the element type of f, Jc, Jp (double or float).  Jc and Jp
 * may both be NULL (residuals only).  cost (nullable, device double) receives
 * F = sum ||f||^2 computed in FP64.  With p->huber = a > 0 (Sec. 5.1) f and J are
 * the IRLS-reweighted sqrt(rho'(s)) f, sqrt(rho'(s)) J of each observation
 * (s = ||f||^2 of the raw residual) and cost is F = sum rho(s); the later calls
 * then solve the reweighted problem.  Uses the workspace for partial sums. */
int stba_residual_jacobian(const stba_problem *p, const stba_dims *dims, int precision, void *f, void *Jc,
                           void *Jp, double *cost, void *ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): stba_residual_jacobian without a
 * workspace, dims or stba_prepare.  Same kernels and results (bit for bit) as
 * stba_residual_jacobian with the same arguments.  The cost's per-workgroup
 * partial sums go to a scratch array of 65536 doubles (512 KiB) that the
 * library keeps in device memory, one copy per GPU it runs on, held until the
 * process ends; nothing is allocated or freed by the call.  The first call on a
 * device looks that device's copy up (hipGetSymbolAddress) with the device
 * current.  Limits: with cost != NULL, q <= 2^24 (65536 partials of 256
 * observations), else STBA_EWORKSPACE before anything is enqueued; other
 * argument errors as stba_residual_jacobian.  Calls that overlap on one GPU
 * (other streams, or other host threads before the first call finishes) share
 * that GPU's scratch and race on the cost: serialise them. */
int stba_residual_jacobian_static(const stba_problem *p, int precision, void *f, void *Jc, void *Jp, double *cost,
                                  hipStream_t stream);

/* Assemble one reduced camera system per cluster (Eq. 10, 13; Alg. 1): draw the
 * sampled constraints as point segments, form the segment blocks C', E', the
 * corrected gradient when lambda >= lambda_corr (Sec. 4.3), then
 * S_k = B_k - E'_k C'^-1 E'_k^T (lower triangle, FP64 storage) and
 * b' = v' - E' C'^-1 w'.  f, Jc, Jp are the outputs of stba_residual_jacobian in
 * the same precision (in FP64 Jc must be 16-byte aligned: the assembly moves it
 * in 16-byte parts; STBA_EINVAL else).  out (host) receives views into the
 * workspace.  The per-point blocks needed by stba_solve_clusters are kept in
 * the workspace. */
int stba_build_cluster_rcs(const stba_problem *p, const stba_dims *dims, const stba_sample *s,
                           const stba_damping *d, int precision, const void *f, const void *Jc, const void *Jp,
                           stba_rcs *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Solve every S_k dc_k = b_k by dense FP64 Cholesky (Eq. 13; plus, in
 * STBA_MIXED, one FP64 refinement step whose residual is formed from J
 * recomputed in FP64 at x, with the damping and the segments of the last
 * stba_build_cluster_rcs), then the point step dp_j = C_j^-1 (w_j - sum_o W_o^T dc)
 * with the physical blocks (Eq. 15).
 * Jc, Jp: the Jacobian passed to stba_build_cluster_rcs.  dcam [m][9], dpt [n][3]
 * (device, FP64).  cluster_status (device int32 [l], nullable): STBA_OK or
 * STBA_ENOTPD per cluster, or STBA_EHIP if a wait between the wavefronts that
 * factor the cluster timed out (the step is then invalid; stba_lm_step rejects
 * it and records STBA_EHIP in the sticky status).  The factorisation overwrites
 * S in the workspace. */
int stba_solve_clusters(const stba_problem *p, const stba_dims *dims, const stba_rcs *rcs, int precision,
                        const void *Jc, const void *Jp, double *dcam, double *dpt,
                        int32_t *cluster_status, void *ws, size_t ws_bytes, hipStream_t stream);

/* The inexact alternative to stba_solve_clusters (App. A, Table 3): every
 * S_k dc_k = b_k by conjugate gradient with the camera-block Jacobi
 * preconditioner M = blockdiag(S_ii) (9 x 9 blocks), from dc_k = 0: q = S p,
 * alpha = r.z / p.q, dc += alpha p, r -= alpha q, stop once ||r|| <= tol ||b_k||
 * or after max_iters iterations, else z = M^-1 r, beta = (r.z)_new / (r.z)_old,
 * p = z + beta p.  The product visits only the 9 x 9 blocks of the camera pairs
 * the plan links, so an iteration costs O(r') in the sampled connections.  Then
 * the point step of Eq. 15 as in stba_solve_clusters.  Reads S and b as
 * stba_build_cluster_rcs left them (S is not modified, so stba_solve_clusters
 * may follow).  Runs in FP64 whatever the precision (which only selects the
 * type of Jc, Jp).
 *   max_iters >= 0; tol >= 0, finite (relative residual).
 *   cluster_iters (device int32 [l], nullable): iterations used per cluster.
 *   cluster_resid (device double [l], nullable): final ||r|| / ||b_k||.
 *   cluster_status (device int32 [l], nullable): STBA_OK, or STBA_ENOTPD when a
 *     camera block is not positive definite or p.q <= 0 (dc_k is then zero).
 * Requires the LDS of one cluster, 8 (5 Np + 9) + n^2 / 8 + 4 (n + 1) + 2 n^2
 * bytes for the largest padded order Np and dims->gamma_max = n, to fit 160 KB
 * (STBA_EINVAL else; n <= 200 fits). */
int stba_solve_clusters_pcg(const stba_problem *p, const stba_dims *dims, const stba_rcs *rcs, int precision,
                            const void *Jc, const void *Jp, double *dcam, double *dpt, int32_t max_iters, double tol,
                            int32_t *cluster_iters, double *cluster_resid, int32_t *cluster_status, void *ws,
                            size_t ws_bytes, hipStream_t stream);

/* Draw the camera clustering {Phi_k} of LM iteration `iter` by stochastic graph
 * clustering (Sec. 4.4, Eq. 16) on the device.  The camera graph weighs the
 * edge (i, j) by the number of points both cameras see (read from the plan of
 * stba_prepare).  From singletons, two neighbouring clusters x, y whose joint
 * size stays within gamma join with probability exp(beta dQ(x, y)) over the sum
 * of the same over all such pairs, dQ = w_xy / s - K_x K_y / (2 s^2) the
 * modularity gain (w_xy: weight between x and y, K: summed incident weight, s:
 * total weight); joining stops when no such pair is left.  The joins are drawn
 * by competing exponential clocks (same law): each eligible pair (a, b), a < b
 * the clusters' smallest cameras, holds T = t + E / exp(beta dQ) with E = -log u,
 * u = ((x0 >> 11) + 1) 2^-53 and x0 word 0 of Philox4x64-10 with key (seed, 2),
 * counter (iter, join step, a, b); the smallest T (ties: smaller (a, b)) joins,
 * and the pairs of the joined cluster draw new clocks with that join's step
 * number (the initial clocks are step 0, the first join step 1).
 *   gamma: size cap, 1 <= gamma <= dims->gamma_max (so the map can be passed to
 *     the per-iteration calls of this workspace); beta >= 0, finite.
 *   cam_cluster [m] (device int32): cluster of each camera, numbered 0..l-1 in
 *     order of each cluster's smallest camera.  n_clusters (device int32): l.
 *   status (device int32): STBA_OK once the map is written.
 * Requires p->m <= 6144 (the clustering runs in one workgroup whose LDS holds
 * 24 bytes per camera), dims->n_pairs < 2^31 (edge weights are 32-bit) and
 * stba_prepare.
 * Keeps its pair labels, clocks and weights in workspace buffers that only
 * stba_prepare otherwise uses (a later stba_prepare rewrites them);
 * asynchronous (one kernel).  A stba_sample can take the map as it stands on the
 * device: cam_cluster, l = m (the bound) and l_dev = n_clusters, with no
 * read-back, so the clustering and the LM step can be captured together. */
int stba_sample_clusters(const stba_problem *p, const stba_dims *dims, int precision, void *ws, size_t ws_bytes,
                         int32_t gamma, double beta, uint64_t seed, uint64_t iter, int32_t *cam_cluster,
                         int32_t *n_clusters, int32_t *status, hipStream_t stream);

/* Initialise a device stba_lm_state (lambda0, lambda_corr, need_jac = 1, lambda_min = 0). */
int stba_lm_init(stba_lm_state *st, double lambda0, double lambda_corr, hipStream_t stream);

/* One full STBA LM iteration (Alg. 1, one pass of the loop) for the given
 * cluster map: residuals/Jacobian (only when x changed), cluster RCS, solves,
 * point update, candidate cost, accept iff F(x+dx) < F(x) strictly, the step is
 * finite and every S_k factorised; then lambda = max(lambda / 3, lambda_min) and
 * x += dx, else lambda *= 3.
 * Every decision is taken on the device; no host synchronisation. */
int stba_lm_step(const stba_problem *p, const stba_dims *dims, const stba_sample *s, stba_lm_state *st,
                 int precision, void *ws, size_t ws_bytes, hipStream_t stream);

/* One LM iteration of many independent problems at once (Alg. 1 per problem):
 * p holds the problems concatenated, with n_prob (1 <= n_prob <= m) problems
 * whose cameras, points and observations lie in contiguous index ranges.
 *   states [n_prob] (device): one stba_lm_state per problem (stba_lm_init each);
 *     each problem keeps its own lambda, cost, accept decision and counters.
 *   prob_cam [m], prob_pt [n] (device int32): the problem of each camera / point.
 *   prob_obs_off [n_prob + 1] (device int64): problem b's observations are
 *     [prob_obs_off[b], prob_obs_off[b + 1]).
 * The cluster map must keep each cluster inside one problem, and each point's
 * observations must see cameras of the point's problem (checked on the device:
 * STBA_EINVAL in every state's status otherwise).  Per problem the step is the
 * one of stba_lm_step: its segments, point blocks and S_k blocks damped with
 * its own lambda, its cost at x and at x + dx summed over its observations in
 * a fixed order, accept iff F(x + dx) < F(x), finite and its clusters
 * factorised; x += dx for its cameras and points only.  f and J are evaluated
 * when any problem accepted its last step.  A non-positive-definite point
 * block, and a sticky data error, reject the step of every problem (they are
 * tracked for the batch as a whole).  Asynchronous, no host synchronisation;
 * errors as stba_lm_step (STBA_EINVAL also for null batch arrays or n_prob out
 * of range). */
int stba_lm_step_batched(const stba_problem *p, const stba_dims *dims, const stba_sample *s, stba_lm_state *states,
                         int32_t n_prob, const int32_t *prob_cam, const int32_t *prob_pt, const int64_t *prob_obs_off,
                         int precision, void *ws, size_t ws_bytes, hipStream_t stream);

/* Same as stba_lm_step, recording events[k] before phase k and events[STBA_NUM_PHASES]
 * after the last (host array of STBA_NUM_PHASES + 1 created hipEvent_t) so that a
 * caller can time each kernel of the iteration on `stream`. */
#define STBA_NUM_PHASES 10   /* clusters, residual_jacobian, points_segments, fill_S,
                                schur_assembly, cluster_cholesky, refinement (STBA_MIXED
                                only; empty otherwise), point_backsub, candidate_cost,
                                accept_update */
int stba_lm_step_profiled(const stba_problem *p, const stba_dims *dims, const stba_sample *s,
                          stba_lm_state *st, int precision, void *ws, size_t ws_bytes, hipStream_t stream,
                          hipEvent_t *events);

/* stba_lm_step with every cluster solve done by conjugate gradient as in
 * stba_solve_clusters_pcg (max_iters, tol as there; an inexact step, App. A);
 * a cluster reporting STBA_ENOTPD rejects the step as in stba_lm_step.  MIXED
 * skips the refinement step (the solve is FP64 and iterative). */
int stba_lm_step_pcg(const stba_problem *p, const stba_dims *dims, const stba_sample *s, stba_lm_state *st,
                     int precision, int32_t max_iters, double tol, void *ws, size_t ws_bytes, hipStream_t stream);

/* Name of phase k of stba_lm_step_profiled (static string, host). */
const char *stba_phase_name(int k);

/* ---- autotuning ---------------------------------------------------------- */

/* What stba_autotune measured (host struct).  Times in ms, the best of three
 * runs each; 0 where a candidate was not run (a form that does not fit). */
#define STBA_TUNE_SCHUR_CANDIDATES 6
typedef struct stba_tune_report {
    int32_t chol_form;                                 /* chosen */
    int32_t schur_blocks;                              /* chosen */
    float chol_ms[4];                                  /* by form: [STBA_CHOL_TILES .. STBA_CHOL_WORKGROUP] */
    int32_t schur_candidates[STBA_TUNE_SCHUR_CANDIDATES];
    float schur_ms[STBA_TUNE_SCHUR_CANDIDATES];        /* the assembly (cluster layout to b) per candidate */
} stba_tune_report;

/* Choose dims->chol_form and dims->schur_blocks for this problem and a
 * representative sample: the residual kernel fills the workspace's f and J,
 * then the assembly (stba_build_cluster_rcs) runs with each Schur workgroup
 * count and the cluster solves with each factorisation form that fits, each
 * timed with HIP events on `stream`; the fastest of each is written to dims.
 * A set-up call: it SYNCHRONISES the stream and creates (and destroys) HIP
 * events; x is not changed.  report (host, nullable) receives the times.
 * Errors as stba_build_cluster_rcs; STBA_EHIP if an event call fails. */
int stba_autotune(const stba_problem *p, stba_dims *dims, const stba_sample *s, const stba_damping *d,
                  int precision, void *ws, size_t ws_bytes, hipStream_t stream, stba_tune_report *report);

/* ---- differentiation (residuals as a differentiable function) ----------- */

/* J^T v for a cotangent v [q][2] of the residuals (FP32 or FP64 per precision):
 * grad_cam[m][9] = sum_o J_c,o^T v_o, grad_pt[n][3] = sum_o J_p,o^T v_o and
 * grad_uv[q][2] = -v_o.  J is recomputed from cam and pt (nothing stored); the
 * residuals differentiated are the raw ones (p->huber is not used).
 * Outputs are written (not accumulated) in the same precision as v; the per-camera
 * and per-point sums use fixed-order segmented reductions.  Requires stba_prepare. */
int stba_residual_vjp(const stba_problem *p, const stba_dims *dims, int precision, const void *v,
                      void *grad_cam, void *grad_pt, void *grad_uv, void *ws, size_t ws_bytes, hipStream_t stream);

/* The same products with J read instead of recomputed: Jc [q][18] and Jp
 * [q][6] (device, same precision as v, row-major as stba_residual_jacobian
 * writes them) must hold the blocks at the x of p (the caller keeps them from
 * the forward evaluation; the memory-for-time choice of the differentiable
 * residual).  Same sums in the same order as stba_residual_vjp (in FP64 the
 * two agree to rounding).  Errors as stba_residual_vjp (STBA_EINVAL also for a
 * null Jc or Jp). */
int stba_residual_vjp_stored(const stba_problem *p, const stba_dims *dims, int precision, const void *v,
                             const void *Jc, const void *Jp, void *grad_cam, void *grad_pt, void *grad_uv, void *ws,
                             size_t ws_bytes, hipStream_t stream);

/* Library version string (host). */
const char *stba_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STBA_H */
