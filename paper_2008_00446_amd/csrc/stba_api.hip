// C ABI of the STBA hot path: argument checks, the workspace layout and the
// order in which one LM iteration (Alg. 1) enqueues its kernels.
#include <math.h>
#include <cmath>
#include <mutex>
#include <stdlib.h>
#include <string.h>

#include "kernels.h"

namespace stba {
namespace {

struct Layout {
    size_t status, lam2;
    // static plan (stba_prepare)
    size_t pt_off, pair_off, scratch_a, keys_in, keys_out, vals_in, pairs, blk_of, blk_key, blk_start, n_blocks,
        diag_blk, blk_chunk_off, chunk_blk, n_chunks, part, vjp_part_off, vjp_part_cam, vjp_part_sum, vjp_obs_off,
        vjp_oj, tmp;
    int64_t blk_cap, chunk_cap, vjp_part_cap;
    size_t tmp_bytes;
    // per iteration
    size_t cl_n, cl_Np, cl_start, cl_cams, cam_local, cl_status, S_off;
    size_t pcg_clus, pcg_minv, pcg_iters, pcg_resid;
    size_t f, Jc, Jp, seg_head, seg_rec, grp_first, obsd, Vinv, wph, S, eref, rres, b, dcam, dpt, partials, chol_flags,
        chol_yx;
    size_t team_flags, team_vec, batch;
    int64_t team_abort_at, team_vec_len;
    bool refine = false;   // STBA_MIXED: eref and rres exist
    int64_t S_cap, n_partials;
    int32_t group_size;
    int32_t max_Np;
    size_t total;
};

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int check_problem(const stba_problem *p) {
    if (!p || p->m < 1 || p->n < 1 || p->q < 1 || p->q >= (int64_t(1) << 31)) return STBA_EINVAL;
    if (!p->cam || !p->pt || !p->obs_cam || !p->obs_pt || !p->obs_uv) return STBA_EINVAL;
    if (p->m > kMaxCamsForClusters) return STBA_EINVAL;
    if (!(p->huber >= 0.0) || !std::isfinite(p->huber)) return STBA_EINVAL;
    return STBA_OK;
}

int check_dims(const stba_problem *p, const stba_dims *d) {
    if (!d || d->n_pairs < p->n || d->n_pairs < p->q || d->gamma_max < 1 || d->gamma_max > p->m)
        return STBA_EINVAL;
    if (d->max_track < 1 || d->max_track > p->q) return STBA_EINVAL;
    if (d->chol_form < STBA_CHOL_AUTO || d->chol_form > STBA_CHOL_WORKGROUP) return STBA_EINVAL;
    if (d->schur_blocks != 0 && (d->schur_blocks < 8 || d->schur_blocks > 65536)) return STBA_EINVAL;
    return STBA_OK;
}

int check_precision(int precision) {
    return (precision == STBA_FP64 || precision == STBA_MIXED || precision == STBA_MIXED_NOREFINE) ? STBA_OK
                                                                                                     : STBA_EINVAL;
}

int check_sample(const stba_problem *p, const stba_sample *s) {
    if (!s || !s->cam_cluster || s->l < 1 || s->l > p->m) return STBA_EINVAL;
    if (!(s->alpha > 0.0 && s->alpha <= 1.0)) return STBA_EINVAL;
    return STBA_OK;
}

// Largest sum of padded S_k sizes over any map with clusters of at most gamma
// cameras: sum_k Np(n_k)^2 = sum_k n_k (Np(n_k)^2 / n_k) <= m max_n Np(n)^2 / n.
int64_t s_capacity(int32_t m, int32_t gamma) {
    double best = 0.0;
    for (int32_t nk = 1; nk <= gamma; ++nk) {
        const double np = (double)round_up(9 * (int64_t)nk, kNB);
        best = fmax(best, np * np / nk);
    }
    return (int64_t)ceil(best * m);
}

bool make_layout(const stba_problem *p, const stba_dims *d, int precision, Layout &L) {
    const size_t es = precision == STBA_FP64 ? sizeof(double) : sizeof(float);
    const size_t m = (size_t)p->m, n = (size_t)p->n, q = (size_t)p->q, np = (size_t)d->n_pairs;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + (bytes ? bytes : 1));
        return o;
    };
    L.status = take(sizeof(int32_t) * kStCount);
    L.lam2 = take(2 * sizeof(double));
    L.pt_off = take(8 * (n + 1));
    L.pair_off = take(8 * (n + 1));
    // scratch_a, keys_in and vals_in serve stba_prepare only; afterwards the
    // device camera clustering keeps its pair labels, clocks and weights there
    L.scratch_a = take(8 * np);
    L.keys_in = take(8 * (np + 1));
    L.keys_out = take(8 * np);
    L.vals_in = take(8 * (np + 1));
    L.pairs = take(8 * np);
    L.blk_of = take(8 * np);
    L.blk_key = take(8 * np);
    L.blk_start = take(8 * (np + 1));
    L.n_blocks = take(8);
    L.diag_blk = take(8 * m);
    // blocks are camera pairs (r, c), r >= c, with at least one pair each
    L.blk_cap = (int64_t)np;
    if ((int64_t)m * ((int64_t)m + 1) / 2 < L.blk_cap) L.blk_cap = (int64_t)m * ((int64_t)m + 1) / 2;
    // a block of len pairs has ceil(len / chunk) <= 1 + len / chunk chunks
    L.chunk_cap = L.blk_cap + (int64_t)np / kSchurChunk + 1;
    L.blk_chunk_off = take(8 * (size_t)(L.blk_cap + 1));
    L.chunk_blk = take(4 * (size_t)L.chunk_cap);
    L.n_chunks = take(8);
    L.part = take(8 * (size_t)kSchurPart * (size_t)L.chunk_cap);
    // camera parts of the J^T v sums: ceil(len / kVjpPart) <= 1 + len / kVjpPart per camera
    L.vjp_part_cap = (int64_t)m + (int64_t)np / kVjpPart + 1;
    L.vjp_part_off = take(8 * (m + 1));
    L.vjp_part_cam = take(4 * (size_t)L.vjp_part_cap);
    L.vjp_part_sum = take(8 * 18 * (size_t)L.vjp_part_cap);
    L.vjp_obs_off = take(8 * (m + 1));
    L.vjp_oj = take(8 * q);
    L.tmp_bytes = prepare_tmp_bytes(d->n_pairs, p->m, 0);
    L.tmp = take(L.tmp_bytes);
    L.cl_n = take(4 * m);
    L.cl_Np = take(4 * m);
    L.cl_start = take(4 * (m + 1));
    L.cl_cams = take(4 * m);
    L.cam_local = take(4 * m);
    L.cl_status = take(4 * m);
    L.S_off = take(8 * (m + 1));
    L.pcg_clus = take(4 * m);
    L.pcg_minv = take(8 * 81 * m);
    L.pcg_iters = take(4 * m);
    L.pcg_resid = take(8 * m);
    L.f = take(es * 2 * q);
    L.Jc = take(es * 18 * q);
    L.Jp = take(es * 6 * q);
    L.seg_head = take(4 * q);
    L.chol_flags = take(4 * (size_t)chol_flag_words());
    L.chol_yx = take(8 * (size_t)chol_yx_doubles());
    L.grp_first = take(4 * (q + 2));
    L.group_size = point_group_size(d->max_track);
    // the staged segment records are used only when the one-lane-per-observation path is off
    L.seg_rec = take(L.group_size > 0 ? 8 : 8 * (size_t)kSegRec * q);
    L.obsd = take(obs_rec_bytes(precision == STBA_FP64) * q);
    L.Vinv = take(8 * 6 * n);
    L.wph = take(8 * 3 * n);
    L.max_Np = (int32_t)round_up(9 * (int64_t)d->gamma_max, kNB);
    L.S_cap = s_capacity(p->m, d->gamma_max);
    L.S = take(8 * (size_t)L.S_cap);
    // batched LM: the costs at x and at x + dx and a scratch word per problem (at most m problems), and a flag
    L.batch = take(8 * 2 * m + 4 * m + 4);
    // flags and block vectors of the team factorisation (many clusters)
    L.team_abort_at = chol_team_flag_words(L.S_cap, p->m) - 3;
    L.team_flags = take(4 * (size_t)(L.team_abort_at + 3));
    L.team_vec_len = chol_team_vec_len(L.S_cap);
    L.team_vec = take(8 * 4 * (size_t)L.team_vec_len);
    // MIXED's refinement step: linearised residuals per observation, residual per camera
    L.refine = precision == STBA_MIXED;
    L.eref = L.refine ? take(8 * 2 * q) : 0;
    L.rres = L.refine ? take(8 * 9 * m) : 0;
    L.b = take(8 * 9 * m);
    L.dcam = take(8 * 9 * m);
    L.dpt = take(8 * 3 * n);
    L.n_partials = rj_blocks(p->q);
    // residual partials, candidate-cost partials, F(x) and have_F before the accept decision
    L.partials = take(8 * (2 * (size_t)L.n_partials + 2));
    L.total = off;
    return true;
}

template <typename P>
P *at(void *ws, size_t off) {
    return reinterpret_cast<P *>(static_cast<char *>(ws) + off);
}

int check_ws(const Layout &L, void *ws, size_t bytes) {
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return STBA_EINVAL;
    if (bytes < L.total) return STBA_EWORKSPACE;
    return STBA_OK;
}

#define STBA_TRY(expr)                          \
    do {                                        \
        const int _rc = (expr);                 \
        if (_rc != STBA_OK) return _rc;         \
    } while (0)

#define STBA_HIP(expr)                          \
    do {                                        \
        if ((expr) != hipSuccess) return STBA_EHIP; \
    } while (0)

uint64_t keep_threshold(double alpha) { return (uint64_t)ceil(alpha * 9007199254740992.0); }

// Common front end of every per-iteration call.
int front(const stba_problem *p, const stba_dims *d, int precision, void *ws, size_t ws_bytes, Layout &L) {
    STBA_TRY(check_problem(p));
    STBA_TRY(check_dims(p, d));
    STBA_TRY(check_precision(precision));
    make_layout(p, d, precision, L);
    return check_ws(L, ws, ws_bytes);
}

SchurChunks chunks_of(const Layout &L, void *ws, const stba_sample *s, const stba_dims *d) {
    SchurChunks c;
    c.all_links = s->alpha >= 1.0 ? 1 : 0;
    c.n_chunks = at<int64_t>(ws, L.n_chunks);
    c.blk_chunk_off = at<int64_t>(ws, L.blk_chunk_off);
    c.chunk_blk = at<int32_t>(ws, L.chunk_blk);
    c.chunk_cap = L.chunk_cap;
    c.part = at<double>(ws, L.part);
    c.blocks = d->schur_blocks;
    return c;
}

template <typename T>
int build_rcs_impl(const stba_problem *p, const stba_dims *d, const stba_sample *s, const double *lam2,
                   const T *f, const T *Jc, const T *Jp, const Layout &L, void *ws, hipStream_t st) {
    int32_t *status = at<int32_t>(ws, L.status);
    STBA_HIP(launch_clusters(s->cam_cluster, p->m, s->l, s->l_dev, d->gamma_max, at<int32_t>(ws, L.cl_n),
                             at<int32_t>(ws, L.cl_Np), at<int32_t>(ws, L.cl_start), at<int32_t>(ws, L.cl_cams),
                             at<int32_t>(ws, L.cam_local), at<int64_t>(ws, L.S_off), at<int32_t>(ws, L.cl_status),
                             status, st));
    STBA_HIP(launch_points<T>(*p, at<int64_t>(ws, L.pt_off), s->cam_cluster, s->l, f, Jc, Jp, lam2, s->seed, s->iter,
                              keep_threshold(s->alpha), at<int32_t>(ws, L.seg_head), at<double>(ws, L.seg_rec), at<T>(ws, L.obsd),
                              at<double>(ws, L.Vinv), at<double>(ws, L.wph), status, L.group_size,
                              at<int32_t>(ws, L.grp_first), st));
    STBA_HIP(launch_fill_S(at<double>(ws, L.S), at<double>(ws, L.b), p->m, at<int64_t>(ws, L.S_off), s->l, L.S_cap,
                           st));
    STBA_HIP(launch_schur<T>(at<int64_t>(ws, L.n_blocks), L.blk_cap, chunks_of(L, ws, s, d), at<int2>(ws, L.blk_key),
                             at<int64_t>(ws, L.blk_start), at<uint64_t>(ws, L.pairs), s->cam_cluster, s->l,
                             at<int32_t>(ws, L.cam_local), at<int32_t>(ws, L.cl_n), at<int32_t>(ws, L.cl_Np),
                             at<int64_t>(ws, L.S_off),
                             at<int32_t>(ws, L.seg_head), Jc, at<T>(ws, L.obsd), lam2, at<double>(ws, L.S),
                             at<double>(ws, L.b), st));
    return STBA_OK;
}

// The camera parts stba_prepare left for the J^T v camera sums.
VjpParts vjp_parts_of(const Layout &L, void *ws) {
    VjpParts v;
    v.off = at<int64_t>(ws, L.vjp_part_off);
    v.cam = at<int32_t>(ws, L.vjp_part_cam);
    v.cap = L.vjp_part_cap;
    v.sum = at<double>(ws, L.vjp_part_sum);
    v.obs_off = at<int64_t>(ws, L.vjp_obs_off);
    v.oj = at<int2>(ws, L.vjp_oj);
    return v;
}

CholTeam team_of(const Layout &L, void *ws, const stba_dims *d) {
    CholTeam t;
    t.flags = at<int32_t>(ws, L.team_flags);
    t.abort_at = L.team_abort_at;
    t.vec = at<double>(ws, L.team_vec);
    t.vec_len = L.team_vec_len;
    t.form = d != nullptr ? d->chol_form : STBA_CHOL_AUTO;
    return t;
}

// The cluster solves of Eq. 13 (FP64 Cholesky of every S_k).
int cluster_solve(const stba_dims *d, int32_t l, bool l_on_device, double *dcam, int32_t *cl_status, const Layout &L,
                  void *ws, hipStream_t st) {
    CholTeam team = team_of(L, ws, d);
    team.l_on_device = l_on_device;
    STBA_HIP(launch_chol(l, at<int32_t>(ws, L.cl_n), at<int32_t>(ws, L.cl_Np), at<int64_t>(ws, L.S_off),
                         at<int32_t>(ws, L.cl_start), at<int32_t>(ws, L.cl_cams), at<double>(ws, L.S),
                         at<double>(ws, L.b), dcam, cl_status, L.max_Np, at<int32_t>(ws, L.chol_flags),
                         at<double>(ws, L.chol_yx), &team, st));
    return STBA_OK;
}

// MIXED: one FP64 refinement step of every cluster solve, dcam += S_k^-1 (b - S x)
// with the residual of the FP64 method's S and b (J recomputed in FP64 at x)
// and the factors of the FP32-assembled S_k.
int refine_solve(const stba_problem *p, int32_t l, const Damp &dm, double *dcam, const Layout &L, void *ws,
                 hipStream_t st) {
    double *r = at<double>(ws, L.rres);
    STBA_HIP(launch_refine_residual(*p, at<int64_t>(ws, L.pt_off), at<int32_t>(ws, L.seg_head), L.group_size,
                                    at<int32_t>(ws, L.grp_first), dm, dcam, at<double>(ws, L.eref),
                                    at<double>(ws, L.Vinv), at<double>(ws, L.wph), at<int64_t>(ws, L.diag_blk),
                                    at<int64_t>(ws, L.blk_start), vjp_parts_of(L, ws), r, st));
    STBA_HIP(launch_sweep(l, at<int32_t>(ws, L.cl_n), at<int32_t>(ws, L.cl_Np), at<int64_t>(ws, L.S_off),
                          at<int32_t>(ws, L.cl_start), at<int32_t>(ws, L.cl_cams), at<double>(ws, L.S), r, dcam,
                          L.max_Np, st));
    return STBA_OK;
}

template <typename T>
int solve_impl(const stba_problem *p, const stba_dims *d, int32_t l, bool l_on_device, const T *Jc, const T *Jp,
               double *dcam, double *dpt, int32_t *cl_status, const Layout &L, void *ws, hipStream_t st) {
    STBA_TRY(cluster_solve(d, l, l_on_device, dcam, cl_status, L, ws, st));
    if (L.refine) STBA_TRY(refine_solve(p, l, at<double>(ws, L.lam2), dcam, L, ws, st));
    STBA_HIP(launch_backsub<T>(*p, at<int64_t>(ws, L.pt_off), Jc, Jp, at<double>(ws, L.Vinv), at<double>(ws, L.wph),
                               dcam, dpt, L.group_size, at<int32_t>(ws, L.grp_first), L.refine, st));
    return STBA_OK;
}

// Autotuning: best of three event-timed runs of the assembly for each Schur
// workgroup count and of the cluster solves for each factorisation form.
constexpr int32_t kSchurCandidates[STBA_TUNE_SCHUR_CANDIDATES] = {1024, 2048, 4096, 8192, 16384, 32768};

template <typename T>
int autotune_impl(const stba_problem *p, stba_dims *dims, const stba_sample *s, const Layout &L, void *ws,
                  hipStream_t st, stba_tune_report *rep) {
    T *f = at<T>(ws, L.f), *Jc = at<T>(ws, L.Jc), *Jp = at<T>(ws, L.Jp);
    const double *lam2 = at<double>(ws, L.lam2);
    STBA_HIP(launch_rj<T>(*p, f, Jc, Jp, nullptr, nullptr, nullptr, ZeroS(), st));
    hipEvent_t e[2];
    if (hipEventCreate(&e[0]) != hipSuccess) return STBA_EHIP;
    if (hipEventCreate(&e[1]) != hipSuccess) {
        (void)hipEventDestroy(e[0]);
        return STBA_EHIP;
    }
    int rc = STBA_OK;
    // best of three runs of fn (with prep before each run, untimed)
    auto best_ms = [&](auto &&prep, auto &&fn, float *out) -> int {
        float best = 0.0f;
        for (int r = 0; r < 3; ++r) {
            STBA_TRY(prep());
            if (hipEventRecord(e[0], st) != hipSuccess) return STBA_EHIP;
            STBA_TRY(fn());
            if (hipEventRecord(e[1], st) != hipSuccess || hipEventSynchronize(e[1]) != hipSuccess) return STBA_EHIP;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e[0], e[1]) != hipSuccess) return STBA_EHIP;
            if (r == 0 || ms < best) best = ms;
        }
        *out = best;
        return STBA_OK;
    };
    auto nothing = []() -> int { return STBA_OK; };
    stba_dims trial = *dims;
    auto build = [&]() -> int { return build_rcs_impl<T>(p, &trial, s, lam2, f, Jc, Jp, L, ws, st); };
    int32_t best_blocks = 0;
    float best = 0.0f;
    for (int i = 0; i < STBA_TUNE_SCHUR_CANDIDATES && rc == STBA_OK; ++i) {
        trial.schur_blocks = kSchurCandidates[i];
        rep->schur_candidates[i] = kSchurCandidates[i];
        rc = best_ms(nothing, build, &rep->schur_ms[i]);
        if (rc == STBA_OK && (best_blocks == 0 || rep->schur_ms[i] < best)) {
            best = rep->schur_ms[i];
            best_blocks = kSchurCandidates[i];
        }
    }
    trial.schur_blocks = best_blocks;
    CholTeam team = team_of(L, ws, &trial);
    team.l_on_device = s->l_dev != nullptr;
    int32_t best_form = STBA_CHOL_AUTO;
    double *dcam = at<double>(ws, L.dcam);
    for (int32_t form = STBA_CHOL_TILES; form <= STBA_CHOL_WORKGROUP && rc == STBA_OK; ++form) {
        rep->chol_ms[form - 1] = 0.0f;
        if (!chol_form_fits(form, s->l, L.max_Np, team.l_on_device, &team)) continue;
        trial.chol_form = form;
        auto solve = [&]() -> int {
            return cluster_solve(&trial, s->l, team.l_on_device, dcam, at<int32_t>(ws, L.cl_status), L, ws, st);
        };
        rc = best_ms(build, solve, &rep->chol_ms[form - 1]);   // the factorisation overwrites S: build first
        if (rc == STBA_OK && (best_form == STBA_CHOL_AUTO || rep->chol_ms[form - 1] < best)) {
            best = rep->chol_ms[form - 1];
            best_form = form;
        }
    }
    (void)hipEventDestroy(e[0]);
    (void)hipEventDestroy(e[1]);
    if (rc != STBA_OK) return rc;
    dims->schur_blocks = best_blocks;
    dims->chol_form = best_form;
    rep->schur_blocks = best_blocks;
    rep->chol_form = best_form;
    return STBA_OK;
}

// Cluster solves by conjugate gradient instead of Cholesky (App. A).
struct PcgOpts {
    int32_t max_iters;
    double tol;
};

template <typename T>
int lm_step_impl(const stba_problem *p, const stba_dims *d, const stba_sample *s, stba_lm_state *stt,
                 const Layout &L, void *ws, hipStream_t st, hipEvent_t *ev, const PcgOpts *pcg = nullptr) {
    int32_t *status = at<int32_t>(ws, L.status);
    const double *lam2 = &stt->lambda;   // lambda and lambda_corr are adjacent
    T *f = at<T>(ws, L.f), *Jc = at<T>(ws, L.Jc), *Jp = at<T>(ws, L.Jp);
    auto mark = [&](int k) -> int {
        if (ev) STBA_HIP(hipEventRecord(ev[k], st));
        return STBA_OK;
    };
    STBA_TRY(mark(0));
    STBA_HIP(launch_clusters(s->cam_cluster, p->m, s->l, s->l_dev, d->gamma_max, at<int32_t>(ws, L.cl_n),
                             at<int32_t>(ws, L.cl_Np), at<int32_t>(ws, L.cl_start), at<int32_t>(ws, L.cl_cams),
                             at<int32_t>(ws, L.cam_local), at<int64_t>(ws, L.S_off), at<int32_t>(ws, L.cl_status),
                             status, st));
    STBA_TRY(mark(1));
    ZeroS z;   // S and b are zeroed by the residual kernel's grid
    z.S = at<double>(ws, L.S);
    z.S_off = at<int64_t>(ws, L.S_off);
    z.l = s->l;
    z.S_cap = L.S_cap;
    z.b = at<double>(ws, L.b);
    z.nb = 9 * (int64_t)p->m;
    STBA_HIP(launch_rj<T>(*p, f, Jc, Jp, at<double>(ws, L.partials), &stt->need_jac, status + kStJacRan, z, st));
    STBA_TRY(mark(2));
    STBA_HIP(launch_points<T>(*p, at<int64_t>(ws, L.pt_off), s->cam_cluster, s->l, f, Jc, Jp, lam2, s->seed, s->iter,
                              keep_threshold(s->alpha), at<int32_t>(ws, L.seg_head), at<double>(ws, L.seg_rec), at<T>(ws, L.obsd),
                              at<double>(ws, L.Vinv), at<double>(ws, L.wph), status, L.group_size,
                              at<int32_t>(ws, L.grp_first), st));
    STBA_TRY(mark(3));
    STBA_TRY(mark(4));   // S was zeroed with the residuals: nothing between the marks
    STBA_HIP(launch_schur<T>(at<int64_t>(ws, L.n_blocks), L.blk_cap, chunks_of(L, ws, s, d), at<int2>(ws, L.blk_key),
                             at<int64_t>(ws, L.blk_start), at<uint64_t>(ws, L.pairs), s->cam_cluster, s->l,
                             at<int32_t>(ws, L.cam_local), at<int32_t>(ws, L.cl_n), at<int32_t>(ws, L.cl_Np),
                             at<int64_t>(ws, L.S_off),
                             at<int32_t>(ws, L.seg_head), Jc, at<T>(ws, L.obsd), lam2, at<double>(ws, L.S),
                             at<double>(ws, L.b), st));
    STBA_TRY(mark(5));
    double *dcam = at<double>(ws, L.dcam), *dpt = at<double>(ws, L.dpt);
    if (pcg)
        STBA_HIP(launch_pcg(s->l, at<int32_t>(ws, L.cl_n), at<int32_t>(ws, L.cl_Np), at<int64_t>(ws, L.S_off),
                            at<int32_t>(ws, L.cl_start), at<int32_t>(ws, L.cl_cams), at<int32_t>(ws, L.cam_local),
                            at<int64_t>(ws, L.n_blocks), at<int2>(ws, L.blk_key), at<double>(ws, L.S),
                            at<double>(ws, L.b), dcam, at<int32_t>(ws, L.pcg_clus), at<double>(ws, L.pcg_minv),
                            L.max_Np, d->gamma_max, pcg->max_iters, pcg->tol, at<int32_t>(ws, L.pcg_iters),
                            at<double>(ws, L.pcg_resid), at<int32_t>(ws, L.cl_status), st));
    else
        STBA_TRY(cluster_solve(d, s->l, s->l_dev != nullptr, dcam, at<int32_t>(ws, L.cl_status), L, ws, st));
    STBA_TRY(mark(6));
    // the conjugate-gradient solves take no refinement step (FP64 and iterative)
    const bool refine = L.refine && pcg == nullptr;
    if (refine) STBA_TRY(refine_solve(p, s->l, lam2, dcam, L, ws, st));
    STBA_TRY(mark(7));
    // The point update takes J in FP64 at x: recomputed from x (48 bytes per
    // observation in) rather than read (200 bytes per observation in FP64).  x
    // is where the residual kernel last evaluated J, so in FP64 the two agree.
    const bool fp64_j = refine || sizeof(T) == sizeof(double);
    STBA_HIP(launch_backsub<T>(*p, at<int64_t>(ws, L.pt_off), Jc, Jp, at<double>(ws, L.Vinv), at<double>(ws, L.wph),
                               dcam, dpt, L.group_size, at<int32_t>(ws, L.grp_first), fp64_j, st));
    STBA_TRY(mark(8));
    double *rj_part = at<double>(ws, L.partials), *cost_part = rj_part + L.n_partials;
    double *F_ref = cost_part + L.n_partials;
    STBA_HIP(launch_cost_at(*p, dcam, dpt, cost_part, stt, F_ref, st));
    STBA_TRY(mark(9));
    STBA_HIP(launch_accept_update(*p, rj_part, cost_part, L.n_partials, F_ref, at<int32_t>(ws, L.cl_status), s->l,
                                  status, stt, dcam, dpt, st));
    STBA_TRY(mark(10));
    return STBA_OK;
}

// One LM step of many problems at once (see stba_lm_step_batched): the
// iteration of lm_step_impl with each problem's damping (Damp over the states'
// lambda and lambda_corr, stba_lm_state apart), f and J evaluated when any
// problem needs them, the cost of each problem summed over its observation
// range, and the decisions taken per problem.
template <typename T>
int lm_step_batched_impl(const stba_problem *p, const stba_dims *d, const stba_sample *s, stba_lm_state *states,
                         int32_t n_prob, const int32_t *prob_cam, const int32_t *prob_pt, const int64_t *obs_off,
                         const Layout &L, void *ws, hipStream_t st) {
    int32_t *status = at<int32_t>(ws, L.status);
    Damp dm;
    dm.lam2 = &states[0].lambda;
    dm.prob_cam = prob_cam;
    dm.prob_pt = prob_pt;
    dm.stride = (int64_t)(sizeof(stba_lm_state) / sizeof(double));
    T *f = at<T>(ws, L.f), *Jc = at<T>(ws, L.Jc), *Jp = at<T>(ws, L.Jp);
    double *F_x = at<double>(ws, L.batch), *F_c = F_x + p->m;
    int32_t *bad = reinterpret_cast<int32_t *>(F_c + p->m), *need = bad + p->m;
    STBA_HIP(launch_clusters(s->cam_cluster, p->m, s->l, s->l_dev, d->gamma_max, at<int32_t>(ws, L.cl_n),
                             at<int32_t>(ws, L.cl_Np), at<int32_t>(ws, L.cl_start), at<int32_t>(ws, L.cl_cams),
                             at<int32_t>(ws, L.cam_local), at<int64_t>(ws, L.S_off), at<int32_t>(ws, L.cl_status),
                             status, st));
    ZeroS z;
    z.S = at<double>(ws, L.S);
    z.S_off = at<int64_t>(ws, L.S_off);
    z.l = s->l;
    z.S_cap = L.S_cap;
    z.b = at<double>(ws, L.b);
    z.nb = 9 * (int64_t)p->m;
    STBA_HIP(launch_batch_need_jac(n_prob, states, need, st));
    STBA_HIP(launch_rj<T>(*p, f, Jc, Jp, at<double>(ws, L.partials), need, status + kStJacRan, z, st));
    STBA_HIP(launch_points<T>(*p, at<int64_t>(ws, L.pt_off), s->cam_cluster, s->l, f, Jc, Jp, dm, s->seed, s->iter,
                              keep_threshold(s->alpha), at<int32_t>(ws, L.seg_head), at<double>(ws, L.seg_rec),
                              at<T>(ws, L.obsd), at<double>(ws, L.Vinv), at<double>(ws, L.wph), status, L.group_size,
                              at<int32_t>(ws, L.grp_first), st));
    STBA_HIP(launch_schur<T>(at<int64_t>(ws, L.n_blocks), L.blk_cap, chunks_of(L, ws, s, d), at<int2>(ws, L.blk_key),
                             at<int64_t>(ws, L.blk_start), at<uint64_t>(ws, L.pairs), s->cam_cluster, s->l,
                             at<int32_t>(ws, L.cam_local), at<int32_t>(ws, L.cl_n), at<int32_t>(ws, L.cl_Np),
                             at<int64_t>(ws, L.S_off), at<int32_t>(ws, L.seg_head), Jc, at<T>(ws, L.obsd), dm,
                             at<double>(ws, L.S), at<double>(ws, L.b), st));
    double *dcam = at<double>(ws, L.dcam), *dpt = at<double>(ws, L.dpt);
    STBA_TRY(cluster_solve(d, s->l, s->l_dev != nullptr, dcam, at<int32_t>(ws, L.cl_status), L, ws, st));
    if (L.refine) STBA_TRY(refine_solve(p, s->l, dm, dcam, L, ws, st));
    const bool fp64_j = L.refine || sizeof(T) == sizeof(double);
    STBA_HIP(launch_backsub<T>(*p, at<int64_t>(ws, L.pt_off), Jc, Jp, at<double>(ws, L.Vinv), at<double>(ws, L.wph),
                               dcam, dpt, L.group_size, at<int32_t>(ws, L.grp_first), fp64_j, st));
    STBA_HIP(launch_cost_problems(*p, n_prob, obs_off, prob_cam, prob_pt, nullptr, nullptr, F_x, status, st));
    STBA_HIP(launch_cost_problems(*p, n_prob, obs_off, prob_cam, prob_pt, dcam, dpt, F_c, status, st));
    STBA_HIP(launch_batch_accept(*p, n_prob, s->l, at<int32_t>(ws, L.cl_start), at<int32_t>(ws, L.cl_cams),
                                 at<int32_t>(ws, L.cl_status), prob_cam, prob_pt, F_x, F_c, bad, status, states, dcam,
                                 dpt, st));
    return STBA_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the entry point that allocates nothing (stba_residual_jacobian_static):
// the per-workgroup cost partials of the residual kernel, one double per 256
// observations, in a file-scope device array of kStaticPartials entries that
// every GPU the library runs on holds until the process ends.  Host code never
// uses the array's name as an address: each device's copy is found once, with
// that device current, by hipGetSymbolAddress, and that pointer is what the
// kernels are given.
// ---------------------------------------------------------------------------
constexpr int64_t kStaticPartials = 65536;           // 512 KiB: up to 2^24 observations
constexpr int kStaticMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticPartials];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kStaticMaxDevices] = {};

// This device's copy of `scratch` (found on the first call on the device).
int static_scratch(double **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return STBA_EHIP;
    if (dev < 0 || dev >= kStaticMaxDevices) return STBA_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return STBA_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<double *>(g_scratch_ptr[dev]);
    return STBA_OK;
}

const char *const kPhaseNames[STBA_NUM_PHASES] = {
    "clusters", "residual_jacobian", "points_segments", "fill_S", "schur_assembly",
    "cluster_cholesky", "refinement", "point_backsub", "candidate_cost", "accept_update"};

}  // namespace
}  // namespace stba

using namespace stba;

extern "C" {

const char *stba_version(void) { return "stba-gfx950 0.1"; }

const char *stba_phase_name(int k) { return (k >= 0 && k < STBA_NUM_PHASES) ? kPhaseNames[k] : ""; }

size_t stba_analyze_scratch_bytes(void) { return 64; }

int stba_analyze(const stba_problem *p, void *d_scratch, stba_dims *dims, hipStream_t stream) {
    STBA_TRY(check_problem(p));
    if (!d_scratch || !dims) return STBA_EINVAL;
    STBA_HIP(launch_analyze(*p, static_cast<int64_t *>(d_scratch), stream));
    int64_t h[4] = {0, 0, 0, 0};
    STBA_HIP(hipMemcpyAsync(h, d_scratch, sizeof(h), hipMemcpyDeviceToHost, stream));
    STBA_HIP(hipStreamSynchronize(stream));
    if (h[2] != 0) return STBA_EDATA;
    dims->n_pairs = h[0];
    dims->max_track = (int32_t)h[1];
    dims->chol_form = STBA_CHOL_AUTO;
    dims->schur_blocks = 0;
    return STBA_OK;
}

size_t stba_workspace_bytes(const stba_problem *p, const stba_dims *dims, int precision) {
    if (check_problem(p) != STBA_OK || check_dims(p, dims) != STBA_OK || check_precision(precision) != STBA_OK)
        return 0;
    Layout L;
    make_layout(p, dims, precision, L);
    return L.total;
}

int stba_prepare(const stba_problem *p, const stba_dims *dims, int precision, void *ws, size_t ws_bytes,
                 hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    PrepBufs b;
    b.pt_off = at<int64_t>(ws, L.pt_off);
    b.pair_off = at<int64_t>(ws, L.pair_off);
    b.scratch_a = at<int64_t>(ws, L.scratch_a);
    b.keys_in = at<uint64_t>(ws, L.keys_in);
    b.keys_out = at<uint64_t>(ws, L.keys_out);
    b.vals_in = at<uint64_t>(ws, L.vals_in);
    b.pairs = at<uint64_t>(ws, L.pairs);
    b.blk_of = at<int64_t>(ws, L.blk_of);
    b.blk_key = at<int2>(ws, L.blk_key);
    b.blk_start = at<int64_t>(ws, L.blk_start);
    b.n_blocks = at<int64_t>(ws, L.n_blocks);
    b.diag_blk = at<int64_t>(ws, L.diag_blk);
    b.blk_chunk_off = at<int64_t>(ws, L.blk_chunk_off);
    b.blk_cap = L.blk_cap;
    b.chunk_blk = at<int32_t>(ws, L.chunk_blk);
    b.chunk_cap = L.chunk_cap;
    b.n_chunks = at<int64_t>(ws, L.n_chunks);
    b.vjp_part_off = at<int64_t>(ws, L.vjp_part_off);
    b.vjp_part_cam = at<int32_t>(ws, L.vjp_part_cam);
    b.vjp_part_cap = L.vjp_part_cap;
    b.vjp_obs_off = at<int64_t>(ws, L.vjp_obs_off);
    b.vjp_oj = at<int2>(ws, L.vjp_oj);
    b.tmp = at<void>(ws, L.tmp);
    b.tmp_bytes = L.tmp_bytes;
    STBA_HIP(launch_reset_status(at<int32_t>(ws, L.status), stream));
    STBA_HIP(launch_prepare(*p, dims->n_pairs, b, at<int32_t>(ws, L.status), stream));
    const CholTeam team = team_of(L, ws, dims);
    STBA_HIP(launch_clear_chol_flags(at<int32_t>(ws, L.chol_flags), at<double>(ws, L.chol_yx), &team, stream));
    if (L.group_size > 0)
        STBA_HIP(launch_point_groups(p->n, b.pt_off, L.group_size, (p->q + L.group_size - 1) / L.group_size,
                                     at<int32_t>(ws, L.grp_first), stream));
    return STBA_OK;
}

int stba_residual_jacobian(const stba_problem *p, const stba_dims *dims, int precision, void *f, void *Jc, void *Jp,
                           double *cost, void *ws, size_t ws_bytes, hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    if (!f || ((Jc == nullptr) != (Jp == nullptr))) return STBA_EINVAL;
    double *partials = cost ? at<double>(ws, L.partials) : nullptr;
    if (precision == STBA_FP64)
        STBA_HIP(launch_rj<double>(*p, (double *)f, (double *)Jc, (double *)Jp, partials, nullptr, nullptr, ZeroS(),
                                   stream));
    else
        STBA_HIP(launch_rj<float>(*p, (float *)f, (float *)Jc, (float *)Jp, partials, nullptr, nullptr, ZeroS(),
                                  stream));
    if (cost) STBA_HIP(launch_sum_partials(partials, L.n_partials, cost, stream));
    return STBA_OK;
}

int stba_residual_jacobian_static(const stba_problem *p, int precision, void *f, void *Jc, void *Jp, double *cost,
                                  hipStream_t stream) {
    STBA_TRY(check_problem(p));
    STBA_TRY(check_precision(precision));
    if (!f || ((Jc == nullptr) != (Jp == nullptr))) return STBA_EINVAL;
    const int64_t nb = rj_blocks(p->q);
    if (cost && nb > kStaticPartials) return STBA_EWORKSPACE;   // more observations than the scratch holds
    double *partials = nullptr;
    if (cost) STBA_TRY(static_scratch(&partials));
    if (precision == STBA_FP64)
        STBA_HIP(launch_rj<double>(*p, (double *)f, (double *)Jc, (double *)Jp, partials, nullptr, nullptr, ZeroS(),
                                   stream));
    else
        STBA_HIP(launch_rj<float>(*p, (float *)f, (float *)Jc, (float *)Jp, partials, nullptr, nullptr, ZeroS(),
                                  stream));
    if (cost) STBA_HIP(launch_sum_partials(partials, nb, cost, stream));
    return STBA_OK;
}

int stba_build_cluster_rcs(const stba_problem *p, const stba_dims *dims, const stba_sample *s, const stba_damping *d,
                           int precision, const void *f, const void *Jc, const void *Jp, stba_rcs *out, void *ws,
                           size_t ws_bytes, hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    STBA_TRY(check_sample(p, s));
    if (!d || !(d->lambda > 0.0) || !(d->lambda_corr >= 0.0) || !f || !Jc || !Jp || !out) return STBA_EINVAL;
    if (precision == STBA_FP64 && (reinterpret_cast<uintptr_t>(Jc) & 15) != 0) return STBA_EINVAL;
    double *lam2 = at<double>(ws, L.lam2);
    STBA_HIP(launch_set_damping(lam2, d->lambda, d->lambda_corr, stream));
    if (precision == STBA_FP64)
        STBA_TRY(build_rcs_impl<double>(p, dims, s, lam2, (const double *)f, (const double *)Jc, (const double *)Jp, L,
                                        ws, stream));
    else
        STBA_TRY(build_rcs_impl<float>(p, dims, s, lam2, (const float *)f, (const float *)Jc, (const float *)Jp, L, ws,
                                       stream));
    out->S = at<double>(ws, L.S);
    out->S_off = at<int64_t>(ws, L.S_off);
    out->cl_n = at<int32_t>(ws, L.cl_n);
    out->cl_Np = at<int32_t>(ws, L.cl_Np);
    out->cl_start = at<int32_t>(ws, L.cl_start);
    out->cl_cams = at<int32_t>(ws, L.cl_cams);
    out->cam_local = at<int32_t>(ws, L.cam_local);
    out->b = at<double>(ws, L.b);
    out->seg_head = at<int32_t>(ws, L.seg_head);
    out->l = s->l;
    out->l_dev = s->l_dev;
    out->precision = precision;
    return STBA_OK;
}

int stba_solve_clusters(const stba_problem *p, const stba_dims *dims, const stba_rcs *rcs, int precision,
                        const void *Jc, const void *Jp, double *dcam, double *dpt, int32_t *cluster_status, void *ws,
                        size_t ws_bytes, hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    if (!rcs || rcs->l < 1 || rcs->l > p->m || rcs->precision != precision || !Jc || !Jp || !dcam || !dpt)
        return STBA_EINVAL;
    int32_t *cs = cluster_status ? cluster_status : at<int32_t>(ws, L.cl_status);
    if (precision == STBA_FP64)
        return solve_impl<double>(p, dims, rcs->l, rcs->l_dev != nullptr, (const double *)Jc, (const double *)Jp,
                                  dcam, dpt, cs, L, ws, stream);
    return solve_impl<float>(p, dims, rcs->l, rcs->l_dev != nullptr, (const float *)Jc, (const float *)Jp, dcam, dpt,
                             cs, L, ws, stream);
}

int stba_sample_clusters(const stba_problem *p, const stba_dims *dims, int precision, void *ws, size_t ws_bytes,
                         int32_t gamma, double beta, uint64_t seed, uint64_t iter, int32_t *cam_cluster,
                         int32_t *n_clusters, int32_t *status, hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    if (p->m > kSgcMaxCams || gamma < 1 || gamma > dims->gamma_max || !(beta >= 0.0) || !std::isfinite(beta))
        return STBA_EINVAL;
    // pair weights and their sums are int32; the total weight is at most n_pairs
    if (dims->n_pairs >= (int64_t(1) << 31)) return STBA_EINVAL;
    if (!cam_cluster || !n_clusters || !status) return STBA_EINVAL;
    // pair labels, clocks and weights per block (at most n_pairs blocks) live in
    // plan buffers that only stba_prepare uses
    STBA_HIP(launch_sgc(p->m, at<int64_t>(ws, L.n_blocks), at<int2>(ws, L.blk_key), at<int64_t>(ws, L.blk_start),
                        gamma, beta, seed, iter, at<uint32_t>(ws, L.scratch_a), at<double>(ws, L.keys_in),
                        at<int32_t>(ws, L.vals_in), cam_cluster, n_clusters, status, stream));
    return STBA_OK;
}

int stba_solve_clusters_pcg(const stba_problem *p, const stba_dims *dims, const stba_rcs *rcs, int precision,
                            const void *Jc, const void *Jp, double *dcam, double *dpt, int32_t max_iters, double tol,
                            int32_t *cluster_iters, double *cluster_resid, int32_t *cluster_status, void *ws,
                            size_t ws_bytes, hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    if (!rcs || rcs->l < 1 || rcs->l > p->m || rcs->precision != precision || !Jc || !Jp || !dcam || !dpt)
        return STBA_EINVAL;
    if (max_iters < 0 || !(tol >= 0.0) || !std::isfinite(tol)) return STBA_EINVAL;
    if (pcg_lds_bytes(L.max_Np, dims->gamma_max) > 160 * 1024) return STBA_EINVAL;
    int32_t *cs = cluster_status ? cluster_status : at<int32_t>(ws, L.cl_status);
    int32_t *its = cluster_iters ? cluster_iters : at<int32_t>(ws, L.pcg_iters);
    double *res = cluster_resid ? cluster_resid : at<double>(ws, L.pcg_resid);
    STBA_HIP(launch_pcg(rcs->l, at<int32_t>(ws, L.cl_n), at<int32_t>(ws, L.cl_Np), at<int64_t>(ws, L.S_off),
                        at<int32_t>(ws, L.cl_start), at<int32_t>(ws, L.cl_cams), at<int32_t>(ws, L.cam_local),
                        at<int64_t>(ws, L.n_blocks), at<int2>(ws, L.blk_key), at<double>(ws, L.S),
                        at<double>(ws, L.b), dcam, at<int32_t>(ws, L.pcg_clus), at<double>(ws, L.pcg_minv),
                        L.max_Np, dims->gamma_max, max_iters, tol, its, res, cs, stream));
    if (precision == STBA_FP64)
        STBA_HIP(launch_backsub<double>(*p, at<int64_t>(ws, L.pt_off), (const double *)Jc, (const double *)Jp,
                                        at<double>(ws, L.Vinv), at<double>(ws, L.wph), dcam, dpt, L.group_size,
                                        at<int32_t>(ws, L.grp_first), false, stream));
    else
        STBA_HIP(launch_backsub<float>(*p, at<int64_t>(ws, L.pt_off), (const float *)Jc, (const float *)Jp,
                                       at<double>(ws, L.Vinv), at<double>(ws, L.wph), dcam, dpt, L.group_size,
                                       at<int32_t>(ws, L.grp_first), false, stream));
    return STBA_OK;
}

int stba_lm_init(stba_lm_state *st, double lambda0, double lambda_corr, hipStream_t stream) {
    if (!st || !(lambda0 > 0.0) || !(lambda_corr >= 0.0)) return STBA_EINVAL;
    STBA_HIP(launch_lm_init(st, lambda0, lambda_corr, stream));
    return STBA_OK;
}

int stba_lm_step_profiled(const stba_problem *p, const stba_dims *dims, const stba_sample *s, stba_lm_state *st,
                          int precision, void *ws, size_t ws_bytes, hipStream_t stream, hipEvent_t *events) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    STBA_TRY(check_sample(p, s));
    if (!st) return STBA_EINVAL;
    if (precision == STBA_FP64) return lm_step_impl<double>(p, dims, s, st, L, ws, stream, events);
    return lm_step_impl<float>(p, dims, s, st, L, ws, stream, events);
}

int stba_lm_step(const stba_problem *p, const stba_dims *dims, const stba_sample *s, stba_lm_state *st, int precision,
                 void *ws, size_t ws_bytes, hipStream_t stream) {
    return stba_lm_step_profiled(p, dims, s, st, precision, ws, ws_bytes, stream, nullptr);
}

int stba_lm_step_pcg(const stba_problem *p, const stba_dims *dims, const stba_sample *s, stba_lm_state *st,
                     int precision, int32_t max_iters, double tol, void *ws, size_t ws_bytes, hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    STBA_TRY(check_sample(p, s));
    if (!st || max_iters < 0 || !(tol >= 0.0) || !std::isfinite(tol)) return STBA_EINVAL;
    if (pcg_lds_bytes(L.max_Np, dims->gamma_max) > 160 * 1024) return STBA_EINVAL;
    const PcgOpts o{max_iters, tol};
    if (precision == STBA_FP64) return lm_step_impl<double>(p, dims, s, st, L, ws, stream, nullptr, &o);
    return lm_step_impl<float>(p, dims, s, st, L, ws, stream, nullptr, &o);
}

int stba_autotune(const stba_problem *p, stba_dims *dims, const stba_sample *s, const stba_damping *d,
                  int precision, void *ws, size_t ws_bytes, hipStream_t stream, stba_tune_report *report) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    STBA_TRY(check_sample(p, s));
    if (!d || !(d->lambda > 0.0) || !(d->lambda_corr >= 0.0)) return STBA_EINVAL;
    STBA_HIP(launch_set_damping(at<double>(ws, L.lam2), d->lambda, d->lambda_corr, stream));
    stba_tune_report local = {};
    stba_tune_report *rep = report ? report : &local;
    *rep = stba_tune_report{};
    if (precision == STBA_FP64) return autotune_impl<double>(p, dims, s, L, ws, stream, rep);
    return autotune_impl<float>(p, dims, s, L, ws, stream, rep);
}

int stba_residual_vjp(const stba_problem *p, const stba_dims *dims, int precision, const void *v, void *grad_cam,
                      void *grad_pt, void *grad_uv, void *ws, size_t ws_bytes, hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    if (!v || !grad_cam || !grad_pt || !grad_uv) return STBA_EINVAL;
    const VjpParts parts = vjp_parts_of(L, ws);
    if (precision == STBA_FP64)
        STBA_HIP(launch_vjp<double>(*p, at<int64_t>(ws, L.pt_off), at<int64_t>(ws, L.diag_blk),
                                    at<int64_t>(ws, L.blk_start), at<uint64_t>(ws, L.pairs), parts, (const double *)v,
                                    (double *)grad_cam, (double *)grad_pt, (double *)grad_uv, stream));
    else
        STBA_HIP(launch_vjp<float>(*p, at<int64_t>(ws, L.pt_off), at<int64_t>(ws, L.diag_blk),
                                   at<int64_t>(ws, L.blk_start), at<uint64_t>(ws, L.pairs), parts, (const float *)v,
                                   (float *)grad_cam, (float *)grad_pt, (float *)grad_uv, stream));
    return STBA_OK;
}

int stba_lm_step_batched(const stba_problem *p, const stba_dims *dims, const stba_sample *s, stba_lm_state *states,
                         int32_t n_prob, const int32_t *prob_cam, const int32_t *prob_pt, const int64_t *prob_obs_off,
                         int precision, void *ws, size_t ws_bytes, hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    STBA_TRY(check_sample(p, s));
    if (!states || !prob_cam || !prob_pt || !prob_obs_off || n_prob < 1 || n_prob > p->m) return STBA_EINVAL;
    if (precision == STBA_FP64)
        return lm_step_batched_impl<double>(p, dims, s, states, n_prob, prob_cam, prob_pt, prob_obs_off, L, ws,
                                            stream);
    return lm_step_batched_impl<float>(p, dims, s, states, n_prob, prob_cam, prob_pt, prob_obs_off, L, ws, stream);
}

int stba_residual_vjp_stored(const stba_problem *p, const stba_dims *dims, int precision, const void *v,
                             const void *Jc, const void *Jp, void *grad_cam, void *grad_pt, void *grad_uv, void *ws,
                             size_t ws_bytes, hipStream_t stream) {
    Layout L;
    STBA_TRY(front(p, dims, precision, ws, ws_bytes, L));
    if (!v || !Jc || !Jp || !grad_cam || !grad_pt || !grad_uv) return STBA_EINVAL;
    const VjpParts parts = vjp_parts_of(L, ws);
    if (precision == STBA_FP64)
        STBA_HIP(launch_vjp_stored<double>(*p, at<int64_t>(ws, L.pt_off), at<int64_t>(ws, L.diag_blk),
                                           at<int64_t>(ws, L.blk_start), at<uint64_t>(ws, L.pairs), parts,
                                           (const double *)v, (const double *)Jc, (const double *)Jp,
                                           (double *)grad_cam, (double *)grad_pt, (double *)grad_uv, stream));
    else
        STBA_HIP(launch_vjp_stored<float>(*p, at<int64_t>(ws, L.pt_off), at<int64_t>(ws, L.diag_blk),
                                          at<int64_t>(ws, L.blk_start), at<uint64_t>(ws, L.pairs), parts,
                                          (const float *)v, (const float *)Jc, (const float *)Jp, (float *)grad_cam,
                                          (float *)grad_pt, (float *)grad_uv, stream));
    return STBA_OK;
}

}  // extern "C"
