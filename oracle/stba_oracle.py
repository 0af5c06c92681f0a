"""Plain, slow, FP64 reference of one LM iteration of plain LM and of STBA.

TEST INFRASTRUCTURE ONLY: called by the tests, by ``__graft_entry__.smoke()`` and
by the ``cpu_baseline`` leg of ``bench.py``.  It never calls the GPU library and
shares no code with it.

Source: L. Zhou et al., "Stochastic Bundle Adjustment for Efficient and Scalable
3D Reconstruction", ECCV 2020 (arXiv 2008.00446).  Citations name the paper's
sections, equations and Algorithm 1 (appendix C).

Every quantity is built from the paper's matrices with scipy.sparse / LAPACK as
the only library steps: J = [J_c, J_p] (Sec. 3), B, C, E, v, w (Eq. 4), the
clustered C', E', v', w' and S' (Eq. 10), the per-cluster systems (Eq. 13), the
point update (Eq. 14-15), the correction (Sec. 4.3) and the LM accept rule
(Alg. 1).  Readings of points the paper leaves open:

* camera model (the paper leaves it open; its experiments use 6-d extrinsics):
  9 parameters (rotation vector w, translation t, focal f, k1, k2); P = R(w) X + t,
  (x, y) = (P_x, P_y) / P_z, pixel = f (1 + k1 r^2 + k2 r^4) (x, y); the camera
  looks along +z, no principal point (pixels are image-centred);
* residual f = predicted - observed and F = ||f||^2 with no 1/2 (Sec. 3);
* w = -J_p^T f (Eq. 4; Alg. 1 prints it without the minus sign) and
  g = -J'^T f (Alg. 1 omits the transpose);
* D = diag(J^T J)^(1/2) with no clamp, and a virtual point is damped by its own
  diagonal (Eq. 7, 10);
* the sampled constraints (Sec. 4.2): a point's observations are ordered by
  (cluster, camera); consecutive same-cluster observations form a link that is
  kept iff a Philox4x64-10 draw falls below alpha; cross-cluster links are always
  dropped, so S' is cluster-diagonal.  alpha = 1 gives Alg. 1 exactly;
* the draw: key (seed, 0), counter (t, point, camera of the later observation, 0),
  output word 0; keep iff (x0 >> 11) < ceil(alpha * 2^53);
* accept iff F(x + dx) < F(x) strictly, the step is finite and every cluster
  system factorises; lambda /= 3 on accept and *= 3 otherwise (Alg. 1);
* the robust loss (Sec. 5.1, optional): Huber on each observation's error norm,
  applied by first-order (IRLS) reweighting of f and J (see `huber_rho`);
* stochastic graph clustering (Sec. 4.4, Eq. 16) draws one join at a time from
  the distribution of Eq. 16 over the neighbouring pairs within the size cap,
  sampled by competing exponential clocks keyed by Philox (see `sgc_clusters`);
* the inexact cluster solve (App. A, Table 3): conjugate gradient with the
  camera-block (9 x 9) Jacobi preconditioner, from x = 0, stopped at a relative
  residual (see `pcg`).

Parity pins live in tests/test_oracle_*.py; every function below is pinned.
"""
from __future__ import annotations

import heapq
import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg
import scipy.sparse as sp

__all__ = [
    "rotation_matrix", "project", "residuals", "cost", "jacobian", "jtv", "gradient",
    "huber_rho", "huber_weight", "robust_cost", "irls",
    "philox4x64_10", "keep_threshold", "link_draws", "segments", "canonical_segments",
    "jc_matrix", "jp_matrix", "damp", "correct_point_gradient", "correction_explicit",
    "StbaStep", "stba_step", "plain_lm_step", "full_normal_step", "relaxed_kkt_step",
    "LmResult", "lm_iteration", "cluster_layout",
    "covisibility_graph", "sgc_uniform", "modularity_gain", "sgc_clusters",
    "block_jacobi_inverse", "pcg",
]

# ---------------------------------------------------------------------------
# O-1 / O-2: projection, residual and cost (Sec. 3)
# ---------------------------------------------------------------------------


def _skew(v):
    z = np.zeros_like(v[..., 0])
    return np.stack([
        np.stack([z, -v[..., 2], v[..., 1]], -1),
        np.stack([v[..., 2], z, -v[..., 0]], -1),
        np.stack([-v[..., 1], v[..., 0], z], -1),
    ], -2)


def _rodrigues_coeffs(theta2):
    """sin(th)/th, (1-cos th)/th^2, (th-sin th)/th^3 with series for small th.

    th^2 is the non-conjugating sum of squares so complex-step differentiation
    goes through unchanged."""
    small = np.real(theta2) < 1e-8
    th2 = np.where(small, 1.0, theta2)
    th = np.sqrt(th2)
    a = np.where(small, 1.0 - theta2 / 6.0, np.sin(th) / th)
    b = np.where(small, 0.5 - theta2 / 24.0, (1.0 - np.cos(th)) / th2)
    c = np.where(small, 1.0 / 6.0 - theta2 / 120.0, (th - np.sin(th)) / (th2 * th))
    return a, b, c


def rotation_matrix(omega):
    """R(w) = I + (sin th / th)[w]x + ((1 - cos th)/th^2)[w]x^2 (Rodrigues)."""
    omega = np.asarray(omega)
    theta2 = np.sum(omega * omega, axis=-1)
    a, b, _ = _rodrigues_coeffs(theta2)
    K = _skew(omega)
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + a[..., None, None] * K + b[..., None, None] * (K @ K)


def project(cam, X):
    """pi(c, X) for matching rows of cam [k,9] and X [k,3] -> [k,2]."""
    R = rotation_matrix(cam[:, 0:3])
    P = np.einsum("kab,kb->ka", R, X) + cam[:, 3:6]
    x = P[:, 0] / P[:, 2]
    y = P[:, 1] / P[:, 2]
    r2 = x * x + y * y
    d = 1.0 + cam[:, 7] * r2 + cam[:, 8] * r2 * r2
    return np.stack([cam[:, 6] * d * x, cam[:, 6] * d * y], axis=1)


def residuals(cam, pt, obs_cam, obs_pt, obs_uv):
    """f_o = pi(c_{i_o}, p_{j_o}) - q_o, stacked [q,2] (Sec. 3)."""
    return project(cam[obs_cam], pt[obs_pt]) - obs_uv


def cost(f):
    """F = ||f||^2, no 1/2 (Sec. 3)."""
    return float(np.sum(np.asarray(f, dtype=np.float64) ** 2))


# ---------------------------------------------------------------------------
# Robust loss (Sec. 5.1): the experiments put a Huber loss of scale 0.5 on the
# errors.  Reading: each observation's squared error s = ||f_o||^2 costs
# rho(s) = s for s <= a^2 and 2 a sqrt(s) - a^2 above (the Huber function of
# the error norm, continuous with its first derivative), F = sum_o rho(s_o), and
# LM is applied to the first-order (IRLS) reweighted problem f~ = sqrt(rho') f,
# J~ = sqrt(rho') J, whose gradient 2 J~^T f~ = 2 sum rho' J^T f is F's.  a = 0
# is the plain squared loss.
# ---------------------------------------------------------------------------


def huber_rho(s, a):
    """rho(s) of the Huber loss with scale a on s = ||f_o||^2."""
    s = np.asarray(s, dtype=np.float64)
    if a <= 0.0:
        return s
    return np.where(s <= a * a, s, 2.0 * a * np.sqrt(s) - a * a)


def huber_weight(s, a):
    """rho'(s): 1 for s <= a^2, a / sqrt(s) above."""
    s = np.asarray(s, dtype=np.float64)
    if a <= 0.0:
        return np.ones_like(s)
    return np.where(s <= a * a, 1.0, a / np.sqrt(np.maximum(s, a * a)))


def robust_cost(f, a):
    """F = sum_o rho(||f_o||^2) (the squared cost for a = 0)."""
    f = np.asarray(f, dtype=np.float64).reshape(-1, 2)
    return float(np.sum(huber_rho(np.sum(f * f, axis=1), a)))


def irls(f, Jc, Jp, a):
    """f~ = sqrt(rho') f, J~_c = sqrt(rho') J_c, J~_p = sqrt(rho') J_p per observation."""
    f = np.asarray(f, dtype=np.float64).reshape(-1, 2)
    r = np.sqrt(huber_weight(np.sum(f * f, axis=1), a))
    return f * r[:, None], Jc * r[:, None, None], Jp * r[:, None, None]


# ---------------------------------------------------------------------------
# O-3: analytic Jacobian J = [J_c, J_p] (Sec. 3)
# ---------------------------------------------------------------------------


def jacobian(cam, pt, obs_cam, obs_pt):
    """Per-observation blocks J_c [q,2,9] and J_p [q,2,3] of f.

    Chain rule: pixel <- (x, y) <- P <- (w, t, X); dP/dw = -R [X]x J_r(w) with the
    right Jacobian of SO(3), J_r = I - ((1-cos)/th^2)[w]x + ((th-sin)/th^3)[w]x^2.
    """
    c = cam[obs_cam]
    X = pt[obs_pt]
    omega = c[:, 0:3]
    theta2 = np.sum(omega * omega, axis=1)
    _, b, cc = _rodrigues_coeffs(theta2)
    K = _skew(omega)
    R = rotation_matrix(omega)
    P = np.einsum("kab,kb->ka", R, X) + c[:, 3:6]
    x = P[:, 0] / P[:, 2]
    y = P[:, 1] / P[:, 2]
    r2 = x * x + y * y
    f, k1, k2 = c[:, 6], c[:, 7], c[:, 8]
    d = 1.0 + k1 * r2 + k2 * r2 * r2
    s = k1 + 2.0 * k2 * r2
    q = c.shape[0]
    # d pixel / d (x, y) = f [d I + 2 s (x,y)^T (x,y)]
    dpix_dxy = np.empty((q, 2, 2))
    dpix_dxy[:, 0, 0] = f * (d + 2.0 * s * x * x)
    dpix_dxy[:, 0, 1] = f * (2.0 * s * x * y)
    dpix_dxy[:, 1, 0] = f * (2.0 * s * x * y)
    dpix_dxy[:, 1, 1] = f * (d + 2.0 * s * y * y)
    # d (x, y) / d P = (1/P_z) [[1, 0, -x], [0, 1, -y]]
    dxy_dP = np.zeros((q, 2, 3))
    dxy_dP[:, 0, 0] = 1.0 / P[:, 2]
    dxy_dP[:, 0, 2] = -x / P[:, 2]
    dxy_dP[:, 1, 1] = 1.0 / P[:, 2]
    dxy_dP[:, 1, 2] = -y / P[:, 2]
    dpix_dP = dpix_dxy @ dxy_dP
    Jr = np.eye(3)[None] - b[:, None, None] * K + cc[:, None, None] * (K @ K)
    dP_dw = -R @ _skew(X) @ Jr
    Jc = np.empty((q, 2, 9))
    Jc[:, :, 0:3] = dpix_dP @ dP_dw
    Jc[:, :, 3:6] = dpix_dP
    Jc[:, :, 6] = np.stack([d * x, d * y], axis=1)
    Jc[:, :, 7] = np.stack([f * r2 * x, f * r2 * y], axis=1)
    Jc[:, :, 8] = np.stack([f * r2 * r2 * x, f * r2 * r2 * y], axis=1)
    Jp = dpix_dP @ R
    return Jc, Jp


def jtv(Jc, Jp, obs_cam, obs_pt, m, n, v):
    """J^T v split into cameras [m,9], points [n,3] and observed pixels [q,2]."""
    gc = np.zeros((m, 9))
    gp = np.zeros((n, 3))
    np.add.at(gc, obs_cam, np.einsum("kab,ka->kb", Jc, v))
    np.add.at(gp, obs_pt, np.einsum("kab,ka->kb", Jp, v))
    return gc, gp, -np.asarray(v, dtype=np.float64)


def gradient(cam, pt, obs_cam, obs_pt, obs_uv):
    """dF/d(cam, pt, obs_uv) = (2 J_c^T f, 2 J_p^T f, -2 f)."""
    f = residuals(cam, pt, obs_cam, obs_pt, obs_uv)
    Jc, Jp = jacobian(cam, pt, obs_cam, obs_pt)
    return jtv(Jc, Jp, obs_cam, obs_pt, cam.shape[0], pt.shape[0], 2.0 * f)


# ---------------------------------------------------------------------------
# the sampler's draw: Philox4x64-10 (Salmon et al., SC'11)
# ---------------------------------------------------------------------------

_M32 = np.uint64(0xFFFFFFFF)
_PHILOX_M = (np.uint64(0xD2E7470EE14C6C93), np.uint64(0xCA5A826395121157))
_PHILOX_W = (np.uint64(0x9E3779B97F4A7C15), np.uint64(0xBB67AE8584CAA73B))


def _mulhilo(a, b):
    a = np.asarray(a, dtype=np.uint64)
    b = np.uint64(b)
    with np.errstate(over="ignore"):
        lo = a * b
        al, ah = a & _M32, a >> np.uint64(32)
        bl, bh = b & _M32, b >> np.uint64(32)
        ll, lh, hl, hh = al * bl, al * bh, ah * bl, ah * bh
        mid = (ll >> np.uint64(32)) + (lh & _M32) + (hl & _M32)
        hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    return hi, lo


def philox4x64_10(counter, key):
    """Philox4x64 with 10 rounds; counter [k,4] uint64, key (k0, k1) -> [k,4]."""
    c = np.array(counter, dtype=np.uint64).reshape(-1, 4)
    c0, c1, c2, c3 = c[:, 0].copy(), c[:, 1].copy(), c[:, 2].copy(), c[:, 3].copy()
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    with np.errstate(over="ignore"):
        for r in range(10):
            hi0, lo0 = _mulhilo(c0, _PHILOX_M[0])
            hi1, lo1 = _mulhilo(c2, _PHILOX_M[1])
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            if r < 9:
                k0 = k0 + _PHILOX_W[0]
                k1 = k1 + _PHILOX_W[1]
    return np.stack([c0, c1, c2, c3], axis=1)


def keep_threshold(alpha: float) -> int:
    """ceil(alpha * 2^53): a 53-bit uniform u keeps a link iff u < threshold."""
    if not (0.0 < alpha <= 1.0):
        raise ValueError("alpha must lie in (0, 1]")
    return int(math.ceil(alpha * float(1 << 53)))


def link_draws(seed, t, point, camera):
    """53-bit uniforms x0 >> 11 for counters (t, point, camera, 0), key (seed, 0)."""
    point = np.asarray(point, dtype=np.uint64)
    ctr = np.stack([np.full_like(point, np.uint64(t)), point,
                    np.asarray(camera, dtype=np.uint64), np.zeros_like(point)], axis=1)
    return philox4x64_10(ctr, (np.uint64(seed), np.uint64(0)))[:, 0] >> np.uint64(11)


# ---------------------------------------------------------------------------
# O-6: the sampled constraint set Theta(alpha) as segments (Sec. 4.1-4.2)
# ---------------------------------------------------------------------------


def segments(obs_cam, obs_pt, cam_cluster, alpha, seed, t, ids=None):
    """Point splitting then point binding (Sec. 4.1-4.2).

    Each observation starts as its own virtual point; the constraints of a
    physical point join consecutive observations (in (cluster, camera) order) of
    the same cluster; a sampled constraint (theta = 1) binds them.  Cross-cluster
    constraints are never bound, which makes S' cluster-diagonal (Sec. 4.2).

    ids: optional (point number, camera number) per observation that key the
    draw, for a problem cut out of a larger one with its cameras and points
    renumbered in increasing order (the draw belongs to the physical point and
    camera, not to their position in the cut-out arrays).

    Returns (seg [q] segment id per observation, n_seg, seg_point [n_seg],
    kept_links [k,2] (earlier obs, later obs), all_links [r,2] intra-point
    constraints of the chain in (cluster, camera) order, and is_cross [r])."""
    obs_cam = np.asarray(obs_cam, dtype=np.int64)
    obs_pt = np.asarray(obs_pt, dtype=np.int64)
    q = obs_cam.shape[0]
    clus = np.asarray(cam_cluster, dtype=np.int64)[obs_cam]
    order = np.lexsort((obs_cam, clus, obs_pt))       # by point, cluster, camera
    p_o, c_o, k_o = obs_pt[order], obs_cam[order], clus[order]
    same_pt = np.r_[False, p_o[1:] == p_o[:-1]]
    same_cl = same_pt & np.r_[False, k_o[1:] == k_o[:-1]]
    if ids is None:
        u = link_draws(seed, t, p_o, c_o)
    else:
        u = link_draws(seed, t, np.asarray(ids[0], dtype=np.int64)[order], np.asarray(ids[1], dtype=np.int64)[order])
    kept = same_cl & (u < np.uint64(keep_threshold(alpha)))
    seg_sorted = np.cumsum(~kept) - 1
    seg = np.empty(q, dtype=np.int64)
    seg[order] = seg_sorted
    n_seg = int(seg_sorted[-1]) + 1 if q else 0
    seg_point = np.empty(n_seg, dtype=np.int64)
    seg_point[seg_sorted] = p_o
    idx = np.flatnonzero(same_pt)
    all_links = np.stack([order[idx - 1], order[idx]], axis=1)
    is_cross = ~same_cl[idx]
    kidx = np.flatnonzero(kept)
    kept_links = np.stack([order[kidx - 1], order[kidx]], axis=1)
    return seg, n_seg, seg_point, kept_links, all_links, is_cross


def canonical_segments(seg):
    """Label each observation by the smallest observation index of its segment."""
    seg = np.asarray(seg)
    first = np.full(int(seg.max()) + 1 if seg.size else 0, np.iinfo(np.int64).max)
    np.minimum.at(first, seg, np.arange(seg.shape[0]))
    return first[seg]


# ---------------------------------------------------------------------------
# sparse J_c, J_p, J'_p (Sec. 3, Eq. 7)
# ---------------------------------------------------------------------------


def jc_matrix(Jc, obs_cam, m):
    """J_c as a sparse [2q, 9m] matrix: rows 2o, 2o+1; columns of camera i_o."""
    q = Jc.shape[0]
    rows = np.broadcast_to((2 * np.arange(q))[:, None, None] + np.arange(2)[None, :, None], (q, 2, 9))
    cols = np.broadcast_to(9 * np.asarray(obs_cam)[:, None, None] + np.arange(9)[None, None, :], (q, 2, 9))
    return sp.csr_matrix((Jc.ravel(), (rows.ravel(), cols.ravel())), shape=(2 * q, 9 * m))


def jp_matrix(Jp, col_of_obs, ncols):
    """J_p (physical points) or J'_p (virtual points) as a sparse [2q, 3 ncols]."""
    q = Jp.shape[0]
    rows = np.broadcast_to((2 * np.arange(q))[:, None, None] + np.arange(2)[None, :, None], (q, 2, 3))
    cols = np.broadcast_to(3 * np.asarray(col_of_obs)[:, None, None] + np.arange(3)[None, None, :], (q, 2, 3))
    return sp.csr_matrix((Jp.ravel(), (rows.ravel(), cols.ravel())), shape=(2 * q, 3 * ncols))


def damp(H, lam):
    """H + lam diag(H), i.e. J^T J + lam D^T D with D = diag(J^T J)^(1/2) (Eq. 2-4)."""
    return (H + lam * sp.diags(H.diagonal())).tocsr()


def _block_diag_inverse(C, bs):
    """Inverse of a block-diagonal sparse matrix with bs x bs blocks."""
    nb = C.shape[0] // bs
    blocks = C.tobsr(blocksize=(bs, bs))
    dense = np.zeros((nb, bs, bs))
    rows = np.repeat(np.arange(nb), np.diff(blocks.indptr))
    if np.any(blocks.indices != rows):
        raise ValueError("matrix is not block diagonal")
    dense[rows] = blocks.data
    inv = np.linalg.inv(dense)
    return sp.bsr_matrix((inv, np.arange(nb), np.arange(nb + 1)), shape=C.shape).tocsr()


# ---------------------------------------------------------------------------
# O-8: steepest-descent correction (Sec. 4.3, Alg. 1)
# ---------------------------------------------------------------------------


def correct_point_gradient(w_seg, h_seg, seg_point, n):
    """g <- g - A^T nu with nu = (A H~^-1 A^T)^-1 A H~^-1 g, H~ = diag(H_lambda).

    A couples only the virtual points of one physical point and has no camera
    columns.  For one point and one coordinate, A's rows span {z : sum z = 0},
    so H~^-1 g' is constant across the point's segments and sum g' = sum g:
    g'_s = h_s * (sum_s g_s) / (sum_s h_s).  Camera entries are unchanged."""
    gsum = np.zeros((n, 3))
    hsum = np.zeros((n, 3))
    np.add.at(gsum, seg_point, w_seg)
    np.add.at(hsum, seg_point, h_seg)
    return h_seg * gsum[seg_point] / hsum[seg_point]


def correction_explicit(w_seg, h_seg, seg_point, spanning="chain"):
    """The same correction with an explicit constraint matrix A and dense solves
    (Alg. 1): rows e_s - e_t over each point's segments, as a chain s_k - s_{k+1}
    or a star s_0 - s_k.  Pins the closed form above; tiny inputs only."""
    S = w_seg.shape[0]
    rows = []
    for j in np.unique(seg_point):
        segs = np.flatnonzero(seg_point == j)
        for k in range(1, segs.shape[0]):
            a = segs[k - 1] if spanning == "chain" else segs[0]
            for d in range(3):
                r = np.zeros(3 * S)
                r[3 * a + d] = 1.0
                r[3 * segs[k] + d] = -1.0
                rows.append(r)
    g = w_seg.reshape(-1).copy()
    if not rows:
        return w_seg.copy()
    A = np.array(rows)
    Hinv = np.diag(1.0 / h_seg.reshape(-1))
    nu = np.linalg.solve(A @ Hinv @ A.T, A @ Hinv @ g)
    return (g - A.T @ nu).reshape(S, 3)


# ---------------------------------------------------------------------------
# O-9 .. O-11: one STBA step (Eq. 10, 13, 15; Alg. 1)
# ---------------------------------------------------------------------------


def cluster_layout(cam_cluster):
    """Cameras of each cluster in ascending id order (the order of S_k's blocks)."""
    cam_cluster = np.asarray(cam_cluster)
    l = int(cam_cluster.max()) + 1
    return [np.flatnonzero(cam_cluster == k) for k in range(l)]


@dataclass
class StbaStep:
    dcam: np.ndarray            # [m,9]
    dpt: np.ndarray             # [n,3]
    S_blocks: list              # dense S_k per cluster (Eq. 13)
    b_blocks: list              # b_k per cluster
    clusters: list              # camera ids per cluster
    ok: bool                    # every S_k factorised
    cluster_ok: np.ndarray
    seg: np.ndarray
    n_seg: int
    cross_max: float            # max |S'_ij| over cameras in different clusters
    corrected: bool
    v_seg_step: np.ndarray      # virtual point steps C'^-1 (w' - E'^T dc)
    b_full: np.ndarray          # b' = v' - E' C'^-1 w'  [9m]


def stba_step(cam, pt, obs_cam, obs_pt, obs_uv, cam_cluster, lam, alpha=1.0, seed=0, t=0,
              lam_corr=0.1, Jc=None, Jp=None, f=None, ids=None, huber=0.0, pcg_opts=None):
    """One STBA step for a given clustering (Alg. 1, one pass of the while loop
    up to the point update).  ids: see `segments`.  huber > 0: the step of the
    IRLS-reweighted problem (robust loss of Sec. 5.1, see `irls`).
    pcg_opts = (max_iters, tol): each cluster system solved by `pcg` (App. A)
    instead of Cholesky."""
    m, n = cam.shape[0], pt.shape[0]
    if f is None:
        f = residuals(cam, pt, obs_cam, obs_pt, obs_uv)
    if Jc is None or Jp is None:
        Jc, Jp = jacobian(cam, pt, obs_cam, obs_pt)
    if huber > 0.0:
        f, Jc, Jp = irls(f, Jc, Jp, huber)
    seg, n_seg, seg_point, _, _, _ = segments(obs_cam, obs_pt, cam_cluster, alpha, seed, t, ids)
    fv = np.asarray(f, dtype=np.float64).reshape(-1)
    Jc_m = jc_matrix(Jc, obs_cam, m)
    Jp_virt = jp_matrix(Jp, seg, n_seg)
    Jp_phys = jp_matrix(Jp, obs_pt, n)
    # Eq. 4 and Eq. 10
    U = (Jc_m.T @ Jc_m).tocsr()
    B = damp(U, lam)
    Cv = damp((Jp_virt.T @ Jp_virt).tocsr(), lam)
    Ev = (Jc_m.T @ Jp_virt).tocsr()
    v = -(Jc_m.T @ fv)
    w_virt = -(Jp_virt.T @ fv)
    corrected = lam >= lam_corr
    if corrected:
        # H~ = diag(H_lambda) on the virtual-point coordinates: (1 + lam) diag(V_s)
        h = (1.0 + lam) * (Jp_virt.T @ Jp_virt).diagonal().reshape(n_seg, 3)
        w_virt = correct_point_gradient(w_virt.reshape(n_seg, 3), h, seg_point, n).reshape(-1)
    Cv_inv = _block_diag_inverse(Cv, 3)
    S_full = (B - Ev @ Cv_inv @ Ev.T).toarray()
    b_full = v - Ev @ (Cv_inv @ w_virt)
    clusters = cluster_layout(cam_cluster)
    cidx = [(9 * c[:, None] + np.arange(9)[None, :]).reshape(-1) for c in clusters]
    lab9 = np.repeat(np.asarray(cam_cluster), 9)
    cross = lab9[:, None] != lab9[None, :]
    cross_max = float(np.max(np.abs(S_full[cross]))) if cross.any() else 0.0
    dc = np.zeros(9 * m)
    S_blocks, b_blocks, okk = [], [], []
    for idx in cidx:
        Sk = S_full[np.ix_(idx, idx)]
        bk = b_full[idx]
        S_blocks.append(Sk)
        b_blocks.append(bk)
        if pcg_opts is not None:
            x, _, _, okp = pcg(Sk, bk, pcg_opts[1], pcg_opts[0])
            dc[idx] = x if okp else 0.0
            okk.append(bool(okp))
            continue
        try:
            fac = scipy.linalg.cho_factor(Sk, lower=True, check_finite=True)
            dc[idx] = scipy.linalg.cho_solve(fac, bk)
            okk.append(True)
        except (np.linalg.LinAlgError, ValueError):
            okk.append(False)
    # Eq. 15: the physical point update with the uncorrected w
    C = damp((Jp_phys.T @ Jp_phys).tocsr(), lam)
    E = (Jc_m.T @ Jp_phys).tocsr()
    w = -(Jp_phys.T @ fv)
    dp = _block_diag_inverse(C, 3) @ (w - E.T @ dc)
    v_seg_step = Cv_inv @ (w_virt - Ev.T @ dc)
    ok_arr = np.array(okk, dtype=bool)
    return StbaStep(dcam=dc.reshape(m, 9), dpt=dp.reshape(n, 3), S_blocks=S_blocks,
                    b_blocks=b_blocks, clusters=clusters, ok=bool(ok_arr.all()),
                    cluster_ok=ok_arr, seg=seg, n_seg=n_seg, cross_max=cross_max,
                    corrected=corrected, v_seg_step=v_seg_step.reshape(n_seg, 3),
                    b_full=b_full)


def plain_lm_step(cam, pt, obs_cam, obs_pt, obs_uv, lam, Jc=None, Jp=None, f=None):
    """The classic LM step by the Schur complement (Eq. 5-6): S dc = v - E C^-1 w,
    dp = C^-1 (w - E^T dc), S = B - E C^-1 E^T dense over all cameras."""
    m, n = cam.shape[0], pt.shape[0]
    if f is None:
        f = residuals(cam, pt, obs_cam, obs_pt, obs_uv)
    if Jc is None or Jp is None:
        Jc, Jp = jacobian(cam, pt, obs_cam, obs_pt)
    fv = np.asarray(f, dtype=np.float64).reshape(-1)
    Jc_m = jc_matrix(Jc, obs_cam, m)
    Jp_m = jp_matrix(Jp, obs_pt, n)
    B = damp((Jc_m.T @ Jc_m).tocsr(), lam)
    C = damp((Jp_m.T @ Jp_m).tocsr(), lam)
    E = (Jc_m.T @ Jp_m).tocsr()
    v = -(Jc_m.T @ fv)
    w = -(Jp_m.T @ fv)
    Cinv = _block_diag_inverse(C, 3)
    S = (B - E @ Cinv @ E.T).toarray()
    rhs = v - E @ (Cinv @ w)
    dc = scipy.linalg.cho_solve(scipy.linalg.cho_factor(S, lower=True), rhs)
    dp = Cinv @ (w - E.T @ dc)
    return dc.reshape(m, 9), dp.reshape(n, 3), S, rhs


def full_normal_step(cam, pt, obs_cam, obs_pt, obs_uv, lam):
    """Brute force: (J^T J + lam diag(J^T J)) dx = -J^T f, dense (Eq. 3)."""
    m, n = cam.shape[0], pt.shape[0]
    f = residuals(cam, pt, obs_cam, obs_pt, obs_uv).reshape(-1)
    Jc, Jp = jacobian(cam, pt, obs_cam, obs_pt)
    J = sp.hstack([jc_matrix(Jc, obs_cam, m), jp_matrix(Jp, obs_pt, n)]).toarray()
    H = J.T @ J
    H = H + lam * np.diag(np.diag(H))
    dx = np.linalg.solve(H, -J.T @ f)
    return dx[:9 * m].reshape(m, 9), dx[9 * m:].reshape(n, 3)


def relaxed_kkt_step(cam, pt, obs_cam, obs_pt, obs_uv, cam_cluster, lam, alpha=1.0, seed=0,
                     t=0, point_gradient_shift=None):
    """Brute force of the relaxed QP (Eq. 7-9, 11-12) at the finest split.

    Every observation gets its own virtual point, damped by its own diagonal;
    each kept link adds the explicit rows dp_a - dp_b = 0; the KKT system
    [[H, A^T], [A, 0]] [dx; nu] = [-J'^T f; 0] is solved densely.
    `point_gradient_shift[o]` (optional, [q,3]) is added to the gradient of
    observation o's virtual point (used to pin the corrected right-hand side).
    Returns (dc [m,9], per-observation virtual steps [q,3])."""
    m = cam.shape[0]
    q = obs_cam.shape[0]
    f = residuals(cam, pt, obs_cam, obs_pt, obs_uv).reshape(-1)
    Jc, Jp = jacobian(cam, pt, obs_cam, obs_pt)
    _, _, _, kept, _, _ = segments(obs_cam, obs_pt, cam_cluster, alpha, seed, t)
    J = sp.hstack([jc_matrix(Jc, obs_cam, m), jp_matrix(Jp, np.arange(q), q)]).toarray()
    H = J.T @ J
    H = H + lam * np.diag(np.diag(H))
    g = -J.T @ f
    if point_gradient_shift is not None:
        g[9 * m:] += np.asarray(point_gradient_shift).reshape(-1)
    nv = 9 * m + 3 * q
    A = np.zeros((3 * kept.shape[0], nv))
    for r, (a, b) in enumerate(kept):
        for d in range(3):
            A[3 * r + d, 9 * m + 3 * a + d] = 1.0
            A[3 * r + d, 9 * m + 3 * b + d] = -1.0
    K = np.block([[H, A.T], [A, np.zeros((A.shape[0], A.shape[0]))]])
    sol = np.linalg.solve(K, np.concatenate([g, np.zeros(A.shape[0])]))
    return sol[:9 * m].reshape(m, 9), sol[9 * m:nv].reshape(q, 3)


# ---------------------------------------------------------------------------
# O-12: the LM accept / reject rule (Alg. 1)
# ---------------------------------------------------------------------------


@dataclass
class LmResult:
    cam: np.ndarray
    pt: np.ndarray
    lam: float
    F: float
    F_new: float
    accepted: bool
    step: StbaStep


def lm_iteration(cam, pt, obs_cam, obs_pt, obs_uv, cam_cluster, lam, alpha=1.0, seed=0, t=0,
                 lam_corr=0.1, F=None, huber=0.0, lam_min=0.0, pcg_opts=None):
    """One pass of Alg. 1's loop: STBA step, then accept iff F(x + dx) < F(x)
    (F the robust cost when huber > 0); lambda / 3 on accept but not below
    lam_min (the lower bound of the correction ablation, Sec. 5.4), x 3 else."""
    if F is None:
        F = robust_cost(residuals(cam, pt, obs_cam, obs_pt, obs_uv), huber)
    st = stba_step(cam, pt, obs_cam, obs_pt, obs_uv, cam_cluster, lam, alpha, seed, t, lam_corr, huber=huber,
                   pcg_opts=pcg_opts)
    cam_new = cam + st.dcam
    pt_new = pt + st.dpt
    F_new = robust_cost(residuals(cam_new, pt_new, obs_cam, obs_pt, obs_uv), huber) if st.ok else float("nan")
    accepted = bool(st.ok and np.isfinite(F_new) and F_new < F)
    if accepted:
        return LmResult(cam_new, pt_new, max(lam / 3.0, lam_min), F_new, F_new, True, st)
    return LmResult(cam.copy(), pt.copy(), lam * 3.0, F, F_new, False, st)


# ---------------------------------------------------------------------------
# O-14: the camera graph and stochastic graph clustering (Sec. 4.4, Eq. 16)
# ---------------------------------------------------------------------------


def covisibility_graph(obs_cam, obs_pt, m, n):
    """Camera graph G_c (Sec. 4.4): edge (i, j), i < j, weighted by the number of
    points both cameras see, i.e. the off-diagonal of V V^T for the m x n
    visibility matrix V.  Returns (edges [E,2] ascending by (i, j), weights [E])."""
    obs_cam = np.asarray(obs_cam, dtype=np.int64)
    obs_pt = np.asarray(obs_pt, dtype=np.int64)
    V = sp.csr_matrix((np.ones(obs_cam.shape[0]), (obs_cam, obs_pt)), shape=(m, n))
    W = sp.triu(V @ V.T, k=1).tocoo()
    order = np.lexsort((W.col, W.row))
    edges = np.stack([W.row[order], W.col[order]], axis=1).astype(np.int64)
    return edges, np.rint(W.data[order]).astype(np.int64)


def sgc_uniform(seed, t, k, a, b):
    """Uniforms in (0, 1] for the clocks of cluster pairs (a, b), a < b, set at
    join step k of LM iteration t: Philox4x64-10 with key (seed, 2) and counter
    (t, k, a, b), u = ((x0 >> 11) + 1) 2^-53."""
    a = np.atleast_1d(np.asarray(a, dtype=np.uint64))
    b = np.atleast_1d(np.asarray(b, dtype=np.uint64))
    ctr = np.stack([np.full_like(a, np.uint64(t)), np.full_like(a, np.uint64(k)), a, b], axis=1)
    x0 = philox4x64_10(ctr, (np.uint64(seed), np.uint64(2)))[:, 0] >> np.uint64(11)
    return (x0.astype(np.float64) + 1.0) * 2.0 ** -53


def modularity_gain(w_xy, K_x, K_y, s):
    """dQ of joining clusters x and y: the change of the modularity of Sec. 4.4,
    w_xy / s - K_x K_y / (2 s^2) (K: summed incident weight, s: total weight)."""
    return w_xy / s - (K_x * K_y) / (2.0 * s * s)


def sgc_clusters(edges, weights, m, gamma, beta, seed, t):
    """Stochastic graph clustering (Sec. 4.4): from singletons, repeatedly join
    two neighbouring clusters x, y with probability exp(beta dQ(x, y)) over the
    sum of the same over all neighbouring pairs (Eq. 16), where only pairs whose
    joint size stays within gamma take part; stop when no such pair is left.

    The draw of each join uses competing exponential clocks: every eligible
    cluster pair holds a clock T = t_now + E / exp(beta dQ), E = -log u with u
    from `sgc_uniform`; the pair with the smallest clock (ties: smaller a m + b
    for the pair (a, b), a < b) joins next.  The smallest of independent
    exponentials with rates r_p is attained at p with probability r_p / sum r,
    and by memorylessness the clocks of pairs the join does not touch stay
    valid, so only the pairs of the joined cluster get new clocks (drawn at
    step k).  A cluster is named by its smallest camera, so joining y into x
    (x < y) keeps the name x.

    Returns (cam_cluster [m] int32 with clusters numbered 0..l-1 by their
    smallest camera, l)."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    weights = np.asarray(weights, dtype=np.int64).reshape(-1)
    adj = [dict() for _ in range(m)]
    for (i, j), w in zip(edges.tolist(), weights.tolist()):
        if i == j or w == 0:
            continue
        adj[i][j] = adj[i].get(j, 0) + w
        adj[j][i] = adj[j].get(i, 0) + w
    K = [sum(a.values()) for a in adj]
    s = float(sum(K)) / 2.0
    lab = np.arange(m, dtype=np.int64)
    size = [1] * m
    clock = {}
    heap = []
    version = [0]

    def set_clocks(pairs, k, t_now):
        if not pairs:
            return
        a = np.array([p[0] for p in pairs], dtype=np.int64)
        b = np.array([p[1] for p in pairs], dtype=np.int64)
        u = sgc_uniform(seed, t, k, a, b)
        for (x, y, w), ui in zip(pairs, u.tolist()):
            version[0] += 1
            if size[x] + size[y] > gamma:
                clock[(x, y)] = (math.inf, version[0])
                continue
            rate = math.exp(beta * modularity_gain(float(w), float(K[x]), float(K[y]), s))
            T = t_now + (-math.log(ui)) / rate
            clock[(x, y)] = (T, version[0])
            heapq.heappush(heap, (T, x * m + y, version[0], x, y))

    if s > 0.0 and gamma > 1:
        set_clocks([(i, j, w) for i in range(m) for j, w in sorted(adj[i].items()) if i < j], 0, 0.0)
        for k in range(1, m):
            while heap and clock.get((heap[0][3], heap[0][4]), (None, -1))[1] != heap[0][2]:
                heapq.heappop(heap)
            if not heap:
                break
            t_now, _, _, x, y = heapq.heappop(heap)
            # join y into x
            del clock[(x, y)]
            del adj[x][y]
            del adj[y][x]
            for z, w in adj[y].items():
                del adj[z][y]
                del clock[(min(y, z), max(y, z))]
                adj[x][z] = adj[x].get(z, 0) + w
                adj[z][x] = adj[x][z]
            adj[y] = {}
            size[x] += size[y]
            K[x] += K[y]
            lab[lab == y] = x
            set_clocks([(min(x, z), max(x, z), w) for z, w in sorted(adj[x].items())], k, t_now)
    names, dense = np.unique(lab, return_inverse=True)
    return dense.astype(np.int32), int(names.shape[0])


# ---------------------------------------------------------------------------
# O-15: the inexact cluster solve by preconditioned conjugate gradient (App. A)
# ---------------------------------------------------------------------------


def block_jacobi_inverse(S, bs=9):
    """M^-1 for the block-Jacobi preconditioner M = blockdiag(S_ii), bs x bs
    diagonal blocks of S (the camera blocks); raises LinAlgError if a block is not
    positive definite."""
    n = S.shape[0] // bs
    out = np.zeros((n, bs, bs))
    for a in range(n):
        blk = S[a * bs:(a + 1) * bs, a * bs:(a + 1) * bs]
        fac = scipy.linalg.cho_factor(blk, lower=True, check_finite=True)
        out[a] = scipy.linalg.cho_solve(fac, np.eye(bs))
    return out


def pcg(S, b, tol, max_iters, bs=9):
    """Preconditioned conjugate gradient on S x = b (App. A: the inexact solver of
    the split reduced camera systems), S symmetric positive definite, with the
    block-Jacobi preconditioner of `block_jacobi_inverse`: x = 0, r = b,
    z = M^-1 r, p = z; each iteration q = S p, alpha = r.z / p.q, x += alpha p,
    r -= alpha q, stop once ||r|| <= tol ||b||, else z = M^-1 r,
    beta = (r.z)_new / (r.z)_old, p = z + beta p.  At most max_iters iterations.
    Returns (x, iterations, ||r|| / ||b||, ok) with ok False when p.q <= 0 or a
    preconditioner block is not positive definite."""
    S = np.asarray(S, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0] // bs
    try:
        Minv = block_jacobi_inverse(S, bs)
    except (np.linalg.LinAlgError, ValueError):
        return np.zeros_like(b), 0, float("nan"), False

    def precond(v):
        return np.einsum("aij,aj->ai", Minv, v.reshape(n, bs)).reshape(-1)

    x = np.zeros_like(b)
    bn = float(np.linalg.norm(b))
    if bn == 0.0:
        return x, 0, 0.0, True
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    while it < max_iters:
        q = S @ p
        pq = float(p @ q)
        if not pq > 0.0:
            return x, it, float(np.linalg.norm(r)) / bn, False
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        if np.linalg.norm(r) <= tol * bn:
            break
        z = precond(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, float(np.linalg.norm(r)) / bn, True
