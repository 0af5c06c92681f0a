"""Synthetic bundle-adjustment scenes shaped like the paper's workloads.

The paper's datasets (1DSfM, KITTI and its private large-scale sets, Sec. 5.1 and
Table 1) are not available, so every scene here is drawn from a seeded
``numpy.random.default_rng`` with the camera counts, track lengths, visibility
structure and pixel-noise levels of the workload it stands in for.

Camera convention used to *synthesise* observations (written in matrix form on
purpose, independent of any angle-axis code): a camera has a world->camera
rotation matrix R (rows are the camera axes, the third one is the viewing
direction), a translation t = -R C, a focal length f and radial distortion
k1, k2.  A world point X maps to P = R X + t, (x, y) = (P_x, P_y) / P_z,
r2 = x^2 + y^2 and pixel = f (1 + k1 r2 + k2 r2^2) (x, y), image-centred.  The
9 stored camera parameters are (rotation vector of R, t, f, k1, k2); the
rotation vector comes from ``scipy.spatial.transform.Rotation``.

Observations are sorted by (point, camera), one per visible (camera, point).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = ["Scene", "tiny_circle", "ring", "small_ring", "internet", "slam", "diff_batch"]


@dataclass
class Scene:
    """A bundle-adjustment problem with its ground truth.

    cam_gt, pt_gt   ground-truth cameras [m,9] and points [n,3]
    cam0, pt0       perturbed starting values (what the solver is given)
    obs_cam, obs_pt int32 [q], sorted by (obs_pt, obs_cam)
    obs_uv          float64 [q,2] noisy pixel observations
    obs_uv_clean    float64 [q,2] the same without noise
    """

    cam_gt: np.ndarray
    pt_gt: np.ndarray
    cam0: np.ndarray
    pt0: np.ndarray
    obs_cam: np.ndarray
    obs_pt: np.ndarray
    obs_uv: np.ndarray
    obs_uv_clean: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.cam_gt.shape[0])

    @property
    def n(self) -> int:
        return int(self.pt_gt.shape[0])

    @property
    def q(self) -> int:
        return int(self.obs_cam.shape[0])


# ----------------------------------------------------------------------------
# geometry helpers (generator side only)
# ----------------------------------------------------------------------------

def _look_at(centres: np.ndarray, targets: np.ndarray, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World->camera rotation matrices [k,3,3] whose third row points at target."""
    z = targets - centres
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    upv = np.broadcast_to(np.asarray(up, dtype=np.float64), z.shape)
    x = np.cross(upv, z)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=1)


def _forward_frames(forward: np.ndarray, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    return _look_at(np.zeros_like(forward), forward, up)


def _cam_space(R: np.ndarray, t: np.ndarray, X: np.ndarray) -> np.ndarray:
    """P = R X + t for matching rows of R [k,3,3], t [k,3], X [k,3]."""
    return np.einsum("kab,kb->ka", R, X) + t


def _pixels(P: np.ndarray, f: np.ndarray, k1: np.ndarray, k2: np.ndarray) -> np.ndarray:
    xy = P[:, :2] / P[:, 2:3]
    r2 = np.sum(xy * xy, axis=1)
    scale = f * (1.0 + k1 * r2 + k2 * r2 * r2)
    return xy * scale[:, None]


def _assemble(name, R, C, intr, X, vis_cam, vis_pt, rng, noise_px, rot_pert=0.01,
              t_pert=0.05, pt_pert=0.05, meta=None, keep_centres=False) -> Scene:
    """Sort the visibility list, synthesise pixels, perturb the start values.

    keep_centres: after the rotation-vector offset, t is recomputed so that each
    camera keeps its centre (then the translation noise is added).  Without it a
    0.01 rad offset turns a camera about the world origin, which on a scene
    kilometres across moves it by tens of metres."""
    m = R.shape[0]
    n = X.shape[0]
    order = np.lexsort((vis_cam, vis_pt))
    obs_cam = vis_cam[order].astype(np.int32)
    obs_pt = vis_pt[order].astype(np.int32)
    t = -np.einsum("kab,kb->ka", R, C)
    P = _cam_space(R[obs_cam], t[obs_cam], X[obs_pt])
    if np.any(P[:, 2] <= 0.5):
        raise ValueError(f"{name}: a visible point lies behind or too close to its camera")
    clean = _pixels(P, intr[obs_cam, 0], intr[obs_cam, 1], intr[obs_cam, 2])
    uv = clean + rng.normal(0.0, noise_px, size=clean.shape)
    omega = Rotation.from_matrix(R).as_rotvec()
    cam_gt = np.concatenate([omega, t, intr], axis=1)
    # start values: a random-direction 0.01 rad offset on the rotation vector,
    # N(0, 0.05^2) on t and on every point coordinate; intrinsics exact.
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    cam0 = cam_gt.copy()
    cam0[:, 0:3] += rot_pert * d
    if keep_centres:
        cam0[:, 3:6] = -np.einsum("kab,kb->ka", Rotation.from_rotvec(cam0[:, 0:3]).as_matrix(), C)
    cam0[:, 3:6] += rng.normal(0.0, t_pert, size=(m, 3))
    pt0 = X + rng.normal(0.0, pt_pert, size=(n, 3))
    return Scene(cam_gt=cam_gt, pt_gt=X.copy(), cam0=cam0, pt0=pt0, obs_cam=obs_cam,
                 obs_pt=obs_pt, obs_uv=uv, obs_uv_clean=clean, name=name, meta=dict(meta or {}))


def _drop_unseen(X, vis_cam, vis_pt, min_views):
    counts = np.bincount(vis_pt, minlength=X.shape[0])
    keep = counts >= min_views
    remap = -np.ones(X.shape[0], dtype=np.int64)
    remap[keep] = np.arange(int(keep.sum()))
    sel = keep[vis_pt]
    return X[keep], vis_cam[sel], remap[vis_pt[sel]]


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def tiny_circle(seed: int = 0) -> Scene:
    """16 cameras on a radius-10 circle (z = 0) looking at the origin, world +z up;
    2000 points ~ U[-2,2]^3, each seen by the 6 cameras nearest to it in azimuth
    (q = 12000); f = 500, k1 = k2 = 0, N(0, 1 px) noise."""
    rng = np.random.default_rng(seed)
    m, n, views = 16, 2000, 6
    az = 2.0 * np.pi * np.arange(m) / m
    C = np.stack([10.0 * np.cos(az), 10.0 * np.sin(az), np.zeros(m)], axis=1)
    R = _look_at(C, np.zeros_like(C))
    intr = np.tile([500.0, 0.0, 0.0], (m, 1))
    X = rng.uniform(-2.0, 2.0, size=(n, 3))
    psi = np.arctan2(X[:, 1], X[:, 0])
    dang = np.abs(np.angle(np.exp(1j * (psi[:, None] - az[None, :]))))
    nearest = np.argsort(dang, axis=1, kind="stable")[:, :views]
    vis_pt = np.repeat(np.arange(n), views)
    vis_cam = nearest.reshape(-1)
    return _assemble("tiny_circle", R, C, intr, X, vis_cam, vis_pt, rng, 1.0,
                     meta=dict(views=views))


def ring(m: int = 200, n: int = 50_000, views: int = 8, seed: int = 0, radius: float = 30.0) -> Scene:
    """Cameras on three perturbed rings (heights 1, 2.5, 4) around the box
    [-10,10]^2 x [0,5]; points uniform in the box, each with a random horizontal
    normal and seen by the `views` cameras at the smallest angle to that normal.
    f ~ N(800, 40), k1 ~ U(-0.1, 0.1), k2 ~ U(-0.01, 0.01), N(0, 1 px) noise."""
    rng = np.random.default_rng(seed)
    counts = [m // 3 + (1 if r < m % 3 else 0) for r in range(3)]
    heights = [1.0, 2.5, 4.0]
    C, T = [], []
    for r, cnt in enumerate(counts):
        spacing = 2.0 * np.pi / cnt
        az = spacing * np.arange(cnt) + rng.uniform(-0.5, 0.5, cnt) * spacing
        rad = radius * (1.0 + rng.normal(0.0, 0.02, cnt))
        h = heights[r] + rng.normal(0.0, 0.2, cnt)
        C.append(np.stack([rad * np.cos(az), rad * np.sin(az), h], axis=1))
        T.append(np.array([0.0, 0.0, 2.5]) + rng.normal(0.0, 0.5, (cnt, 3)))
    C = np.concatenate(C)
    T = np.concatenate(T)
    R = _look_at(C, T)
    intr = np.stack([rng.normal(800.0, 40.0, m), rng.uniform(-0.1, 0.1, m),
                     rng.uniform(-0.01, 0.01, m)], axis=1)
    X = np.stack([rng.uniform(-10, 10, n), rng.uniform(-10, 10, n), rng.uniform(0, 5, n)], axis=1)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    normal = np.stack([np.cos(phi), np.sin(phi), np.zeros(n)], axis=1)
    views = min(views, m)
    vis_cam = np.empty((n, views), dtype=np.int64)
    for a in range(0, n, 8192):
        b = min(n, a + 8192)
        d = C[None, :, :] - X[a:b, None, :]
        d /= np.linalg.norm(d, axis=2, keepdims=True)
        cosang = np.einsum("pcd,pd->pc", d, normal[a:b])
        vis_cam[a:b] = np.argsort(-cosang, axis=1, kind="stable")[:, :views]
    vis_pt = np.repeat(np.arange(n), views)
    return _assemble(f"ring_m{m}_n{n}", R, C, intr, X, vis_cam.reshape(-1), vis_pt, rng, 1.0,
                     meta=dict(views=views))


def small_ring(m: int = 40, n: int = 3000, views: int = 8, seed: int = 1) -> Scene:
    """A scaled-down ring scene for parity tests (same recipe as `ring`)."""
    return ring(m=m, n=n, views=views, seed=seed)


def internet(seed: int = 0, m: int = 1000, n: int = 300_000, landmarks: int = 10,
             mean_views: float = 2400.0, lo: int = 200, hi: int = 5000) -> Scene:
    """Internet-photo-like scene: `landmarks` sites over a 200 x 200 m area, an
    equal share of the points on each (uniform in a 30 x 30 x 20 m block), an
    equal share of cameras per site at 20-60 m distance with azimuths from a
    von Mises mixture over 3 popular directions; camera i keeps
    clip(LogNormal(mu, 1), lo, hi) of its site's in-view points (mu bisected so
    the mean is `mean_views`).  Points seen fewer than twice are dropped."""
    rng = np.random.default_rng(seed)
    centres = np.stack([rng.uniform(-100, 100, landmarks), rng.uniform(-100, 100, landmarks),
                        np.zeros(landmarks)], axis=1)
    site_of_pt = np.repeat(np.arange(landmarks), n // landmarks)
    n = site_of_pt.shape[0]
    X = centres[site_of_pt] + np.stack([rng.uniform(-15, 15, n), rng.uniform(-15, 15, n),
                                        rng.uniform(0, 20, n)], axis=1)
    site_of_cam = np.repeat(np.arange(landmarks), m // landmarks)
    m = site_of_cam.shape[0]
    popular = rng.uniform(0, 2 * np.pi, (landmarks, 3))
    which = rng.integers(0, 3, m)
    az = rng.vonmises(popular[site_of_cam, which], 4.0)
    dist = np.clip(np.where(rng.random(m) < 0.6, rng.normal(30, 5, m), rng.normal(50, 5, m)), 20, 60)
    C = centres[site_of_cam] + np.stack([dist * np.cos(az), dist * np.sin(az),
                                         1.7 + np.abs(rng.normal(0, 1.0, m))], axis=1)
    T = centres[site_of_cam] + np.array([0.0, 0.0, 10.0]) + rng.normal(0, 3.0, (m, 3))
    R = _look_at(C, T)
    intr = np.stack([rng.normal(800.0, 40.0, m), rng.uniform(-0.1, 0.1, m),
                     rng.uniform(-0.01, 0.01, m)], axis=1)
    z = rng.normal(size=m)

    def clipped_mean(mu):
        return float(np.mean(np.clip(np.exp(mu + z), lo, hi)))

    a, b = np.log(lo), np.log(hi)
    for _ in range(60):
        mid = 0.5 * (a + b)
        a, b = (mid, b) if clipped_mean(mid) < mean_views else (a, mid)
    nviews = np.clip(np.exp(0.5 * (a + b) + z), lo, hi).astype(np.int64)
    t = -np.einsum("kab,kb->ka", R, C)
    pts_of_site = [np.nonzero(site_of_pt == s)[0] for s in range(landmarks)]
    vis_cam, vis_pt = [], []
    for i in range(m):
        cand = pts_of_site[site_of_cam[i]]
        P = X[cand] @ R[i].T + t[i]
        xy = P[:, :2] / P[:, 2:3]
        ok = (P[:, 2] > 2.0) & (np.abs(xy[:, 0]) < 0.6) & (np.abs(xy[:, 1]) < 0.6)
        cand = cand[ok]
        k = min(int(nviews[i]), cand.shape[0])
        pick = rng.choice(cand, size=k, replace=False)
        vis_pt.append(pick)
        vis_cam.append(np.full(k, i))
    vis_cam = np.concatenate(vis_cam)
    vis_pt = np.concatenate(vis_pt)
    X, vis_cam, vis_pt = _drop_unseen(X, vis_cam, vis_pt, 2)
    return _assemble("internet", R, C, intr, X, vis_cam, vis_pt, rng, 1.0,
                     meta=dict(landmarks=landmarks, site_of_cam=site_of_cam))


def slam(seed: int = 0, m: int = 5000, n: int = 1_000_000, p_geom: float = 0.25,
         lmin: int = 3, lmax: int = 15) -> Scene:
    """Sequential SLAM-like scene: m cameras along a smooth sum-of-sinusoids path
    resampled to 1 m spacing, each looking along the tangent with up to 2 deg of
    jitter; n points with track length L = min(lmin + Geom(p_geom), lmax), a
    uniformly drawn first camera s and visibility in cameras s..s+L-1 (banded),
    each point at depth U(5, 40) m and within a 25 deg cone of its last camera;
    N(0, 0.7 px) noise."""
    rng = np.random.default_rng(seed)
    s = np.linspace(0.0, 1.3 * m, 40 * m)
    path = np.stack([s, 40.0 * np.sin(s / 300.0) + 15.0 * np.sin(s / 97.0),
                     3.0 * np.sin(s / 211.0)], axis=1)
    seg = np.linalg.norm(np.diff(path, axis=0), axis=1)
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    want = np.arange(m, dtype=np.float64)
    C = np.stack([np.interp(want, arc, path[:, k]) for k in range(3)], axis=1)
    fwd = np.gradient(C, axis=0)
    fwd /= np.linalg.norm(fwd, axis=1, keepdims=True)
    R = _forward_frames(fwd)
    jit = Rotation.from_rotvec(np.deg2rad(2.0) * rng.uniform(-1, 1, (m, 1)) *
                               _unit(rng.normal(size=(m, 3))))
    R = np.einsum("kab,kbc->kac", jit.as_matrix(), R)
    intr = np.stack([rng.normal(800.0, 40.0, m), rng.uniform(-0.1, 0.1, m),
                     rng.uniform(-0.01, 0.01, m)], axis=1)
    t = -np.einsum("kab,kb->ka", R, C)
    L = np.minimum(lmin + rng.geometric(p_geom, n) - 1, lmax)
    first = rng.integers(0, m - L + 1)
    X = np.empty((n, 3))
    todo = np.arange(n)
    for _ in range(50):
        if todo.size == 0:
            break
        last = first[todo] + L[todo] - 1
        k = todo.size
        ang = np.deg2rad(25.0) * np.sqrt(rng.random(k))
        phi = rng.uniform(0, 2 * np.pi, k)
        ray = np.stack([np.sin(ang) * np.cos(phi), np.sin(ang) * np.sin(phi), np.cos(ang)], axis=1)
        depth = rng.uniform(5.0, 40.0, k)
        Pc = ray * (depth / ray[:, 2])[:, None]
        X[todo] = np.einsum("kba,kb->ka", R[last], Pc - t[last])
        ok = np.ones(k, dtype=bool)
        for d in range(lmax):
            sel = d < L[todo]
            ci = np.where(sel, first[todo] + d, last)
            P = np.einsum("kab,kb->ka", R[ci], X[todo]) + t[ci]
            xy = P[:, :2] / P[:, 2:3]
            good = (P[:, 2] > 2.0) & (np.abs(xy[:, 0]) < 0.8) & (np.abs(xy[:, 1]) < 0.8)
            ok &= good | ~sel
        todo = todo[~ok]
    if todo.size:
        raise RuntimeError("slam: could not place every point in view")
    vis_pt = np.repeat(np.arange(n), L)
    offs = np.arange(vis_pt.shape[0]) - np.repeat(np.cumsum(L) - L, L)
    vis_cam = first[vis_pt] + offs
    return _assemble("slam", R, C, intr, X, vis_cam, vis_pt, rng, 0.7,
                     meta=dict(track_mean=float(L.mean())), keep_centres=True)


def _unit(v):
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def diff_batch(seeds=range(64), views: int = 7):
    """Many independent small ring problems: m_b ~ U{30..120}, n_b ~ U{5k..30k},
    `views` observations per point; problem b uses seed b."""
    out = []
    for s in seeds:
        rng = np.random.default_rng(10_000 + int(s))
        mb = int(rng.integers(30, 121))
        nb = int(rng.integers(5_000, 30_001))
        out.append(ring(m=mb, n=nb, views=views, seed=int(s)))
    return out
