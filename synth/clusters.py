"""Camera->cluster maps, the per-iteration input of the STBA hot path.

The hot path takes the camera clustering {Phi_k} of an iteration as an input
(Alg. 1 draws it first, then builds A from it).  This module makes those maps on
the host:

* ``sgc_map``: stochastic graph clustering (Sec. 4.4, Eq. 16).  The camera graph
  weighs an edge by the number of points both cameras see.  Starting from
  singletons, two neighbouring clusters x, y whose joint size stays within Gamma
  are joined with probability proportional to exp(beta * dQ(x, y)), with the
  modularity gain dQ(x, y) = w_xy / s - K_x K_y / (2 s^2) (w_xy: weight between
  the clusters, K: summed incident weight, s: total weight).  Joining stops when
  no eligible pair is left.
* ``sequential_map``: contiguous runs of U{lo..hi} cameras (sequential data).
* ``halves_map``: a fixed split into equal contiguous halves.

Every map is relabelled so cluster ids are 0..l-1 in order of each cluster's
smallest camera id.  Randomness comes from numpy's Philox keyed by
(seed, domain 1) with the iteration t in the counter.
"""
from __future__ import annotations

import numpy as np

__all__ = ["camera_graph", "sgc_map", "sequential_map", "halves_map", "relabel", "map_rng"]


def map_rng(seed: int, t: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=np.array([seed, 1], dtype=np.uint64),
                                                counter=np.array([t, 0, 0, 0], dtype=np.uint64)))


def relabel(cam_cluster: np.ndarray) -> np.ndarray:
    """Renumber clusters 0..l-1 by their smallest camera id."""
    lab = np.asarray(cam_cluster)
    _, first, inv = np.unique(lab, return_index=True, return_inverse=True)
    rank = np.empty(first.shape[0], dtype=np.int32)
    rank[np.argsort(first, kind="stable")] = np.arange(first.shape[0], dtype=np.int32)
    return rank[inv.reshape(-1)]


def camera_graph(obs_cam: np.ndarray, obs_pt: np.ndarray, m: int):
    """Edges (i < j) of the covisibility graph and their weights (shared points)."""
    obs_cam = np.asarray(obs_cam, dtype=np.int64)
    obs_pt = np.asarray(obs_pt, dtype=np.int64)
    starts = np.flatnonzero(np.r_[True, obs_pt[1:] != obs_pt[:-1]])
    ends = np.r_[starts[1:], obs_pt.shape[0]]
    keys = []
    lens = ends - starts
    for v in np.unique(lens):
        if v < 2:
            continue
        s = starts[lens == v]
        block = obs_cam[s[:, None] + np.arange(v)[None, :]]
        a, b = np.triu_indices(v, 1)
        i = np.minimum(block[:, a], block[:, b]).reshape(-1)
        j = np.maximum(block[:, a], block[:, b]).reshape(-1)
        keys.append(i * m + j)
    if not keys:
        return np.zeros((0, 2), dtype=np.int64), np.zeros(0, dtype=np.float64)
    keys, w = np.unique(np.concatenate(keys), return_counts=True)
    return np.stack([keys // m, keys % m], axis=1), w.astype(np.float64)


def sgc_map(edges: np.ndarray, weights: np.ndarray, m: int, gamma: int, beta: float = 10.0,
            seed: int = 0, t: int = 0) -> np.ndarray:
    """Stochastic graph clustering with cluster-size cap `gamma`."""
    rng = map_rng(seed, t)
    lab = np.arange(m)
    size = np.ones(m, dtype=np.int64)
    s = float(weights.sum())
    if s == 0.0 or gamma <= 1:
        return relabel(lab)
    deg = np.zeros(m)
    np.add.at(deg, edges[:, 0], weights)
    np.add.at(deg, edges[:, 1], weights)
    K = deg.copy()
    ex, ey, ew = edges[:, 0].copy(), edges[:, 1].copy(), weights.copy()
    while ex.size:
        ok = size[ex] + size[ey] <= gamma
        if not ok.any():
            break
        idx = np.flatnonzero(ok)
        dq = ew[idx] / s - K[ex[idx]] * K[ey[idx]] / (2.0 * s * s)
        p = np.exp(beta * (dq - dq.max()))
        e = idx[rng.choice(idx.size, p=p / p.sum())]
        x, y = ex[e], ey[e]
        lab[lab == y] = x
        size[x] += size[y]
        K[x] += K[y]
        ex = np.where(ex == y, x, ex)
        ey = np.where(ey == y, x, ey)
        keep = ex != ey
        a = np.minimum(ex[keep], ey[keep])
        b = np.maximum(ex[keep], ey[keep])
        key, inv = np.unique(a * m + b, return_inverse=True)
        ew = np.bincount(inv, weights=ew[keep])
        ex, ey = key // m, key % m
    return relabel(lab)


def sequential_map(m: int, lo: int, hi: int, seed: int = 0, t: int = 0) -> np.ndarray:
    """Contiguous runs of U{lo..hi} cameras; the last run takes the remainder."""
    rng = map_rng(seed, t)
    lab = np.empty(m, dtype=np.int32)
    start, k = 0, 0
    while start < m:
        size = int(rng.integers(lo, hi + 1))
        lab[start:start + size] = k
        start += size
        k += 1
    return lab


def halves_map(m: int, parts: int = 2) -> np.ndarray:
    return (np.arange(m) * parts // m).astype(np.int32)
