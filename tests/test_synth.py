"""Checks of the synthetic inputs and of the host clustering harness (Sec. 4.4)."""
import numpy as np
import pytest

import synth


def _check_problem(s):
    assert s.obs_cam.dtype == np.int32 and s.obs_pt.dtype == np.int32
    key = s.obs_pt.astype(np.int64) * s.m + s.obs_cam
    assert np.all(np.diff(key) > 0)          # sorted by (point, camera), no duplicates
    assert s.obs_cam.min() >= 0 and s.obs_cam.max() < s.m
    assert np.array_equal(np.unique(s.obs_pt), np.arange(s.n))
    assert s.obs_uv.shape == (s.q, 2) and np.all(np.isfinite(s.obs_uv))


def test_tiny_circle_shape():
    s = synth.tiny_circle()
    assert (s.m, s.n, s.q) == (16, 2000, 12000)
    _check_problem(s)
    assert np.all(s.cam_gt[:, 6] == 500.0) and np.all(s.cam_gt[:, 7:] == 0.0)


def test_ring_shape_small():
    s = synth.small_ring(m=30, n=2000, views=8)
    _check_problem(s)
    assert s.q == 16000
    assert np.all(np.bincount(s.obs_pt) == 8)


def test_slam_banded_small():
    s = synth.slam(m=300, n=3000, seed=1)
    _check_problem(s)
    counts = np.bincount(s.obs_pt)
    assert counts.min() >= 3 and counts.max() <= 15
    # banded: a point's cameras are consecutive
    starts = np.r_[0, np.cumsum(counts)[:-1]]
    span = s.obs_cam[starts + counts - 1] - s.obs_cam[starts] + 1
    assert np.array_equal(span, counts)


def _modularity(edges, w, lab):
    s = w.sum()
    k = np.zeros(lab.shape[0])
    np.add.at(k, edges[:, 0], w)
    np.add.at(k, edges[:, 1], w)
    inside = sum(w[e] for e in range(len(w)) if lab[edges[e, 0]] == lab[edges[e, 1]])
    K = np.zeros(lab.max() + 1)
    np.add.at(K, lab, k)
    return inside / s - np.sum(K * K) / (4 * s * s)


def test_sgc_respects_cap_and_raises_modularity():
    s = synth.small_ring(m=60, n=3000, views=6, seed=5)
    e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
    for t in range(3):
        lab = synth.sgc_map(e, w, s.m, gamma=15, beta=10.0, seed=2, t=t)
        sizes = np.bincount(lab)
        assert sizes.max() <= 15 and sizes.sum() == s.m
        q = _modularity(e, w, lab)
        assert -1.0 <= q <= 1.0 and q > _modularity(e, w, np.arange(s.m))
        # ids are 0..l-1 in order of each cluster's first camera
        first = [np.flatnonzero(lab == k)[0] for k in range(lab.max() + 1)]
        assert first == sorted(first)
    # a new iteration index draws a different clustering
    a = synth.sgc_map(e, w, s.m, 15, 10.0, 2, 0)
    b = synth.sgc_map(e, w, s.m, 15, 10.0, 2, 1)
    assert not np.array_equal(a, b)


def test_modularity_gain_formula_matches_brute_force():
    s = synth.small_ring(m=20, n=800, views=5, seed=6)
    e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
    lab = np.arange(s.m)
    x, y = e[0]
    tot = w.sum()
    k = np.zeros(s.m)
    np.add.at(k, e[:, 0], w)
    np.add.at(k, e[:, 1], w)
    dq = w[0] / tot - k[x] * k[y] / (2 * tot * tot)
    lab2 = lab.copy()
    lab2[lab2 == y] = x
    assert np.isclose(_modularity(e, w, lab2) - _modularity(e, w, lab), dq, rtol=1e-12)


def test_sequential_and_halves_maps():
    lab = synth.sequential_map(1000, 20, 120, seed=0, t=4)
    sizes = np.bincount(lab)
    assert np.all(np.diff(lab) >= 0) and np.all(sizes[:-1] >= 20) and np.all(sizes <= 120)
    assert np.array_equal(synth.halves_map(16), np.repeat([0, 1], 8))
