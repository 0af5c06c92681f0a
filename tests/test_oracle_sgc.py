"""Pins of the oracle's camera graph and stochastic graph clustering (Sec. 4.4,
Eq. 16) against definitions written out here: the camera graph from sets of
seen points, the modularity of Sec. 4.4 summed over all camera pairs, and the
exact law of the final clustering under one-join-at-a-time draws, enumerated
over every join sequence of small graphs."""
import functools
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.stats

import oracle
import synth

# a 6-camera graph whose joins have very different probabilities at beta = 10
G6_EDGES = np.array([[0, 1], [1, 2], [2, 3], [3, 4], [0, 4], [1, 3], [4, 5], [2, 5]])
G6_W = np.array([6, 2, 5, 1, 3, 2, 4, 1])


def _adjacency(edges, w, m):
    A = np.zeros((m, m))
    for (i, j), x in zip(edges, w):
        A[i, j] += x
        A[j, i] += x
    return A


def _modularity(A, lab):
    """Q = 1/(2s) sum over all camera pairs (i, j) of (A_ij - k_i k_j / (2s)) [same cluster]."""
    k = A.sum(axis=1)
    two_s = A.sum()
    same = lab[:, None] == lab[None, :]
    return float(((A - np.outer(k, k) / two_s) * same).sum() / two_s)


def _canonical(lab):
    names, dense = np.unique(np.asarray(lab), return_inverse=True)
    return tuple(int(v) for v in dense)


def _exact_law(edges, w, m, gamma, beta, gain=None):
    """Law of the final map when each step joins one pair of neighbouring
    clusters within the cap with probability exp(beta dQ) / sum (Eq. 16), dQ the
    change of Q; `gain` replaces dQ (to show the test tells laws apart)."""
    A = _adjacency(edges, w, m)

    @functools.lru_cache(maxsize=None)
    def final(state):
        lab = np.array(state)
        q0 = _modularity(A, lab)
        cand = []
        ids = sorted(set(state))
        for ai, x in enumerate(ids):
            for y in ids[ai + 1:]:
                mx, my = lab == x, lab == y
                if A[np.ix_(mx, my)].sum() == 0 or mx.sum() + my.sum() > gamma:
                    continue
                joined = lab.copy()
                joined[my] = x
                dq = _modularity(A, joined) - q0 if gain is None else gain(A, lab, x, y)
                cand.append((dq, _canonical(joined)))
        if not cand:
            return {state: 1.0}
        z = sum(math.exp(beta * dq) for dq, _ in cand)
        out = {}
        for dq, nxt in cand:
            for fin, p in final(nxt).items():
                out[fin] = out.get(fin, 0.0) + p * math.exp(beta * dq) / z
        return out

    return final(tuple(range(m)))


def _chi2_pvalue(law, counts, n):
    keys = sorted(law, key=lambda k: -law[k])
    exp_, obs = [], []
    rest_e = rest_o = 0.0
    for k in keys:
        if law[k] * n >= 10:
            exp_.append(law[k] * n)
            obs.append(counts.get(k, 0))
        else:
            rest_e += law[k] * n
            rest_o += counts.get(k, 0)
    assert sum(counts.values()) == n and set(counts) <= set(law), "a map outside the law's support"
    if rest_e > 0:
        exp_.append(rest_e)
        obs.append(rest_o)
    return scipy.stats.chisquare(obs, exp_).pvalue


def test_covisibility_graph_counts_shared_points():
    rng = np.random.default_rng(3)
    m, n = 9, 60
    seen = [set(rng.choice(m, size=rng.integers(1, 5), replace=False).tolist()) for _ in range(n)]
    obs = sorted((j, i) for j, cams in enumerate(seen) for i in cams)
    obs_pt = np.array([o[0] for o in obs])
    obs_cam = np.array([o[1] for o in obs])
    edges, w = oracle.covisibility_graph(obs_cam, obs_pt, m, n)
    expect = {}
    for cams in seen:
        for i in cams:
            for j in cams:
                if i < j:
                    expect[(i, j)] = expect.get((i, j), 0) + 1
    assert {(int(i), int(j)): int(x) for (i, j), x in zip(edges, w)} == expect
    assert [tuple(e) for e in edges.tolist()] == sorted(expect)


def test_modularity_gain_is_the_change_of_q():
    rng = np.random.default_rng(11)
    m = 10
    iu = np.triu_indices(m, 1)
    keep = rng.random(iu[0].shape[0]) < 0.5
    edges = np.stack([iu[0][keep], iu[1][keep]], axis=1)
    w = rng.integers(1, 9, size=edges.shape[0])
    A = _adjacency(edges, w, m)
    s = A.sum() / 2.0
    for _ in range(20):
        lab = rng.integers(0, 4, size=m)
        x, y = sorted(rng.choice(np.unique(lab), size=2, replace=False)) if len(np.unique(lab)) > 1 else (0, 0)
        if x == y:
            continue
        mx, my = lab == x, lab == y
        w_xy = A[np.ix_(mx, my)].sum()
        Kx, Ky = A[mx].sum(), A[my].sum()
        joined = lab.copy()
        joined[my] = x
        assert oracle.modularity_gain(w_xy, Kx, Ky, s) == pytest.approx(
            _modularity(A, joined) - _modularity(A, lab), rel=1e-12, abs=1e-15)


def test_uniforms_lie_in_the_unit_interval_and_are_uniform():
    a = np.repeat(np.arange(100), 100)
    b = np.tile(np.arange(100), 100) + 100
    u = oracle.sgc_uniform(5, 3, 7, a, b)
    assert np.all(u > 0.0) and np.all(u <= 1.0)
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-3
    # the counter names the draw: another step, pair or iteration gives other numbers
    assert not np.array_equal(u, oracle.sgc_uniform(5, 3, 8, a, b))
    assert not np.array_equal(u, oracle.sgc_uniform(5, 4, 7, a, b))
    assert oracle.sgc_uniform(5, 3, 7, [4], [9])[0] == oracle.sgc_uniform(5, 3, 7, [4, 1], [9, 2])[0]


@pytest.mark.parametrize("gamma", [2, 3, 4])
def test_final_maps_follow_the_exact_law(gamma):
    m, beta, n = 6, 10.0, 3000
    law = _exact_law(G6_EDGES, G6_W, m, gamma, beta)
    assert abs(sum(law.values()) - 1.0) < 1e-12
    counts = {}
    for t in range(n):
        lab, l = oracle.sgc_clusters(G6_EDGES, G6_W, m, gamma, beta, seed=7, t=t)
        key = _canonical(lab)
        assert l == max(key) + 1
        counts[key] = counts.get(key, 0) + 1
    assert _chi2_pvalue(law, counts, n) > 1e-3
    # the same sample rejects plausible mistakes: no modularity term, the sign of
    # dQ flipped, beta dropped
    wrong = [
        lambda A, lab, x, y: A[np.ix_(lab == x, lab == y)].sum() / (A.sum() / 2),
        lambda A, lab, x, y: -(_modularity(A, np.where(lab == y, x, lab)) - _modularity(A, lab)),
        lambda A, lab, x, y: 0.0,
    ]
    for g in wrong:
        bad = _exact_law(G6_EDGES, G6_W, m, gamma, beta, gain=g)
        if max(abs(bad.get(k, 0.0) - law.get(k, 0.0)) for k in set(bad) | set(law)) > 0.05:
            assert _chi2_pvalue(bad, counts, n) < 1e-6


# a second graph: two dense triangles joined through camera 6 by weak edges, with
# one heavy edge across, so that the cap decides which communities can form
G7_EDGES = np.array([[0, 1], [1, 2], [0, 2], [3, 4], [4, 5], [3, 5], [2, 6], [6, 3], [1, 4], [0, 6]])
G7_W = np.array([9, 7, 8, 6, 9, 5, 1, 2, 12, 1])


@pytest.mark.parametrize("gamma,beta", [(5, 25.0), (6, 4.0)])
def test_final_maps_follow_the_exact_law_second_graph(gamma, beta):
    m, n = 7, 3000
    law = _exact_law(G7_EDGES, G7_W, m, gamma, beta)
    assert abs(sum(law.values()) - 1.0) < 1e-12
    assert len(law) > 3
    counts = {}
    for t in range(n):
        lab, l = oracle.sgc_clusters(G7_EDGES, G7_W, m, gamma, beta, seed=13, t=t)
        key = _canonical(lab)
        assert l == max(key) + 1 and np.bincount(lab).max() <= gamma
        counts[key] = counts.get(key, 0) + 1
    assert _chi2_pvalue(law, counts, n) > 1e-3
    wrong = [
        lambda A, lab, x, y: A[np.ix_(lab == x, lab == y)].sum() / (A.sum() / 2),
        lambda A, lab, x, y: -(_modularity(A, np.where(lab == y, x, lab)) - _modularity(A, lab)),
        lambda A, lab, x, y: 0.0,
    ]
    for g in wrong:
        bad = _exact_law(G7_EDGES, G7_W, m, gamma, beta, gain=g)
        if max(abs(bad.get(k, 0.0) - law.get(k, 0.0)) for k in set(bad) | set(law)) > 0.05:
            assert _chi2_pvalue(bad, counts, n) < 1e-6


def test_host_harness_draws_the_same_law():
    m, gamma, beta, n = 6, 3, 10.0, 3000
    law = _exact_law(G6_EDGES, G6_W, m, gamma, beta)
    counts = {}
    for t in range(n):
        key = _canonical(synth.sgc_map(G6_EDGES, G6_W.astype(float), m, gamma, beta, seed=1, t=t))
        counts[key] = counts.get(key, 0) + 1
    assert _chi2_pvalue(law, counts, n) > 1e-3


def test_cap_and_maximality_on_a_ring():
    s = synth.small_ring(m=40, n=3000, views=8, seed=1)
    edges, w = oracle.covisibility_graph(s.obs_cam, s.obs_pt, s.m, s.n)
    for gamma in (5, 12):
        for t in range(3):
            lab, l = oracle.sgc_clusters(edges, w, s.m, gamma, 10.0, seed=0, t=t)
            sizes = np.bincount(lab)
            assert sizes.shape[0] == l and sizes.max() <= gamma
            # no two neighbouring clusters could still join
            a, b = lab[edges[:, 0]], lab[edges[:, 1]]
            cross = a != b
            assert np.all(sizes[a[cross]] + sizes[b[cross]] > gamma)
            # numbered by smallest camera
            first = [int(np.flatnonzero(lab == k)[0]) for k in range(l)]
            assert first == sorted(first)


def test_uncapped_clustering_gives_the_connected_components():
    m = 12
    edges = np.array([[0, 1], [1, 2], [2, 3], [5, 6], [6, 8], [5, 8], [9, 11]])
    w = np.array([3, 1, 2, 4, 1, 1, 2])
    lab, l = oracle.sgc_clusters(edges, w, m, m, 10.0, seed=3, t=0)
    ncomp, comp = csgraph.connected_components(sp.csr_matrix((w, (edges[:, 0], edges[:, 1])), shape=(m, m)),
                                              directed=False)
    assert l == ncomp
    assert _canonical(lab) == _canonical(comp)


def test_degenerate_cases_keep_singletons():
    ident = tuple(range(7))
    edges = np.array([[0, 1], [1, 2], [3, 4]])
    w = np.array([1, 2, 3])
    assert _canonical(oracle.sgc_clusters(edges, w, 7, 1, 10.0, 0, 0)[0]) == ident
    assert oracle.sgc_clusters(np.zeros((0, 2)), np.zeros(0), 7, 5, 10.0, 0, 0)[1] == 7
    assert oracle.sgc_clusters(np.zeros((0, 2)), np.zeros(0), 1, 5, 10.0, 0, 0)[1] == 1


def test_maps_are_reproducible_and_change_with_the_iteration():
    s = synth.small_ring(m=40, n=3000, views=8, seed=1)
    edges, w = oracle.covisibility_graph(s.obs_cam, s.obs_pt, s.m, s.n)
    a, _ = oracle.sgc_clusters(edges, w, s.m, 10, 10.0, seed=4, t=2)
    b, _ = oracle.sgc_clusters(edges, w, s.m, 10, 10.0, seed=4, t=2)
    c, _ = oracle.sgc_clusters(edges, w, s.m, 10, 10.0, seed=4, t=3)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
