"""Stochastic graph clustering on the device (Sec. 4.4, Eq. 16) against the
oracle: the map of every camera and the number of clusters, bit-exact, on the
200-camera ring (graph of 1713 edges, clocks in registers), a 600-camera ring
and the 1000-camera Internet-like scene (graphs above 4096 blocks, clocks in
the workspace), over several iterations, caps and scales; the degenerate caps;
argument errors; and an LM iteration driven by a device-drawn map."""
import functools

import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_00446_amd as S
import synth
from gpu_helpers import GpuProblem, dev

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _scene(name):
    if name == "ring200":
        return synth.ring(m=200, n=50_000, views=8, seed=0)
    if name == "ring600":
        return synth.ring(m=600, n=30_000, views=8, seed=2)
    if name == "internet":
        return synth.internet(seed=0)
    if name == "small":
        return synth.small_ring(m=40, n=3000, views=8, seed=1)
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def _graph(name):
    s = _scene(name)
    return O.covisibility_graph(s.obs_cam, s.obs_pt, s.m, s.n)


@functools.lru_cache(maxsize=None)
def _problem(name, gamma_max):
    return GpuProblem(_scene(name), gamma_max=gamma_max)


def _device_map(g, gamma, beta, seed, t):
    m = g.prob.m
    cc = torch.full((m,), -7, dtype=torch.int32, device="cuda")
    out = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    S.stba_sample_clusters(g.prob, g.dims, g.precision, g.ws, gamma, beta, seed, t, cc, out[0:1], out[1:2])
    torch.cuda.synchronize()
    l, status = out.cpu().tolist()
    return cc.cpu().numpy(), l, status


def _check(name, gamma, beta, seed, t, gamma_max=None):
    g = _problem(name, gamma_max or gamma)
    edges, w = _graph(name)
    lab, l = O.sgc_clusters(edges, w, g.prob.m, gamma, beta, seed, t)
    got, gl, status = _device_map(g, gamma, beta, seed, t)
    print(f"sgc {name} gamma={gamma} beta={beta} seed={seed} t={t}: l={l} (device {gl})", flush=True)
    assert status == 0
    assert gl == l
    np.testing.assert_array_equal(got, lab)
    return lab


@pytest.mark.parametrize("t", [0, 1, 2, 7])
def test_ring_maps_match_oracle(t):
    lab = _check("ring200", 50, 10.0, 0, t)
    assert np.bincount(lab).max() <= 50


@pytest.mark.parametrize("gamma,beta,seed", [(2, 10.0, 3), (13, 10.0, 1), (40, 0.0, 5), (40, 25.0, 9)])
def test_small_ring_caps_and_scales(gamma, beta, seed):
    _check("small", gamma, beta, seed, 4, gamma_max=40)


def test_uncapped_map_is_one_cluster_and_cap_one_is_singletons():
    lab = _check("small", 40, 10.0, 0, 0, gamma_max=40)
    assert lab.max() == 0
    lab = _check("small", 1, 10.0, 0, 0, gamma_max=40)
    np.testing.assert_array_equal(lab, np.arange(40))


@pytest.mark.parametrize("t", [0, 3])
def test_large_graph_in_workspace_matches_oracle(t):
    edges, _ = _graph("ring600")
    assert edges.shape[0] + 600 > 4096      # the blocks do not fit the register slots
    _check("ring600", 60, 10.0, 11, t)


def test_internet_like_scene_matches_oracle():
    lab = _check("internet", 100, 10.0, 0, 0)
    assert np.bincount(lab).max() <= 100


def test_repeated_calls_reuse_the_workspace():
    # two maps in a row on the same workspace, the second one of another cap
    _check("small", 13, 10.0, 2, 0, gamma_max=40)
    _check("small", 6, 10.0, 2, 1, gamma_max=40)
    _check("small", 13, 10.0, 2, 0, gamma_max=40)


def test_bad_arguments_are_rejected():
    g = _problem("small", 40)
    cc = torch.zeros(40, dtype=torch.int32, device="cuda")
    out = torch.zeros(2, dtype=torch.int32, device="cuda")
    for gamma, beta in [(0, 10.0), (41, 10.0), (5, -1.0), (5, float("nan")), (5, float("inf"))]:
        with pytest.raises(S.StbaError):
            S.stba_sample_clusters(g.prob, g.dims, g.precision, g.ws, gamma, beta, 0, 0, cc, out[0:1], out[1:2])


def test_more_cameras_than_one_workgroup_holds_is_rejected():
    m = 6145   # one workgroup's LDS holds the clustering of up to 6144 cameras
    obs_pt = np.repeat(np.arange(m - 1), 2).astype(np.int32)
    obs_cam = np.stack([np.arange(m - 1), np.arange(1, m)], axis=1).reshape(-1).astype(np.int32)
    cam = np.zeros((m, 9))
    cam[:, 5] = 10.0
    cam[:, 6] = 500.0
    pt = np.zeros((m - 1, 3))
    uv = np.zeros((obs_pt.shape[0], 2))
    prob = S.make_problem(dev(cam, torch.float64), dev(pt, torch.float64), dev(obs_cam, torch.int32),
                          dev(obs_pt, torch.int32), dev(uv, torch.float64))
    dims = S.stba_analyze(prob)
    dims.gamma_max = 4
    ws = S.alloc_workspace(S.stba_workspace_bytes(prob, dims, S.STBA_FP64))
    S.stba_prepare(prob, dims, S.STBA_FP64, ws)
    cc = torch.zeros(m, dtype=torch.int32, device="cuda")
    out = torch.zeros(2, dtype=torch.int32, device="cuda")
    with pytest.raises(S.StbaError):
        S.stba_sample_clusters(prob, dims, S.STBA_FP64, ws, 4, 10.0, 0, 0, cc, out[0:1], out[1:2])


def test_lm_iteration_on_a_device_map_matches_oracle():
    s = _scene("small")
    edges, w = _graph("small")
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=12, lambda0=1e-3)
    for t in range(2):
        samp = sol.sample_clusters(12, beta=10.0, seed=5, it=t)
        lab, l = O.sgc_clusters(edges, w, s.m, 12, 10.0, 5, t)
        assert samp.l == l
        cam0 = sol.cam.cpu().numpy()
        pt0 = sol.pt.cpu().numpy()
        lam = sol.read_state()["lambda_"]
        sol.step(samp)
        st = sol.read_state()
        ref = O.lm_iteration(cam0, pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, 1.0, 5, t)
        assert bool(st["accepted"]) == ref.accepted
        assert st["F_new"] == pytest.approx(ref.F_new, rel=1e-9)
        np.testing.assert_allclose(sol.cam.cpu().numpy(), ref.cam, rtol=0, atol=1e-9 * np.abs(ref.cam).max())


def test_uncapped_ring_is_plain_lm_in_one_cluster():
    # Gamma = m: every camera joins one cluster (the ring's graph is connected), so
    # the iteration is one dense 1800 x 1800 solve (App. B: STBA equals LM there)
    s = _scene("ring200")
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=s.m, lambda0=1e-4)
    samp = sol.sample_clusters(s.m, beta=10.0, seed=0, it=0)
    assert samp.l == 1
    sol.step(samp)
    st = sol.read_state()
    ref = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, np.zeros(s.m, dtype=np.int64), 1e-4, 1.0, 0, 0)
    assert st["status"] == 0 and bool(st["accepted"]) == ref.accepted
    assert st["F_new"] == pytest.approx(ref.F_new, rel=1e-9)
    dc = sol.cam.cpu().numpy() - s.cam0
    assert np.linalg.norm(dc - (ref.cam - s.cam0)) <= 1e-9 * np.linalg.norm(ref.cam - s.cam0)

