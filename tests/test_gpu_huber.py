"""The robust loss of the experiments (Sec. 5.1, Huber of scale 0.5 by IRLS
reweighting) on the GPU against the oracle: robust cost, reweighted residuals,
the cluster step (FP64 and MIXED) and one LM iteration, on scenes with 5%
gross outliers so that both branches of the loss are exercised."""
import copy

import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_00446_amd as S
import synth
from gpu_helpers import GpuProblem, rel

pytestmark = pytest.mark.gpu

A = 0.5


def _with_outliers(s, seed=3, frac=0.05, sigma=20.0):
    rng = np.random.default_rng(seed)
    t = copy.copy(s)
    t.obs_uv = s.obs_uv.copy()
    idx = rng.choice(s.q, size=int(frac * s.q), replace=False)
    t.obs_uv[idx] += rng.normal(0.0, sigma, size=(idx.size, 2))
    return t


def _sgc(scene, gamma, t, seed=0):
    e, w = synth.camera_graph(scene.obs_cam, scene.obs_pt, scene.m)
    return synth.sgc_map(e, w, scene.m, gamma, 10.0, seed, t)


def test_huber_residuals_and_cost_match_oracle():
    s = _with_outliers(synth.small_ring(m=40, n=3000, views=8, seed=1))
    g = GpuProblem(s, gamma_max=12, huber=A)
    f, Jc, Jp, cost = g.residual_jacobian()
    f0 = O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)
    Jc0, Jp0 = O.jacobian(s.cam0, s.pt0, s.obs_cam, s.obs_pt)
    ft, Jct, Jpt = O.irls(f0, Jc0, Jp0, A)
    w = O.huber_weight(np.sum(f0 * f0, axis=1), A)
    print(f"weights below 1: {np.mean(w < 1):.2f} of the observations")
    assert 0.05 < np.mean(w < 1) < 0.99          # both branches are exercised
    assert rel(f.cpu().numpy(), ft) < 1e-12
    assert rel(Jc.cpu().numpy().reshape(-1, 2, 9), Jct) < 1e-12
    assert rel(Jp.cpu().numpy().reshape(-1, 2, 3), Jpt) < 1e-12
    F = float(cost.cpu().numpy()[0])
    assert abs(F - O.robust_cost(f0, A)) <= 1e-12 * O.robust_cost(f0, A)


@pytest.mark.parametrize("precision,tol", [(S.STBA_FP64, 1e-9), (S.STBA_MIXED, 1e-4)])
def test_huber_cluster_step_matches_oracle(precision, tol):
    s = _with_outliers(synth.small_ring(m=40, n=3000, views=8, seed=1))
    lab = _sgc(s, 12, 1)
    g = GpuProblem(s, gamma_max=12, precision=precision, huber=A)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3, 0.8, 2, 1)
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3, 0.8, 2, 1, huber=A)
    assert np.all(cs == 0)
    print(f"precision {precision}: dcam rel {rel(dcam, ref.dcam):.2e} dpt rel {rel(dpt, ref.dpt):.2e}")
    assert rel(dcam, ref.dcam) < tol
    assert rel(dpt, ref.dpt) < tol


@pytest.mark.parametrize("precision,tol", [(S.STBA_FP64, 1e-9), (S.STBA_MIXED, 1e-4)])
def test_huber_lm_iteration_matches_oracle(precision, tol):
    s = _with_outliers(synth.small_ring(m=40, n=3000, views=8, seed=1))
    lab = _sgc(s, 12, 0)
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=12, lambda0=1e-3,
                       precision=precision, huber=A)
    sol.step(sol.sample(lab, alpha=1.0, seed=0, it=0))
    st = sol.read_state()
    ref = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3, 1.0, 0, 0, huber=A)
    print(f"precision {precision}: F_new {st['F_new']:.12e} oracle {ref.F_new:.12e}")
    assert st["status"] == 0
    assert bool(st["accepted"]) == ref.accepted
    assert abs(st["F_new"] - ref.F_new) <= tol * ref.F_new
    assert rel(sol.cam.cpu().numpy() - s.cam0, ref.cam - s.cam0) < tol


@pytest.mark.parametrize("bad", [-0.5, float("nan"), float("inf")])
def test_invalid_huber_scale_is_rejected(bad):
    s = synth.tiny_circle()
    with pytest.raises(S.StbaError):
        S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=8, huber=bad)
