"""Many problems through one LM iteration (stba_lm_step_batched): each problem
of the batch keeps its own damping, cost and accept decision (Alg. 1 per
problem).  Checked against stepping every problem alone with stba_lm_step on
the same cluster maps (alpha = 1, so the constraint draws, keyed by global
indices, keep every link alike): the same accept decisions and damping, the
same costs and the same parameters to rounding (the batch sums each problem's
cost over its observations in another order than the one-problem path).  The
one-problem path is itself checked against the oracle in test_gpu_parity."""
import numpy as np
import pytest
import torch

import paper_2008_00446_amd as S
import synth
from gpu_helpers import rel

pytestmark = pytest.mark.gpu


def _batch(P=5):
    scenes = synth.diff_batch(seeds=range(P))
    # perturbed starts, so that the problems take different accept sequences
    out = []
    for b, s in enumerate(scenes):
        rng = np.random.default_rng(100 + b)
        cam = s.cam0.copy()
        cam[:, :6] += rng.normal(0.0, 1e-3 * (1 + b), size=(s.m, 6))
        out.append((cam, s.pt0.copy(), s.obs_cam, s.obs_pt, s.obs_uv))
    return scenes, out


@pytest.mark.parametrize("precision", [S.STBA_FP64, S.STBA_MIXED], ids=["fp64", "mixed"])
def test_batched_step_matches_each_problem_alone(precision):
    scenes, probs = _batch()
    K = 5
    maps = [[synth.sequential_map(s.m, 10, 40, b, t) for b, s in enumerate(scenes)] for t in range(K)]
    gamma = 40
    bs = S.BatchSolver(probs, gamma, precision=precision, lambda0=1e-3)
    for t in range(K):
        bs.step(bs.sample(maps[t], alpha=1.0, seed=0, it=t))
    torch.cuda.synchronize()
    got = bs.read_states()
    for b, (cam, pt, oc, op, uv) in enumerate(probs):
        sol = S.StbaSolver(cam, pt, oc, op, uv, min(gamma, cam.shape[0]), precision=precision, lambda0=1e-3)
        for t in range(K):
            sol.step(sol.sample(maps[t][b], alpha=1.0, seed=0, it=t))
        ref = sol.read_state()
        st = got[b]
        assert st["status"] == 0 and ref["status"] == 0
        assert st["n_accept"] == ref["n_accept"] and st["accepted"] == ref["accepted"], (b, st, ref)
        assert st["lambda_"] == ref["lambda_"], (b, st["lambda_"], ref["lambda_"])
        assert abs(st["F"] - ref["F"]) <= 1e-12 * ref["F"], (b, st["F"], ref["F"])
        tol = 1e-9 if precision == S.STBA_FP64 else 1e-5
        assert rel(bs.cam_of(b).cpu().numpy(), sol.cam.cpu().numpy()) < tol
        assert rel(bs.pt_of(b).cpu().numpy(), sol.pt.cpu().numpy()) < tol
    # every problem moved
    assert all(s["n_accept"] >= 1 for s in got)


def test_batched_step_rejects_a_cluster_spanning_two_problems():
    scenes, probs = _batch(P=2)
    m0 = scenes[0].m
    bs = S.BatchSolver(probs, m0 + scenes[1].m, precision=S.STBA_FP64)
    # one cluster over every camera of both problems
    cc = torch.zeros(bs.cam.shape[0], dtype=torch.int32, device="cuda")
    smp = S.make_sample(cc, 1, 1.0, 0, 0)
    cam0 = bs.cam.clone()
    bs.step(smp)
    torch.cuda.synchronize()
    for st in bs.read_states():
        assert st["status"] == -1   # STBA_EINVAL
        assert st["accepted"] == 0
    assert torch.equal(bs.cam, cam0) and m0 > 0


def test_batched_step_argument_checks():
    _, probs = _batch(P=2)
    bs = S.BatchSolver(probs, 40, precision=S.STBA_FP64)
    smp = bs.sample([synth.sequential_map(p[0].shape[0], 10, 40, 0, 0) for p in probs])
    with pytest.raises(S.StbaError):
        S.stba_lm_step_batched(bs.problem, bs.dims, smp, bs.states, 0, bs.prob_cam, bs.prob_pt, bs.prob_obs_off,
                               bs.precision, bs.ws)
    with pytest.raises(S.StbaError):
        S.stba_lm_step_batched(bs.problem, bs.dims, smp, bs.states, bs.n_prob, None, bs.prob_pt, bs.prob_obs_off,
                               bs.precision, bs.ws)
