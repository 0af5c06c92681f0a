"""The per-iteration calls under HIP graph capture: three LM iterations
captured once (through torch.cuda.graph, on its capture stream) and replayed
three times, with eager work between the replays (x and the LM state reset);
every replay must reproduce the eager iterations bit for bit, since every sum
in the path has a fixed order."""
import numpy as np
import pytest
import torch

import paper_2008_00446_amd as S
import synth

pytestmark = pytest.mark.gpu


def _maps(s, gamma, k):
    e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
    return [synth.sgc_map(e, w, s.m, gamma, 10.0, 0, t) for t in range(k)]


@pytest.mark.parametrize("precision", [S.STBA_FP64, S.STBA_MIXED], ids=["fp64", "mixed"])
def test_captured_iterations_replay_the_eager_ones(precision):
    s = synth.small_ring(m=40, n=3000, views=8, seed=1)
    K, lam0 = 3, 1e-3
    maps = _maps(s, 12, K)
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=12, precision=precision,
                       lambda0=lam0)
    samples = [sol.sample(maps[t], it=t) for t in range(K)]
    cam0, pt0 = sol.cam.clone(), sol.pt.clone()

    def reset():
        sol.cam.copy_(cam0)
        sol.pt.copy_(pt0)
        S.stba_lm_init(sol.state, lam0, 0.1)

    # eager reference (also initialises everything the launches query once)
    reset()
    for t in range(K):
        sol.step(samples[t])
    torch.cuda.synchronize()
    ref_cam, ref_pt, ref_state = sol.cam.clone(), sol.pt.clone(), sol.read_state()
    assert ref_state["status"] == 0 and ref_state["n_accept"] >= 1

    reset()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for t in range(K):
            sol.step(samples[t])
    torch.cuda.synchronize()
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        st = sol.read_state()
        print(f"graph replay {rep}: F={st['F']} accepted={st['n_accept']}", flush=True)
        assert torch.equal(sol.cam, ref_cam) and torch.equal(sol.pt, ref_pt), rep
        for key in ("F", "lambda_", "n_accept", "n_jac", "status"):
            assert st[key] == ref_state[key], (rep, key)
