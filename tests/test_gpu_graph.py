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


def test_profiled_step_matches_the_plain_step():
    """stba_lm_step_profiled records events between the phases and otherwise
    runs the same iteration: identical results, ordered events, named phases."""
    s = synth.small_ring(m=40, n=3000, views=8, seed=1)
    K = 3
    maps = _maps(s, 12, K)
    out = []
    for profiled in (False, True):
        sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=12, lambda0=1e-3)
        evs = [S.hip_events(S.STBA_NUM_PHASES + 1) for _ in range(K)] if profiled else None
        for t in range(K):
            sol.step(sol.sample(maps[t], it=t), events=None if evs is None else evs[t])
        torch.cuda.synchronize()
        out.append((sol.cam.cpu().numpy(), sol.pt.cpu().numpy(), sol.read_state()))
        if profiled:
            for ev in evs:
                ms = [S.event_ms(ev[k], ev[k + 1]) for k in range(S.STBA_NUM_PHASES)]
                assert all(v >= 0.0 for v in ms) and sum(ms) > 0.0
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2]["F"] == out[1][2]["F"] and out[0][2]["lambda_"] == out[1][2]["lambda_"]
    names = [S.stba_phase_name(k) for k in range(S.STBA_NUM_PHASES)]
    assert len(set(names)) == S.STBA_NUM_PHASES and all(names)
