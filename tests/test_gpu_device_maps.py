"""Camera clusterings drawn on the device feeding the LM step with no
read-back: the number of clusters is read on the device (stba_sample.l_dev,
l = m a bound).  Checked against the same steps with the count read back to
the host (bit for bit), the device clustering against the oracle above the
former 2048-camera limit, a HIP graph of draw + step replayed against the eager
iterations, and a device count out of range rejecting the step."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_00446_amd as S
import synth

pytestmark = pytest.mark.gpu


def _state_equal(a, b):
    return all(a[k] == b[k] or (np.isnan(a[k]) and np.isnan(b[k])) for k in a)


@pytest.mark.parametrize("which,gamma", [("ring", 50), ("slam3000", 60)])
def test_device_count_step_matches_host_count_step(which, gamma):
    """With the count on the device the cluster factorisation takes the team
    form (its tile grid cannot be sized on the host); choosing that form for
    the host-count run as well, the two runs agree bit for bit."""
    if which == "ring":
        s = synth.ring(m=200, n=50000, views=8, seed=0)
    else:
        s = synth.slam(seed=1, m=3000, n=150000)
    sols = [S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=gamma, lambda0=1e-4)
            for _ in range(2)]
    for sol in sols:
        sol.dims.chol_form = S.STBA_CHOL_TEAM
    for t in range(3):
        host = sols[0].sample_clusters(gamma, 10.0, alpha=1.0, seed=0, it=t)   # count read back
        sols[0].step(host)
        dev = sols[1].sample_clusters_device(gamma, 10.0, alpha=1.0, seed=0, it=t)
        sols[1].step(dev)
        a, b = sols[0].read_state(), sols[1].read_state()
        print(f"{which} t {t}: clusters {host.l} F {a['F']:.10e} accepted {a['accepted']}", flush=True)
        assert a["status"] == 0 and _state_equal(a, b), (a, b)
        assert torch.equal(sols[0].cam, sols[1].cam) and torch.equal(sols[0].pt, sols[1].pt)


def test_device_clustering_above_2048_cameras_matches_oracle():
    s = synth.slam(seed=1, m=3000, n=150000)
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=60)
    e, w = O.covisibility_graph(s.obs_cam, s.obs_pt, s.m, s.n)
    for t in (0, 4):
        smp = sol.sample_clusters(60, 10.0, alpha=1.0, seed=3, it=t)
        ref, l = O.sgc_clusters(e, w, s.m, 60, 10.0, 3, t)
        got = smp._keep[0].cpu().numpy()
        print(f"t {t}: clusters {smp.l} (oracle {l})", flush=True)
        assert smp.l == l and np.array_equal(got, ref)


@pytest.mark.parametrize("precision", [S.STBA_FP64, S.STBA_MIXED])
def test_captured_draw_and_step_replay_the_eager_iterations(precision):
    s = synth.ring(m=200, n=50000, views=8, seed=0)
    K = 3
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=50, lambda0=1e-4,
                       precision=precision)
    cam0, pt0 = sol.cam.clone(), sol.pt.clone()

    def reset():
        sol.cam.copy_(cam0)
        sol.pt.copy_(pt0)
        S.stba_lm_init(sol.state, 1e-4, 0.1)

    reset()
    for t in range(K):
        sol.step(sol.sample_clusters_device(50, 10.0, it=t))
    torch.cuda.synchronize()
    eager = sol.read_state()
    eager_cam = sol.cam.clone()
    reset()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for t in range(K):
            sol.step(sol.sample_clusters_device(50, 10.0, it=t))
    for rep in range(3):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        st = sol.read_state()
        print(f"replay {rep}: F {st['F']:.12e} (eager {eager['F']:.12e})", flush=True)
        assert _state_equal(st, eager)
        assert torch.equal(sol.cam, eager_cam)
        # the program's own eager work between replays
        sol.step(sol.sample_clusters_device(50, 10.0, it=K))
        torch.cuda.synchronize()


@pytest.mark.parametrize("count", [0, 201, -1, 1])
def test_device_count_out_of_range_rejects_the_step(count):
    """One cluster of all 200 cameras under the bound l = 200: a device count of
    1 is that map (199 empty clusters follow it); 0, -1 or above the bound
    reject the step as a bad id does."""
    s = synth.small_ring(m=200, n=3000, views=6, seed=2)
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=200, lambda0=1e-3)
    lab = torch.zeros(s.m, dtype=torch.int32, device="cuda")
    ldev = torch.tensor([count], dtype=torch.int32, device="cuda")
    sol.step(S.make_sample(lab, s.m, l_dev=ldev))
    st = sol.read_state()
    if count == 1:
        ref = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, np.zeros(s.m, dtype=np.int64),
                             1e-3, 1.0, 0, 0)
        assert st["status"] == 0 and bool(st["accepted"]) == ref.accepted
        assert st["F_new"] == pytest.approx(ref.F_new, rel=1e-9)
    else:
        assert st["accepted"] == 0 and st["status"] == -1
        assert np.array_equal(sol.cam.cpu().numpy(), s.cam0)
