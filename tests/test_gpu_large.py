"""GPU parity at the full sizes of the Internet-like (1000 cameras, 2.4M
observations, graph clusters of up to 100 cameras) and SLAM-like (5000 cameras,
5.9M observations, sequential clusters of 20-120 cameras) workloads, in FP64
and mixed precision.

The oracle's dense S over all cameras does not fit at these sizes, so it runs
one cluster at a time on the cluster's own observations (see cluster_cut): the
largest, the smallest and a median cluster are compared entry by entry (S_k,
b_k, the camera step, the steps of points seen only inside the cluster), the
cost F(x) over every observation, and one LM iteration through the library's
whole-iteration entry point on the same map and draw."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_00446_amd as S
import synth
from synth.cluster_cut import cut_args, cut_cluster
from gpu_helpers import GpuProblem, rel, rel_max

pytestmark = pytest.mark.gpu

# bars: FP64 as in the small parity tests; mixed 1e-4 relative on steps and cost
BARS = {S.STBA_FP64: dict(S=1e-11, b=1e-9, step=1e-9, F=1e-12),
        S.STBA_MIXED: dict(S=1e-4, b=1e-4, step=1e-4, F=1e-5)}


def _workload(which):
    if which == "internet":
        s = synth.internet(seed=0)
        e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
        lab = synth.sgc_map(e, w, s.m, 100, 10.0, 0, 1)
        return s, lab, 100, 1e-3, 0.8, 3, 1
    s = synth.slam(seed=0)
    lab = synth.sequential_map(s.m, 20, 120, 0, 0)
    return s, lab, 120, 1e-4, 1.0, 0, 0


@pytest.mark.parametrize("which", ["internet", "slam"])
@pytest.mark.parametrize("precision", [S.STBA_FP64, S.STBA_MIXED])
def test_full_size_sampled_clusters_match_oracle(which, precision):
    s, lab, gamma, lam, alpha, seed, t = _workload(which)
    bar = BARS[precision]
    print(f"{which}: m {s.m} n {s.n} q {s.q} clusters {lab.max() + 1} precision {precision}", flush=True)
    g = GpuProblem(s, gamma_max=gamma, precision=precision)
    f, Jc, Jp, cost = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, lam, alpha, seed, t)
    sizes = np.bincount(lab)
    picks = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2])})
    built = {k: g.read_cluster(rcs, k) for k in picks}   # before the solve factorises S in place
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    assert np.all(cs == 0)
    F0 = O.cost(O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv))
    assert abs(cost.item() - F0) <= bar["F"] * F0

    refs = {}
    for k in picks:
        cut = cut_cluster(s.obs_cam, s.obs_pt, lab, k)
        args, ids = cut_args(s, cut)
        ref = O.stba_step(*args, lam, alpha, seed, t, ids=ids)
        assert ref.ok and not ref.corrected
        Sk, b = built[k]
        print(f"  cluster {k}: {cut.cams.size} cameras, {cut.obs.size} observations, "
              f"S {rel_max(Sk, ref.S_blocks[0]):.2e} dc {rel(dcam[cut.cams], ref.dcam):.2e}", flush=True)
        assert rel_max(Sk, ref.S_blocks[0]) < bar["S"]
        assert rel(b[cut.cams].ravel(), ref.b_blocks[0]) < bar["b"]
        assert rel(dcam[cut.cams], ref.dcam) < bar["step"]
        assert cut.interior.size > 0
        assert rel(dpt[cut.pts[cut.interior]], ref.dpt[cut.interior]) < bar["step"]
        refs[k] = (cut, ref)

    # the same iteration through the whole-iteration entry point
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=gamma, lambda0=lam,
                       precision=precision)
    sol.step(sol.sample(lab, alpha=alpha, seed=seed, it=t))
    st = sol.read_state()
    F_gpu = cost.item()   # the same residual kernel and summation order as the iteration's F(x)
    print(f"  iteration: accepted {st['accepted']} F {F_gpu:.10e} -> {st['F_new']:.10e}", flush=True)
    assert st["status"] == 0
    assert bool(st["accepted"]) == (st["F_new"] < F_gpu)
    assert st["F"] == (st["F_new"] if st["accepted"] else F_gpu)
    cam = sol.cam.cpu().numpy()
    for k, (cut, ref) in refs.items():
        moved = cam[cut.cams] - s.cam0[cut.cams]
        if st["accepted"]:
            assert rel(moved, ref.dcam) < bar["step"]
        else:
            assert np.all(moved == 0)
