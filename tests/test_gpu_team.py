"""The team form of the cluster factorisation (many clusters, tiles in memory,
a band wavefront per cluster and workers sized by the cluster's work), chosen
with stba_dims.chol_form = STBA_CHOL_TEAM on scenes the oracle solves whole, against the oracle's
steps: clusters of 1 to 15 block rows (the band alone below three), FP64 and
MIXED, a cluster made indefinite, one cluster per camera, repeated runs bit
for bit.  The SLAM-like workload, where the form is the default, is checked
cluster by cluster in test_gpu_large."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_00446_amd as S
import synth
from gpu_helpers import GpuProblem, kappa_scaled, rel, ws_view

pytestmark = pytest.mark.gpu


def _team(obj):
    """the team form for a GpuProblem or a StbaSolver"""
    obj.dims.chol_form = S.STBA_CHOL_TEAM
    return obj


def _sgc(scene, gamma, t, seed=0):
    e, w = synth.camera_graph(scene.obs_cam, scene.obs_pt, scene.m)
    return synth.sgc_map(e, w, scene.m, gamma, 10.0, seed, t)


@pytest.mark.parametrize("gamma,lam,alpha", [(12, 1e-3, 1.0), (12, 0.3, 0.7), (40, 1e-4, 1.0), (1, 1e-3, 1.0)])
def test_team_steps_match_oracle(gamma, lam, alpha):
    s = synth.small_ring(m=40, n=3000, views=8, seed=1)
    lab = _sgc(s, gamma, 2)
    g = _team(GpuProblem(s, gamma_max=gamma))
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, lam, alpha, 5, 2)
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, alpha, 5, 2)
    kap = max(kappa_scaled(Sk) for Sk in ref.S_blocks)
    print(f"gamma {gamma}: clusters {lab.max() + 1}, block rows up to {(9 * np.bincount(lab).max() + 31) // 32}, "
          f"kappa {kap:.2e}, dcam {rel(dcam, ref.dcam):.2e} dpt {rel(dpt, ref.dpt):.2e}", flush=True)
    assert np.all(cs == 0)
    assert rel(dcam, ref.dcam) < 1e-9
    assert rel(dpt, ref.dpt) < 1e-9


@pytest.mark.parametrize("precision,bar", [(S.STBA_FP64, 1e-9), (S.STBA_MIXED, 1e-4)])
def test_team_full_size_ring_iteration(precision, bar):
    """One LM iteration of the 200-camera ring (Gamma 50: up to 15 block rows)."""
    s = synth.ring(m=200, n=50000, views=8, seed=0)
    lab = _sgc(s, 50, 0)
    sol = _team(S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=50, lambda0=1e-4,
                             precision=precision))
    sol.step(sol.sample(lab, alpha=1.0, seed=0, it=0))
    st = sol.read_state()
    ref = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-4, 1.0, 0, 0)
    dc = rel(sol.cam.cpu().numpy() - s.cam0, ref.cam - s.cam0)
    print(f"ring team precision {precision}: accepted {st['accepted']} F_new {st['F_new']:.12e} "
          f"oracle {ref.F_new:.12e} dcam {dc:.2e}", flush=True)
    assert st["status"] == 0 and st["last_status"] == 0
    assert bool(st["accepted"]) == ref.accepted
    assert abs(st["F_new"] - ref.F_new) <= bar * ref.F_new
    assert dc < bar
    assert rel(sol.pt.cpu().numpy() - s.pt0, ref.pt - s.pt0) < bar


def test_team_reports_a_cluster_that_is_not_positive_definite():
    s = synth.small_ring(m=40, n=3000, views=8, seed=1)
    lab = _sgc(s, 40, 1)
    g = _team(GpuProblem(s, gamma_max=40))
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3)
    torch.cuda.synchronize()
    S_off = ws_view(g.ws, rcs.S_off, torch.int64, rcs.l + 1).cpu().numpy()
    Sbuf = ws_view(g.ws, rcs.S, torch.float64, int(S_off[rcs.l]))
    bad = int(np.argmax(np.bincount(lab)))
    Sbuf[int(S_off[bad])] = -1.0   # entry (0, 0) of the largest cluster
    torch.cuda.synchronize()
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    assert cs[bad] == -2
    assert np.all(np.delete(cs, bad) == 0)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3)
    good = lab != bad
    assert rel(dcam[good], ref.dcam[good]) < 1e-9
    # the flags and vectors were returned to their initial state: the next solve is clean
    rcs = g.build(f, Jc, Jp, lab, 1e-3)
    dcam2, _, cs2 = g.solve(rcs, Jc, Jp)
    assert np.all(cs2 == 0)
    assert rel(dcam2, ref.dcam) < 1e-9


def test_team_solves_are_bit_for_bit_repeatable():
    s = synth.ring(m=200, n=50000, views=8, seed=0)
    lab = _sgc(s, 50, 3)
    g = _team(GpuProblem(s, gamma_max=50))
    f, Jc, Jp, _ = g.residual_jacobian()
    out = []
    for _ in range(3):
        rcs = g.build(f, Jc, Jp, lab, 1e-4)
        dcam, dpt, cs = g.solve(rcs, Jc, Jp)
        assert np.all(cs == 0)
        out.append((dcam, dpt))
    for dcam, dpt in out[1:]:
        assert np.array_equal(dcam, out[0][0]) and np.array_equal(dpt, out[0][1])
