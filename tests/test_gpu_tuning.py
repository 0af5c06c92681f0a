"""Launch settings: every factorisation form chosen through stba_dims.chol_form
and every Schur workgroup count give the oracle's step; stba_autotune measures
the candidates, writes the fastest into dims and reports the times (forms that
do not fit are not run); the shape-class cache reuses a choice without
measuring again."""
import json

import numpy as np
import pytest

import oracle as O
import paper_2008_00446_amd as S
import synth
from gpu_helpers import GpuProblem, rel

pytestmark = pytest.mark.gpu


def _sgc(scene, gamma, t, seed=0):
    e, w = synth.camera_graph(scene.obs_cam, scene.obs_pt, scene.m)
    return synth.sgc_map(e, w, scene.m, gamma, 10.0, seed, t)


@pytest.mark.parametrize("form", [S.STBA_CHOL_AUTO, S.STBA_CHOL_TILES, S.STBA_CHOL_TEAM, S.STBA_CHOL_WORKGROUP])
@pytest.mark.parametrize("blocks", [0, 8, 4096])
def test_every_form_and_block_count_gives_the_oracle_step(form, blocks):
    s = synth.small_ring(m=40, n=3000, views=8, seed=1)
    lab = _sgc(s, 12, 2)
    g = GpuProblem(s, gamma_max=12)
    g.dims.chol_form = form
    g.dims.schur_blocks = blocks
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3, 1.0, 5, 2)
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3, 1.0, 5, 2)
    assert np.all(cs == 0)
    assert rel(dcam, ref.dcam) < 1e-9 and rel(dpt, ref.dpt) < 1e-9


def test_bad_launch_settings_are_rejected():
    s = synth.small_ring(m=20, n=500, views=5, seed=6)
    g = GpuProblem(s, gamma_max=10)
    for form, blocks in [(4, 0), (-1, 0), (0, 7), (0, 65537)]:
        g.dims.chol_form, g.dims.schur_blocks = form, blocks
        with pytest.raises(S.StbaError):
            g.residual_jacobian()


@pytest.mark.parametrize("which", ["ring", "singletons"])
def test_autotune_picks_a_measured_setting_and_keeps_the_step(which, tmp_path):
    s = synth.ring(m=200, n=50000, views=8, seed=0)
    lab = _sgc(s, 50, 0) if which == "ring" else np.arange(s.m, dtype=np.int32)
    gamma = 50 if which == "ring" else 1
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=gamma, lambda0=1e-4)
    smp = sol.sample(lab, it=0)
    cache = str(tmp_path / "tune.json")
    res = sol.autotune(smp, cache_path=cache)
    print(f"{which}: {res}", flush=True)
    assert not res["cached"]
    assert res["chol_form"] in ("tiles", "team", "workgroup") and res["chol_form"] in res["chol_ms"]
    assert res["schur_blocks"] in res["schur_ms"]
    assert res["chol_ms"][res["chol_form"]] == min(res["chol_ms"].values())
    assert res["schur_ms"][res["schur_blocks"]] == min(res["schur_ms"].values())
    assert "workgroup" in res["chol_ms"]   # the workgroup form always fits
    assert sol.dims.chol_form != S.STBA_CHOL_AUTO and sol.dims.schur_blocks == res["schur_blocks"]
    # x is untouched by the tuning; the tuned step matches the oracle
    assert np.array_equal(sol.cam.cpu().numpy(), s.cam0)
    sol.step(smp)
    st = sol.read_state()
    ref = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-4, 1.0, 0, 0)
    assert st["status"] == 0 and bool(st["accepted"]) == ref.accepted
    assert abs(st["F_new"] - ref.F_new) <= 1e-9 * ref.F_new
    # the same shape class again: taken from the cache, nothing measured
    sol2 = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=gamma, lambda0=1e-4)
    res2 = sol2.autotune(sol2.sample(lab, it=0), cache_path=cache)
    assert res2["cached"] and res2["chol_form"] == res["chol_form"] and res2["schur_blocks"] == res["schur_blocks"]
    assert sol2.dims.chol_form == sol.dims.chol_form
    with open(cache) as fh:
        assert res["class"] in json.load(fh)
