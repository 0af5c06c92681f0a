"""GPU parity at the edges of the method's arithmetic and of the LM rule:

* residuals and Jacobian at rotation vectors of norm 0, 1e-9 and 1e-5 (the
  series branch of the Rodrigues coefficients), and just either side of the
  branch switch, element by element against the oracle;
* a step whose candidate cost is not finite (a NaN observed pixel: J and S stay
  finite, b and the step do not) and a camera whose focal length is NaN (the
  cluster system is not positive definite): both rejected as the oracle's LM
  rule rejects them, lambda x3, x bit for bit unchanged, the reason in
  last_status;
* one LM iteration of the full-size 200-camera ring with the correction active
  (lambda 0.3 >= 0.1) and a random constraint draw (alpha 0.7), against the
  oracle's whole iteration;
* every cluster system's condition number after diagonal scaling,
  kappa(D^-1 S_k D^-1), printed beside the step errors."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_00446_amd as S
import synth
from gpu_helpers import GpuProblem, kappa_scaled, rel, rel_max

pytestmark = pytest.mark.gpu


def _near_identity_scene(norms, seed=3):
    """tiny_circle with some cameras replaced by near-identity rotations: camera
    c gets a rotation vector of norm norms[c] in a random direction and looks
    along +z from 10 units in front of the point cube (every point at depth 8-12)."""
    s = synth.tiny_circle(seed=0)
    rng = np.random.default_rng(seed)
    cam = s.cam0.copy()
    for c, th in enumerate(norms):
        u = rng.normal(size=3)
        cam[c, 0:3] = th * u / np.linalg.norm(u)
        cam[c, 3:6] = (0.1, -0.2, 10.0)
    return s, cam


@pytest.mark.parametrize("norms", [(0.0, 1e-9, 1e-5, 0.0, 1e-9, 1e-5),
                                   (1e-4 * (1 - 1e-3), 1e-4 * (1 + 1e-3), 3e-5, 2e-4)],
                         ids=["series_branch", "branch_switch"])
def test_residual_jacobian_at_small_rotations(norms):
    s, cam = _near_identity_scene(norms)
    g = GpuProblem(s, gamma_max=s.m, cam=cam)
    f, Jc, Jp, cost = g.residual_jacobian()
    torch.cuda.synchronize()
    f_ref = O.residuals(cam, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)
    Jc_ref, Jp_ref = O.jacobian(cam, s.pt0, s.obs_cam, s.obs_pt)
    Jc_g = Jc.cpu().numpy().reshape(-1, 2, 9)
    Jp_g = Jp.cpu().numpy().reshape(-1, 2, 3)
    f_g = f.cpu().numpy()
    sel = np.flatnonzero(s.obs_cam < len(norms))
    assert sel.size > 100
    # element by element, each observation's block against its own largest entry
    for got, ref in ((f_g, f_ref), (Jc_g, Jc_ref), (Jp_g, Jp_ref)):
        g_s = got[sel].reshape(sel.size, -1)
        r_s = ref[sel].reshape(sel.size, -1)
        scale = np.max(np.abs(r_s), axis=1, keepdims=True)
        err = np.max(np.abs(g_s - r_s) / scale)
        print(f"max element error / block scale: {err:.2e}")
        assert err < 1e-12
    # the rotation columns of J_c at theta = 0: dP/dw = -R [X]x, R = I
    if norms[0] == 0.0:
        assert rel_max(Jc_g[s.obs_cam == 0], Jc_ref[s.obs_cam == 0]) < 1e-13
    assert abs(cost.item() - O.cost(f_ref)) <= 1e-12 * O.cost(f_ref)


@pytest.mark.parametrize("what", ["nan_pixel", "nan_focal"])
def test_non_finite_step_is_rejected(what):
    """The LM rule (Alg. 1) accepts only a finite candidate cost below F(x) from
    factorised cluster systems; anything else is a rejected step."""
    s = synth.small_ring(m=24, n=1500, views=6, seed=5)
    lab = (np.arange(s.m) * 3 // s.m).astype(np.int32)
    cam, uv = s.cam0.copy(), s.obs_uv.copy()
    if what == "nan_pixel":
        uv[7, 0] = np.nan          # f and b carry the NaN; J and S do not
    else:
        cam[5, 6] = np.nan         # camera 5's rows of J and S are NaN
    sol = S.StbaSolver(cam, s.pt0, s.obs_cam, s.obs_pt, uv, gamma_max=8, lambda0=1e-3)
    sol.step(sol.sample(lab, alpha=1.0, seed=0, it=0))
    st = sol.read_state()
    ref = O.lm_iteration(cam, s.pt0, s.obs_cam, s.obs_pt, uv, lab, 1e-3, 1.0, 0, 0)
    print(f"{what}: last_status {st['last_status']} F_new {st['F_new']} oracle ok {ref.step.ok}")
    assert not ref.accepted
    assert st["accepted"] == 0
    assert st["lambda_"] == ref.lam == 3e-3
    assert st["status"] == 0                      # not a data error: the step alone is rejected
    if what == "nan_pixel":
        assert st["last_status"] == -3            # STBA_ENONFINITE: S factorised, the cost is not finite
        assert not np.isfinite(st["F_new"])
    else:
        assert st["last_status"] == -2            # STBA_ENOTPD: NaN pivots in camera 5's cluster
    got_cam = sol.cam.cpu().numpy()
    got_pt = sol.pt.cpu().numpy()
    assert np.array_equal(np.isnan(got_cam), np.isnan(cam))
    assert np.array_equal(got_cam[~np.isnan(cam)], cam[~np.isnan(cam)])
    assert np.array_equal(got_pt, s.pt0)
    # the next iteration (lambda 3e-3) is rejected the same way and lambda grows again
    sol.step(sol.sample(lab, alpha=1.0, seed=0, it=1))
    st2 = sol.read_state()
    assert st2["accepted"] == 0 and st2["lambda_"] == (1e-3 * 3.0) * 3.0


def test_full_size_ring_iteration_with_correction_and_draw():
    """One LM iteration on the 200-camera ring (400k observations), Gamma = 50
    graph clusters, lambda 0.3 (the correction of Sec. 4.3 applies), alpha 0.7
    (each intra-cluster link kept with probability 0.7), against the oracle."""
    s = synth.ring(m=200, n=50000, views=8, seed=0)
    e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
    lab = synth.sgc_map(e, w, s.m, 50, 10.0, 0, 2)
    lam, alpha, seed, t = 0.3, 0.7, 4, 2
    g = GpuProblem(s, gamma_max=50)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, lam, alpha, seed, t)
    blocks, b, seg, cl_n = g.read_rcs(rcs, lab)
    ref_step = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, alpha, seed, t)
    assert ref_step.corrected
    assert np.array_equal(seg.astype(np.int64), O.canonical_segments(ref_step.seg))
    for k, (Sk, Rk) in enumerate(zip(blocks, ref_step.S_blocks)):
        print(f"cluster {k}: {cl_n[k]} cameras, kappa(D^-1 S D^-1) {kappa_scaled(Rk):.2e}, "
              f"S {rel_max(np.tril(Sk), np.tril(Rk)):.2e}")
        assert rel_max(np.tril(Sk), np.tril(Rk)) < 1e-11
    assert rel(b.reshape(-1), ref_step.b_full) < 1e-9
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=50, lambda0=lam)
    sol.step(sol.sample(lab, alpha=alpha, seed=seed, it=t))
    st = sol.read_state()
    ref = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, alpha, seed, t)
    dc = sol.cam.cpu().numpy() - s.cam0
    dp = sol.pt.cpu().numpy() - s.pt0
    print(f"ring lambda {lam} alpha {alpha}: accepted {st['accepted']} F_new {st['F_new']:.12e} "
          f"oracle {ref.F_new:.12e}")
    assert st["status"] == 0 and st["last_status"] == 0
    assert bool(st["accepted"]) == ref.accepted
    assert st["lambda_"] == ref.lam
    assert abs(st["F_new"] - ref.F_new) <= 1e-9 * ref.F_new
    if ref.accepted:
        assert rel(dc, ref.cam - s.cam0) < 1e-9
        assert rel(dp, ref.pt - s.pt0) < 1e-9
