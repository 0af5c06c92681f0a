"""Pins of the oracle's LM / STBA step against brute force and stated invariants.

* Schur step (Eq. 5-6) == dense damped normal equations (Eq. 3).
* one cluster and alpha = 1 makes STBA plain LM (Gamma = infinity, appendix B).
* for any map and alpha, STBA's camera step == the camera part of a dense KKT
  solve of the relaxed QP at the finest split with explicit kept-link rows
  (Eq. 7-9, 11-12); with lambda >= 0.1 the corrected gradient is fed to the KKT.
* the closed-form correction == explicit nu with dense solves for two different
  spanning sets of A (Alg. 1).
* S' is cluster-diagonal and symmetric; with one camera per cluster each 9x9 block
  has its closed form; the point step satisfies Eq. 6 for the computed dc.
* LM: accepted steps lower F, rejected steps leave x unchanged, lambda /3 and x3.
* below the correction threshold, one cluster cut out of the problem (cameras and
  points renumbered, draws keyed by the original numbers) gives the same S_k,
  b_k, camera step and interior point steps as the whole problem.
"""
import numpy as np
import pytest

import oracle as O
import synth
from synth.cluster_cut import cut_args, cut_cluster


def _tiny(seed=3, m=5, n=12, views=3):
    s = synth.small_ring(m=m, n=n, views=views, seed=seed)
    return s, (s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("lam", [1e-4, 1e-2, 1.0])
def test_schur_step_equals_full_normal_equations(lam):
    s, args = _tiny(m=6, n=20, views=4)
    dc_full, dp_full = O.full_normal_step(*args, lam)
    dc, dp, S, _ = O.plain_lm_step(*args, lam)
    assert _rel(dc, dc_full) < 1e-9
    assert _rel(dp, dp_full) < 1e-9
    assert np.allclose(S, S.T, atol=1e-9 * np.abs(S).max())


@pytest.mark.parametrize("lam", [1e-4, 0.05])
def test_one_cluster_alpha_one_is_plain_lm(lam):
    s, args = _tiny(m=8, n=60, views=5, seed=6)
    dc, dp, _, _ = O.plain_lm_step(*args, lam)
    st = O.stba_step(*args, np.zeros(s.m, dtype=np.int32), lam, alpha=1.0)
    assert _rel(st.dcam, dc) < 1e-12
    assert _rel(st.dpt, dp) < 1e-12


def _kkt_shift(s, st, lam, lab, alpha, seed, t):
    """Gradient shift that carries the corrected w'_s into the finest split."""
    q = s.q
    f = O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)
    Jc, Jp = O.jacobian(s.cam0, s.pt0, s.obs_cam, s.obs_pt)
    seg, n_seg, seg_point, _, _, _ = O.segments(s.obs_cam, s.obs_pt, lab, alpha, seed, t)
    w_fine = -np.einsum("kab,ka->kb", Jp, f)
    w_seg = np.zeros((n_seg, 3))
    np.add.at(w_seg, seg, w_fine)
    V_diag = np.zeros((n_seg, 3))
    np.add.at(V_diag, seg, np.einsum("kab,kab->kb", Jp, Jp))
    w_corr = O.correct_point_gradient(w_seg, (1 + lam) * V_diag, seg_point, s.n)
    shift = np.zeros((q, 3))
    first = O.canonical_segments(seg)
    heads = np.flatnonzero(first == np.arange(q))
    shift[heads] = (w_corr - w_seg)[seg[heads]]
    return shift


@pytest.mark.parametrize("alpha", [1.0, 0.6])
@pytest.mark.parametrize("lam", [1e-3, 0.3])
@pytest.mark.parametrize("lab", [[0, 0, 1, 1, 1], [0, 1, 0, 1, 2], [0, 1, 2, 3, 4]])
def test_stba_step_equals_relaxed_kkt(alpha, lam, lab):
    s, args = _tiny(seed=3, m=5, n=14, views=4)
    lab = np.array(lab, dtype=np.int32)
    seed, t = 7, 2
    st = O.stba_step(*args, lab, lam, alpha=alpha, seed=seed, t=t)
    shift = _kkt_shift(s, st, lam, lab, alpha, seed, t) if lam >= 0.1 else None
    dc, vsteps = O.relaxed_kkt_step(*args, lab, lam, alpha=alpha, seed=seed, t=t,
                                    point_gradient_shift=shift)
    assert st.corrected == (lam >= 0.1)
    assert _rel(st.dcam, dc) < 1e-8
    # the virtual-point steps of the segments match the KKT's bound virtual points
    assert _rel(st.v_seg_step[st.seg], vsteps) < 1e-8
    assert st.cross_max == 0.0


def test_correction_closed_form_equals_explicit_nu():
    rng = np.random.default_rng(3)
    seg_point = np.array([0, 0, 0, 1, 2, 2, 3, 3, 3, 3])
    w = rng.normal(size=(10, 3))
    h = rng.uniform(0.5, 3.0, (10, 3))
    closed = O.correct_point_gradient(w, h, seg_point, 4)
    for span in ("chain", "star"):
        ex = O.correction_explicit(w, h, seg_point, span)
        assert _rel(closed, ex) < 1e-12
    # the corrected step H~^-1 g' is equal across a point's segments, sums preserved
    step = closed / h
    for j in range(4):
        sel = seg_point == j
        assert np.allclose(step[sel], step[sel][0], rtol=1e-12)
        assert np.allclose(closed[sel].sum(0), w[sel].sum(0), rtol=1e-12)


def test_singleton_clusters_closed_form():
    s, args = _tiny(m=5, n=14, views=4, seed=8)
    lam = 1e-3
    lab = np.arange(s.m, dtype=np.int32)
    st = O.stba_step(*args, lab, lam, alpha=1.0)
    f = O.residuals(*args)
    Jc, Jp = O.jacobian(s.cam0, s.pt0, s.obs_cam, s.obs_pt)
    for i in range(s.m):
        obs = np.flatnonzero(s.obs_cam == i)
        U = sum(Jc[o].T @ Jc[o] for o in obs)
        S = U + lam * np.diag(np.diag(U))
        b = -sum(Jc[o].T @ f[o] for o in obs)
        for o in obs:
            V = Jp[o].T @ Jp[o]
            Vs = V + lam * np.diag(np.diag(V))
            W = Jc[o].T @ Jp[o]
            S -= W @ np.linalg.solve(Vs, W.T)
            b -= W @ np.linalg.solve(Vs, -Jp[o].T @ f[o])
        # b = v - E C^-1 w cancels strongly; 1e-8 still catches any dropped term
        assert _rel(st.S_blocks[i], S) < 1e-10
        assert _rel(st.b_blocks[i], b) < 1e-8
        assert np.all(np.linalg.eigvalsh(st.S_blocks[i]) > 0)


def test_cluster_solve_and_point_update_identities():
    s, args = _tiny(m=8, n=50, views=5, seed=10)
    lam = 1e-2
    lab = np.array([0, 0, 0, 1, 1, 2, 2, 2], dtype=np.int32)
    st = O.stba_step(*args, lab, lam, alpha=0.8, seed=1, t=5)
    for Sk, bk, cams in zip(st.S_blocks, st.b_blocks, st.clusters):
        assert np.allclose(Sk, Sk.T, rtol=0, atol=1e-12 * np.abs(Sk).max())
        ref = np.linalg.solve(Sk, bk)
        assert _rel(st.dcam[cams].reshape(-1), ref) < 1e-9
    # Eq. 6 with the physical C, E, w: C dp = w - E^T dc
    f = O.residuals(*args).reshape(-1)
    Jc, Jp = O.jacobian(s.cam0, s.pt0, s.obs_cam, s.obs_pt)
    Jcm = O.jc_matrix(Jc, s.obs_cam, s.m).toarray()
    Jpm = O.jp_matrix(Jp, s.obs_pt, s.n).toarray()
    C = Jpm.T @ Jpm
    C = C + lam * np.diag(np.diag(C))
    lhs = C @ st.dpt.reshape(-1)
    rhs = -Jpm.T @ f - (Jcm.T @ Jpm).T @ st.dcam.reshape(-1)
    assert _rel(lhs, rhs) < 1e-9
    # sum over clusters of the virtual-point Jacobians is the physical J_p (Eq. 15)
    Jv = O.jp_matrix(Jp, st.seg, st.n_seg).toarray()
    seg_point = np.zeros(st.n_seg, dtype=int)
    seg_point[st.seg] = s.obs_pt
    folded = np.zeros_like(Jpm)
    for sg in range(st.n_seg):
        folded[:, 3 * seg_point[sg]:3 * seg_point[sg] + 3] += Jv[:, 3 * sg:3 * sg + 3]
    assert np.array_equal(folded, Jpm)


def test_lm_loop_accept_reject_and_lambda():
    s = synth.small_ring(m=12, n=300, views=5, seed=12)
    lab = synth.halves_map(s.m, 3)
    cam, pt, lam = s.cam0.copy(), s.pt0.copy(), 1e-4
    F = O.cost(O.residuals(cam, pt, s.obs_cam, s.obs_pt, s.obs_uv))
    seen_accept = False
    for t in range(6):
        r = O.lm_iteration(cam, pt, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, alpha=0.9, seed=3,
                           t=t, F=F)
        if r.accepted:
            seen_accept = True
            assert r.F < F and np.isclose(r.lam, lam / 3.0)
            assert not np.array_equal(r.cam, cam)
        else:
            assert np.array_equal(r.cam, cam) and np.array_equal(r.pt, pt)
            assert np.isclose(r.lam, lam * 3.0) and r.F == F
        cam, pt, lam, F = r.cam, r.pt, r.lam, r.F
    assert seen_accept


def test_lm_rejects_non_finite_step_and_keeps_x():
    s = synth.small_ring(m=8, n=100, views=4, seed=13)
    cam = s.cam0.copy()
    cam[2, 6] = np.nan                       # a broken focal length
    F = 1.0e6
    r = O.lm_iteration(cam, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, synth.halves_map(s.m), 1e-3,
                       F=F)
    assert not r.accepted and r.F == F and np.isclose(r.lam, 3e-3)
    assert np.array_equal(r.cam, cam, equal_nan=True) and np.array_equal(r.pt, s.pt0)


@pytest.mark.parametrize("alpha,lam", [(1.0, 1e-4), (0.6, 1e-3), (0.3, 0.05)])
def test_cluster_cut_reproduces_the_whole_problem(alpha, lam):
    s = synth.small_ring(m=24, n=600, views=6, seed=8)
    e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
    lab = synth.sgc_map(e, w, s.m, 8, 10.0, 1, 2)
    assert lab.max() >= 2
    full = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, alpha, 5, 2)
    assert not full.corrected
    differs = False
    for k in range(int(lab.max()) + 1):
        cut = cut_cluster(s.obs_cam, s.obs_pt, lab, k)
        args, ids = cut_args(s, cut)
        sub = O.stba_step(*args, lam, alpha, 5, 2, ids=ids)
        assert _rel(sub.S_blocks[0], full.S_blocks[k]) < 1e-13
        assert _rel(sub.b_blocks[0], full.b_blocks[k]) < 1e-12
        assert _rel(sub.dcam, full.dcam[cut.cams]) < 1e-10
        if cut.interior.size:
            assert _rel(sub.dpt[cut.interior], full.dpt[cut.pts[cut.interior]]) < 1e-10
        # the draw belongs to the original numbers: renumbered draws split differently
        plain = O.segments(args[2], args[3], args[5], alpha, 5, 2)[0]
        keyed = O.segments(args[2], args[3], args[5], alpha, 5, 2, ids)[0]
        differs |= not np.array_equal(O.canonical_segments(plain), O.canonical_segments(keyed))
    assert differs == (alpha < 1.0)
