"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (FP64): residuals/Jacobians 1e-12 (same formulas, different rounding order),
cluster matrices 1e-11 of their largest entry, right-hand sides and steps 1e-9
relative (2-norm), the constraint selection bit-exact (segment heads compared as
integers), accept decisions and lambda exactly."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_00446_amd as S
import synth
from gpu_helpers import GpuProblem, dev, kappa_scaled, rel, rel_max, ws_view

pytestmark = pytest.mark.gpu


def _small():
    return synth.small_ring(m=40, n=3000, views=8, seed=1)


def _sgc(scene, gamma, t, seed=0):
    e, w = synth.camera_graph(scene.obs_cam, scene.obs_pt, scene.m)
    return synth.sgc_map(e, w, scene.m, gamma, 10.0, seed, t)


@pytest.mark.parametrize("which", ["tiny_circle", "small_ring"])
def test_residual_jacobian_matches_oracle(which):
    s = synth.tiny_circle() if which == "tiny_circle" else _small()
    g = GpuProblem(s, gamma_max=s.m)
    f, Jc, Jp, cost = g.residual_jacobian()
    torch.cuda.synchronize()
    f_ref = O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)
    Jc_ref, Jp_ref = O.jacobian(s.cam0, s.pt0, s.obs_cam, s.obs_pt)
    assert rel_max(f.cpu().numpy(), f_ref) < 1e-12
    assert rel_max(Jc.cpu().numpy().reshape(-1, 2, 9), Jc_ref) < 1e-12
    assert rel_max(Jp.cpu().numpy().reshape(-1, 2, 3), Jp_ref) < 1e-12
    assert abs(cost.item() - O.cost(f_ref)) <= 1e-12 * O.cost(f_ref)


@pytest.mark.parametrize("alpha,seed,t", [(1.0, 0, 0), (0.5, 3, 1), (0.2, 9, 7)])
def test_constraint_selection_bit_exact(alpha, seed, t):
    s = _small()
    lab = _sgc(s, 12, t)
    g = GpuProblem(s, gamma_max=12)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3, alpha, seed, t)
    _, _, seg, _ = g.read_rcs(rcs, lab)
    ref_seg = O.segments(s.obs_cam, s.obs_pt, lab, alpha, seed, t)[0]
    assert np.array_equal(seg.astype(np.int64), O.canonical_segments(ref_seg))


@pytest.mark.parametrize("lam,alpha", [(1e-4, 1.0), (1e-3, 0.6), (0.3, 1.0), (0.5, 0.7)])
def test_cluster_systems_and_steps_match_oracle(lam, alpha):
    s = _small()
    seed, t = 5, 2
    lab = _sgc(s, 12, t)
    g = GpuProblem(s, gamma_max=12)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, lam, alpha, seed, t)
    blocks, b, _, cl_n = g.read_rcs(rcs, lab)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, alpha, seed, t)
    assert ref.corrected == (lam >= 0.1)
    assert len(blocks) == len(ref.S_blocks)
    for k, (Sk, Rk) in enumerate(zip(blocks, ref.S_blocks)):
        assert cl_n[k] * 9 == Rk.shape[0]
        assert rel_max(np.tril(Sk), np.tril(Rk)) < 1e-11, k
    assert rel(b.reshape(-1), ref.b_full) < 1e-9
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    kap = max(kappa_scaled(Rk) for Rk in ref.S_blocks)
    print(f"lam {lam} alpha {alpha}: max kappa(D^-1 S_k D^-1) {kap:.2e} (kappa 1e-16 = {kap * 1e-16:.1e}), "
          f"dcam {rel(dcam, ref.dcam):.2e} dpt {rel(dpt, ref.dpt):.2e}")
    assert kap * 1e-16 < 1e-9   # the FP64 bar is meaningful for these systems
    assert np.all(cs == 0)
    assert rel(dcam, ref.dcam) < 1e-9
    assert rel(dpt, ref.dpt) < 1e-9


def test_tiny_circle_one_iteration_matches_oracle():
    """16 cameras, 2 fixed clusters of 8, lambda 1e-3, seed 0, alpha 1: one LM iteration."""
    s = synth.tiny_circle()
    lab = synth.halves_map(16)
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=8, lambda0=1e-3)
    sol.step(sol.sample(lab, alpha=1.0, seed=0, it=0))
    st = sol.read_state()
    ref = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3, 1.0, 0, 0)
    F0 = O.cost(O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv))
    assert st["status"] == 0 and st["last_status"] == 0
    assert bool(st["accepted"]) == ref.accepted
    assert st["lambda_"] == ref.lam
    assert abs(st["F_new"] - ref.F_new) <= 1e-9 * ref.F_new
    assert abs(st["F"] - (ref.F_new if ref.accepted else F0)) <= 1e-9 * F0
    cam = sol.cam.cpu().numpy()
    pt = sol.pt.cpu().numpy()
    assert rel(cam - s.cam0, ref.cam - s.cam0) < 1e-9
    assert rel(pt - s.pt0, ref.pt - s.pt0) < 1e-9


@pytest.mark.parametrize("lam_corr", [0.1, float("inf")], ids=["stba", "stba_star"])
def test_lambda_floor_and_correction_ablation_match_oracle(lam_corr):
    # Sec. 5.4: lambda kept >= 0.1 so that the correction (STBA) is active at every
    # iteration, against the same iterations without it (STBA*)
    s = _small()
    lam0, alpha, seed = 0.1, 1.0, 4
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=12, lambda0=lam0,
                       lambda_corr=lam_corr, lambda_min=0.1)
    cam, pt, lam = s.cam0.copy(), s.pt0.copy(), lam0
    F = O.cost(O.residuals(cam, pt, s.obs_cam, s.obs_pt, s.obs_uv))
    accepted = 0
    for t in range(4):
        lab = _sgc(s, 12, t, seed)
        sol.step(sol.sample(lab, alpha=alpha, seed=seed, it=t))
        st = sol.read_state()
        r = O.lm_iteration(cam, pt, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, alpha, seed, t, lam_corr=lam_corr,
                           F=F, lam_min=0.1)
        assert bool(st["accepted"]) == r.accepted, t
        assert st["lambda_"] == r.lam and r.lam >= 0.1, t
        assert abs(st["F"] - r.F) <= 1e-9 * r.F, t
        cam, pt, lam, F = r.cam, r.pt, r.lam, r.F
        accepted += r.accepted
        assert rel(sol.cam.cpu().numpy() - s.cam0, cam - s.cam0) < 1e-8, t
    assert accepted >= 1


def test_lm_iterations_with_changing_maps_match_oracle():
    s = _small()
    lam0, alpha, seed = 0.2, 0.8, 11
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=12, lambda0=lam0)
    cam, pt, lam = s.cam0.copy(), s.pt0.copy(), lam0
    F = O.cost(O.residuals(cam, pt, s.obs_cam, s.obs_pt, s.obs_uv))
    decisions = []
    for t in range(4):
        lab = _sgc(s, 12, t, seed)
        sol.step(sol.sample(lab, alpha=alpha, seed=seed, it=t))
        st = sol.read_state()
        r = O.lm_iteration(cam, pt, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, alpha, seed, t, F=F)
        assert bool(st["accepted"]) == r.accepted, t
        assert np.isclose(st["lambda_"], r.lam, rtol=1e-15), t
        assert abs(st["F"] - r.F) <= 1e-9 * r.F, t
        cam, pt, lam, F = r.cam, r.pt, r.lam, r.F
        decisions.append(r.accepted)
        assert rel(sol.cam.cpu().numpy() - s.cam0, cam - s.cam0) < 1e-8, t
        assert rel(sol.pt.cpu().numpy() - s.pt0, pt - s.pt0) < 1e-8, t
    st = sol.read_state()
    assert st["n_rcs"] == 4 and st["n_accept"] == sum(decisions)
    assert st["n_jac"] == 1 + sum(decisions[:-1])


@pytest.mark.parametrize("mode", ["one_cluster", "singletons"])
def test_extreme_clusterings(mode):
    s = synth.small_ring(m=30, n=1500, views=6, seed=4)
    lam = 1e-3
    if mode == "one_cluster":
        lab, gamma = np.zeros(s.m, dtype=np.int32), s.m
    else:
        lab, gamma = np.arange(s.m, dtype=np.int32), 1
    g = GpuProblem(s, gamma_max=gamma)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, lam)
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    if mode == "one_cluster":
        ref_c, ref_p, _, _ = O.plain_lm_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lam)
    else:
        st = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam)
        ref_c, ref_p = st.dcam, st.dpt
    assert np.all(cs == 0)
    assert rel(dcam, ref_c) < 1e-9
    assert rel(dpt, ref_p) < 1e-9


@pytest.mark.parametrize("m,l", [(200, 23), (1100, 150), (5000, 70), (5000, 1300)])
def test_cluster_layout_bit_exact(m, l):
    """Cameras grouped by cluster (ascending ids), sizes, padded orders and S_k
    offsets; 200 cameras take the one-workgroup layout, 1100 and 5000 the
    many-workgroup one.  Some cluster ids are left unused (empty clusters)."""
    s = synth.small_ring(m=m, n=2500, views=4, seed=11)
    rng = np.random.default_rng(4)
    lab = rng.integers(0, l - 3, size=m).astype(np.int32)   # ids l-3 .. l-1 stay empty
    gamma = max(40, int(np.bincount(lab).max()))
    g = GpuProblem(s, gamma_max=gamma)
    f, Jc, Jp, _ = g.residual_jacobian()
    lab_d = dev(lab, torch.int32)
    rcs = S.stba_build_cluster_rcs(g.prob, g.dims, S.make_sample(lab_d, l), S.StbaDamping(1e-3, 0.1),
                                   S.STBA_FP64, f, Jc, Jp, g.ws)
    torch.cuda.synchronize()
    got = {k: ws_view(g.ws, getattr(rcs, k), dt, cnt).cpu().numpy() for k, dt, cnt in [
        ("cl_n", torch.int32, l), ("cl_Np", torch.int32, l), ("cl_start", torch.int32, l + 1),
        ("cl_cams", torch.int32, m), ("cam_local", torch.int32, m), ("S_off", torch.int64, l + 1)]}
    n_k = np.bincount(lab, minlength=l)
    Np = (9 * n_k + 31) // 32 * 32
    order = np.argsort(lab, kind="stable")
    local = np.empty(m, dtype=np.int64)
    start = np.concatenate([[0], np.cumsum(n_k)])
    local[order] = np.arange(m) - start[lab[order]]
    assert np.array_equal(got["cl_n"], n_k)
    assert np.array_equal(got["cl_Np"], Np)
    assert np.array_equal(got["cl_start"], start)
    assert np.array_equal(got["cl_cams"], order)
    assert np.array_equal(got["cam_local"], local)
    assert np.array_equal(got["S_off"], np.concatenate([[0], np.cumsum(Np.astype(np.int64) ** 2)]))


def test_invalid_maps_are_rejected_on_device():
    s = synth.small_ring(m=20, n=500, views=5, seed=6)
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=10, lambda0=1e-3)
    bad = synth.halves_map(20)
    bad[3] = 7                                 # id outside [0, l)
    sol.step(sol.sample(bad, l=2))
    st = sol.read_state()
    assert st["status"] == -1 and st["accepted"] == 0 and np.isclose(st["lambda_"], 3e-3)
    assert np.array_equal(sol.cam.cpu().numpy(), s.cam0)
    big = np.zeros(20, dtype=np.int32)         # one cluster of 20 > gamma_max 10
    sol2 = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=10, lambda0=1e-3)
    sol2.step(sol2.sample(big, l=1))
    st2 = sol2.read_state()
    assert st2["status"] == -1 and st2["accepted"] == 0
    assert np.array_equal(sol2.pt.cpu().numpy(), s.pt0)


def test_host_argument_checks():
    s = synth.small_ring(m=10, n=200, views=4, seed=7)
    g = GpuProblem(s, gamma_max=5)
    f, Jc, Jp, _ = g.residual_jacobian()
    lab = dev(synth.halves_map(10), torch.int32)
    with pytest.raises(S.StbaError):
        S.stba_build_cluster_rcs(g.prob, g.dims, S.make_sample(lab, 2, alpha=0.0), S.StbaDamping(1e-3, 0.1),
                                 S.STBA_FP64, f, Jc, Jp, g.ws)
    with pytest.raises(S.StbaError):
        S.stba_build_cluster_rcs(g.prob, g.dims, S.make_sample(lab, 2), S.StbaDamping(-1.0, 0.1),
                                 S.STBA_FP64, f, Jc, Jp, g.ws)
    with pytest.raises(S.StbaError):
        S.stba_residual_jacobian(g.prob, g.dims, S.STBA_FP64, f, Jc, Jp, None, g.ws[:1024])
    # unsorted observations are found by the analysis
    uv = dev(s.obs_uv, torch.float64)
    oc = dev(s.obs_cam[::-1].copy(), torch.int32)
    op = dev(s.obs_pt[::-1].copy(), torch.int32)
    prob = S.make_problem(g.cam, g.pt, oc, op, uv)
    with pytest.raises(S.StbaError) as e:
        S.stba_analyze(prob)
    assert e.value.code == -6


def test_step_is_deterministic():
    s = _small()
    lab = _sgc(s, 12, 0)
    out = []
    for _ in range(2):
        sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=12, lambda0=1e-4)
        for t in range(2):
            sol.step(sol.sample(lab, alpha=0.7, seed=1, it=t))
        out.append((sol.cam.cpu().numpy(), sol.pt.cpu().numpy(), sol.read_state()["F"]))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


@pytest.mark.parametrize("precision,tol", [(S.STBA_FP64, 1e-12), (S.STBA_MIXED, 1e-5)])
def test_residual_vjp_matches_oracle_gradient(precision, tol):
    s = synth.small_ring(m=30, n=2000, views=7, seed=8)
    plan = S.ResidualPlan(s.obs_cam, s.obs_pt, s.m, s.n, precision)
    cam = dev(s.cam0, torch.float64).requires_grad_(True)
    pt = dev(s.pt0, torch.float64).requires_grad_(True)
    uv = dev(s.obs_uv, torch.float64).requires_grad_(True)
    f = S.residuals(cam, pt, uv, plan)
    loss = (f.double() ** 2).sum()
    loss.backward()
    gc, gp, gu = O.gradient(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)
    assert abs(loss.item() - O.cost(O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv))) <= tol * loss.item()
    assert rel(cam.grad.cpu().numpy(), gc) < tol
    assert rel(pt.grad.cpu().numpy(), gp) < tol
    assert rel(uv.grad.cpu().numpy(), gu) < tol


@pytest.mark.parametrize("gamma", [3, 7, 11])
def test_tile_parallel_cholesky_small_tile_counts(gamma):
    """Cluster caps giving 1, 2 and 4 diagonal tiles per cluster (tile-parallel solve)."""
    s = _small()
    lab = _sgc(s, gamma, 1)
    g = GpuProblem(s, gamma_max=gamma)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3, 0.8, 2, 1)
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3, 0.8, 2, 1)
    assert np.all(cs == 0)
    assert rel(dcam, ref.dcam) < 1e-9
    assert rel(dpt, ref.dpt) < 1e-9


@pytest.mark.parametrize("precision,tol", [(S.STBA_FP64, 1e-9), (S.STBA_MIXED, 1e-4)])
def test_many_clusters_use_workgroup_cholesky(precision, tol):
    """40 singleton clusters with a cap of 40 cameras: too many tile wavefronts,
    so every cluster is solved by one workgroup."""
    s = _small()
    lab = np.arange(s.m, dtype=np.int32)
    g = GpuProblem(s, gamma_max=s.m, precision=precision)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-2)
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-2)
    assert np.all(cs == 0)
    print(f"precision {precision}: dcam rel {rel(dcam, ref.dcam):.2e} dpt rel {rel(dpt, ref.dpt):.2e}")
    assert rel(dcam, ref.dcam) < tol
    assert rel(dpt, ref.dpt) < tol


@pytest.mark.parametrize("lam", [1e-3, 1e-1])
def test_mixed_precision_steps_match_oracle(lam):
    """FP32 Jacobian and Schur assembly, FP64 Cholesky plus one refinement step:
    steps and the candidate cost within 1e-4 relative of the FP64 oracle."""
    s = _small()
    seed, t = 5, 2
    lab = _sgc(s, 12, t)
    g = GpuProblem(s, gamma_max=12, precision=S.STBA_MIXED)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, lam, 1.0, seed, t)
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, 1.0, seed, t)
    assert np.all(cs == 0)
    ec, ep = rel(dcam, ref.dcam), rel(dpt, ref.dpt)
    F_gpu = O.cost(O.residuals(s.cam0 + dcam, s.pt0 + dpt, s.obs_cam, s.obs_pt, s.obs_uv))
    F_ref = O.cost(O.residuals(s.cam0 + ref.dcam, s.pt0 + ref.dpt, s.obs_cam, s.obs_pt, s.obs_uv))
    print(f"lambda {lam}: dcam rel {ec:.2e} dpt rel {ep:.2e} F rel {abs(F_gpu - F_ref) / F_ref:.2e}")
    assert ec < 1e-4 and ep < 1e-4
    assert abs(F_gpu - F_ref) <= 1e-4 * F_ref


def test_mixed_lm_iteration_matches_oracle():
    s = synth.tiny_circle()
    lab = synth.halves_map(16)
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=8, lambda0=1e-3,
                       precision=S.STBA_MIXED)
    sol.step(sol.sample(lab, alpha=1.0, seed=0, it=0))
    st = sol.read_state()
    ref = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3, 1.0, 0, 0)
    print(f"mixed F_new {st['F_new']:.9e} oracle {ref.F_new:.9e}")
    assert st["status"] == 0
    assert bool(st["accepted"]) == ref.accepted
    assert abs(st["F_new"] - ref.F_new) <= 1e-4 * ref.F_new
    assert rel(sol.cam.cpu().numpy() - s.cam0, ref.cam - s.cam0) < 1e-4


def test_full_size_ring_iteration_matches_oracle():
    """One LM iteration on the 200-camera ring (50k points, 400k observations)
    with a Gamma = 50 graph-clustering map, against the FP64 oracle."""
    s = synth.ring(m=200, n=50000, views=8, seed=0)
    lab = _sgc(s, 50, 0)
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=50, lambda0=1e-4)
    sol.step(sol.sample(lab, alpha=1.0, seed=0, it=0))
    st = sol.read_state()
    ref = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-4, 1.0, 0, 0)
    print(f"ring: accepted {st['accepted']} F_new {st['F_new']:.12e} oracle {ref.F_new:.12e} "
          f"dcam {rel(sol.cam.cpu().numpy() - s.cam0, ref.cam - s.cam0):.2e} "
          f"dpt {rel(sol.pt.cpu().numpy() - s.pt0, ref.pt - s.pt0):.2e}")
    assert st["status"] == 0
    assert bool(st["accepted"]) == ref.accepted
    assert abs(st["F_new"] - ref.F_new) <= 1e-9 * ref.F_new
    assert rel(sol.cam.cpu().numpy() - s.cam0, ref.cam - s.cam0) < 1e-9
    assert rel(sol.pt.cpu().numpy() - s.pt0, ref.pt - s.pt0) < 1e-9


def test_long_tracks_use_thread_per_point_path():
    """Points seen by 40 cameras: the one-lane-per-observation kernel does not
    apply (tracks above 32), the thread-per-point path runs instead."""
    s = synth.small_ring(m=50, n=400, views=40, seed=3)
    lab = _sgc(s, 20, 0)
    g = GpuProblem(s, gamma_max=20)
    assert g.dims.max_track > 32
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 0.2, 0.7, 4, 0)
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 0.2, 0.7, 4, 0)
    assert np.all(cs == 0)
    assert rel(dcam, ref.dcam) < 1e-9
    assert rel(dpt, ref.dpt) < 1e-9


@pytest.mark.parametrize("path", ["tile", "workgroup"])
def test_non_positive_definite_cluster_is_reported(path):
    """A cluster system made indefinite (its first diagonal entry set to -1 after
    the assembly) reports STBA_ENOTPD from the device, in the tile-parallel and in
    the one-workgroup-per-cluster factorisation, while every other cluster's step
    still matches the oracle."""
    s = _small()
    lab = _sgc(s, 12, 1) if path == "tile" else np.arange(s.m, dtype=np.int32)
    g = GpuProblem(s, gamma_max=12 if path == "tile" else s.m)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3)
    torch.cuda.synchronize()
    S_off = ws_view(g.ws, rcs.S_off, torch.int64, rcs.l + 1).cpu().numpy()
    Sbuf = ws_view(g.ws, rcs.S, torch.float64, int(S_off[rcs.l]))
    bad = 1
    Sbuf[int(S_off[bad])] = -1.0   # entry (0, 0) of cluster 1 (column-major)
    torch.cuda.synchronize()
    dcam, dpt, cs = g.solve(rcs, Jc, Jp)
    assert cs[bad] == -2                                   # STBA_ENOTPD
    assert np.all(np.delete(cs, bad) == 0)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3)
    good = lab != bad
    assert rel(dcam[good], ref.dcam[good]) < 1e-9
