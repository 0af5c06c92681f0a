"""The inexact cluster solve (App. A, Table 3: conjugate gradient with the
camera-block Jacobi preconditioner) on the GPU against the oracle: the first
iterates against the oracle's PCG on the oracle's own S_k and b_k, converged
steps against the exact (Cholesky) STBA step on a small ring and on the
200-camera ring, MIXED, a non-positive-definite cluster, and argument errors."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_00446_amd as S
import synth
from gpu_helpers import GpuProblem, kappa_scaled, rel, solve_pcg, ws_view


def _kappas(ref):
    """kappa(S_k) and kappa(D^-1 S_k D^-1) of every cluster system of the oracle's step."""
    return [(float(np.linalg.cond(Sk)), kappa_scaled(Sk)) for Sk in ref.S_blocks]


def _report(tag, kap, dc_err, dp_err, tol):
    k_max = max(k for k, _ in kap)
    ks_max = max(k for _, k in kap)
    # stopping at ||r|| <= tol ||b|| bounds the relative error of each cluster's
    # step by kappa(S_k) tol; with FP64 rounding of S_k alone the bound is
    # about kappa_scaled 1e-16
    print(f"{tag}: max kappa(S_k) {k_max:.2e}, max kappa(D^-1 S_k D^-1) {ks_max:.2e}, "
          f"kappa tol {k_max * tol:.1e}, kappa_scaled eps {ks_max * 1e-16:.1e}; "
          f"errors dcam {dc_err:.2e} dpt {dp_err:.2e}", flush=True)
    return k_max, ks_max


pytestmark = pytest.mark.gpu


def _small():
    return synth.small_ring(m=40, n=3000, views=8, seed=1)


def _map(s, gamma, t, seed=0):
    e, w = O.covisibility_graph(s.obs_cam, s.obs_pt, s.m, s.n)
    return O.sgc_clusters(e, w, s.m, gamma, 10.0, seed, t)[0]


@pytest.mark.parametrize("k", [1, 2, 5])
def test_first_iterates_match_oracle_pcg(k):
    s = _small()
    lab = _map(s, 12, 0)
    g = GpuProblem(s, gamma_max=12)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3)
    dcam, _, cs, its, _ = solve_pcg(g, rcs, Jc, Jp, k, 0.0)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3)
    assert np.all(cs == 0) and np.all(its == k)
    for Sk, bk, cams in zip(ref.S_blocks, ref.b_blocks, ref.clusters):
        x, it, _, ok = O.pcg(Sk, bk, 0.0, k)
        assert ok and it == k
        assert rel(dcam[cams].reshape(-1), x) < 1e-9


@pytest.mark.parametrize("lam,alpha", [(1e-3, 1.0), (0.3, 0.7)])
def test_converged_pcg_matches_the_exact_step(lam, alpha):
    s = _small()
    lab = _map(s, 12, 2)
    g = GpuProblem(s, gamma_max=12)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, lam, alpha=alpha, seed=3)
    dcam, dpt, cs, its, res = solve_pcg(g, rcs, Jc, Jp, 1000, 1e-12)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, alpha, 3)
    print(f"pcg small ring lam={lam} alpha={alpha}: iterations {its.tolist()}", flush=True)
    k_max, _ = _report("small ring", _kappas(ref), rel(dcam, ref.dcam), rel(dpt, ref.dpt), 1e-12)
    assert np.all(cs == 0) and np.all(res <= 1e-12) and np.all(its < 1000)
    # the stopping rule's bound, not below the FP64 bar
    bar = max(1e-9, 10.0 * k_max * 1e-12)
    assert rel(dcam, ref.dcam) < bar
    assert rel(dpt, ref.dpt) < bar


def test_ring_pcg_matches_the_exact_step():
    s = synth.ring(m=200, n=50_000, views=8, seed=0)
    lab = _map(s, 50, 0)
    g = GpuProblem(s, gamma_max=50)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-4)
    dcam, dpt, cs, its, res = solve_pcg(g, rcs, Jc, Jp, 2000, 1e-12)
    print(f"pcg ring: iterations {its.tolist()} residuals {res.tolist()}", flush=True)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-4)
    k_max, _ = _report("ring", _kappas(ref), rel(dcam, ref.dcam), rel(dpt, ref.dpt), 1e-12)
    assert np.all(cs == 0) and np.all(res <= 1e-12)
    bar = max(1e-9, 10.0 * k_max * 1e-12)
    assert rel(dcam, ref.dcam) < bar
    assert rel(dpt, ref.dpt) < bar


def test_mixed_precision_pcg_within_the_mixed_bar():
    s = _small()
    lab = _map(s, 12, 1)
    g = GpuProblem(s, gamma_max=12, precision=S.STBA_MIXED)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3)
    dcam, dpt, cs, its, res = solve_pcg(g, rcs, Jc, Jp, 1000, 1e-12)
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3)
    assert np.all(cs == 0)
    assert rel(dcam, ref.dcam) < 1e-4
    assert rel(dpt, ref.dpt) < 1e-4


def test_non_positive_definite_cluster_is_reported():
    s = _small()
    lab = _map(s, 12, 1)
    g = GpuProblem(s, gamma_max=12)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3)
    torch.cuda.synchronize()
    S_off = ws_view(g.ws, rcs.S_off, torch.int64, rcs.l + 1).cpu().numpy()
    Sbuf = ws_view(g.ws, rcs.S, torch.float64, int(S_off[rcs.l]))
    bad = 1
    Sbuf[int(S_off[bad])] = -1.0   # entry (0, 0) of cluster 1
    torch.cuda.synchronize()
    dcam, _, cs, _, _ = solve_pcg(g, rcs, Jc, Jp, 500, 1e-12)
    assert cs[bad] == -2 and np.all(np.delete(cs, bad) == 0)
    assert not dcam[lab == bad].any()
    ref = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3)
    good = lab != bad
    k_max, _ = _report("non-PD cluster", _kappas(ref), rel(dcam[good], ref.dcam[good]), 0.0, 1e-12)
    assert rel(dcam[good], ref.dcam[good]) < max(1e-9, 10.0 * k_max * 1e-12)


def test_bad_arguments_are_rejected():
    s = _small()
    lab = _map(s, 12, 0)
    g = GpuProblem(s, gamma_max=12)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-3)
    for it, tol in [(-1, 1e-6), (10, float("nan")), (10, -1.0), (10, float("inf"))]:
        with pytest.raises(S.StbaError):
            solve_pcg(g, rcs, Jc, Jp, it, tol)


@pytest.mark.parametrize("max_iters,tol", [(10, 0.0), (2000, 1e-12)])
def test_lm_iterations_with_pcg_solves_match_oracle(max_iters, tol):
    s = _small()
    lam0 = 1e-3
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=12, lambda0=lam0)
    cam, pt, lam = s.cam0.copy(), s.pt0.copy(), lam0
    F = O.cost(O.residuals(cam, pt, s.obs_cam, s.obs_pt, s.obs_uv))
    for t in range(3):
        lab = _map(s, 12, t)
        sol.step(sol.sample(lab, it=t), pcg=(max_iters, tol))
        st = sol.read_state()
        r = O.lm_iteration(cam, pt, s.obs_cam, s.obs_pt, s.obs_uv, lab, lam, 1.0, 0, t, F=F,
                           pcg_opts=(max_iters, tol))
        assert st["status"] == 0 and bool(st["accepted"]) == r.accepted, t
        assert st["lambda_"] == r.lam, t
        assert abs(st["F"] - r.F) <= 1e-9 * r.F, t
        cam, pt, lam, F = r.cam, r.pt, r.lam, r.F
        err = rel(sol.cam.cpu().numpy() - s.cam0, cam - s.cam0)
        kap = _kappas(r.step)
        _report(f"LM iteration {t}, {max_iters} iterations tol {tol:g}", kap, err, 0.0, tol)
        # both sides run the same recurrence on S_k that differ by FP64 assembly
        # rounding; conjugate gradient passes such differences on to its
        # iterates scaled by up to kappa(D^-1 S_k D^-1), and a converged solve
        # is bounded by the stopping rule
        ks_max = max(k for _, k in kap)
        k_max = max(k for k, _ in kap)
        bar = max(1e-9, 1e3 * ks_max * 1e-16, 10.0 * k_max * tol if tol > 0 else 0.0)
        assert err < bar, t
