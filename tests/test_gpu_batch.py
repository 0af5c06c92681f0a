"""The differentiation batch: many independent ring problems concatenated into
one with index offsets (cameras and points renumbered per problem), residuals
forward and J^T v backward through the autograd function in one launch each,
FP64 and FP32.  Checked per problem against the oracle's gradient 2 J^T f and
against central differences of the oracle's FP64 cost on sampled coordinates
(only the observations a coordinate touches change the cost)."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2008_00446_amd as S
import synth
from gpu_helpers import dev, rel

pytestmark = pytest.mark.gpu


def _concat(batch):
    cams, pts, oc, op, uv, spans = [], [], [], [], [], []
    c0 = p0 = 0
    for s in batch:
        cams.append(s.cam0)
        pts.append(s.pt0)
        oc.append(s.obs_cam + c0)
        op.append(s.obs_pt + p0)
        uv.append(s.obs_uv)
        spans.append((c0, c0 + s.m, p0, p0 + s.n))
        c0 += s.m
        p0 += s.n
    return (np.vstack(cams), np.vstack(pts), np.concatenate(oc).astype(np.int32),
            np.concatenate(op).astype(np.int32), np.vstack(uv), spans)


def _local_cost(s, cam, pt, obs):
    f = O.residuals(cam, pt, s.obs_cam[obs], s.obs_pt[obs], s.obs_uv[obs])
    return float(np.sum(f * f))


@pytest.mark.parametrize("precision,tol", [(S.STBA_FP64, 1e-12), (S.STBA_MIXED, 1e-5)], ids=["fp64", "fp32"])
def test_batched_gradient_matches_oracle_per_problem(precision, tol):
    batch = synth.diff_batch(seeds=range(6))
    cam, pt, oc, op, uv, spans = _concat(batch)
    plan = S.ResidualPlan(oc, op, cam.shape[0], pt.shape[0], precision)
    tc = dev(cam, torch.float64).requires_grad_(True)
    tp = dev(pt, torch.float64).requires_grad_(True)
    tu = dev(uv, torch.float64).requires_grad_(True)
    f = S.residuals(tc, tp, tu, plan)
    loss = (f.double() ** 2).sum()
    loss.backward()
    gc, gp, gu = tc.grad.cpu().numpy(), tp.grad.cpu().numpy(), tu.grad.cpu().numpy()
    q0 = 0
    F_all = 0.0
    heavy = 0
    for s, (c0, c1, p0, p1) in zip(batch, spans):
        rc, rp, ru = O.gradient(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)
        assert rel(gc[c0:c1], rc) < tol and rel(gp[p0:p1], rp) < tol
        assert rel(gu[q0:q0 + s.q], ru) < tol
        # cameras with more observations than one wavefront takes (1792): their
        # sums come from several parts, each row checked on its own
        for i in np.flatnonzero(np.bincount(s.obs_cam, minlength=s.m) > 1792):
            assert rel(gc[c0 + i], rc[i]) < tol, (s.m, i)
            heavy += 1
        q0 += s.q
        F_all += O.cost(O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv))
    assert heavy > 0
    assert abs(loss.item() - F_all) <= tol * F_all


def test_batched_gradient_matches_central_differences():
    batch = synth.diff_batch(seeds=range(3))
    cam, pt, oc, op, uv, spans = _concat(batch)
    plan = S.ResidualPlan(oc, op, cam.shape[0], pt.shape[0], S.STBA_FP64)
    tc = dev(cam, torch.float64).requires_grad_(True)
    tp = dev(pt, torch.float64).requires_grad_(True)
    f = S.residuals(tc, tp, dev(uv, torch.float64), plan)
    (f ** 2).sum().backward()
    gc, gp = tc.grad.cpu().numpy(), tp.grad.cpu().numpy()
    rng = np.random.default_rng(5)
    h = 1e-4
    for s, (c0, c1, p0, p1) in zip(batch, spans):
        for _ in range(20):
            i, k = int(rng.integers(s.m)), int(rng.integers(9))
            obs = np.flatnonzero(s.obs_cam == i)
            cp, cm = s.cam0.copy(), s.cam0.copy()
            cp[i, k] += h
            cm[i, k] -= h
            fd = (_local_cost(s, cp, s.pt0, obs) - _local_cost(s, cm, s.pt0, obs)) / (2 * h)
            assert abs(gc[c0 + i, k] - fd) <= 1e-5 * max(1.0, abs(fd)) + 1e-4 * abs(fd), (i, k)
        for _ in range(20):
            j, k = int(rng.integers(s.n)), int(rng.integers(3))
            obs = np.flatnonzero(s.obs_pt == j)
            pp, pm = s.pt0.copy(), s.pt0.copy()
            pp[j, k] += h
            pm[j, k] -= h
            fd = (_local_cost(s, s.cam0, pp, obs) - _local_cost(s, s.cam0, pm, obs)) / (2 * h)
            assert abs(gp[p0 + j, k] - fd) <= 1e-5 * max(1.0, abs(fd)) + 1e-4 * abs(fd), (j, k)


def _richardson(cost_at, h):
    """d/dt of cost_at(t) at 0 by central differences at h and h / 2 combined
    by Richardson extrapolation (truncation O(h^4))."""
    d1 = (cost_at(h) - cost_at(-h)) / (2 * h)
    d2 = (cost_at(h / 2) - cost_at(-h / 2)) / h
    return (4 * d2 - d1) / 3


@pytest.mark.parametrize("precision,rtol", [(S.STBA_FP64, 1e-7), (S.STBA_MIXED, 1e-4)], ids=["fp64", "fp32"])
def test_64_problem_batch_gradient_against_central_differences(precision, rtol):
    """The full 64-problem batch in one launch each way; on every problem 200
    coordinates (100 camera, 100 point, drawn at random) against central
    differences of the oracle's FP64 cost over the observations the coordinate
    touches (h = 1e-3 and 5e-4, Richardson-extrapolated: truncation near
    1e-12 relative, rounding near 1e-9).  FP32 stores f and the gradients in
    FP32."""
    batch = synth.diff_batch(seeds=range(64))
    cam, pt, oc, op, uv, spans = _concat(batch)
    plan = S.ResidualPlan(oc, op, cam.shape[0], pt.shape[0], precision)
    tc = dev(cam, torch.float64).requires_grad_(True)
    tp = dev(pt, torch.float64).requires_grad_(True)
    f = S.residuals(tc, tp, dev(uv, torch.float64), plan)
    (f.double() ** 2).sum().backward()
    gc, gp = tc.grad.cpu().numpy(), tp.grad.cpu().numpy()
    rng = np.random.default_rng(11)
    h = 1e-3
    worst = 0.0
    for s, (c0, c1, p0, p1) in zip(batch, spans):
        by_cam = np.argsort(s.obs_cam, kind="stable")
        cam_start = np.searchsorted(s.obs_cam[by_cam], np.arange(s.m + 1))
        pt_start = np.searchsorted(s.obs_pt, np.arange(s.n + 1))
        for _ in range(100):
            i, k = int(rng.integers(s.m)), int(rng.integers(9))
            obs = by_cam[cam_start[i]:cam_start[i + 1]]

            def at(t):
                c = s.cam0.copy()
                c[i, k] += t
                return _local_cost(s, c, s.pt0, obs)
            fd = _richardson(at, h)
            err = abs(gc[c0 + i, k] - fd) / max(1.0, abs(fd))
            worst = max(worst, err)
            assert err <= rtol, (s.m, i, k, gc[c0 + i, k], fd)
        for _ in range(100):
            j, k = int(rng.integers(s.n)), int(rng.integers(3))
            obs = np.arange(pt_start[j], pt_start[j + 1])

            def at(t):
                p = s.pt0.copy()
                p[j, k] += t
                return _local_cost(s, s.cam0, p, obs)
            fd = _richardson(at, h)
            err = abs(gp[p0 + j, k] - fd) / max(1.0, abs(fd))
            worst = max(worst, err)
            assert err <= rtol, (s.n, j, k, gp[p0 + j, k], fd)
    print(f"64 problems x 200 coordinates: worst |g - fd| / max(1, |fd|) = {worst:.2e}", flush=True)


@pytest.mark.parametrize("precision", [S.STBA_FP64, S.STBA_MIXED], ids=["fp64", "fp32"])
def test_stored_jacobian_vjp_matches_recompute_and_oracle(precision):
    """The stored-Jacobian backward pass (J kept from the forward evaluation)
    against the recomputing one: the same sums in the same order, so FP64 agrees
    to rounding (the compiler fuses the block's last products into the sums
    differently in the two kernels); FP32 stores rounded blocks and agrees to
    FP32 rounding.  Both against the oracle's gradient 2 J^T f per problem."""
    batch = synth.diff_batch(seeds=range(6))
    cam, pt, oc, op, uv, spans = _concat(batch)
    grads = {}
    for store in (False, True):
        plan = S.ResidualPlan(oc, op, cam.shape[0], pt.shape[0], precision, store_jacobian=store)
        tc = dev(cam, torch.float64).requires_grad_(True)
        tp = dev(pt, torch.float64).requires_grad_(True)
        tu = dev(uv, torch.float64).requires_grad_(True)
        f = S.residuals(tc, tp, tu, plan)
        (f.double() ** 2).sum().backward()
        grads[store] = [t.grad.cpu().numpy() for t in (tc, tp, tu)]
    for a, b in zip(grads[False], grads[True]):
        assert rel(b, a) < (1e-13 if precision == S.STBA_FP64 else 1e-5)
    tol = 1e-12 if precision == S.STBA_FP64 else 1e-5
    gc, gp, gu = grads[True]
    q0 = 0
    for s, (c0, c1, p0, p1) in zip(batch, spans):
        rc, rp, ru = O.gradient(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)
        assert rel(gc[c0:c1], rc) < tol and rel(gp[p0:p1], rp) < tol
        assert rel(gu[q0:q0 + s.q], ru) < tol
        q0 += s.q


def test_stored_jacobian_vjp_rejects_missing_blocks():
    batch = synth.diff_batch(seeds=range(1))
    cam, pt, oc, op, uv, _ = _concat(batch)
    plan = S.ResidualPlan(oc, op, cam.shape[0], pt.shape[0], S.STBA_FP64, store_jacobian=True)
    prob = plan.problem(dev(cam, torch.float64), dev(pt, torch.float64), dev(uv, torch.float64))
    v = torch.zeros((plan.q, 2), dtype=torch.float64, device="cuda")
    gc = torch.empty((plan.m, 9), dtype=torch.float64, device="cuda")
    gp = torch.empty((plan.n, 3), dtype=torch.float64, device="cuda")
    gu = torch.empty((plan.q, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(S.StbaError):
        S.stba_residual_vjp_stored(prob, plan.dims, S.STBA_FP64, v, None, None, gc, gp, gu, plan.ws)


@pytest.mark.parametrize("precision,tol", [(S.STBA_FP64, 1e-12), (S.STBA_MIXED, 1e-5)], ids=["fp64", "fp32"])
def test_camera_sums_at_the_part_boundaries(precision, tol):
    """The camera sums of J^T v run over each camera's observations in parts
    of at most 1792 (one wavefront each) added in part order: cameras of
    exactly one part (1792), one past it (1793), exactly two parts (3584), a
    small one (100) and one that sees nothing, each camera's gradient row
    against the oracle's."""
    rng = np.random.default_rng(5)
    sizes = [1792, 1793, 3584, 100, 0]
    m, n = len(sizes), max(sizes)
    pt = np.column_stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(6, 9, n)])
    cam = np.zeros((m, 9))
    cam[:, :3] = rng.normal(0, 0.02, (m, 3))
    cam[:, 3:6] = rng.normal(0, 0.1, (m, 3))
    cam[:, 6], cam[:, 7], cam[:, 8] = 500.0, 1e-3, -1e-4
    # observations sorted by point, then camera: camera i sees points 0 .. sizes[i] - 1
    pairs = sorted((j, i) for i, k in enumerate(sizes) for j in range(k))
    op = np.array([j for j, _ in pairs], dtype=np.int32)
    oc = np.array([i for _, i in pairs], dtype=np.int32)
    uv = O.residuals(cam, pt, oc, op, np.zeros((len(op), 2))) + rng.normal(0, 1.0, (len(op), 2))
    plan = S.ResidualPlan(oc, op, m, n, precision)
    tc = dev(cam, torch.float64).requires_grad_(True)
    tp = dev(pt, torch.float64).requires_grad_(True)
    f = S.residuals(tc, tp, dev(uv, torch.float64), plan)
    (f.double() ** 2).sum().backward()
    gc = tc.grad.cpu().numpy()
    rc, rp, _ = O.gradient(cam, pt, oc, op, uv)
    for i, k in enumerate(sizes):
        if k == 0:
            assert np.all(gc[i] == 0.0)
        else:
            assert rel(gc[i], rc[i]) < tol, (i, k)
    assert rel(tp.grad.cpu().numpy(), rp) < tol
