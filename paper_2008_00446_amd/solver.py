"""Python conveniences over the C ABI: a solver object that owns the workspace
and the device LM state, and residuals as a differentiable function.

Both only marshal arguments; every step of the method runs in libstba.so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import binding as B


class StbaSolver:
    """One bundle-adjustment problem resident on the GPU.

    cam [m,9], pt [n,3] (FP64, copied to the device and updated in place on
    accepted steps), obs_cam / obs_pt [q] int32 sorted by (point, camera),
    obs_uv [q,2] FP64.  gamma_max bounds the cluster sizes of every map later
    passed to `step`.  huber > 0: the robust (Huber) loss of that scale.
    lambda_min > 0: lambda never drops below it after an accepted step."""

    def __init__(self, cam, pt, obs_cam, obs_pt, obs_uv, gamma_max, precision=B.STBA_FP64,
                 lambda0=1e-4, lambda_corr=0.1, device="cuda", huber=0.0, lambda_min=0.0):
        as_dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)  # noqa: E731
        self.cam = as_dev(cam, torch.float64).clone()
        self.pt = as_dev(pt, torch.float64).clone()
        self.obs_cam = as_dev(obs_cam, torch.int32)
        self.obs_pt = as_dev(obs_pt, torch.int32)
        self.obs_uv = as_dev(obs_uv, torch.float64)
        self.precision = int(precision)
        self.problem = B.make_problem(self.cam, self.pt, self.obs_cam, self.obs_pt, self.obs_uv, huber)
        self.dims = B.stba_analyze(self.problem)
        self.dims.gamma_max = int(gamma_max)
        self.ws = B.alloc_workspace(B.stba_workspace_bytes(self.problem, self.dims, self.precision))
        B.stba_prepare(self.problem, self.dims, self.precision, self.ws)
        self.state = B.new_state(device)
        B.stba_lm_init(self.state, lambda0, lambda_corr)
        if lambda_min:
            B.set_lambda_min(self.state, lambda_min)
        self._events = None
        self._sgc = None

    @property
    def m(self):
        return self.problem.m

    @property
    def q(self):
        return self.problem.q

    def sample(self, cam_cluster, alpha=1.0, seed=0, it=0, l=None):
        cc = cam_cluster if torch.is_tensor(cam_cluster) else torch.as_tensor(
            np.asarray(cam_cluster, dtype=np.int32)).to(self.cam.device)
        if l is None:
            l = int(np.asarray(cam_cluster.cpu() if torch.is_tensor(cam_cluster) else cam_cluster).max()) + 1
        return B.make_sample(cc, l, alpha, seed, it)

    def sample_clusters(self, gamma, beta=10.0, alpha=1.0, seed=0, it=0, stream=None):
        """Draw iteration `it`'s camera clustering on the device (stochastic graph
        clustering, cap gamma) and return the sample for `step`.  The map stays on
        the device; only l is read back (the call waits for the kernel).  The map
        buffer is reused by the next call, after the work queued before it."""
        if self._sgc is None:
            self._sgc = (torch.empty(self.m, dtype=torch.int32, device=self.cam.device),
                         torch.zeros(2, dtype=torch.int32, device=self.cam.device))
        cc, out = self._sgc
        B.stba_sample_clusters(self.problem, self.dims, self.precision, self.ws, gamma, beta, seed, it, cc,
                               out[0:1], out[1:2], stream)
        l, status = (int(v) for v in out.cpu().tolist())
        if status != 0:
            raise B.StbaError("stba_sample_clusters", status)
        return B.make_sample(cc, l, alpha, seed, it)

    def sample_clusters_device(self, gamma, beta=10.0, alpha=1.0, seed=0, it=0, stream=None):
        """Draw iteration `it`'s camera clustering on the device and return a sample
        that reads the number of clusters on the device (l = m as the bound), so
        nothing is read back and the draw can be captured with the step.  The map
        buffer is reused by the next call, after the work queued before it."""
        if self._sgc is None:
            self._sgc = (torch.empty(self.m, dtype=torch.int32, device=self.cam.device),
                         torch.zeros(2, dtype=torch.int32, device=self.cam.device))
        cc, out = self._sgc
        B.stba_sample_clusters(self.problem, self.dims, self.precision, self.ws, gamma, beta, seed, it, cc,
                               out[0:1], out[1:2], stream)
        return B.make_sample(cc, self.m, alpha, seed, it, l_dev=out[0:1])

    def autotune(self, sample, cache_path=None):
        """Choose the Schur workgroup count and the factorisation form for this
        problem's shape class (measured once per class; see tuning.py)."""
        from .tuning import autotune_solver
        return autotune_solver(self, sample, cache_path)

    def step(self, sample, events=None, pcg=None):
        """One LM iteration (asynchronous); pcg = (max_iters, tol): the cluster
        solves by conjugate gradient instead of Cholesky."""
        if pcg is not None:
            B.stba_lm_step_pcg(self.problem, self.dims, sample, self.state, self.precision, pcg[0], pcg[1], self.ws)
        elif events is None:
            B.stba_lm_step(self.problem, self.dims, sample, self.state, self.precision, self.ws)
        else:
            B.stba_lm_step_profiled(self.problem, self.dims, sample, self.state, self.precision, self.ws, events)

    def read_state(self):
        return B.read_state(self.state)


class BatchSolver:
    """Many independent bundle-adjustment problems stepped by one LM iteration
    (stba_lm_step_batched): the problems are concatenated with index offsets,
    and each keeps its own damping, cost and accept decision.

    problems: a list of (cam [m_b,9], pt [n_b,3], obs_cam [q_b], obs_pt [q_b],
    obs_uv [q_b,2]) with local indices, each sorted by (point, camera)."""

    def __init__(self, problems, gamma_max, precision=B.STBA_FP64, lambda0=1e-4, lambda_corr=0.1, device="cuda",
                 huber=0.0):
        cams, pts, oc, op, uv = [], [], [], [], []
        self.cam_off, self.pt_off, self.obs_off = [0], [0], [0]
        for cam, pt, c_, p_, u_ in problems:
            cams.append(np.asarray(cam, dtype=np.float64))
            pts.append(np.asarray(pt, dtype=np.float64))
            oc.append(np.asarray(c_, dtype=np.int64) + self.cam_off[-1])
            op.append(np.asarray(p_, dtype=np.int64) + self.pt_off[-1])
            uv.append(np.asarray(u_, dtype=np.float64))
            self.cam_off.append(self.cam_off[-1] + len(cams[-1]))
            self.pt_off.append(self.pt_off[-1] + len(pts[-1]))
            self.obs_off.append(self.obs_off[-1] + len(oc[-1]))
        self.n_prob = len(problems)
        as_dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)  # noqa: E731
        self.cam = as_dev(np.vstack(cams), torch.float64).clone()
        self.pt = as_dev(np.vstack(pts), torch.float64).clone()
        self.obs_cam = as_dev(np.concatenate(oc), torch.int32)
        self.obs_pt = as_dev(np.concatenate(op), torch.int32)
        self.obs_uv = as_dev(np.vstack(uv), torch.float64)
        sizes = np.diff(self.cam_off)
        self.prob_cam = as_dev(np.repeat(np.arange(self.n_prob), sizes), torch.int32)
        self.prob_pt = as_dev(np.repeat(np.arange(self.n_prob), np.diff(self.pt_off)), torch.int32)
        self.prob_obs_off = as_dev(np.asarray(self.obs_off), torch.int64)
        self.precision = int(precision)
        self.problem = B.make_problem(self.cam, self.pt, self.obs_cam, self.obs_pt, self.obs_uv, huber)
        self.dims = B.stba_analyze(self.problem)
        self.dims.gamma_max = int(gamma_max)
        self.ws = B.alloc_workspace(B.stba_workspace_bytes(self.problem, self.dims, self.precision))
        B.stba_prepare(self.problem, self.dims, self.precision, self.ws)
        self.states = B.new_states(self.n_prob, device)
        for b in range(self.n_prob):
            B.stba_lm_init(self.states[b], lambda0, lambda_corr)

    def sample(self, maps, alpha=1.0, seed=0, it=0):
        """maps: one cluster map per problem (local cluster ids); the clusters are
        numbered across the batch in problem order."""
        full, base = [], 0
        for mp in maps:
            mp = np.asarray(mp, dtype=np.int64)
            full.append(mp + base)
            base += int(mp.max()) + 1
        cc = torch.as_tensor(np.concatenate(full).astype(np.int32)).to(self.cam.device)
        return B.make_sample(cc, base, alpha, seed, it)

    def step(self, sample):
        """One LM iteration of every problem (asynchronous)."""
        B.stba_lm_step_batched(self.problem, self.dims, sample, self.states, self.n_prob, self.prob_cam,
                               self.prob_pt, self.prob_obs_off, self.precision, self.ws)

    def read_states(self):
        return [B.read_state(self.states[b]) for b in range(self.n_prob)]

    def cam_of(self, b):
        return self.cam[self.cam_off[b]:self.cam_off[b + 1]]

    def pt_of(self, b):
        return self.pt[self.pt_off[b]:self.pt_off[b + 1]]


class ResidualPlan:
    """Static structure (visibility graph) for repeated residual / J^T v calls.

    store_jacobian: keep J (24 values per observation) from the forward pass and
    read it in the backward pass, instead of recomputing it (the default, for
    when memory is short)."""

    def __init__(self, obs_cam, obs_pt, m, n, precision=B.STBA_FP64, device="cuda", store_jacobian=False):
        self.store_jacobian = bool(store_jacobian)
        self.obs_cam = torch.as_tensor(obs_cam, dtype=torch.int32).to(device).contiguous()
        self.obs_pt = torch.as_tensor(obs_pt, dtype=torch.int32).to(device).contiguous()
        self.m, self.n, self.q = int(m), int(n), int(self.obs_cam.shape[0])
        self.precision = int(precision)
        self.dtype = torch.float64 if self.precision == B.STBA_FP64 else torch.float32
        cam = torch.zeros((self.m, 9), dtype=torch.float64, device=device)
        pt = torch.zeros((self.n, 3), dtype=torch.float64, device=device)
        uv = torch.zeros((self.q, 2), dtype=torch.float64, device=device)
        prob = B.make_problem(cam, pt, self.obs_cam, self.obs_pt, uv)
        self.dims = B.stba_analyze(prob)
        self.dims.gamma_max = 1
        self.ws = B.alloc_workspace(B.stba_workspace_bytes(prob, self.dims, self.precision))
        B.stba_prepare(prob, self.dims, self.precision, self.ws)

    def problem(self, cam, pt, uv):
        return B.make_problem(cam.contiguous(), pt.contiguous(), self.obs_cam, self.obs_pt, uv.contiguous())


class _Residuals(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cam, pt, obs_uv, plan):
        cam_d, pt_d, uv_d = cam.detach(), pt.detach(), obs_uv.detach()
        prob = plan.problem(cam_d, pt_d, uv_d)
        f = torch.empty((plan.q, 2), dtype=plan.dtype, device=cam.device)
        if plan.store_jacobian:
            Jc = torch.empty((plan.q, 18), dtype=plan.dtype, device=cam.device)
            Jp = torch.empty((plan.q, 6), dtype=plan.dtype, device=cam.device)
            B.stba_residual_jacobian(prob, plan.dims, plan.precision, f, Jc, Jp, None, plan.ws)
            ctx.save_for_backward(cam_d, pt_d, uv_d, Jc, Jp)
        else:
            B.stba_residual_jacobian(prob, plan.dims, plan.precision, f, None, None, None, plan.ws)
            ctx.save_for_backward(cam_d, pt_d, uv_d)
        ctx.plan = plan
        return f

    @staticmethod
    def backward(ctx, grad_f):
        plan = ctx.plan
        cam, pt, uv = ctx.saved_tensors[:3]
        prob = plan.problem(cam, pt, uv)
        v = grad_f.to(plan.dtype).contiguous()
        gc = torch.empty((plan.m, 9), dtype=plan.dtype, device=cam.device)
        gp = torch.empty((plan.n, 3), dtype=plan.dtype, device=cam.device)
        gu = torch.empty((plan.q, 2), dtype=plan.dtype, device=cam.device)
        if plan.store_jacobian:
            Jc, Jp = ctx.saved_tensors[3:]
            B.stba_residual_vjp_stored(prob, plan.dims, plan.precision, v, Jc, Jp, gc, gp, gu, plan.ws)
        else:
            B.stba_residual_vjp(prob, plan.dims, plan.precision, v, gc, gp, gu, plan.ws)
        return gc.to(cam.dtype), gp.to(pt.dtype), gu.to(uv.dtype), None


def residuals(cam, pt, obs_uv, plan: ResidualPlan):
    """Reprojection residuals f (pixel - observed) as a differentiable function of
    cam, pt and obs_uv; the backward pass is J^T v on the GPU, with J recomputed
    or, for a plan made with store_jacobian=True, kept from the forward pass."""
    return _Residuals.apply(cam, pt, obs_uv, plan)


def hip_events(count):
    """Create `count` timing events through the HIP runtime (for stba_lm_step_profiled)."""
    hip = ctypes.CDLL("libamdhip64.so")
    arr = (ctypes.c_void_p * count)()
    for i in range(count):
        rc = hip.hipEventCreate(ctypes.byref(arr, i * ctypes.sizeof(ctypes.c_void_p)))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed: {rc}")
    return arr


def event_ms(start, stop) -> float:
    hip = ctypes.CDLL("libamdhip64.so")
    ms = ctypes.c_float(0.0)
    rc = hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(start), ctypes.c_void_p(stop))
    if rc != 0:
        raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
    return float(ms.value)
