"""Helpers for the GPU parity tests: run the C ABI calls on a synthetic scene and
copy results back.  Only the tests import this module."""
from __future__ import annotations

import numpy as np
import torch

import paper_2008_00446_amd as S


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def ws_view(ws, ptr, dtype, count):
    """A tensor view of `count` elements of `dtype` at device address `ptr` inside ws."""
    es = torch.tensor([], dtype=dtype).element_size()
    off = int(ptr) - ws.data_ptr()
    assert 0 <= off and off + count * es <= ws.numel()
    return ws[off:off + count * es].view(dtype)


class GpuProblem:
    """The scene's start values and observations on the device, analysed and prepared."""

    def __init__(self, scene, gamma_max, precision=S.STBA_FP64, cam=None, pt=None, huber=0.0):
        self.scene = scene
        self.precision = precision
        self.T = torch.float64 if precision == S.STBA_FP64 else torch.float32
        self.cam = dev(scene.cam0 if cam is None else cam, torch.float64)
        self.pt = dev(scene.pt0 if pt is None else pt, torch.float64)
        self.obs_cam = dev(scene.obs_cam, torch.int32)
        self.obs_pt = dev(scene.obs_pt, torch.int32)
        self.obs_uv = dev(scene.obs_uv, torch.float64)
        self.prob = S.make_problem(self.cam, self.pt, self.obs_cam, self.obs_pt, self.obs_uv, huber)
        self.dims = S.stba_analyze(self.prob)
        self.dims.gamma_max = int(gamma_max)
        self.ws = S.alloc_workspace(S.stba_workspace_bytes(self.prob, self.dims, precision))
        S.stba_prepare(self.prob, self.dims, precision, self.ws)

    @property
    def q(self):
        return self.prob.q

    def residual_jacobian(self):
        q = self.q
        f = torch.empty((q, 2), dtype=self.T, device="cuda")
        Jc = torch.empty((q, 18), dtype=self.T, device="cuda")
        Jp = torch.empty((q, 6), dtype=self.T, device="cuda")
        cost = torch.empty(1, dtype=torch.float64, device="cuda")
        S.stba_residual_jacobian(self.prob, self.dims, self.precision, f, Jc, Jp, cost, self.ws)
        return f, Jc, Jp, cost

    def build(self, f, Jc, Jp, lab, lam, alpha=1.0, seed=0, t=0, lam_corr=0.1):
        lab = np.asarray(lab, dtype=np.int32)
        self._lab = dev(lab, torch.int32)
        samp = S.make_sample(self._lab, int(lab.max()) + 1, alpha, seed, t)
        rcs = S.stba_build_cluster_rcs(self.prob, self.dims, samp, S.StbaDamping(lam, lam_corr), self.precision,
                                       f, Jc, Jp, self.ws)
        return rcs

    def read_rcs(self, rcs, lab):
        """Dense lower-triangular S_k (as full symmetric from the lower part), b, seg heads."""
        torch.cuda.synchronize()
        l = rcs.l
        S_off = ws_view(self.ws, rcs.S_off, torch.int64, l + 1).cpu().numpy()
        cl_Np = ws_view(self.ws, rcs.cl_Np, torch.int32, l).cpu().numpy()
        cl_n = ws_view(self.ws, rcs.cl_n, torch.int32, l).cpu().numpy()
        Sflat = ws_view(self.ws, rcs.S, torch.float64, int(S_off[l])).cpu().numpy()
        blocks = []
        for k in range(l):
            Np, N = int(cl_Np[k]), 9 * int(cl_n[k])
            A = Sflat[S_off[k]:S_off[k] + Np * Np].reshape(Np, Np).T[:N, :N]   # column-major storage
            L = np.tril(A)
            blocks.append(L + np.tril(A, -1).T)
        b = ws_view(self.ws, rcs.b, torch.float64, 9 * self.prob.m).cpu().numpy().reshape(-1, 9)
        seg = ws_view(self.ws, rcs.seg_head, torch.int32, self.q).cpu().numpy()
        return blocks, b, seg, cl_n

    def read_cluster(self, rcs, k):
        """Cluster k's S_k (symmetric, from its lower part) and the b of all cameras."""
        torch.cuda.synchronize()
        l = rcs.l
        S_off = ws_view(self.ws, rcs.S_off, torch.int64, l + 1).cpu().numpy()
        Np = int(ws_view(self.ws, rcs.cl_Np, torch.int32, l).cpu().numpy()[k])
        N = 9 * int(ws_view(self.ws, rcs.cl_n, torch.int32, l).cpu().numpy()[k])
        base = ws_view(self.ws, rcs.S, torch.float64, int(S_off[l]))
        A = base[int(S_off[k]):int(S_off[k]) + Np * Np].cpu().numpy().reshape(Np, Np).T[:N, :N]
        b = ws_view(self.ws, rcs.b, torch.float64, 9 * self.prob.m).cpu().numpy().reshape(-1, 9)
        return np.tril(A) + np.tril(A, -1).T, b

    def solve(self, rcs, Jc, Jp):
        m, n = self.prob.m, self.prob.n
        dcam = torch.empty((m, 9), dtype=torch.float64, device="cuda")
        dpt = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        cs = torch.empty(rcs.l, dtype=torch.int32, device="cuda")
        S.stba_solve_clusters(self.prob, self.dims, rcs, self.precision, Jc, Jp, dcam, dpt, cs, self.ws)
        torch.cuda.synchronize()
        return dcam.cpu().numpy(), dpt.cpu().numpy(), cs.cpu().numpy()


def solve_pcg(g, rcs, Jc, Jp, max_iters, tol):
    """stba_solve_clusters_pcg on a GpuProblem: (dcam, dpt, status, iterations, residuals)."""
    m, n = g.prob.m, g.prob.n
    dcam = torch.empty((m, 9), dtype=torch.float64, device="cuda")
    dpt = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    cs = torch.empty(rcs.l, dtype=torch.int32, device="cuda")
    its = torch.empty(rcs.l, dtype=torch.int32, device="cuda")
    res = torch.empty(rcs.l, dtype=torch.float64, device="cuda")
    S.stba_solve_clusters_pcg(g.prob, g.dims, rcs, g.precision, Jc, Jp, dcam, dpt, max_iters, tol, its, res, cs,
                              g.ws)
    torch.cuda.synchronize()
    return (dcam.cpu().numpy(), dpt.cpu().numpy(), cs.cpu().numpy(), its.cpu().numpy(), res.cpu().numpy())


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def kappa_scaled(Sk):
    """kappa(D^-1 S_k D^-1), D = diag(S_k)^(1/2): the condition number that bounds
    how much FP64 rounding in S_k or b_k (about 1e-16 relative) can move the step."""
    Sk = np.asarray(Sk, dtype=np.float64)
    d = np.sqrt(np.diag(Sk))
    return float(np.linalg.cond(Sk / np.outer(d, d)))
