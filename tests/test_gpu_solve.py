"""Cluster solves against the matrices they solve (no oracle needed): every
cluster's camera step satisfies the assembled system S_k dc_k = b_k (Eq. 13)
to FP64 rounding, whether FP64 or FP32 (STBA_MIXED_NOREFINE) assembled S_k.
STBA_MIXED's refinement step aims at the FP64 method's system instead: its
step is checked against the FP64-assembled S_k and b_k.  On the 200-camera
ring with Gamma = 50 (5 clusters of up to 50 cameras, 13-15 tile rows) this
runs the tile-parallel factorisation and its substitution chains, then for
MIXED the refinement residual and the sweeps with the stored factors."""
import numpy as np
import pytest

import paper_2008_00446_amd as S
import synth
from gpu_helpers import GpuProblem

pytestmark = pytest.mark.gpu




def _backward_error(A, x, b):
    """Normwise backward error ||A x - b|| / (||A|| ||x|| + ||b||), infinity norms."""
    r = A @ x - b
    return float(np.abs(r).max() / (np.abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()))


# A Cholesky solve is backward stable with an error of order N u (N <= 450
# here, u = 1.1e-16).
BOUND = 1e-13


@pytest.mark.parametrize("precision", [S.STBA_FP64, S.STBA_MIXED_NOREFINE])
def test_ring_cluster_solves_are_backward_stable(precision):
    s = synth.ring(m=200, n=50000, views=8, seed=0)
    e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
    lab = synth.sgc_map(e, w, s.m, 50, 10.0, 0, 0)
    g = GpuProblem(s, gamma_max=50, precision=precision)
    f, Jc, Jp, _ = g.residual_jacobian()
    rcs = g.build(f, Jc, Jp, lab, 1e-4)
    systems = [g.read_cluster(rcs, k) for k in range(rcs.l)]   # before the solve factorises S in place
    dcam, _, cs = g.solve(rcs, Jc, Jp)
    assert np.all(cs == 0)
    for k, (A, b_all) in enumerate(systems):
        cams = np.nonzero(lab == k)[0]          # a cluster's cameras in increasing order
        x = dcam[cams].reshape(-1)
        b = b_all[cams].reshape(-1)
        eta = _backward_error(A, x, b)
        print(f"precision {precision} cluster {k} ({len(cams)} cameras, N = {A.shape[0]}): backward error {eta:.2e}")
        assert eta < BOUND


def test_refined_mixed_steps_solve_the_fp64_systems():
    """STBA_MIXED's step against the FP64-assembled S_k and b_k: the unrefined
    step's backward error there is that of the FP32 assembly (about 2^-24 times
    the cancellation in S_k); one refinement step leaves about that error times
    kappa 2^-24."""
    s = synth.ring(m=200, n=50000, views=8, seed=0)
    e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
    lab = synth.sgc_map(e, w, s.m, 50, 10.0, 0, 0)
    g64 = GpuProblem(s, gamma_max=50, precision=S.STBA_FP64)
    f, Jc, Jp, _ = g64.residual_jacobian()
    rcs = g64.build(f, Jc, Jp, lab, 1e-4)
    systems = [g64.read_cluster(rcs, k) for k in range(rcs.l)]
    steps = {}
    for precision in (S.STBA_MIXED_NOREFINE, S.STBA_MIXED):
        g = GpuProblem(s, gamma_max=50, precision=precision)
        f, Jc, Jp, _ = g.residual_jacobian()
        rcs = g.build(f, Jc, Jp, lab, 1e-4)
        dcam, _, cs = g.solve(rcs, Jc, Jp)
        assert np.all(cs == 0)
        steps[precision] = dcam
    for k, (A, b_all) in enumerate(systems):
        cams = np.nonzero(lab == k)[0]
        b = b_all[cams].reshape(-1)
        eta0 = _backward_error(A, steps[S.STBA_MIXED_NOREFINE][cams].reshape(-1), b)
        eta1 = _backward_error(A, steps[S.STBA_MIXED][cams].reshape(-1), b)
        print(f"cluster {k} ({len(cams)} cameras): backward error in the FP64 system, unrefined {eta0:.2e}, "
              f"refined {eta1:.2e}", flush=True)
        assert eta1 < max(BOUND, 1e-2 * eta0)
