"""Cluster solves against the matrices they solve (no oracle needed): every
cluster's camera step satisfies the assembled system S_k dc_k = b_k (Eq. 13)
to FP64 rounding, whatever precision assembled S_k.  On the 200-camera ring
with Gamma = 50 (5 clusters of up to 50 cameras, 13-15 tile rows) this runs the
tile-parallel factorisation, its substitution chains and, for MIXED, the FP64
refinement step in the same launch."""
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
# here, u = 1.1e-16); the refinement step of MIXED only lowers it.
BOUND = 1e-13


@pytest.mark.parametrize("precision", [S.STBA_FP64, S.STBA_MIXED])
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
