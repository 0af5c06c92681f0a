"""Cutting one cluster's observations out of a problem, for checks of large
problems one cluster at a time.  Indexing only: no arithmetic of the method.

Without the correction of Sec. 4.3 (lambda below its threshold) a cluster's
system S_k, b_k (Eq. 13) depends only on the observations of its cameras: the
virtual points of the cluster are chains of those observations (Sec. 4.2), which
are consecutive in (cluster, camera) order.  The cut-out renumbers cameras and
points in increasing order and keeps their original numbers for the draw."""
from dataclasses import dataclass

import numpy as np


@dataclass
class ClusterCut:
    cams: np.ndarray        # original camera numbers, ascending (the order of S_k)
    pts: np.ndarray         # original point numbers, ascending
    obs: np.ndarray         # original observation indices (ascending)
    obs_cam: np.ndarray     # renumbered
    obs_pt: np.ndarray      # renumbered
    interior: np.ndarray    # renumbered points whose observations all lie in the cluster


def cut_cluster(obs_cam, obs_pt, cam_cluster, k):
    obs_cam = np.asarray(obs_cam)
    obs_pt = np.asarray(obs_pt)
    cams = np.flatnonzero(np.asarray(cam_cluster) == k)
    obs = np.flatnonzero(np.isin(obs_cam, cams))
    pts, pt_local = np.unique(obs_pt[obs], return_inverse=True)
    cam_local = np.searchsorted(cams, obs_cam[obs])
    total = np.bincount(obs_pt, minlength=int(obs_pt.max()) + 1)[pts]
    inside = np.bincount(pt_local, minlength=pts.shape[0])
    return ClusterCut(cams, pts, obs, cam_local, pt_local, np.flatnonzero(inside == total))


def cut_args(scene, cut):
    """Arguments of the oracle's step for the cut-out: cameras, points,
    observations, a one-cluster map and the draw numbers."""
    return (scene.cam0[cut.cams], scene.pt0[cut.pts], cut.obs_cam, cut.obs_pt, scene.obs_uv[cut.obs],
            np.zeros(cut.cams.shape[0], dtype=np.int64)), (scene.obs_pt[cut.obs], scene.obs_cam[cut.obs])
