"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and bench.py.

This package only *makes inputs*: camera rigs, 3-D points, visibility, noisy pixel
observations, per-iteration camera->cluster maps, and cut-outs of one cluster's
cameras and observations (indexing only).  It holds none of the bundle
adjustment arithmetic (no residual, Jacobian, Schur complement, solve or LM logic),
and it imports neither the oracle nor the HIP library.
"""
from .scenes import Scene, tiny_circle, ring, internet, slam, diff_batch, small_ring
from .clusters import camera_graph, sgc_map, sequential_map, halves_map, relabel
from .cluster_cut import ClusterCut, cut_cluster, cut_args

__all__ = [
    "Scene", "tiny_circle", "ring", "internet", "slam", "diff_batch", "small_ring",
    "camera_graph", "sgc_map", "sequential_map", "halves_map", "relabel",
    "ClusterCut", "cut_cluster", "cut_args",
]
