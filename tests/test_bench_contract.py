"""Host-side checks of the benchmark: it refuses more than one GPU with a
message, and its algorithmic model (the numerator of the roofline fraction)
counts what it says, checked against brute force on a small scene."""
import os
import subprocess
import sys

import numpy as np

import bench
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_algorithmic_model_counts_pairs_and_flops():
    """Segments, same-segment observation pairs, Cholesky flops (N^3/3 + 4 N^2)
    and lower-triangle entries of the model against brute force (alpha = 1: one
    segment per point and cluster)."""
    s = synth.small_ring(m=20, n=400, views=5, seed=2)
    e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
    maps = [synth.sgc_map(e, w, s.m, 6, 10.0, 0, t) for t in range(2)]
    model, stats = bench.algorithmic_model(s, maps, 8)
    off_pairs, segs, flops, entries = [], [], [], []
    for lab in maps:
        p, ns = 0, 0
        for j in range(s.n):
            cams = s.obs_cam[s.obs_pt == j]
            ns += len({int(lab[c]) for c in cams})
            for a in range(cams.shape[0]):
                for b in range(a):
                    p += int(lab[cams[a]] == lab[cams[b]])
        off_pairs.append(p)
        segs.append(ns)
        N = [9 * int((lab == k).sum()) for k in range(lab.max() + 1)]
        flops.append(sum(x ** 3 / 3 + 4 * x ** 2 for x in N))
        entries.append(sum(x * (x + 1) / 2 for x in N))
    assert stats["off_pairs"] == np.mean(off_pairs)
    assert stats["n_seg"] == np.mean(segs)
    assert np.isclose(stats["chol_flops"], np.mean(flops), rtol=1e-12)
    assert np.isclose(stats["S_lower"], np.mean(entries), rtol=1e-12)
    assert np.isclose(model["schur_assembly"]["flops"], 486 * np.mean(off_pairs) + 576 * s.q, rtol=1e-12)
    assert np.isclose(model["schur_assembly"]["bytes"], s.q * 216 + 8 * np.mean(entries), rtol=1e-12)
    assert np.isclose(model["cluster_cholesky"]["flops"], np.mean(flops), rtol=1e-12)
    assert np.isclose(model["point_backsub"]["bytes"], s.q * 48 + 72 * s.m + 24 * s.n + 72 * s.n, rtol=1e-12)
    m4, _ = bench.algorithmic_model(s, maps, 4)
    assert np.isclose(m4["schur_assembly"]["bytes"], s.q * 112 + 8 * np.mean(entries), rtol=1e-12)
    assert "refinement" not in m4
    assert np.isclose(m4["point_backsub"]["bytes"], s.q * 104 + 72 * s.n, rtol=1e-12)
    # STBA_MIXED: the refinement's inputs once, the factor twice; the point
    # update reads ids, pixel and point to form J in FP64
    mr, _ = bench.algorithmic_model(s, maps, 4, refine=True)
    params = 72 * s.m + 24 * s.n
    assert np.isclose(mr["refinement"]["bytes"], 48 * s.q + params + 72 * s.m + 16 * np.mean(entries), rtol=1e-12)
    assert np.isclose(mr["point_backsub"]["bytes"], 48 * s.q + params + 72 * s.n, rtol=1e-12)
