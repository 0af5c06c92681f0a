"""Pins of the oracle's constraint draw (Sec. 4.2: theta_i with Prob(theta_i = 1) >= alpha).

numpy.random.Philox is an independent Philox4x64-10; it increments its counter
before producing a block, so the block for counter c comes out of a generator
whose counter was set to c - 1."""
import numpy as np
import pytest

import oracle as O
import synth


def _numpy_block(counter, key):
    c = [int(x) for x in counter]
    prev = list(c)
    for i in range(4):                      # c - 1 with borrow
        if prev[i] > 0:
            prev[i] -= 1
            break
        prev[i] = (1 << 64) - 1
    bg = np.random.Philox(counter=np.array(prev, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


def test_philox_bit_equal_to_numpy():
    rng = np.random.default_rng(5)
    cases = [([1, 0, 0, 0], [0, 0]), ([0, 1, 0, 0], [7, 0]), ([2**64 - 1, 3, 0, 9], [1, 2])]
    for _ in range(30):
        cases.append((rng.integers(0, 2**63, 4, dtype=np.uint64).tolist(),
                      rng.integers(0, 2**63, 2, dtype=np.uint64).tolist()))
    for ctr, key in cases:
        ours = O.philox4x64_10([ctr], key)[0]
        assert np.array_equal(ours, _numpy_block(ctr, key)), (ctr, key)


def test_link_draw_uses_counter_t_point_camera():
    u = O.link_draws(seed=11, t=3, point=[5, 6], camera=[2, 9])
    for k, (j, i) in enumerate([(5, 2), (6, 9)]):
        ref = _numpy_block([3, j, i, 0], [11, 0])[0] >> np.uint64(11)
        assert u[k] == ref


def test_keep_threshold_edges():
    assert O.keep_threshold(1.0) == 2 ** 53
    assert O.keep_threshold(0.5) == 2 ** 52
    with pytest.raises(ValueError):
        O.keep_threshold(0.0)


@pytest.mark.parametrize("alpha", [0.3, 0.7, 1.0])
def test_kept_fraction_within_binomial_band(alpha):
    s = synth.small_ring(m=30, n=3000, views=8, seed=2)
    lab = synth.halves_map(s.m, 3)
    _, _, _, kept, links, cross = O.segments(s.obs_cam, s.obs_pt, lab, alpha, seed=4, t=1)
    r = int((~cross).sum())
    k = kept.shape[0]
    if alpha == 1.0:
        assert k == r
    else:
        sd = np.sqrt(r * alpha * (1 - alpha))
        assert abs(k - alpha * r) < 5 * sd


def test_alpha_one_segments_are_point_cluster_pairs():
    s = synth.small_ring(m=20, n=500, views=6, seed=3)
    lab = synth.halves_map(s.m, 4)
    seg, n_seg, seg_point, _, _, _ = O.segments(s.obs_cam, s.obs_pt, lab, 1.0, 0, 0)
    key = s.obs_pt.astype(np.int64) * 10 + lab[s.obs_cam]
    _, inv = np.unique(key, return_inverse=True)
    # same partition: bijection between segment ids and (point, cluster) ids
    pairs = set(zip(seg.tolist(), inv.reshape(-1).tolist()))
    assert len(pairs) == n_seg == len(np.unique(inv))
    assert np.all(seg_point[seg] == s.obs_pt)
