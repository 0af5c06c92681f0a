"""Pins of the oracle's camera model, residuals, Jacobian and gradient (Sec. 3).

Nothing here compares the oracle with itself: rotations against scipy, residuals
against the generator's independent matrix-form camera, derivatives against
complex-step and central differences of the oracle's own residual function."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
import synth


def test_rotation_matches_scipy_and_is_orthonormal():
    rng = np.random.default_rng(0)
    om = rng.normal(size=(200, 3)) * rng.uniform(0, 3, (200, 1))
    om[:4] = [[0, 0, 0], [1e-9, 0, 0], [0, 1e-5, -1e-5], [np.pi - 1e-3, 0, 0]]
    R = O.rotation_matrix(om)
    ref = Rotation.from_rotvec(om).as_matrix()
    assert np.max(np.abs(R - ref)) < 1e-14
    assert np.max(np.abs(R @ np.swapaxes(R, 1, 2) - np.eye(3))) < 1e-14
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-14)


@pytest.mark.parametrize("maker", [synth.tiny_circle, lambda: synth.small_ring(m=12, n=400)])
def test_zero_residual_at_ground_truth(maker):
    s = maker()
    f = O.residuals(s.cam_gt, s.pt_gt, s.obs_cam, s.obs_pt, s.obs_uv_clean)
    scale = np.max(np.abs(s.obs_uv_clean))
    assert np.max(np.abs(f)) < 1e-12 * scale
    # the noisy observations differ by the injected pixel noise only
    fn = O.residuals(s.cam_gt, s.pt_gt, s.obs_cam, s.obs_pt, s.obs_uv)
    assert 0.5 < np.std(fn) < 1.5


def _tiny_with_rotations(theta):
    s = synth.small_ring(m=5, n=30, views=3, seed=4)
    cam = s.cam0.copy()
    if theta is not None:
        d = np.array([0.3, -0.5, 0.81])
        cam[:, 0:3] = theta * d / np.linalg.norm(d)
        cam[:, 3:6] = [0.0, 0.0, 30.0]
    return s, cam


@pytest.mark.parametrize("theta", [None, 0.0, 1e-9, 1e-5])
def test_jacobian_matches_complex_step(theta):
    s, cam = _tiny_with_rotations(theta)
    pt = s.pt0
    Jc, Jp = O.jacobian(cam, pt, s.obs_cam, s.obs_pt)
    h = 1e-30
    for k in range(9):
        cc = cam.astype(complex)
        cc[:, k] += 1j * h
        d = O.residuals(cc, pt.astype(complex), s.obs_cam, s.obs_pt, s.obs_uv).imag / h
        assert np.max(np.abs(d - Jc[:, :, k])) <= 1e-13 * max(1.0, np.max(np.abs(Jc[:, :, k])))
    for k in range(3):
        pc = pt.astype(complex)
        pc[:, k] += 1j * h
        d = O.residuals(cam.astype(complex), pc, s.obs_cam, s.obs_pt, s.obs_uv).imag / h
        assert np.max(np.abs(d - Jp[:, :, k])) <= 1e-13 * max(1.0, np.max(np.abs(Jp[:, :, k])))


def test_jacobian_matches_central_differences():
    s, cam = _tiny_with_rotations(None)
    Jc, Jp = O.jacobian(cam, s.pt0, s.obs_cam, s.obs_pt)
    for k in range(9):
        h = 1e-6 * max(1.0, np.max(np.abs(cam[:, k])))
        cp, cm = cam.copy(), cam.copy()
        cp[:, k] += h
        cm[:, k] -= h
        d = (O.residuals(cp, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)
             - O.residuals(cm, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv)) / (2 * h)
        assert np.max(np.abs(d - Jc[:, :, k])) <= 1e-6 * max(1.0, np.max(np.abs(Jc[:, :, k])))


def test_gradient_matches_central_differences_of_cost():
    s = synth.small_ring(m=6, n=40, views=4, seed=9)
    args = (s.obs_cam, s.obs_pt)
    gc, gp, guv = O.gradient(s.cam0, s.pt0, *args, s.obs_uv)

    def F(c, p, uv):
        return O.cost(O.residuals(c, p, *args, uv))

    h = 1e-4
    rng = np.random.default_rng(1)
    for _ in range(20):
        i, k = rng.integers(0, s.m), rng.integers(0, 9)
        cp, cm = s.cam0.copy(), s.cam0.copy()
        cp[i, k] += h
        cm[i, k] -= h
        fd = (F(cp, s.pt0, s.obs_uv) - F(cm, s.pt0, s.obs_uv)) / (2 * h)
        assert abs(fd - gc[i, k]) <= 1e-5 * max(1.0, abs(gc[i, k]))
        j, d = rng.integers(0, s.n), rng.integers(0, 3)
        pp, pm = s.pt0.copy(), s.pt0.copy()
        pp[j, d] += h
        pm[j, d] -= h
        fd = (F(s.cam0, pp, s.obs_uv) - F(s.cam0, pm, s.obs_uv)) / (2 * h)
        assert abs(fd - gp[j, d]) <= 1e-5 * max(1.0, abs(gp[j, d]))
        o, a = rng.integers(0, s.q), rng.integers(0, 2)
        up, um = s.obs_uv.copy(), s.obs_uv.copy()
        up[o, a] += h
        um[o, a] -= h
        fd = (F(s.cam0, s.pt0, up) - F(s.cam0, s.pt0, um)) / (2 * h)
        assert abs(fd - guv[o, a]) <= 1e-6 * max(1.0, abs(guv[o, a]))
