"""Pins of the oracle's robust loss (Sec. 5.1: Huber, scale 0.5, applied by
IRLS reweighting): closed-form values, continuity of rho and rho' at the
threshold, rho' against finite differences of rho, the IRLS gradient against
finite differences of the robust cost, the squared loss as the large-scale
limit, and descent of an accepted step."""
import numpy as np
import pytest

import oracle as O
import synth


def _outlier_scene(seed=3, frac=0.05, sigma=20.0):
    s = synth.tiny_circle()
    rng = np.random.default_rng(seed)
    uv = s.obs_uv.copy()
    idx = rng.choice(s.q, size=int(frac * s.q), replace=False)
    uv[idx] += rng.normal(0.0, sigma, size=(idx.size, 2))
    return s, uv


def test_huber_closed_form_values():
    a = 0.5
    s = np.array([0.0, 0.1, 0.25, 1.0, 4.0])
    # s <= a^2: s; above: 2 a sqrt(s) - a^2
    np.testing.assert_array_equal(O.huber_rho(s, a), [0.0, 0.1, 0.25, 0.75, 1.75])
    np.testing.assert_array_equal(O.huber_weight(s, a), [1.0, 1.0, 1.0, 0.5, 0.25])
    # a = 0 is the squared loss
    np.testing.assert_array_equal(O.huber_rho(s, 0.0), s)
    np.testing.assert_array_equal(O.huber_weight(s, 0.0), np.ones_like(s))


@pytest.mark.parametrize("a", [0.5, 2.0])
def test_huber_rho_and_its_derivative_are_continuous(a):
    t = a * a
    eps = 1e-9 * t
    lo, hi = O.huber_rho(t - eps, a), O.huber_rho(t + eps, a)
    assert abs(float(hi - lo)) < 3 * eps
    assert abs(float(O.huber_weight(t - eps, a) - O.huber_weight(t + eps, a))) < 1e-8


@pytest.mark.parametrize("a", [0.5, 2.0])
def test_huber_weight_is_the_derivative_of_rho(a):
    s = np.array([0.01, 0.2, 0.9, 3.0, 50.0, 1e4]) * a * a
    h = 1e-6 * s
    fd = (O.huber_rho(s + h, a) - O.huber_rho(s - h, a)) / (2 * h)
    np.testing.assert_allclose(O.huber_weight(s, a), fd, rtol=1e-7)


def test_irls_gradient_matches_finite_differences_of_robust_cost():
    """2 J~^T f~ = 2 sum_o rho'(s_o) J_o^T f_o is the gradient of F = sum rho(s)."""
    s, uv = _outlier_scene()
    a = 0.5
    f = O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, uv)
    Jc, Jp = O.jacobian(s.cam0, s.pt0, s.obs_cam, s.obs_pt)
    ft, Jct, Jpt = O.irls(f, Jc, Jp, a)
    gc, gp, _ = O.jtv(Jct, Jpt, s.obs_cam, s.obs_pt, s.m, s.n, ft)
    gc, gp = 2 * gc, 2 * gp
    rng = np.random.default_rng(0)
    for _ in range(12):
        if rng.random() < 0.5:
            i, k = rng.integers(s.m), rng.integers(9)
            h = 1e-6 * max(1.0, abs(s.cam0[i, k]))
            cp, cm = s.cam0.copy(), s.cam0.copy()
            cp[i, k] += h
            cm[i, k] -= h
            Fp = O.robust_cost(O.residuals(cp, s.pt0, s.obs_cam, s.obs_pt, uv), a)
            Fm = O.robust_cost(O.residuals(cm, s.pt0, s.obs_cam, s.obs_pt, uv), a)
            g = gc[i, k]
        else:
            j, k = rng.integers(s.n), rng.integers(3)
            h = 1e-6
            pp, pm = s.pt0.copy(), s.pt0.copy()
            pp[j, k] += h
            pm[j, k] -= h
            Fp = O.robust_cost(O.residuals(s.cam0, pp, s.obs_cam, s.obs_pt, uv), a)
            Fm = O.robust_cost(O.residuals(s.cam0, pm, s.obs_cam, s.obs_pt, uv), a)
            g = gp[j, k]
        fd = (Fp - Fm) / (2 * h)
        assert abs(fd - g) <= 1e-5 * max(1.0, abs(g)), (fd, g)


def test_large_scale_reduces_to_the_squared_loss():
    s, uv = _outlier_scene()
    lab = synth.halves_map(16)
    big = 1e6   # above every residual: every weight is exactly 1
    a = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, uv, lab, 1e-3, 1.0, 0, 0, huber=big)
    b = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, uv, lab, 1e-3, 1.0, 0, 0)
    np.testing.assert_array_equal(a.dcam, b.dcam)
    np.testing.assert_array_equal(a.dpt, b.dpt)
    f = O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, uv)
    assert O.robust_cost(f, big) == pytest.approx(O.cost(f), rel=1e-14)


def test_robust_step_lowers_the_robust_cost():
    s, uv = _outlier_scene()
    lab = synth.halves_map(16)
    F0 = O.robust_cost(O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, uv), 0.5)
    r = O.lm_iteration(s.cam0, s.pt0, s.obs_cam, s.obs_pt, uv, lab, 1e-3, huber=0.5)
    assert r.accepted and r.F_new < F0
    assert r.F_new == O.robust_cost(O.residuals(r.cam, r.pt, s.obs_cam, s.obs_pt, uv), 0.5)
