"""Pins of the oracle's preconditioned conjugate gradient (App. A, Table 3: the
inexact solver of the split reduced camera systems) against mathematics that
fixes it: the exact solution, the Krylov-subspace optimality of every iterate
(built here from an explicit basis), one step when the preconditioner is the
matrix, finite termination, and the failure cases."""
import numpy as np
import pytest

import oracle as O
import synth


def _spd(nb, seed, coupling=0.3, bs=9):
    rng = np.random.default_rng(seed)
    n = nb * bs
    G = rng.normal(size=(n, n))
    A = G @ G.T / n + np.eye(n) * 0.5
    # make the camera blocks dominate so block-Jacobi is a sensible preconditioner
    mask = np.kron(np.eye(nb), np.ones((bs, bs)))
    A = A * (mask + coupling * (1 - mask))
    w = np.linalg.eigvalsh(A)
    assert w.min() > 0
    return A, rng.normal(size=n)


def _block_jacobi_apply(S, v, bs=9):
    out = np.empty_like(v)
    for a in range(S.shape[0] // bs):
        sl = slice(a * bs, (a + 1) * bs)
        out[sl] = np.linalg.solve(S[sl, sl], v[sl])
    return out


@pytest.mark.parametrize("nb,seed", [(3, 0), (6, 1), (12, 2)])
def test_pcg_reaches_the_exact_solution(nb, seed):
    S, b = _spd(nb, seed)
    x, it, res, ok = O.pcg(S, b, tol=1e-13, max_iters=10 * S.shape[0])
    xs = np.linalg.solve(S, b)
    assert ok and it <= S.shape[0] + 5
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert res == pytest.approx(np.linalg.norm(b - S @ x) / np.linalg.norm(b), abs=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_every_iterate_minimises_the_energy_error_over_the_krylov_space(k):
    # x_k = argmin over span{M^-1 b, (M^-1 S) M^-1 b, ...} (k vectors) of ||x - x*||_S
    S, b = _spd(6, 7)
    V = [_block_jacobi_apply(S, b)]
    for _ in range(k - 1):
        V.append(_block_jacobi_apply(S, S @ V[-1]))
    V = np.linalg.qr(np.stack(V, axis=1))[0]
    y = np.linalg.solve(V.T @ S @ V, V.T @ b)
    x_ref = V @ y
    x, it, _, ok = O.pcg(S, b, tol=0.0, max_iters=k)
    assert ok and it == k
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


def test_block_diagonal_system_is_solved_in_one_step():
    S, b = _spd(5, 3, coupling=0.0)
    x, it, res, ok = O.pcg(S, b, tol=1e-12, max_iters=50)
    assert ok and it == 1 and res < 1e-12
    assert np.allclose(x, np.linalg.solve(S, b), rtol=1e-12, atol=0)


def test_zero_right_hand_side_and_failures():
    S, b = _spd(3, 4)
    x, it, res, ok = O.pcg(S, np.zeros_like(b), tol=1e-12, max_iters=10)
    assert ok and it == 0 and not x.any()
    bad = S.copy()
    bad[:9, :9] = -np.eye(9)
    assert not O.pcg(bad, b, 1e-12, 50)[3]
    # positive definite camera blocks, indefinite whole: p.q <= 0 is met
    ind = np.kron(np.array([[1.0, 2.0], [2.0, 1.0]]), np.eye(9))
    assert not O.pcg(ind, np.r_[np.ones(9), np.zeros(9)], 1e-12, 50)[3]


def test_pcg_on_a_cluster_system_approaches_the_cholesky_step():
    s = synth.small_ring(m=24, n=1500, views=6, seed=3)
    lab = (np.arange(s.m) * 2 // s.m).astype(np.int64)
    st = O.stba_step(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, lab, 1e-3)
    for Sk, bk, cams in zip(st.S_blocks, st.b_blocks, st.clusters):
        x, it, res, ok = O.pcg(Sk, bk, tol=1e-12, max_iters=2000)
        ref = st.dcam[cams].reshape(-1)
        assert ok and res <= 1e-12
        assert np.linalg.norm(x - ref) <= 1e-6 * np.linalg.norm(ref)
