"""The entry point that allocates nothing (stba_residual_jacobian_static): its
f, J and cost equal stba_residual_jacobian's bit for bit on the same inputs,
over two calls in a row (the second on a smaller problem, so the scratch holds
the first call's partials beyond the second's), in FP64 and FP32, and a problem
beyond its scratch is refused before anything runs."""
import numpy as np
import pytest
import torch

import paper_2008_00446_amd as S
import synth

pytestmark = pytest.mark.gpu


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)


def _outputs(q, T):
    return (torch.empty((q, 2), dtype=T, device="cuda"), torch.empty((q, 18), dtype=T, device="cuda"),
            torch.empty((q, 6), dtype=T, device="cuda"), torch.empty(1, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("precision", [S.STBA_FP64, S.STBA_MIXED])
def test_static_scratch_entry_matches_workspace_entry(precision):
    T = torch.float64 if precision == S.STBA_FP64 else torch.float32
    scenes = [synth.ring(m=200, n=50_000, views=8, seed=0), synth.small_ring(m=40, n=3000, views=8, seed=1)]
    assert scenes[1].q < scenes[0].q
    for s in scenes:
        print(f"precision {precision}: q {s.q}", flush=True)
        cam, pt = _dev(s.cam0, torch.float64), _dev(s.pt0, torch.float64)
        oc, op, uv = _dev(s.obs_cam, torch.int32), _dev(s.obs_pt, torch.int32), _dev(s.obs_uv, torch.float64)
        prob = S.make_problem(cam, pt, oc, op, uv)
        dims = S.stba_analyze(prob)
        dims.gamma_max = 1
        ws = S.alloc_workspace(S.stba_workspace_bytes(prob, dims, precision))
        S.stba_prepare(prob, dims, precision, ws)
        ref = _outputs(s.q, T)
        S.stba_residual_jacobian(prob, dims, precision, *ref, ws)
        got = _outputs(s.q, T)
        S.stba_residual_jacobian_static(prob, precision, *got)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        # residuals only, without the cost
        f_only = torch.empty((s.q, 2), dtype=T, device="cuda")
        S.stba_residual_jacobian_static(prob, precision, f_only, None, None, None)
        torch.cuda.synchronize()
        assert torch.equal(f_only, ref[0])


def test_static_scratch_entry_refuses_a_problem_beyond_its_scratch():
    # q above 2^24 with a cost asked for: refused on the host, nothing enqueued
    # (the arrays are never touched, so small stand-ins suffice)
    idx = torch.zeros(16, dtype=torch.int32, device="cuda")
    prob = S.make_problem(torch.zeros((1, 9), dtype=torch.float64, device="cuda"),
                          torch.zeros((1, 3), dtype=torch.float64, device="cuda"), idx, idx,
                          torch.zeros((16, 2), dtype=torch.float64, device="cuda"))
    prob.q = (1 << 24) + 1
    f = torch.empty(2, dtype=torch.float64, device="cuda")
    cost = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(S.StbaError) as e:
        S.stba_residual_jacobian_static(prob, S.STBA_FP64, f, None, None, cost)
    assert e.value.code == -4   # STBA_EWORKSPACE
