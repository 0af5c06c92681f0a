"""ctypes binding of libstba.so: the C ABI in include/stba.h under the same names.

Argument marshalling only: every call passes device pointers (torch CUDA/HIP
tensors' data_ptr()) and the current HIP stream to the library.  There is no
fallback: if the shared library is missing or a call fails, an exception is
raised.
"""
from __future__ import annotations

import ctypes
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libstba.so")

STBA_FP64 = 0
STBA_MIXED = 1
STBA_MIXED_NOREFINE = 2
STBA_CHOL_AUTO, STBA_CHOL_TILES, STBA_CHOL_TEAM, STBA_CHOL_WORKGROUP = 0, 1, 2, 3
STBA_TUNE_SCHUR_CANDIDATES = 6
STBA_NUM_PHASES = 10
STATUS_NAMES = {0: "STBA_OK", -1: "STBA_EINVAL", -2: "STBA_ENOTPD", -3: "STBA_ENONFINITE",
                -4: "STBA_EWORKSPACE", -5: "STBA_EHIP", -6: "STBA_EDATA"}


class StbaError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} returned {code} ({STATUS_NAMES.get(code, '?')})")
        self.code = code


class StbaProblem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("q", ctypes.c_int64),
                ("cam", ctypes.c_void_p), ("pt", ctypes.c_void_p), ("obs_cam", ctypes.c_void_p),
                ("obs_pt", ctypes.c_void_p), ("obs_uv", ctypes.c_void_p), ("huber", ctypes.c_double)]


class StbaDims(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("max_track", ctypes.c_int32), ("gamma_max", ctypes.c_int32),
                ("chol_form", ctypes.c_int32), ("schur_blocks", ctypes.c_int32)]


class StbaTuneReport(ctypes.Structure):
    _fields_ = [("chol_form", ctypes.c_int32), ("schur_blocks", ctypes.c_int32), ("chol_ms", ctypes.c_float * 4),
                ("schur_candidates", ctypes.c_int32 * STBA_TUNE_SCHUR_CANDIDATES),
                ("schur_ms", ctypes.c_float * STBA_TUNE_SCHUR_CANDIDATES)]


class StbaSample(ctypes.Structure):
    _fields_ = [("cam_cluster", ctypes.c_void_p), ("l", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("seed", ctypes.c_uint64), ("iter", ctypes.c_uint64),
                ("l_dev", ctypes.c_void_p)]


class StbaDamping(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("lambda_corr", ctypes.c_double)]


class StbaLmState(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("lambda_corr", ctypes.c_double), ("F", ctypes.c_double),
                ("F_new", ctypes.c_double), ("accepted", ctypes.c_int32), ("status", ctypes.c_int32),
                ("need_jac", ctypes.c_int32), ("have_F", ctypes.c_int32), ("last_status", ctypes.c_int32),
                ("pad0", ctypes.c_int32), ("n_jac", ctypes.c_int64), ("n_rcs", ctypes.c_int64),
                ("n_accept", ctypes.c_int64), ("lambda_min", ctypes.c_double)]


class StbaRcs(ctypes.Structure):
    _fields_ = [("S", ctypes.c_void_p), ("S_off", ctypes.c_void_p), ("cl_n", ctypes.c_void_p),
                ("cl_Np", ctypes.c_void_p), ("cl_start", ctypes.c_void_p), ("cl_cams", ctypes.c_void_p),
                ("cam_local", ctypes.c_void_p), ("b", ctypes.c_void_p), ("seg_head", ctypes.c_void_p),
                ("l", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("l_dev", ctypes.c_void_p)]


_P = ctypes.c_void_p
_SIGS = {
    "stba_version": (ctypes.c_char_p, []),
    "stba_phase_name": (ctypes.c_char_p, [ctypes.c_int]),
    "stba_analyze_scratch_bytes": (ctypes.c_size_t, []),
    "stba_analyze": (ctypes.c_int, [_P, _P, _P, _P]),
    "stba_workspace_bytes": (ctypes.c_size_t, [_P, _P, ctypes.c_int]),
    "stba_prepare": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, ctypes.c_size_t, _P]),
    "stba_residual_jacobian": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "stba_residual_jacobian_static": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, _P]),
    "stba_build_cluster_rcs": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, _P, _P, _P, _P, _P,
                                              ctypes.c_size_t, _P]),
    "stba_solve_clusters": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "stba_solve_clusters_pcg": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, _P, _P, _P, ctypes.c_int32,
                                               ctypes.c_double, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "stba_sample_clusters": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, ctypes.c_size_t, ctypes.c_int32,
                                            ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, _P, _P, _P, _P]),
    "stba_lm_init": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, _P]),
    "stba_lm_step": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, _P, ctypes.c_size_t, _P]),
    "stba_lm_step_batched": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, _P, _P, _P, ctypes.c_int, _P,
                                            ctypes.c_size_t, _P]),
    "stba_lm_step_pcg": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, ctypes.c_int32, ctypes.c_double, _P,
                                        ctypes.c_size_t, _P]),
    "stba_lm_step_profiled": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, _P, ctypes.c_size_t, _P, _P]),
    "stba_residual_vjp": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "stba_residual_vjp_stored": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "stba_autotune": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, _P, ctypes.c_size_t, _P, _P]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libstba.so (built by paper_2008_00446_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libstba.so not found at {path}; build it with `python -m paper_2008_00446_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(fn, rc):
    if rc != 0:
        raise StbaError(fn, rc)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("STBA calls take device tensors")
    if not t.is_contiguous():
        raise ValueError("STBA calls take contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ref(struct):
    return ctypes.byref(struct)


# ---------------------------------------------------------------------------
# argument structs from tensors
# ---------------------------------------------------------------------------

def make_problem(cam, pt, obs_cam, obs_pt, obs_uv, huber=0.0) -> StbaProblem:
    """stba_problem from device tensors: cam [m,9] f64, pt [n,3] f64, obs_cam/obs_pt [q] int32, obs_uv [q,2] f64;
    huber: the robust loss scale (0: squared loss)."""
    assert cam.dtype == torch.float64 and pt.dtype == torch.float64 and obs_uv.dtype == torch.float64
    assert obs_cam.dtype == torch.int32 and obs_pt.dtype == torch.int32
    assert cam.shape[1] == 9 and pt.shape[1] == 3 and obs_uv.shape[1] == 2
    p = StbaProblem(cam.shape[0], pt.shape[0], obs_cam.shape[0], _ptr(cam), _ptr(pt), _ptr(obs_cam),
                    _ptr(obs_pt), _ptr(obs_uv), float(huber))
    p._keep = (cam, pt, obs_cam, obs_pt, obs_uv)
    return p


def make_sample(cam_cluster, l, alpha=1.0, seed=0, it=0, l_dev=None) -> StbaSample:
    """l_dev (device int32 tensor of one element, optional): the number of clusters on the
    device; l is then an upper bound."""
    assert cam_cluster.dtype == torch.int32
    assert l_dev is None or (l_dev.dtype == torch.int32 and l_dev.numel() >= 1)
    s = StbaSample(_ptr(cam_cluster), int(l), 0, float(alpha), int(seed), int(it), _ptr(l_dev))
    s._keep = (cam_cluster, l_dev)
    return s


# ---------------------------------------------------------------------------
# the ABI under its own names
# ---------------------------------------------------------------------------

def stba_version() -> str:
    return load_library().stba_version().decode()


def stba_phase_name(k: int) -> str:
    return load_library().stba_phase_name(k).decode()


def stba_analyze_scratch_bytes() -> int:
    return int(load_library().stba_analyze_scratch_bytes())


def stba_analyze(problem: StbaProblem, stream=None) -> StbaDims:
    lib = load_library()
    scratch = torch.empty(stba_analyze_scratch_bytes(), dtype=torch.uint8, device="cuda")
    dims = StbaDims(0, 0, 0)
    _check("stba_analyze", lib.stba_analyze(_ref(problem), _ptr(scratch), _ref(dims), _stream(stream)))
    return dims


def stba_workspace_bytes(problem: StbaProblem, dims: StbaDims, precision: int) -> int:
    n = load_library().stba_workspace_bytes(_ref(problem), _ref(dims), precision)
    if n == 0:
        raise StbaError("stba_workspace_bytes", -1)
    return int(n)


def alloc_workspace(nbytes: int) -> torch.Tensor:
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def stba_prepare(problem, dims, precision, ws, stream=None):
    _check("stba_prepare", load_library().stba_prepare(_ref(problem), _ref(dims), precision, _ptr(ws),
                                                       ws.numel(), _stream(stream)))


def stba_residual_jacobian(problem, dims, precision, f, Jc, Jp, cost, ws, stream=None):
    _check("stba_residual_jacobian", load_library().stba_residual_jacobian(
        _ref(problem), _ref(dims), precision, _ptr(f), _ptr(Jc), _ptr(Jp), _ptr(cost), _ptr(ws), ws.numel(),
        _stream(stream)))


def stba_residual_jacobian_static(problem, precision, f, Jc, Jp, cost, stream=None):
    """stba_residual_jacobian without a workspace (the library's own scratch, no allocation)."""
    _check("stba_residual_jacobian_static", load_library().stba_residual_jacobian_static(
        _ref(problem), precision, _ptr(f), _ptr(Jc), _ptr(Jp), _ptr(cost), _stream(stream)))


def stba_build_cluster_rcs(problem, dims, sample, damping, precision, f, Jc, Jp, ws, stream=None) -> StbaRcs:
    out = StbaRcs()
    _check("stba_build_cluster_rcs", load_library().stba_build_cluster_rcs(
        _ref(problem), _ref(dims), _ref(sample), _ref(damping), precision, _ptr(f), _ptr(Jc), _ptr(Jp),
        _ref(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def stba_autotune(problem, dims, sample, damping, precision, ws, stream=None) -> dict:
    """Fill dims.chol_form and dims.schur_blocks with the fastest settings for this
    problem and sample (synchronises); returns what was measured."""
    rep = StbaTuneReport()
    _check("stba_autotune", load_library().stba_autotune(
        _ref(problem), _ref(dims), _ref(sample), _ref(damping), precision, _ptr(ws), ws.numel(), _stream(stream),
        _ref(rep)))
    names = {STBA_CHOL_TILES: "tiles", STBA_CHOL_TEAM: "team", STBA_CHOL_WORKGROUP: "workgroup"}
    return {"chol_form": names.get(rep.chol_form, "auto"), "schur_blocks": int(rep.schur_blocks),
            "chol_ms": {names[f]: float(rep.chol_ms[f - 1]) for f in names if rep.chol_ms[f - 1] > 0},
            "schur_ms": {int(rep.schur_candidates[i]): float(rep.schur_ms[i])
                         for i in range(STBA_TUNE_SCHUR_CANDIDATES)}}


def stba_solve_clusters(problem, dims, rcs, precision, Jc, Jp, dcam, dpt, cluster_status, ws, stream=None):
    _check("stba_solve_clusters", load_library().stba_solve_clusters(
        _ref(problem), _ref(dims), _ref(rcs), precision, _ptr(Jc), _ptr(Jp), _ptr(dcam), _ptr(dpt),
        _ptr(cluster_status), _ptr(ws), ws.numel(), _stream(stream)))


def stba_solve_clusters_pcg(problem, dims, rcs, precision, Jc, Jp, dcam, dpt, max_iters, tol, cluster_iters,
                            cluster_resid, cluster_status, ws, stream=None):
    """Cluster solves by block-Jacobi preconditioned conjugate gradient, then the point step."""
    _check("stba_solve_clusters_pcg", load_library().stba_solve_clusters_pcg(
        _ref(problem), _ref(dims), _ref(rcs), precision, _ptr(Jc), _ptr(Jp), _ptr(dcam), _ptr(dpt), int(max_iters),
        float(tol), _ptr(cluster_iters), _ptr(cluster_resid), _ptr(cluster_status), _ptr(ws), ws.numel(),
        _stream(stream)))


def stba_sample_clusters(problem, dims, precision, ws, gamma, beta, seed, it, cam_cluster, n_clusters, status,
                         stream=None):
    """Device stochastic graph clustering; cam_cluster [m], n_clusters [1], status [1] int32 tensors."""
    _check("stba_sample_clusters", load_library().stba_sample_clusters(
        _ref(problem), _ref(dims), precision, _ptr(ws), ws.numel(), int(gamma), float(beta), int(seed), int(it),
        _ptr(cam_cluster), _ptr(n_clusters), _ptr(status), _stream(stream)))


def stba_lm_init(state, lambda0, lambda_corr=0.1, stream=None):
    _check("stba_lm_init", load_library().stba_lm_init(_ptr(state), float(lambda0), float(lambda_corr),
                                                       _stream(stream)))


def stba_lm_step(problem, dims, sample, state, precision, ws, stream=None):
    _check("stba_lm_step", load_library().stba_lm_step(_ref(problem), _ref(dims), _ref(sample), _ptr(state),
                                                       precision, _ptr(ws), ws.numel(), _stream(stream)))


def stba_lm_step_batched(problem, dims, sample, states, n_prob, prob_cam, prob_pt, prob_obs_off, precision, ws,
                         stream=None):
    """states: n_prob stba_lm_state structs back to back in one device tensor."""
    _check("stba_lm_step_batched", load_library().stba_lm_step_batched(
        _ref(problem), _ref(dims), _ref(sample), _ptr(states), int(n_prob), _ptr(prob_cam), _ptr(prob_pt),
        _ptr(prob_obs_off), precision, _ptr(ws), ws.numel(), _stream(stream)))


def stba_lm_step_pcg(problem, dims, sample, state, precision, max_iters, tol, ws, stream=None):
    _check("stba_lm_step_pcg", load_library().stba_lm_step_pcg(
        _ref(problem), _ref(dims), _ref(sample), _ptr(state), precision, int(max_iters), float(tol), _ptr(ws),
        ws.numel(), _stream(stream)))


def stba_lm_step_profiled(problem, dims, sample, state, precision, ws, events, stream=None):
    """events: a ctypes array of STBA_NUM_PHASES + 1 hipEvent_t handles."""
    _check("stba_lm_step_profiled", load_library().stba_lm_step_profiled(
        _ref(problem), _ref(dims), _ref(sample), _ptr(state), precision, _ptr(ws), ws.numel(),
        _stream(stream), ctypes.cast(events, ctypes.c_void_p)))


def stba_residual_vjp(problem, dims, precision, v, grad_cam, grad_pt, grad_uv, ws, stream=None):
    _check("stba_residual_vjp", load_library().stba_residual_vjp(
        _ref(problem), _ref(dims), precision, _ptr(v), _ptr(grad_cam), _ptr(grad_pt), _ptr(grad_uv), _ptr(ws),
        ws.numel(), _stream(stream)))


def stba_residual_vjp_stored(problem, dims, precision, v, Jc, Jp, grad_cam, grad_pt, grad_uv, ws, stream=None):
    _check("stba_residual_vjp_stored", load_library().stba_residual_vjp_stored(
        _ref(problem), _ref(dims), precision, _ptr(v), _ptr(Jc), _ptr(Jp), _ptr(grad_cam), _ptr(grad_pt),
        _ptr(grad_uv), _ptr(ws), ws.numel(), _stream(stream)))


def read_state(state: torch.Tensor) -> dict:
    """Copy a device stba_lm_state to the host (synchronising) as a dict."""
    raw = state.cpu().numpy().tobytes()
    s = StbaLmState.from_buffer_copy(raw[:ctypes.sizeof(StbaLmState)])
    return {name: getattr(s, name) for name, _ in StbaLmState._fields_ if not name.startswith("pad")}


def set_lambda_min(state: torch.Tensor, value: float) -> None:
    """Write stba_lm_state.lambda_min in place (a host-to-device copy on the current stream)."""
    off = StbaLmState.lambda_min.offset
    state[off:off + 8].copy_(torch.tensor([float(value)], dtype=torch.float64).view(torch.uint8))


def new_state(device="cuda") -> torch.Tensor:
    return torch.zeros(ctypes.sizeof(StbaLmState), dtype=torch.uint8, device=device)


def new_states(count, device="cuda") -> torch.Tensor:
    """count device stba_lm_state structs back to back ([count, size] bytes)."""
    return torch.zeros((count, ctypes.sizeof(StbaLmState)), dtype=torch.uint8, device=device)
