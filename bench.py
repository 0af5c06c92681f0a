"""Benchmark of the STBA hot path on one MI355X.

Headline workload: the SLAM-like scene (5000 cameras along a smooth path at 1 m
spacing, 1M points, geometric track lengths of mean about 6, banded visibility,
about 5.9M observations, 0.7 px noise), sequential camera clusters of U{20..120}
cameras redrawn every LM iteration, lambda0 = 1e-4, alpha = 1, FP64: 20 LM
iterations.  One step = one full LM iteration of STBA (cluster layout,
residuals/Jacobian when x changed, segments and correction, Schur assembly,
cluster Cholesky, point update, candidate cost, accept).  Inputs are resident in
HBM before the timed region; the cluster maps of all timed iterations are drawn
and uploaded beforehand.

Prints ONE JSON line.  `value` is LM iterations per second of the timed FP64 run
(no events inside it); `obs_per_s` is q x iterations/s.  The per-phase split
comes from a second, identical pass with HIP events between the phases on the
library's stream; the residual phase is reported per launch that evaluated the
Jacobian and per launch that only cleared S.  `roofline` describes the phase
with the largest time per iteration, against the algorithmic work of the method
(bytes or flops per launch, the per-unit figures stated in `model`).
`mixed_vs_fp64` runs the same iterations in MIXED precision (FP32 Jacobian and
Schur assembly, FP64 Cholesky and cost) from the same start and maps: the FP64
cost after K iterations is the target, and MIXED is timed until it reaches it
(the time-to-target idea of the performance profiles, Sec. 5.2); the profile at
tau = 0.1, 0.01, 0.001 (F_tau = F* + tau (F0 - F*)) is reported beside it.
`cpu_baseline` times the FP64 oracle on the host on a bounded sample of the
first iteration (whole clusters cut out of the problem, scaled to the full
iteration by observations) and reports the GPU's FP64 and MIXED results on the
same clusters against it.  `secondary` times the 200-camera ring and the
Internet-like workloads; `diff_batch` the 64-problem differentiation batch;
`batched_lm` the same 64 problems through one LM iteration against stepping
them one by one; `ablations` the paper's ablations on the SLAM-like and Internet-like scenes;
`huber`, `pcg` and `sgc` the robust loss, the inexact cluster solve and the
device graph clustering.

--pmc-summary turns rocprofv3 counter CSVs (FETCH_SIZE and WRITE_SIZE runs of
this benchmark and of --copy-calibration) into profiles/pmc_<phase>_<workload>.txt,
the HBM traffic that `roofline.traffic` reports while the sources are unchanged.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from dataclasses import dataclass
from typing import Callable

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def source_hash() -> str:
    csrc = os.path.join(ROOT, "paper_2008_00446_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "stba.h"), "rb").read())
    return h.hexdigest()[:16]


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="LM iterations timed (default: 20 slam, 10 others)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["slam", "ring", "internet"], default="slam")
    ap.add_argument("--precision", choices=["fp64", "mixed", "mixed_norefine"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work in cpu_baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (to scale HBM counters)")
    ap.add_argument("--only-timed", action="store_true",
                    help="only the warm-up and the timed iterations (for profiler runs)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-secondary", action="store_true", help="skip the ring and Internet-like workloads")
    ap.add_argument("--no-huber", action="store_true", help="skip the robust-loss (Huber) leg")
    ap.add_argument("--no-sgc", action="store_true", help="skip the device graph-clustering leg")
    ap.add_argument("--no-ablations", action="store_true", help="skip the synthetic ablations")
    ap.add_argument("--no-pcg", action="store_true", help="skip the inexact (PCG) cluster-solve leg")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay of the timed iterations")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in launch settings instead of measuring them (stba_autotune) first")
    ap.add_argument("--no-diff-batch", action="store_true", help="skip the 64-problem differentiation batch")
    ap.add_argument("--no-batched-lm", action="store_true", help="skip the many-problem LM iteration leg")
    ap.add_argument("--ablation-iters", type=int, default=20)
    ap.add_argument("--pmc-summary", action="store_true",
                    help="write a profiles/pmc_*.txt summary from counter CSVs (no GPU work)")
    ap.add_argument("--phase", default="cluster_cholesky")
    ap.add_argument("--kernels", default="k_chol",
                    help="comma-separated kernel name fragments belonging to --phase")
    ap.add_argument("--fetch-csv")
    ap.add_argument("--write-csv")
    ap.add_argument("--calib-fetch-csv")
    ap.add_argument("--calib-write-csv")
    ap.add_argument("--command", default="", help="the commands that produced the CSVs (recorded)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# workloads: scene, per-iteration cluster maps, cap, lambda0
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    kind: str
    scene: object
    map_of: Callable          # t -> cam_cluster (int32 [m])
    gamma: int
    lam0: float
    steps: int
    maps_desc: str

    @property
    def name(self):
        s = self.scene
        return f"{self.kind}_m{s.m}_n{s.n}_q{s.q}"


def make_workload(kind: str) -> Workload:
    import synth
    if kind == "slam":
        s = synth.slam(seed=0)
        return Workload(kind, s, lambda t: synth.sequential_map(s.m, 20, 120, 0, t), 120, 1e-4, 20,
                        "sequential runs of U{20..120} cameras, redrawn per iteration from Philox(0, t)")
    if kind == "ring":
        s = synth.ring(m=200, n=50_000, views=8, seed=0)
        e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
        return Workload(kind, s, lambda t: synth.sgc_map(e, w, s.m, 50, 10.0, 0, t), 50, 1e-4, 10,
                        "stochastic graph clustering (host harness), cap 50, beta 10, redrawn per iteration")
    if kind == "internet":
        s = synth.internet(seed=0)
        return Workload(kind, s, None, 100, 1e-4, 10,
                        "stochastic graph clustering on the device, cap 100, beta 10, redrawn per iteration")
    raise ValueError(kind)


def draw_maps(S, wl, total):
    """The maps of iterations 0..total-1 (host arrays).  The Internet-like
    workload draws them with the device clustering (its host harness takes
    about a second per map on this graph)."""
    if wl.map_of is not None:
        return [np.asarray(wl.map_of(t), dtype=np.int32) for t in range(total)]
    s = wl.scene
    sol = S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=wl.gamma, precision=S.STBA_FP64)
    out = [sol.sample_clusters(wl.gamma, SGC_BETA, alpha=1.0, seed=0, it=t)._keep[0].cpu().numpy().copy()
           for t in range(total)]
    del sol
    return out


# ---------------------------------------------------------------------------
# HBM counter summaries
# ---------------------------------------------------------------------------

def copy_calibration():
    import torch
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")     # 1 GiB
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8, "launches": 3}))


def _counter_rows(path, counter):
    import csv
    return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in csv.DictReader(open(path))
            if r["Counter_Name"] == counter]


def pmc_summary(args, workload):
    """Average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the phase's kernels,
    scaled by what the same counters read for a copy of known size."""
    frags = [k for k in args.kernels.split(",") if k]

    def named(n, f):
        # f as a whole kernel name (k_schur does not match k_schur_reduce)
        return any(f + t in n for t in ("<", "("))

    def per_step(path, counter):
        rows = [(n, v) for n, v in _counter_rows(path, counter) if any(named(n, f) for f in frags)]
        main = [v for n, v in rows if named(n, frags[0])]
        # dispatches of the first kernel = phase launches; all kernels of the phase summed per launch
        return sum(v for _, v in rows) / max(1, len(main)), len(main)

    def calib(path, counter):
        rows = [v for n, v in _counter_rows(path, counter) if "copyBuffer" in n or "copy" in n.lower()]
        return max(rows)

    fetch_kib, n_f = per_step(args.fetch_csv, "FETCH_SIZE")
    write_kib, n_w = per_step(args.write_csv, "WRITE_SIZE")
    copy_bytes = float(1 << 30)
    cf = copy_bytes / (calib(args.calib_fetch_csv, "FETCH_SIZE"))   # bytes per counted KiB (fetch)
    cw = copy_bytes / (calib(args.calib_write_csv, "WRITE_SIZE"))
    traffic = fetch_kib * cf + write_kib * cw
    path = os.path.join(ROOT, "profiles", f"pmc_{args.phase}_{workload}.txt")
    with open(path, "w") as fh:
        fh.write(f"# HBM traffic of phase {args.phase} (kernels {args.kernels}) on {workload}\n")
        fh.write("# rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, over bench.py; the same counters over\n")
        fh.write("# bench.py --copy-calibration (1 GiB read + 1 GiB written per copy) give the scale.\n")
        fh.write(f"# commands: {args.command}\n")
        fh.write(f"source_hash = {source_hash()}\n")
        fh.write(f"dispatches_fetch = {n_f}\ndispatches_write = {n_w}\n")
        fh.write(f"fetch_kib_per_launch = {fetch_kib:.1f}\nwrite_kib_per_launch = {write_kib:.1f}\n")
        fh.write(f"copy_bytes_per_fetch_kib = {cf:.2f}\ncopy_bytes_per_write_kib = {cw:.2f}\n")
        fh.write(f"traffic_bytes_per_launch = {traffic:.0f}\n")
    print(open(path).read())


def load_traffic(phase: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was
    measured on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_{phase}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# the algorithmic work of each phase
# ---------------------------------------------------------------------------

def algorithmic_model(scene, maps, es, refine=False):
    """Algorithmic bytes / flops per launch of each phase, averaged over `maps`
    (alpha = 1: one segment per point and cluster).  es: bytes per element of
    f, J and the Schur data (8 FP64, 4 MIXED); refine: STBA_MIXED's refinement
    step runs (and the point update takes J in FP64 at x).

    Per unit (the method's own inputs and outputs of each step, not this
    implementation's intermediate records):
      residual_jacobian  24 + 26 es bytes per observation (ids and pixel in,
                         f, J_c, J_p out) + the camera and point rows, per
                         Jacobian evaluation; every launch also clears the
                         padded cluster matrices (8 bytes per entry) and b
      points_segments    8 + 26 es bytes per observation (ids, f, J in) +
                         72 per segment (V_s, w'_s) + 72 per point (V*_j, w_j)
                         + 432 per camera (U, v)
      schur_assembly     8 + 26 es bytes per observation + 8 per entry of the
                         lower triangle of S_k; 576 flop per observation + 486
                         per pair of distinct observations of one segment
      cluster_cholesky   sum_k N_k^3 / 3 + 4 N_k^2 flop (N_k = 9 n_k),
                         16 bytes per lower entry
      refinement         (MIXED) 48 bytes per observation (ids, pixel, point)
                         + the parameters, 72 per camera out, and the factor
                         of S_k twice (forward and backward): 16 per lower entry
      point_backsub      72 per point + 48 per observation (ids, pixel, point:
                         J formed in FP64 at x; FP64 and MIXED) or 8 + 24 es
                         (the FP32 J read; MIXED_NOREFINE)
      candidate_cost     24 bytes per observation + the parameters twice"""
    q, n, m = scene.q, scene.n, scene.m
    acc = {k: [] for k in ("chol_flops", "S_lower", "S_padded", "n_seg", "off_pairs", "clusters")}
    for lab in maps:
        lab = np.asarray(lab)
        sizes = np.bincount(lab)
        N = 9 * sizes.astype(np.float64)
        Np = np.ceil(N / 32.0) * 32.0
        acc["chol_flops"].append(float(np.sum(N ** 3 / 3.0 + 4.0 * N ** 2)))
        acc["S_lower"].append(float(np.sum(N * (N + 1) / 2)))
        acc["S_padded"].append(float(np.sum(Np ** 2)))
        key = scene.obs_pt.astype(np.int64) * (int(lab.max()) + 1) + lab[scene.obs_cam]
        _, c = np.unique(key, return_counts=True)
        acc["n_seg"].append(float(c.size))
        acc["off_pairs"].append(float(np.sum(c * (c - 1) / 2)))
        acc["clusters"].append(float(sizes.size))
    st = {k: float(np.mean(v)) for k, v in acc.items()}
    params = m * 72 + n * 24
    model = {
        "residual_jacobian": dict(bound="hbm", bytes=q * (24 + 26 * es) + params,
                                  clear_bytes=8 * st["S_padded"] + 72 * m),
        "points_segments": dict(bound="hbm", bytes=q * (8 + 26 * es) + 72 * st["n_seg"] + 72 * n + 432 * m,
                                record_bytes=q * 32 * es),
        "schur_assembly": dict(bound="alu", flops=576 * q + 486 * st["off_pairs"],
                               bytes=q * (8 + 26 * es) + 8 * st["S_lower"]),
        "cluster_cholesky": dict(bound="mfma", flops=st["chol_flops"], bytes=16 * st["S_lower"]),
        "point_backsub": dict(bound="hbm", bytes=(q * 48 + params if (refine or es == 8) else q * (8 + 24 * es))
                              + 72 * n),
        "candidate_cost": dict(bound="hbm", bytes=q * 24 + 2 * params),
    }
    if refine:
        model["refinement"] = dict(bound="hbm", bytes=q * 48 + params + 72 * m + 16 * st["S_lower"])
    return model, st


# ---------------------------------------------------------------------------
# running iterations
# ---------------------------------------------------------------------------

def run_iterations(sol, samples, cam0, pt0, lam0, steps, events=None, snapshots=None, jac_flags=None):
    """LM iterations 0..steps-1 from x0 (asynchronous unless jac_flags is given).
    events: per-iteration phase events; snapshots: a device tensor receiving the
    cost after each iteration; jac_flags: a list receiving, per iteration, whether
    it evaluated the Jacobian (reads the state back after every iteration)."""
    import paper_2008_00446_amd as S
    sol.cam.copy_(cam0)
    sol.pt.copy_(pt0)
    S.stba_lm_init(sol.state, lam0, 0.1)
    F_dev = sol.state[16:24].view(sol.cam.dtype)     # stba_lm_state.F
    n_jac = 0
    for t in range(steps):
        sol.step(samples[t], events=None if events is None else events[t])
        if snapshots is not None:
            snapshots[t:t + 1].copy_(F_dev)
        if jac_flags is not None:
            nj = int(sol.read_state()["n_jac"])
            jac_flags.append(nj > n_jac)
            n_jac = nj


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def make_solver(S, wl, precision, **kw):
    s = wl.scene
    return S.StbaSolver(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv, gamma_max=kw.pop("gamma", wl.gamma),
                        precision=precision, lambda0=kw.pop("lam0", wl.lam0), **kw)


def phase_split(S, sol, samples, cam0, pt0, lam0, steps, model):
    """Per-phase times (HIP events between the phases on the library's stream),
    the residual phase split into launches that evaluated the Jacobian and
    launches that only cleared S."""
    import torch
    P = S.STBA_NUM_PHASES
    evs = [S.hip_events(P + 1) for _ in range(steps)]
    jac = []
    run_iterations(sol, samples, cam0, pt0, lam0, steps, events=evs, jac_flags=jac)
    torch.cuda.synchronize()
    ms = np.array([[S.event_ms(ev[k], ev[k + 1]) for k in range(P)] for ev in evs])
    names = [S.stba_phase_name(k) for k in range(P)]
    out = {}
    for k, nm in enumerate(names):
        e = {"ms": round(float(ms[:, k].mean()), 4)}
        mm = model.get(nm)
        if nm == "residual_jacobian":
            jm = ms[np.array(jac), k] if any(jac) else np.array([])
            cm = ms[~np.array(jac), k] if not all(jac) else np.array([])
            e["launches_with_jacobian"] = int(np.sum(jac))
            if jm.size:
                e["ms_with_jacobian"] = round(float(jm.mean()), 4)
                e["GB/s_with_jacobian"] = round((mm["bytes"] + mm["clear_bytes"]) / (jm.mean() * 1e-3) / 1e9, 1)
            if cm.size:
                e["ms_clear_only"] = round(float(cm.mean()), 4)
                e["GB/s_clear_only"] = round(mm["clear_bytes"] / (cm.mean() * 1e-3) / 1e9, 1)
        elif mm is not None:
            sec = ms[:, k].mean() * 1e-3
            if "bytes" in mm:
                e["GB/s"] = round(mm["bytes"] / sec / 1e9, 1)
                e["hbm_frac"] = round(mm["bytes"] / sec / 1e9 / HBM_PEAK_GBS, 4)
            if "flops" in mm:
                e["TFLOP/s"] = round(mm["flops"] / sec / 1e12, 3)
        out[nm] = e
    return out, names, ms, jac


def roofline_of(phases, model, precision_fp64, workload):
    """The phase with the largest time against its bound."""
    dom = max((nm for nm in phases if nm in model and nm != "residual_jacobian"),
              key=lambda nm: phases[nm]["ms"])
    rj = phases.get("residual_jacobian", {})
    if rj.get("ms", 0.0) > phases[dom]["ms"]:
        dom = "residual_jacobian"
    mdl = model[dom]
    if dom == "residual_jacobian":
        dur = rj.get("ms_with_jacobian", rj["ms"]) * 1e-3
        achieved, peak, unit = (mdl["bytes"] + mdl["clear_bytes"]) / dur / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        dur = phases[dom]["ms"] * 1e-3
        if mdl["bound"] == "hbm":
            achieved, peak, unit = mdl["bytes"] / dur / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            achieved = mdl["flops"] / dur / 1e12
            peak = FP64_PEAK_TFLOPS if (precision_fp64 or dom == "cluster_cholesky") else FP32_PEAK_TFLOPS
            unit = "TFLOP/s"
    return {"kernel": dom, "bound": mdl["bound"], "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": load_traffic(dom, workload), "duration_ms": dur * 1e3}


TUNE = True   # measure the launch settings (stba_autotune) on the first map before timing


def tune(sol, sample):
    """stba_autotune on a representative sample (the first map); the choices
    and what was measured, or None when tuning is off."""
    return sol.autotune(sample) if TUNE else None


def timed_run(S, wl, precision, maps, steps, warmup, graph=True):
    """Warm-up, the timed K iterations and (optionally) their HIP-graph replay;
    the launch settings tuned on the first map first (sol.tuning)."""
    import torch
    sol = make_solver(S, wl, precision)
    samples = [sol.sample(maps[t], alpha=1.0, seed=0, it=t) for t in range(len(maps))]
    sol.tuning = tune(sol, samples[0])
    cam0, pt0 = sol.cam.clone(), sol.pt.clone()
    run_iterations(sol, samples, cam0, pt0, wl.lam0, warmup)
    elapsed = timed(lambda: run_iterations(sol, samples, cam0, pt0, wl.lam0, steps))
    st = sol.read_state()
    graph_ips = None
    if graph:
        g = torch.cuda.CUDAGraph()
        run_iterations(sol, samples, cam0, pt0, wl.lam0, 0)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            for t in range(steps):
                sol.step(samples[t])
        run_iterations(sol, samples, cam0, pt0, wl.lam0, 0)
        g.replay()
        run_iterations(sol, samples, cam0, pt0, wl.lam0, 0)
        graph_elapsed = timed(g.replay)
        graph_ips = steps / graph_elapsed
        assert sol.read_state()["F"] == st["F"], "graph replay diverged from the eager iterations"
        del g
    return sol, samples, cam0, pt0, elapsed, st, graph_ips


def main():
    args = parse_args()
    global TUNE
    TUNE = not args.no_tune
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.pmc_summary:
        import synth
        s = {"slam": synth.slam, "ring": lambda: synth.ring(m=200, n=50_000, views=8, seed=0),
             "internet": synth.internet}[args.workload]()
        pmc_summary(args, f"{args.workload}_m{s.m}_n{s.n}_q{s.q}")
        return
    import torch
    import paper_2008_00446_amd as S

    precision = {"fp64": S.STBA_FP64, "mixed": S.STBA_MIXED, "mixed_norefine": S.STBA_MIXED_NOREFINE}[args.precision]
    es = 8 if precision == S.STBA_FP64 else 4
    wl = make_workload(args.workload)
    scene = wl.scene
    steps = args.steps or wl.steps
    mixed_max = 3 * steps
    total = max(steps, args.warmup, mixed_max)
    maps = draw_maps(S, wl, total)
    sol, samples, cam0, pt0, elapsed, st, graph_ips = timed_run(
        S, wl, precision, maps, steps, args.warmup, graph=not (args.no_graph or args.only_timed))
    out = {
        "metric": "STBA LM iterations/s (and observations/s)", "value": steps / elapsed, "unit": "iter/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == S.STBA_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": wl.name, "scene": wl.kind, "cameras": scene.m, "points": scene.n,
                   "observations": scene.q, "maps": wl.maps_desc, "cluster_cap": wl.gamma,
                   "clusters_mean": float(np.mean([mp.max() + 1 for mp in maps[:steps]])), "lambda0": wl.lam0,
                   "alpha": 1.0, "lm_iterations": steps, "precision": args.precision},
        "obs_per_s": scene.q * steps / elapsed,
        "graph_iter_per_s": graph_ips,
        "lm": {"F_final": st["F"], "accepted": st["n_accept"], "jacobian_evals": st["n_jac"],
               "rcs_builds": st["n_rcs"], "lambda_final": st["lambda_"], "status": st["status"]},
        "source_hash": source_hash(),
        "tuning": sol.tuning,
    }
    if args.only_timed:
        print(json.dumps(out))
        return
    model, stats = algorithmic_model(scene, maps[:steps], es, refine=precision == S.STBA_MIXED)
    phases, names, _, _ = phase_split(S, sol, samples, cam0, pt0, wl.lam0, steps, model)
    out["roofline"] = roofline_of(phases, model, precision == S.STBA_FP64, wl.name)
    out["phases"] = phases
    out["model"] = {"per_launch": {k: {kk: vv for kk, vv in v.items()} for k, v in model.items()}, **stats}
    mixed = None
    if not args.no_mixed and precision == S.STBA_FP64:
        mixed = mixed_leg(S, wl, sol, samples, maps, steps, args.warmup, cam0, pt0)
        out["mixed_vs_fp64"] = mixed
    del sol
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(S, wl, maps[0], args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    if not args.no_huber and precision == S.STBA_FP64:
        out["huber"] = huber_leg(S, wl, maps, steps, args.warmup)
    if not args.no_ablations and precision == S.STBA_FP64:
        out["ablations"] = {wl.kind: ablation_leg(S, wl, args.ablation_iters)}
    torch.cuda.empty_cache()
    if not args.no_secondary:
        sec = {}
        for kind in ("ring", "internet"):
            if kind == wl.kind:
                continue
            w2 = make_workload(kind)
            sec[kind] = secondary_leg(S, w2, args.warmup)
            if kind == "internet" and not args.no_ablations:
                out.setdefault("ablations", {})[kind] = ablation_leg(S, w2, args.ablation_iters)
            if kind == "ring":
                if not args.no_pcg:
                    out["pcg"] = pcg_leg(S, w2)
                if not args.no_sgc:
                    out["sgc"] = sgc_leg(S, w2, args.warmup)
            del w2
            torch.cuda.empty_cache()
        out["secondary"] = sec
    if not args.no_diff_batch:
        out["diff_batch"] = diff_batch_leg(S, args)
        torch.cuda.empty_cache()
    if not args.no_batched_lm:
        out["batched_lm"] = batched_lm_leg(S, args)
    print(json.dumps(out))


# ---------------------------------------------------------------------------
# legs
# ---------------------------------------------------------------------------

TAUS = (0.1, 0.01, 0.001)


def mixed_leg(S, wl, sol64, samples64, maps, K, warmup, cam0, pt0):
    """The two mixed-precision modes against FP64 from the same x0 with the same
    maps: STBA_MIXED (FP32 assembly, FP64 factorisation and one FP64 refinement
    step) and STBA_MIXED_NOREFINE (the same without the refinement).  The target
    is the FP64 cost after K iterations; each mode is run until its cost reaches
    it (up to 3K iterations) and the wall times to reach it are compared.  The
    profile at tau = 0.1, 0.01, 0.001 (F_tau = F* + tau (F0 - F*), F* the lowest
    of the costs after K iterations) is reported beside it."""
    import torch
    kmax = 3 * K
    runs = {"fp64": (sol64, samples64)}
    for name, prec in (("mixed", S.STBA_MIXED), ("mixed_norefine", S.STBA_MIXED_NOREFINE)):
        sol = make_solver(S, wl, prec)
        runs[name] = (sol, [sol.sample(maps[t], alpha=1.0, seed=0, it=t) for t in range(kmax)])
        tune(sol, runs[name][1][0])
    hist = {}
    for name, (sol, smp) in runs.items():
        run_iterations(sol, smp, cam0, pt0, wl.lam0, warmup)
        Fs = torch.empty(kmax, dtype=torch.float64, device="cuda")
        run_iterations(sol, smp, cam0, pt0, wl.lam0, kmax, snapshots=Fs)
        hist[name] = Fs.cpu().numpy()
    s = wl.scene
    plan = S.ResidualPlan(s.obs_cam, s.obs_pt, s.m, s.n, precision=S.STBA_FP64)
    uv = torch.as_tensor(s.obs_uv, dtype=torch.float64, device="cuda")
    F0 = float((S.residuals(cam0, pt0, uv, plan) ** 2).sum())
    del plan
    cache = {}

    def seconds(name, n):
        if (name, n) not in cache:
            sol, smp = runs[name]
            cache[(name, n)] = timed(lambda: run_iterations(sol, smp, cam0, pt0, wl.lam0, n))
        return cache[(name, n)]

    def first_at_or_below(name, F):
        hit = np.nonzero(hist[name] <= F)[0]
        return int(hit[0]) + 1 if hit.size else None

    F_target = float(hist["fp64"][K - 1])
    t64 = seconds("fp64", K)
    F_star = float(min(h[K - 1] for h in hist.values()))
    profile = []
    for tau in TAUS:
        F_tau = F_star + tau * (F0 - F_star)
        row = {"tau": tau, "F_tau": F_tau}
        for name in runs:
            n = first_at_or_below(name, F_tau)
            row[f"{name}_iterations"] = n
            row[f"{name}_seconds"] = None if n is None else seconds(name, n)
        for name in ("mixed", "mixed_norefine"):
            row[f"{name}_speedup"] = (row["fp64_seconds"] / row[f"{name}_seconds"]
                                      if row["fp64_seconds"] and row[f"{name}_seconds"] else None)
        profile.append(row)
    variants = {}
    for name in ("mixed", "mixed_norefine"):
        n = first_at_or_below(name, F_target)
        # the same target up to FP64 rounding of the cost sum (1e-9 relative)
        n9 = first_at_or_below(name, F_target * (1.0 + 1e-9))
        tk = seconds(name, K)
        variants[name] = {
            "iterations_to_target": n,
            "seconds_to_target": None if n is None else seconds(name, n),
            "speedup_at_equal_cost_reduction": None if n is None else t64 / seconds(name, n),
            "iterations_to_target_rel_1e-9": n9,
            "speedup_at_target_rel_1e-9": None if n9 is None else t64 / seconds(name, n9),
            "F_after_K": float(hist[name][K - 1]),
            "minus_fp64_F_after_K_rel": float((hist[name][K - 1] - hist["fp64"][K - 1]) / hist["fp64"][K - 1]),
            "iter_per_s": K / tk, "obs_per_s": s.q * K / tk,
        }
    out = {
        "F0": F0, "iterations": K, "F_target": F_target,
        "fp64_seconds_to_target": t64, "fp64_iter_per_s": K / t64, "fp64_F_after_K": float(hist["fp64"][K - 1]),
        # the headline: STBA_MIXED (with its refinement step)
        "speedup_at_equal_cost_reduction": variants["mixed"]["speedup_at_equal_cost_reduction"],
        "variants": variants, "profile_tau": profile,
    }
    for name in ("mixed", "mixed_norefine"):
        del runs[name]
    return out


def _cluster_blocks(ws, rcs, l, ks):
    """Dense symmetric S_k (from the stored lower triangle) of clusters ks."""
    import torch
    torch.cuda.synchronize()
    base = ws.data_ptr()

    def view(ptr, dt, count):
        es = torch.tensor([], dtype=dt).element_size()
        off = int(ptr) - base
        return ws[off:off + count * es].view(dt)

    S_off = view(rcs.S_off, torch.int64, l + 1).cpu().numpy()
    Np = view(rcs.cl_Np, torch.int32, l).cpu().numpy()
    nk = view(rcs.cl_n, torch.int32, l).cpu().numpy()
    Sflat = view(rcs.S, torch.float64, int(S_off[l]))
    out = {}
    for k in ks:
        P, N = int(Np[k]), 9 * int(nk[k])
        A = Sflat[int(S_off[k]):int(S_off[k]) + P * P].cpu().numpy().reshape(P, P).T[:N, :N]
        out[k] = np.tril(A) + np.tril(A, -1).T
    return out


def _gpu_cluster_results(S, wl, precision, lab, ks):
    """One build and solve at x0 with map `lab`: S_k of clusters ks, b, dcam, dpt, F(x0)."""
    import torch
    s = wl.scene
    sol = make_solver(S, wl, precision)
    T = torch.float64 if precision == S.STBA_FP64 else torch.float32
    q, m, n = s.q, s.m, s.n
    f = torch.empty((q, 2), dtype=T, device="cuda")
    Jc = torch.empty((q, 18), dtype=T, device="cuda")
    Jp = torch.empty((q, 6), dtype=T, device="cuda")
    cost = torch.empty(1, dtype=torch.float64, device="cuda")
    S.stba_residual_jacobian(sol.problem, sol.dims, precision, f, Jc, Jp, cost, sol.ws)
    smp = sol.sample(lab, alpha=1.0, seed=0, it=0)
    rcs = S.stba_build_cluster_rcs(sol.problem, sol.dims, smp, S.StbaDamping(wl.lam0, 0.1), precision, f, Jc, Jp,
                                   sol.ws)
    blocks = _cluster_blocks(sol.ws, rcs, smp.l, ks)
    b = (sol.ws[int(rcs.b) - sol.ws.data_ptr():][:72 * m]).view(torch.float64).cpu().numpy().reshape(m, 9)
    dcam = torch.empty((m, 9), dtype=torch.float64, device="cuda")
    dpt = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    cs = torch.empty(smp.l, dtype=torch.int32, device="cuda")
    S.stba_solve_clusters(sol.problem, sol.dims, rcs, precision, Jc, Jp, dcam, dpt, cs, sol.ws)
    torch.cuda.synchronize()
    res = dict(S=blocks, b=b, dcam=dcam.cpu().numpy(), dpt=dpt.cpu().numpy(), F=float(cost.item()),
               status_ok=bool((cs == 0).all().item()))
    del sol, f, Jc, Jp
    torch.cuda.empty_cache()
    return res


def cpu_baseline(S, wl, lab, budget_s):
    """The FP64 oracle on the host for a bounded sample of the first iteration:
    whole clusters of its map cut out of the problem (their cameras and every
    observation of them; below the correction threshold a cluster's system
    depends on nothing else) and run through the oracle's LM iteration, largest,
    smallest and median first and then alternating, until about `budget_s`
    seconds.  The per-iteration time is scaled to the whole problem by
    observations (every observation belongs to exactly one cluster).  The
    GPU's FP64, MIXED and MIXED_NOREFINE results on the same clusters (S_k, b_k, camera steps,
    steps of points seen only inside the cluster) and the cost F(x0) are
    compared with the oracle's."""
    import psutil
    import oracle as O
    import synth
    s = wl.scene
    lab = np.asarray(lab)
    sizes = np.bincount(lab)
    order = np.argsort(sizes, kind="stable")
    pick_order, lo, hi = [], 0, len(order) - 1
    mid = len(order) // 2
    seen = set()
    for k in [order[hi], order[lo], order[mid]] + [order[i] for pair in zip(range(hi - 1, -1, -1), range(lo + 1, hi))
                                                   for i in pair]:
        if int(k) not in seen:
            seen.add(int(k))
            pick_order.append(int(k))
    proc = psutil.Process()
    c0 = proc.cpu_times()
    t_wall, q_done, refs = 0.0, 0, {}
    for k in pick_order:
        cut = synth.cut_cluster(s.obs_cam, s.obs_pt, lab, k)
        args, ids = synth.cut_args(s, cut)
        t0 = time.perf_counter()
        r = O.lm_iteration(*args, wl.lam0, 1.0, 0, 0)
        t_wall += time.perf_counter() - t0
        q_done += cut.obs.size
        refs[k] = (cut, r)
        if t_wall >= budget_s:
            break
    c1 = proc.cpu_times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    per_iter = t_wall * s.q / q_done
    t0 = time.perf_counter()
    F_ref = O.cost(O.residuals(s.cam0, s.pt0, s.obs_cam, s.obs_pt, s.obs_uv))
    t_cost = time.perf_counter() - t0
    # kappa(D^-1 S_k D^-1) of the sampled systems: FP64 rounding of S_k moves a
    # step by up to about kappa 1e-16, FP32 assembly by up to about kappa 6e-8
    kap = []
    for k, (cut, r) in refs.items():
        Sk = r.step.S_blocks[0]
        d = np.sqrt(np.diag(Sk))
        kap.append(float(np.linalg.cond(Sk / np.outer(d, d))))
    errors = {"kappa_scaled_max": max(kap), "kappa_scaled_median": float(np.median(kap))}
    for name, prec in (("fp64", S.STBA_FP64), ("mixed", S.STBA_MIXED), ("mixed_norefine", S.STBA_MIXED_NOREFINE)):
        g = _gpu_cluster_results(S, wl, prec, lab, list(refs))
        e = {"S_maxabs_rel": 0.0, "b_rel": 0.0, "dcam_rel": 0.0, "dpt_interior_rel": 0.0,
             "F_x0_rel": abs(g["F"] - F_ref) / F_ref, "status_ok": g["status_ok"]}
        for k, (cut, r) in refs.items():
            st = r.step
            Sk = g["S"][k]
            e["S_maxabs_rel"] = max(e["S_maxabs_rel"], float(np.max(np.abs(Sk - st.S_blocks[0])) /
                                                              np.max(np.abs(st.S_blocks[0]))))
            e["b_rel"] = max(e["b_rel"], _rel(g["b"][cut.cams].ravel(), st.b_blocks[0]))
            e["dcam_rel"] = max(e["dcam_rel"], _rel(g["dcam"][cut.cams], st.dcam))
            if cut.interior.size:
                e["dpt_interior_rel"] = max(e["dpt_interior_rel"],
                                            _rel(g["dpt"][cut.pts[cut.interior]], st.dpt[cut.interior]))
        errors[name] = e
    return {"value": 1.0 / per_iter, "unit": "iter/s", "cores": int(round(max(1.0, cpu / max(t_wall, 1e-9)))),
            "kind": "oracle",
            "sample": (f"first LM iteration, {len(refs)} of {sizes.size} clusters cut out whole "
                       f"({q_done} of {s.q} observations), FP64 NumPy/SciPy, {t_wall:.1f} s wall, "
                       f"{cpu:.1f} s CPU, scaled to the whole iteration by observations; host cpus "
                       f"{len(os.sched_getaffinity(0))}"),
            "oracle_cost_x0_s": t_cost,
            "gpu_vs_oracle_on_sample": errors}


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def secondary_leg(S, wl, warmup):
    """A secondary workload: FP64, MIXED and MIXED_NOREFINE iterations/s (eager and graph replay)."""
    import torch
    K = wl.steps
    maps = draw_maps(S, wl, max(K, warmup))
    out = {"workload": wl.name, "iterations": K, "maps": wl.maps_desc, "cluster_cap": wl.gamma,
           "clusters_mean": float(np.mean([mp.max() + 1 for mp in maps[:K]]))}
    for name, prec in (("fp64", S.STBA_FP64), ("mixed", S.STBA_MIXED), ("mixed_norefine", S.STBA_MIXED_NOREFINE)):
        sol, _, _, _, el, st, gips = timed_run(S, wl, prec, maps, K, warmup, graph=True)
        out[name] = {"iter_per_s": K / el, "obs_per_s": wl.scene.q * K / el, "graph_iter_per_s": gips,
                     "F_after_K": st["F"], "accepted": st["n_accept"], "status": st["status"],
                     "tuning": sol.tuning}
        del sol
        torch.cuda.empty_cache()
    return out


HUBER_SCALE = 0.5   # the experiments' robust loss (Sec. 5.1)


def huber_leg(S, wl, maps, K, warmup):
    """The same K FP64 iterations under the Huber loss of scale 0.5 (IRLS)."""
    solh = make_solver(S, wl, S.STBA_FP64, huber=HUBER_SCALE)
    samples = [solh.sample(maps[t], alpha=1.0, seed=0, it=t) for t in range(max(K, warmup))]
    cam0, pt0 = solh.cam.clone(), solh.pt.clone()
    run_iterations(solh, samples, cam0, pt0, wl.lam0, warmup)
    t = timed(lambda: run_iterations(solh, samples, cam0, pt0, wl.lam0, K))
    st = solh.read_state()
    return {"scale": HUBER_SCALE, "iter_per_s": K / t, "obs_per_s": wl.scene.q * K / t,
            "F_after_K": st["F"], "accepted": st["n_accept"], "status": st["status"]}


def diff_batch_leg(S, args):
    """The differentiation batch: 64 ring problems (m ~ U{30..120}, n ~ U{5k..30k},
    7 views per point, seeds 0-63) concatenated with index offsets into one
    problem; one forward (residuals, stba_residual_jacobian without J) and one
    backward (stba_residual_vjp of v = 2 f, the gradient of sum ||f||^2 with the
    Jacobian recomputed) per pass, in FP32, timed over K passes.  Algorithmic
    bytes per pass: forward ids, pixel and f (24 + 2 es per observation),
    backward ids, v and the pixel gradient (8 + 4 es per observation), plus the
    gathered and reduced camera and point rows.  The same with the Jacobian
    stored: the forward pass also writes J and the backward pass reads it
    (stba_residual_vjp_stored), 48 es more per observation."""
    import torch
    import synth
    batch = synth.diff_batch(seeds=range(64))
    cam = np.vstack([b.cam0 for b in batch])
    pt = np.vstack([b.pt0 for b in batch])
    co = np.cumsum([0] + [b.m for b in batch])
    po = np.cumsum([0] + [b.n for b in batch])
    oc = np.concatenate([b.obs_cam + co[i] for i, b in enumerate(batch)]).astype(np.int32)
    op = np.concatenate([b.obs_pt + po[i] for i, b in enumerate(batch)]).astype(np.int32)
    uv = np.vstack([b.obs_uv for b in batch])
    m, n, q = cam.shape[0], pt.shape[0], oc.shape[0]
    plan = S.ResidualPlan(oc, op, m, n, S.STBA_MIXED)
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt)  # noqa: E731
    tc, tp, tu = dev(cam, torch.float64), dev(pt, torch.float64), dev(uv, torch.float64)
    prob = plan.problem(tc, tp, tu)
    f = torch.empty((q, 2), dtype=torch.float32, device="cuda")
    v = torch.empty_like(f)
    gc = torch.empty((m, 9), dtype=torch.float32, device="cuda")
    gp = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    gu = torch.empty((q, 2), dtype=torch.float32, device="cuda")

    Jc = torch.empty((q, 18), dtype=torch.float32, device="cuda")
    Jp = torch.empty((q, 6), dtype=torch.float32, device="cuda")

    def one():
        S.stba_residual_jacobian(prob, plan.dims, S.STBA_MIXED, f, None, None, None, plan.ws)
        torch.mul(f, 2.0, out=v)
        S.stba_residual_vjp(prob, plan.dims, S.STBA_MIXED, v, gc, gp, gu, plan.ws)

    def one_stored():
        # J kept from the forward pass (24 values per observation) and read back
        S.stba_residual_jacobian(prob, plan.dims, S.STBA_MIXED, f, Jc, Jp, None, plan.ws)
        torch.mul(f, 2.0, out=v)
        S.stba_residual_vjp_stored(prob, plan.dims, S.STBA_MIXED, v, Jc, Jp, gc, gp, gu, plan.ws)

    K = 20
    es = 4
    algo = q * ((24 + 2 * es) + (8 + 4 * es) + 2 * es) + (m * 72 + n * 24) + (m * 9 + n * 3) * es
    algo_st = algo + q * 2 * 24 * es   # the blocks written forward and read back
    res = {"problems": len(batch), "observations": q, "cameras": m, "points": n, "passes": K}
    for name, fn, a in (("recompute", one, algo), ("stored", one_stored, algo_st)):
        for _ in range(args.warmup):
            fn()
        dt = timed(lambda: [fn() for _ in range(K)])
        leg = {"us_per_fwd_bwd": 1e6 * dt / K, "GB_per_s_algorithmic": a * K / dt / 1e9,
               "hbm_frac": a * K / dt / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_pass": a}
        if name == "recompute":
            res.update(leg)
        else:
            res["stored_jacobian"] = leg
    return res


def batched_lm_leg(S, args, P=64, K=10):
    """Many problems through one LM iteration (stba_lm_step_batched): the 64
    ring problems of the differentiation batch (m_b ~ U{30..120}, n_b ~
    U{5k..30k}, 7 views per point), cameras perturbed, each with its own map of
    runs of U{10..40} cameras per iteration and its own damping and accept
    decisions; FP64, K iterations of the whole batch against the same K
    iterations taken problem by problem with stba_lm_step."""
    import torch
    import synth
    scenes = synth.diff_batch(seeds=range(P))
    probs = []
    for b, s in enumerate(scenes):
        rng = np.random.default_rng(100 + b)
        cam = s.cam0.copy()
        cam[:, :6] += rng.normal(0.0, 1e-3, size=(s.m, 6))
        probs.append((cam, s.pt0.copy(), s.obs_cam, s.obs_pt, s.obs_uv))
    gamma = 40
    maps = [[synth.sequential_map(s.m, 10, gamma, b, t) for b, s in enumerate(scenes)] for t in range(K)]
    bs = S.BatchSolver(probs, gamma, precision=S.STBA_FP64, lambda0=1e-3)
    samples = [bs.sample(maps[t], alpha=1.0, seed=0, it=t) for t in range(K)]
    cam0, pt0, st0 = bs.cam.clone(), bs.pt.clone(), bs.states.clone()

    def batch_run(n):
        bs.cam.copy_(cam0)
        bs.pt.copy_(pt0)
        bs.states.copy_(st0)
        for t in range(n):
            bs.step(samples[t])

    batch_run(min(args.warmup, K))
    t_batch = timed(lambda: batch_run(K))
    got = bs.read_states()
    sols = [S.StbaSolver(*pr, min(gamma, s.m), precision=S.STBA_FP64, lambda0=1e-3) for pr, s in zip(probs, scenes)]
    one = [[sol.sample(maps[t][b], alpha=1.0, seed=0, it=t) for t in range(K)] for b, sol in enumerate(sols)]
    c0 = [(sol.cam.clone(), sol.pt.clone()) for sol in sols]

    def single_run(n):
        for b, sol in enumerate(sols):
            sol.cam.copy_(c0[b][0])
            sol.pt.copy_(c0[b][1])
            S.stba_lm_init(sol.state, 1e-3, 0.1)
            for t in range(n):
                sol.step(one[b][t])

    single_run(min(args.warmup, K))
    t_single = timed(lambda: single_run(K))
    ref = [sol.read_state() for sol in sols]
    same = all(g["n_accept"] == r["n_accept"] and g["lambda_"] == r["lambda_"] for g, r in zip(got, ref))
    q = sum(s.q for s in scenes)
    return {"problems": P, "observations": q, "cameras": sum(s.m for s in scenes), "iterations": K,
            "batch_iter_per_s": K / t_batch, "problem_iter_per_s": P * K / t_batch,
            "obs_per_s": q * K / t_batch, "one_by_one_problem_iter_per_s": P * K / t_single,
            "speedup_over_one_by_one": t_single / t_batch, "same_decisions_as_one_by_one": bool(same),
            "accepted_total": int(sum(g["n_accept"] for g in got))}


SGC_BETA = 10.0   # the clustering's scale beta


def sgc_leg(S, wl, warmup):
    """Maps drawn on the device by stochastic graph clustering (Sec. 4.4, Eq. 16):
    the clustering kernel alone (K maps back to back, HIP events on the stream it
    runs on), then K FP64 LM iterations each preceded by its own device map (the
    number of clusters read back before each step), against the host harness's
    time per map on the same camera graph; then the same K iterations with the
    number of clusters left on the device (no read-back), eager and as one
    captured HIP graph, whose final state must equal the eager one's."""
    import torch
    import synth
    s = wl.scene
    sol = make_solver(S, wl, S.STBA_FP64)
    K = wl.steps
    cc = torch.empty(s.m, dtype=torch.int32, device="cuda")
    out = torch.zeros(2, dtype=torch.int32, device="cuda")

    def draw(t):
        S.stba_sample_clusters(sol.problem, sol.dims, sol.precision, sol.ws, wl.gamma, SGC_BETA, 0, t, cc,
                               out[0:1], out[1:2])

    for t in range(warmup):
        draw(t)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for t in range(K):
        draw(t)
    e1.record(stream)
    torch.cuda.synchronize()
    kernel_ms = e0.elapsed_time(e1) / K
    cam0, pt0 = sol.cam.clone(), sol.pt.clone()

    def reset():
        sol.cam.copy_(cam0)
        sol.pt.copy_(pt0)
        S.stba_lm_init(sol.state, wl.lam0, 0.1)

    def iterations(steps):
        reset()
        ls = []
        for t in range(steps):
            smp = sol.sample_clusters(wl.gamma, SGC_BETA, alpha=1.0, seed=0, it=t)
            ls.append(smp.l)
            sol.step(smp)
        return ls

    def device_iterations(steps):
        # the number of clusters stays on the device: nothing is read back
        for t in range(steps):
            sol.step(sol.sample_clusters_device(wl.gamma, SGC_BETA, alpha=1.0, seed=0, it=t))

    iterations(warmup)
    ls = []
    t_iter = timed(lambda: ls.extend(iterations(K)))
    st = sol.read_state()
    reset()
    device_iterations(warmup)
    reset()
    t_dev = timed(lambda: device_iterations(K))
    st_dev = sol.read_state()
    g = torch.cuda.CUDAGraph()
    reset()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        device_iterations(K)
    reset()
    g.replay()
    torch.cuda.synchronize()
    st_cap = sol.read_state()
    reset()
    t_cap = timed(g.replay)
    del g
    e, w = synth.camera_graph(s.obs_cam, s.obs_pt, s.m)
    t0 = time.perf_counter()
    n_host = 3
    for t in range(n_host):
        synth.sgc_map(e, w, s.m, wl.gamma, SGC_BETA, 0, t)
    host_ms = 1e3 * (time.perf_counter() - t0) / n_host
    # the captured iterations replay the eager device-count ones bit for bit; the
    # host-count run factors with the tile form (the device count takes the team
    # form), so it agrees to rounding only
    same = all(st_cap[k] == st_dev[k] for k in ("F", "lambda_", "accepted", "status"))
    return {"workload": wl.name, "beta": SGC_BETA, "cap": wl.gamma, "kernel_ms_per_map": kernel_ms,
            "iter_per_s_with_device_maps": K / t_iter, "iter_per_s_device_count": K / t_dev,
            "iter_per_s_captured_device_maps": K / t_cap, "captured_equals_eager": bool(same),
            "device_count_minus_host_count_F_rel": float((st_dev["F"] - st["F"]) / st["F"]),
            "clusters_mean": float(np.mean(ls)), "F_after_K": st["F"], "status": st["status"],
            "host_harness_ms_per_map": host_ms}


PCG_TOLS = (1e-4, 1e-6, 1e-10)


def pcg_leg(S, wl):
    """The inexact cluster solve (App. A, Table 3) against the Cholesky solve on
    the first iteration's cluster systems: for each tolerance the time of
    stba_solve_clusters_pcg (conjugate gradient, camera-block Jacobi, then the
    point step), the largest iteration count over the clusters and the camera
    step's distance from the Cholesky one; the Cholesky solve's time beside it.
    Each solve is timed with events on its stream after a fresh assembly."""
    import torch
    s = wl.scene
    K = wl.steps
    maps = draw_maps(S, wl, K)
    sol = make_solver(S, wl, S.STBA_FP64)
    m, n, q = s.m, s.n, s.q
    f = torch.empty((q, 2), dtype=torch.float64, device="cuda")
    Jc = torch.empty((q, 18), dtype=torch.float64, device="cuda")
    Jp = torch.empty((q, 6), dtype=torch.float64, device="cuda")
    S.stba_residual_jacobian(sol.problem, sol.dims, sol.precision, f, Jc, Jp, None, sol.ws)
    smp = sol.sample(maps[0], alpha=1.0, seed=0, it=0)
    l = smp.l
    dcam = torch.empty((m, 9), dtype=torch.float64, device="cuda")
    dpt = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    cs = torch.empty(l, dtype=torch.int32, device="cuda")
    its = torch.empty(l, dtype=torch.int32, device="cuda")
    res = torch.empty(l, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def timed_solve(fn, reps=3):
        ms = []
        for _ in range(reps):
            rcs = S.stba_build_cluster_rcs(sol.problem, sol.dims, smp, S.StbaDamping(wl.lam0, 0.1), sol.precision,
                                           f, Jc, Jp, sol.ws)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn(rcs)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    chol_ms = timed_solve(lambda rcs: S.stba_solve_clusters(sol.problem, sol.dims, rcs, sol.precision, Jc, Jp,
                                                            dcam, dpt, cs, sol.ws))
    ref = dcam.cpu().numpy()
    out = {"workload": wl.name, "clusters": l, "cholesky_ms": chol_ms, "tolerances": {}}
    for tol in PCG_TOLS:
        ms = timed_solve(lambda rcs: S.stba_solve_clusters_pcg(sol.problem, sol.dims, rcs, sol.precision, Jc, Jp,
                                                               dcam, dpt, 5000, tol, its, res, cs, sol.ws))
        x = dcam.cpu().numpy()
        out["tolerances"][f"{tol:g}"] = {
            "ms": ms, "iterations_max": int(its.max().item()), "iterations_mean": float(its.double().mean().item()),
            "step_rel_diff_vs_cholesky": float(np.linalg.norm(x - ref) / np.linalg.norm(ref)),
            "status_ok": bool((cs == 0).all().item())}
    cam0, pt0 = sol.cam.clone(), sol.pt.clone()
    samples = [sol.sample(maps[t], alpha=1.0, seed=0, it=t) for t in range(K)]

    def lm(pcg):
        sol.cam.copy_(cam0)
        sol.pt.copy_(pt0)
        S.stba_lm_init(sol.state, wl.lam0, 0.1)
        for t in range(K):
            sol.step(samples[t], pcg=pcg)

    lm(None)
    F_chol = sol.read_state()["F"]
    dt = timed(lambda: lm((5000, 1e-6)))
    st = sol.read_state()
    out["lm_tol_1e-6"] = {"iter_per_s": K / dt, "F_after_K": st["F"], "F_after_K_cholesky": F_chol,
                          "accepted": st["n_accept"], "status": st["status"]}
    return out


def ablation_leg(S, wl, K):
    """Synthetic versions of the paper's ablations, each K FP64 LM iterations
    from the same start, maps redrawn per iteration unless fixed (SLAM-like:
    sequential runs; otherwise the device graph clustering, beta 10):
    - correction (Sec. 5.4): lambda kept >= 0.1 (lambda0 0.1), STBA (correction
      whenever lambda >= 0.1, so at every iteration) against STBA* (none);
    - fixed clustering (Sec. 5.2): STBA against STBA-fixed (the first map at every
      iteration), lambda0 1e-4;
    - cluster cap (App. B): Gamma in {1, 25, 50, 100, cap} (sequential runs of
      exactly Gamma cameras on the SLAM-like scene), final costs normalised by
      the smallest, as the paper's figure does.
    Each entry gives the cost after every iteration and the iteration rate."""
    import synth
    s = wl.scene
    seq = wl.kind == "slam"

    def run(gamma, lam0, lam_corr=0.1, lam_min=0.0, fixed=False):
        sol = make_solver(S, wl, S.STBA_FP64, gamma=gamma, lam0=lam0, lambda_corr=lam_corr, lambda_min=lam_min)
        Fs, ls, first = [], [], None
        t0 = time.perf_counter()
        for t in range(K):
            if first is None or not fixed:
                if seq:
                    lo = 20 if gamma == wl.gamma else gamma
                    smp = sol.sample(synth.sequential_map(s.m, lo, gamma, 0, 0 if fixed else t), 1.0, 0, t)
                else:
                    smp = sol.sample_clusters(gamma, SGC_BETA, alpha=1.0, seed=0, it=t)
                first = first or smp
            use = first if fixed else smp
            if fixed:
                use = S.make_sample(first._keep[0], first.l, 1.0, 0, t)
            sol.step(use)
            st = sol.read_state()
            Fs.append(float(st["F"]))
            ls.append(use.l)
        dt = time.perf_counter() - t0
        del sol
        return {"F": [float(f"{f:.7g}") for f in Fs], "F_final": Fs[-1], "clusters_mean": float(np.mean(ls)),
                "iter_per_s": K / dt, "status": int(st["status"])}

    out = {"workload": wl.name, "iterations": K}
    stba, star = run(wl.gamma, 0.1, 0.1, 0.1), run(wl.gamma, 0.1, float("inf"), 0.1)
    out["correction"] = {"lambda_min": 0.1, "stba": stba, "stba_star": star,
                         "final_ratio_star_over_stba": star["F_final"] / stba["F_final"]}
    redrawn, fixed = run(wl.gamma, wl.lam0), run(wl.gamma, wl.lam0, fixed=True)
    out["fixed_clustering"] = {"stba": redrawn, "stba_fixed": fixed,
                               "final_ratio_fixed_over_stba": fixed["F_final"] / redrawn["F_final"]}
    caps = {}
    for g in (1, 25, 50, 100, wl.gamma if seq else 200):
        caps[str(g)] = run(g, wl.lam0)
    best = min(c["F_final"] for c in caps.values())
    for c in caps.values():
        c["normalized_final"] = c["F_final"] / best
        del c["F"]
    out["cluster_cap"] = caps
    return out


if __name__ == "__main__":
    main()
