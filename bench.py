"""Benchmark of the STBA hot path on one MI355X.

Workload (default): the 200-camera ring scene (3 rings around a 20 x 20 x 5 box,
50k points, 8 views per point, q = 400k observations, 1 px noise), camera
clusters of at most 50 from stochastic graph clustering redrawn every LM
iteration, lambda0 = 1e-4, alpha = 1, FP64: 10 LM iterations.  One step = one
full LM iteration of STBA (cluster layout, residuals/Jacobian when x changed,
segments and correction, Schur assembly, cluster Cholesky, point update,
candidate cost, accept).  Inputs are resident in HBM before the timed region;
the cluster maps of all timed iterations are drawn and uploaded beforehand.

Prints ONE JSON line.  `value` is LM iterations per second of the timed FP64
run (no events inside it); `obs_per_s` is q x iterations/s.  The per-phase
split comes from a second, identical pass with HIP events between the phases on
the library's stream.  `roofline` describes the phase with the largest time per
iteration.  `mixed_vs_fp64` runs the same iterations in MIXED precision (FP32
Jacobian and Schur assembly, FP64 Cholesky with one refinement step and FP64
cost) from the same start and maps and compares the two at equal cost
reduction as the performance profiles of Sec. 5.2 do: the time each needs to
reach F_tau = F* + tau (F0 - F*) for tau = 0.1, 0.01, 0.001 (F* the lower of
their costs after K iterations); the headline speedup is the one at 0.001.
`huber` runs the same iterations under the robust loss (Sec. 5.1).  `pcg` times the inexact
cluster solve (App. A) against the Cholesky one.  `ablations`
repeats the paper's ablations on this scene (correction, Sec. 5.4; fixed
clustering, Sec. 5.2; cluster cap, App. B).  `sgc` draws
the maps on the device instead (stochastic graph clustering, Sec. 4.4): the
clustering kernel's time per map and the iteration rate with a device map drawn
before every step.  `cpu_baseline` times the FP64 oracle on the host for the
first iterations of the same run.

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
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--gamma", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2, help="oracle iterations timed for cpu_baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (to scale HBM counters)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-huber", action="store_true", help="skip the robust-loss (Huber) leg")
    ap.add_argument("--no-sgc", action="store_true", help="skip the device graph-clustering leg")
    ap.add_argument("--no-ablations", action="store_true", help="skip the synthetic ablations")
    ap.add_argument("--no-pcg", action="store_true", help="skip the inexact (PCG) cluster-solve leg")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay of the timed iterations")
    ap.add_argument("--diff-batch", action="store_true",
                    help="also time residuals + J^T v on the 64-problem differentiation batch (FP32)")
    ap.add_argument("--ablation-iters", type=int, default=20)
    ap.add_argument("--pmc-summary", action="store_true",
                    help="write a profiles/pmc_*.txt summary from counter CSVs (no GPU work)")
    ap.add_argument("--phase", default="cluster_cholesky")
    ap.add_argument("--kernels", default="k_chol_tiles",
                    help="comma-separated kernel name fragments belonging to --phase")
    ap.add_argument("--fetch-csv")
    ap.add_argument("--write-csv")
    ap.add_argument("--calib-fetch-csv")
    ap.add_argument("--calib-write-csv")
    ap.add_argument("--command", default="", help="the commands that produced the CSVs (recorded)")
    return ap.parse_args()


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

    def per_step(path, counter):
        rows = [(n, v) for n, v in _counter_rows(path, counter) if any(f in n for f in frags)]
        main = [v for n, v in rows if frags[0] in n]
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
        fh.write(f"# rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, over bench.py; the same counters over\n")
        fh.write(f"# bench.py --copy-calibration (1 GiB read + 1 GiB written per copy) give the scale.\n")
        fh.write(f"# commands: {args.command}\n")
        fh.write(f"source_hash = {source_hash()}\n")
        fh.write(f"dispatches_fetch = {n_f}\ndispatches_write = {n_w}\n")
        fh.write(f"fetch_kib_per_launch = {fetch_kib:.1f}\nwrite_kib_per_launch = {write_kib:.1f}\n")
        fh.write(f"copy_bytes_per_fetch_kib = {cf:.2f}\ncopy_bytes_per_write_kib = {cw:.2f}\n")
        fh.write(f"traffic_bytes_per_launch = {traffic:.0f}\n")
    print(open(path).read())


def algorithmic_model(scene, maps, es):
    """Algorithmic bytes / flops per launch of each phase (averaged over `maps`).

    es: bytes per element of f/J/Schur data (8 FP64, 4 mixed)."""
    q, n, m = scene.q, scene.n, scene.m
    counts = np.bincount(scene.obs_pt, minlength=n)
    chol_flops, schur_pairs, S_entries = [], [], []
    for lab in maps:
        sizes = np.bincount(lab)
        N = 9 * sizes.astype(np.float64)
        chol_flops.append(float(np.sum(N ** 3 / 3.0 + 2.0 * N ** 2)))
        S_entries.append(float(np.sum(N * (N + 1) / 2)))
        # same-cluster observation pairs of each point (alpha = 1: one segment per point and cluster)
        key = scene.obs_pt.astype(np.int64) * (lab.max() + 1) + lab[scene.obs_cam]
        _, c = np.unique(key, return_counts=True)
        schur_pairs.append(float(np.sum(c * (c + 1) / 2)))
    chol_flops, schur_pairs, S_entries = map(np.mean, (chol_flops, schur_pairs, S_entries))
    diag_pairs = float(q)
    off_pairs = schur_pairs - diag_pairs
    model = {
        # reads ids (8) + uv (16) + gathered cam/pt; writes f, Jc, Jp (26 elements)
        "residual_jacobian": dict(bound="hbm", bytes=q * (24 + 26 * es) + m * 72 + n * 24),
        # reads f, Jp, Jc (26 el.) + ids; writes segment record (32 el.) + head; point blocks (72 B)
        "points_segments": dict(bound="hbm", bytes=q * (26 * es + 32 * es + 12) + n * (72 + 16)),
        # zero the lower-triangle storage of S (counted as written once)
        "fill_S": dict(bound="hbm", bytes=8 * S_entries),
        # 486 flop per off-diagonal pair (Y_u Y_w^T), 400 per diagonal pair; each record read once
        "schur_assembly": dict(bound="alu", flops=486 * off_pairs + 400 * diag_pairs,
                               bytes=q * (32 + 18) * es + 8 * S_entries + 8 * schur_pairs),
        "cluster_cholesky": dict(bound="mfma", flops=chol_flops, bytes=8 * 2 * S_entries),
        # reads Jc, Jp (24 el.) + dc gathers; point blocks (72 B); writes dp
        "point_backsub": dict(bound="hbm", bytes=q * (24 * es + 4) + n * (72 + 24 + 16)),
        # reads ids, uv, gathered x and dx
        "candidate_cost": dict(bound="hbm", bytes=q * 24 + (m * 72 + n * 24) * 2),
    }
    return model, dict(chol_flops=chol_flops, schur_pairs=schur_pairs, S_lower_entries=S_entries,
                       counts_mean=float(counts.mean()))


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was
    measured on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}.txt")
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


def cpu_baseline(scene, maps, lam0, iters):
    import psutil
    import oracle as O
    proc = psutil.Process()
    cam, pt, lam = scene.cam0.copy(), scene.pt0.copy(), lam0
    F = O.cost(O.residuals(cam, pt, scene.obs_cam, scene.obs_pt, scene.obs_uv))
    c0 = proc.cpu_times()
    t0 = time.perf_counter()
    for t in range(iters):
        r = O.lm_iteration(cam, pt, scene.obs_cam, scene.obs_pt, scene.obs_uv, maps[t], lam, 1.0, 0, t, F=F)
        cam, pt, lam, F = r.cam, r.pt, r.lam, r.F
    wall = time.perf_counter() - t0
    c1 = proc.cpu_times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas = 1
    return {"value": iters / wall, "unit": "iter/s", "cores": int(round(max(1.0, cpu / wall))),
            "kind": "oracle",
            "sample": f"first {iters} LM iterations of the same workload, same maps and seeds "
                      f"(FP64 NumPy/SciPy, {wall:.1f} s wall, {cpu:.1f} s CPU; BLAS threads available {blas}, "
                      f"host cpus {len(os.sched_getaffinity(0))})",
            "F_after": F}


def run_iterations(sol, samples, cam0, pt0, lam0, steps, events=None, snapshots=None):
    """LM iterations 0..steps-1 from x0 (asynchronous).  events: per-iteration
    phase events; snapshots: a device tensor receiving the cost after each
    iteration."""
    import paper_2008_00446_amd as S
    sol.cam.copy_(cam0)
    sol.pt.copy_(pt0)
    S.stba_lm_init(sol.state, lam0, 0.1)
    F_dev = sol.state[16:24].view(sol.cam.dtype)     # stba_lm_state.F
    for t in range(steps):
        sol.step(samples[t], events=None if events is None else events[t])
        if snapshots is not None:
            snapshots[t:t + 1].copy_(F_dev)


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.pmc_summary:
        pmc_summary(args, "ring_m200_n50000_q400000")
        return
    import torch
    import paper_2008_00446_amd as S
    import synth

    precision = S.STBA_FP64 if args.precision == "fp64" else S.STBA_MIXED
    es = 8 if precision == S.STBA_FP64 else 4
    scene = synth.ring(m=200, n=50_000, views=8, seed=0)
    workload = f"ring_m{scene.m}_n{scene.n}_q{scene.q}"
    e, w = synth.camera_graph(scene.obs_cam, scene.obs_pt, scene.m)
    mixed_max = 3 * args.steps
    total = max(args.steps, args.warmup, args.cpu_iters, mixed_max)
    maps = [synth.sgc_map(e, w, scene.m, args.gamma, 10.0, 0, t) for t in range(total)]
    lam0 = 1e-4
    sol = S.StbaSolver(scene.cam0, scene.pt0, scene.obs_cam, scene.obs_pt, scene.obs_uv,
                       gamma_max=args.gamma, precision=precision, lambda0=lam0)
    samples = [sol.sample(maps[t], alpha=1.0, seed=0, it=t) for t in range(total)]
    cam0 = sol.cam.clone()
    pt0 = sol.pt.clone()
    run_iterations(sol, samples, cam0, pt0, lam0, args.warmup)
    # timed: K iterations, nothing else on the stream
    elapsed = timed(lambda: run_iterations(sol, samples, cam0, pt0, lam0, args.steps))
    st = sol.read_state()
    # the same K iterations captured once in a HIP graph and replayed (timed replay)
    graph_ips = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        run_iterations(sol, samples, cam0, pt0, lam0, 0)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            for t in range(args.steps):
                sol.step(samples[t])
        run_iterations(sol, samples, cam0, pt0, lam0, 0)
        g.replay()
        run_iterations(sol, samples, cam0, pt0, lam0, 0)
        graph_elapsed = timed(g.replay)
        graph_ips = args.steps / graph_elapsed
        assert sol.read_state()["F"] == st["F"], "graph replay diverged from the eager iterations"
    # per-phase split: the same iterations again with events between the phases
    P = S.STBA_NUM_PHASES
    evs = [S.hip_events(P + 1) for _ in range(args.steps)]
    run_iterations(sol, samples, cam0, pt0, lam0, args.steps, events=evs)
    torch.cuda.synchronize()
    phase_ms = np.zeros(P)
    for ev in evs:
        for k in range(P):
            phase_ms[k] += S.event_ms(ev[k], ev[k + 1])
    phase_ms /= args.steps
    names = [S.stba_phase_name(k) for k in range(P)]
    model, stats = algorithmic_model(scene, maps[:args.steps], es)
    ms_per_step = 1e3 * elapsed / args.steps
    dom = max((nm for nm in names if nm in model), key=lambda nm: phase_ms[names.index(nm)])
    dur_s = phase_ms[names.index(dom)] * 1e-3
    mdl = model[dom]
    if mdl["bound"] == "hbm":
        achieved, peak, unit = mdl["bytes"] / dur_s / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        achieved = mdl["flops"] / dur_s / 1e12
        peak = FP64_PEAK_TFLOPS if (precision == S.STBA_FP64 or dom == "cluster_cholesky") else FP32_PEAK_TFLOPS
        unit = "TFLOP/s"
    roofline = {"kernel": dom, "bound": mdl["bound"], "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": load_traffic(dom, workload),
                "duration_ms": phase_ms[names.index(dom)]}
    per_phase = {}
    for k, nm in enumerate(names):
        entry = {"ms": round(float(phase_ms[k]), 4)}
        if nm in model:
            mm = model[nm]
            if "bytes" in mm:
                entry["GB/s"] = round(mm["bytes"] / (phase_ms[k] * 1e-3) / 1e9, 1)
            if "flops" in mm:
                entry["TFLOP/s"] = round(mm["flops"] / (phase_ms[k] * 1e-3) / 1e12, 3)
        per_phase[nm] = entry
    out = {
        "metric": "STBA LM iterations/s (and observations/s)", "value": args.steps / elapsed, "unit": "iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == S.STBA_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": workload, "cameras": scene.m, "points": scene.n, "observations": scene.q,
                   "views_per_point": 8, "cluster_cap": args.gamma, "clusters_mean": float(
                       np.mean([mp.max() + 1 for mp in maps[:args.steps]])), "lambda0": lam0, "alpha": 1.0,
                   "lm_iterations": args.steps, "precision": args.precision},
        "obs_per_s": scene.q * args.steps / elapsed,
        "graph_iter_per_s": graph_ips,
        "roofline": roofline,
        "phases": per_phase,
        "lm": {"F_final": st["F"],
               "accepted": st["n_accept"], "jacobian_evals": st["n_jac"], "rcs_builds": st["n_rcs"],
               "lambda_final": st["lambda_"], "status": st["status"]},
        "model": stats, "source_hash": source_hash(),
    }
    if not args.no_mixed and precision == S.STBA_FP64:
        out["mixed_vs_fp64"] = mixed_leg(S, scene, sol, samples, samples_maps=maps, args=args, lam0=lam0,
                                         cam0=cam0, pt0=pt0)
    if not args.no_huber and precision == S.STBA_FP64:
        out["huber"] = huber_leg(S, scene, maps, args, lam0, cam0, pt0)
    if not args.no_sgc and precision == S.STBA_FP64:
        out["sgc"] = sgc_leg(S, scene, e, w, args, lam0, cam0, pt0)
    if not args.no_pcg and precision == S.STBA_FP64:
        out["pcg"] = pcg_leg(S, scene, maps, args, lam0)
    if not args.no_ablations and precision == S.STBA_FP64:
        out["ablations"] = ablation_leg(S, scene, args)
    if args.diff_batch:
        out["diff_batch"] = diff_batch_leg(S, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, maps, lam0, args.cpu_iters)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


HUBER_SCALE = 0.5   # the experiments' robust loss (Sec. 5.1)


def huber_leg(S, scene, maps, args, lam0, cam0, pt0):
    """The same K FP64 iterations under the Huber loss of scale 0.5 (IRLS)."""
    solh = S.StbaSolver(scene.cam0, scene.pt0, scene.obs_cam, scene.obs_pt, scene.obs_uv,
                        gamma_max=args.gamma, precision=S.STBA_FP64, lambda0=lam0, huber=HUBER_SCALE)
    samples = [solh.sample(maps[t], alpha=1.0, seed=0, it=t) for t in range(max(args.steps, args.warmup))]
    run_iterations(solh, samples, cam0, pt0, lam0, args.warmup)
    t = timed(lambda: run_iterations(solh, samples, cam0, pt0, lam0, args.steps))
    st = solh.read_state()
    return {"scale": HUBER_SCALE, "iter_per_s": args.steps / t, "obs_per_s": scene.q * args.steps / t,
            "F_after_K": st["F"], "accepted": st["n_accept"], "status": st["status"]}


def diff_batch_leg(S, args):
    """The differentiation batch: 64 ring problems (m ~ U{30..120}, n ~ U{5k..30k},
    7 views per point, seeds 0-63) concatenated with index offsets into one
    problem; one forward (residuals, stba_residual_jacobian without J) and one
    backward (stba_residual_vjp of v = 2 f, the gradient of sum ||f||^2 with the
    Jacobian recomputed) per pass, in FP32, timed over K passes.  Algorithmic
    bytes per pass: forward ids, pixel and f (24 + 2 es per observation),
    backward ids, v and the pixel gradient (8 + 4 es per observation), plus the
    gathered and reduced camera and point rows."""
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

    def one():
        S.stba_residual_jacobian(prob, plan.dims, S.STBA_MIXED, f, None, None, None, plan.ws)
        torch.mul(f, 2.0, out=v)
        S.stba_residual_vjp(prob, plan.dims, S.STBA_MIXED, v, gc, gp, gu, plan.ws)

    for _ in range(args.warmup):
        one()
    K = args.steps
    dt = timed(lambda: [one() for _ in range(K)])
    es = 4
    algo = q * ((24 + 2 * es) + (8 + 4 * es) + 2 * es) + (m * 72 + n * 24) + (m * 9 + n * 3) * es
    return {"problems": len(batch), "observations": q, "cameras": m, "points": n,
            "us_per_fwd_bwd": 1e6 * dt / K, "GB_per_s_algorithmic": algo * K / dt / 1e9,
            "algorithmic_bytes_per_pass": algo}


SGC_BETA = 10.0   # the clustering's scale beta


def sgc_leg(S, scene, e, w, args, lam0, cam0, pt0):
    """Maps drawn on the device by stochastic graph clustering (Sec. 4.4, Eq. 16):
    the clustering kernel alone (K maps back to back, HIP events on the stream it
    runs on), then K FP64 LM iterations each preceded by its own device map (the
    number of clusters read back before each step), against the host harness's
    time per map on the same camera graph."""
    import torch
    import synth
    sol = S.StbaSolver(scene.cam0, scene.pt0, scene.obs_cam, scene.obs_pt, scene.obs_uv,
                       gamma_max=args.gamma, precision=S.STBA_FP64, lambda0=lam0)
    K = args.steps
    cc = torch.empty(scene.m, dtype=torch.int32, device="cuda")
    out = torch.zeros(2, dtype=torch.int32, device="cuda")

    def draw(t):
        S.stba_sample_clusters(sol.problem, sol.dims, sol.precision, sol.ws, args.gamma, SGC_BETA, 0, t, cc,
                               out[0:1], out[1:2])

    for t in range(args.warmup):
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

    def iterations(steps):
        sol.cam.copy_(cam0)
        sol.pt.copy_(pt0)
        S.stba_lm_init(sol.state, lam0, 0.1)
        ls = []
        for t in range(steps):
            smp = sol.sample_clusters(args.gamma, SGC_BETA, alpha=1.0, seed=0, it=t)
            ls.append(smp.l)
            sol.step(smp)
        return ls

    iterations(args.warmup)
    ls = []
    t_iter = timed(lambda: ls.extend(iterations(K)))
    st = sol.read_state()
    t0 = time.perf_counter()
    n_host = 3
    for t in range(n_host):
        synth.sgc_map(e, w, scene.m, args.gamma, SGC_BETA, 0, t)
    host_ms = 1e3 * (time.perf_counter() - t0) / n_host
    return {"beta": SGC_BETA, "cap": args.gamma, "kernel_ms_per_map": kernel_ms,
            "iter_per_s_with_device_maps": K / t_iter, "clusters_mean": float(np.mean(ls)),
            "F_after_K": st["F"], "status": st["status"], "host_harness_ms_per_map": host_ms}


PCG_TOLS = (1e-4, 1e-6, 1e-10)


def pcg_leg(S, scene, maps, args, lam0):
    """The inexact cluster solve (App. A, Table 3) against the Cholesky solve on
    the first iteration's cluster systems: for each tolerance the time of
    stba_solve_clusters_pcg (conjugate gradient, camera-block Jacobi, then the
    point step), the largest iteration count over the clusters and the camera
    step's distance from the Cholesky one; the Cholesky solve's time beside it.
    Each solve is timed with events on its stream after a fresh assembly."""
    import torch
    sol = S.StbaSolver(scene.cam0, scene.pt0, scene.obs_cam, scene.obs_pt, scene.obs_uv, gamma_max=args.gamma,
                       precision=S.STBA_FP64, lambda0=lam0)
    m, n, q = scene.m, scene.n, scene.q
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
            rcs = S.stba_build_cluster_rcs(sol.problem, sol.dims, smp, S.StbaDamping(lam0, 0.1), sol.precision,
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
    out = {"clusters": l, "cholesky_ms": chol_ms, "tolerances": {}}
    for tol in PCG_TOLS:
        ms = timed_solve(lambda rcs: S.stba_solve_clusters_pcg(sol.problem, sol.dims, rcs, sol.precision, Jc, Jp,
                                                               dcam, dpt, 5000, tol, its, res, cs, sol.ws))
        x = dcam.cpu().numpy()
        out["tolerances"][f"{tol:g}"] = {
            "ms": ms, "iterations_max": int(its.max().item()), "iterations_mean": float(its.double().mean().item()),
            "step_rel_diff_vs_cholesky": float(np.linalg.norm(x - ref) / np.linalg.norm(ref)),
            "status_ok": bool((cs == 0).all().item())}
    # K LM iterations with the PCG solves (tol 1e-6) from x0 on the same maps
    cam0, pt0 = sol.cam.clone(), sol.pt.clone()
    samples = [sol.sample(maps[t], alpha=1.0, seed=0, it=t) for t in range(args.steps)]

    def lm(pcg):
        sol.cam.copy_(cam0)
        sol.pt.copy_(pt0)
        S.stba_lm_init(sol.state, lam0, 0.1)
        for t in range(args.steps):
            sol.step(samples[t], pcg=pcg)

    lm(None)
    F_chol = sol.read_state()["F"]
    dt = timed(lambda: lm((5000, 1e-6)))
    st = sol.read_state()
    out["lm_tol_1e-6"] = {"iter_per_s": args.steps / dt, "F_after_K": st["F"], "F_after_K_cholesky": F_chol,
                          "accepted": st["n_accept"], "status": st["status"]}
    return out


def ablation_leg(S, scene, args):
    """Synthetic versions of the paper's ablations on the same scene, each
    `--ablation-iters` FP64 LM iterations from the same start, every map drawn
    on the device (stochastic graph clustering, beta 10, seed 0, redrawn per
    iteration unless fixed):
    - correction (Sec. 5.4): lambda kept >= 0.1 (lambda0 0.1), STBA (correction
      whenever lambda >= 0.1, so at every iteration) against STBA* (none);
    - fixed clustering (Sec. 5.2): STBA against STBA-fixed (the first map at every
      iteration), lambda0 1e-4;
    - cluster cap (App. B): Gamma in {1, 25, 50, 100, m} (m: one cluster, plain
      LM), final costs normalised by the smallest, as the paper's figure does.
    Each entry gives the cost after every iteration and the iteration rate."""
    K = args.ablation_iters

    def run(gamma, lam0, lam_corr=0.1, lam_min=0.0, fixed=False):
        sol = S.StbaSolver(scene.cam0, scene.pt0, scene.obs_cam, scene.obs_pt, scene.obs_uv, gamma_max=gamma,
                           precision=S.STBA_FP64, lambda0=lam0, lambda_corr=lam_corr, lambda_min=lam_min)
        Fs, ls, first = [], [], None
        t0 = time.perf_counter()
        for t in range(K):
            if first is None or not fixed:
                smp = sol.sample_clusters(gamma, SGC_BETA, alpha=1.0, seed=0, it=t)
                first = first or smp
            sol.step(first if fixed else smp)
            st = sol.read_state()
            Fs.append(float(st["F"]))
            ls.append((first if fixed else smp).l)
        dt = time.perf_counter() - t0
        return {"F": [float(f"{f:.7g}") for f in Fs], "F_final": Fs[-1], "clusters_mean": float(np.mean(ls)),
                "iter_per_s": K / dt, "status": int(st["status"])}

    out = {"iterations": K}
    stba, star = run(args.gamma, 0.1, 0.1, 0.1), run(args.gamma, 0.1, float("inf"), 0.1)
    out["correction"] = {"lambda_min": 0.1, "stba": stba, "stba_star": star,
                         "final_ratio_star_over_stba": star["F_final"] / stba["F_final"]}
    redrawn, fixed = run(args.gamma, 1e-4), run(args.gamma, 1e-4, fixed=True)
    out["fixed_clustering"] = {"stba": redrawn, "stba_fixed": fixed,
                               "final_ratio_fixed_over_stba": fixed["F_final"] / redrawn["F_final"]}
    caps = {}
    for g in (1, 25, 50, 100, scene.m):
        caps[str(g)] = run(g, 1e-4)
    best = min(c["F_final"] for c in caps.values())
    for c in caps.values():
        c["normalized_final"] = c["F_final"] / best
        del c["F"]
    out["cluster_cap"] = caps
    return out


TAUS = (0.1, 0.01, 0.001)


def mixed_leg(S, scene, sol64, samples64, samples_maps, args, lam0, cam0, pt0):
    """MIXED against FP64 at equal cost reduction, measured as in the performance
    profiles of Sec. 5.2: both precisions run from the same x0 with the same
    cluster maps; F0 is the cost at x0, F* the lower of their costs after K
    iterations, F_tau = F* + tau (F0 - F*), and T_tau is the wall time of the
    iterations a precision needs to bring its cost to F_tau or below."""
    import torch
    solm = S.StbaSolver(scene.cam0, scene.pt0, scene.obs_cam, scene.obs_pt, scene.obs_uv,
                        gamma_max=args.gamma, precision=S.STBA_MIXED, lambda0=lam0)
    kmax = 3 * args.steps
    samplesm = [solm.sample(samples_maps[t], alpha=1.0, seed=0, it=t) for t in range(kmax)]
    runs = {"fp64": (sol64, samples64), "mixed": (solm, samplesm)}
    hist = {}
    for name, (sol, smp) in runs.items():
        run_iterations(sol, smp, cam0, pt0, lam0, args.warmup)
        Fs = torch.empty(kmax, dtype=torch.float64, device="cuda")
        run_iterations(sol, smp, cam0, pt0, lam0, kmax, snapshots=Fs)
        hist[name] = Fs.cpu().numpy()
    plan = S.ResidualPlan(scene.obs_cam, scene.obs_pt, scene.m, scene.n, precision=S.STBA_FP64)
    uv = torch.as_tensor(scene.obs_uv, dtype=torch.float64, device="cuda")
    F0 = float((S.residuals(cam0, pt0, uv, plan) ** 2).sum())
    K = args.steps
    F_star = float(min(hist["fp64"][K - 1], hist["mixed"][K - 1]))
    cache = {}

    def seconds(name, n):
        if (name, n) not in cache:
            sol, smp = runs[name]
            cache[(name, n)] = timed(lambda: run_iterations(sol, smp, cam0, pt0, lam0, n))
        return cache[(name, n)]

    def first_at_or_below(name, F):
        hit = np.nonzero(hist[name] <= F)[0]
        return int(hit[0]) + 1 if hit.size else None

    profile = []
    for tau in TAUS:
        F_tau = F_star + tau * (F0 - F_star)
        row = {"tau": tau, "F_tau": F_tau}
        for name in runs:
            n = first_at_or_below(name, F_tau)
            row[f"{name}_iterations"] = n
            row[f"{name}_seconds"] = None if n is None else seconds(name, n)
        row["speedup"] = (row["fp64_seconds"] / row["mixed_seconds"]
                          if row["fp64_seconds"] and row["mixed_seconds"] else None)
        profile.append(row)
    t64, tmx = seconds("fp64", K), seconds("mixed", K)
    n_strict = first_at_or_below("mixed", hist["fp64"][K - 1])
    return {
        "F0": F0, "F_star": F_star, "iterations": K,
        "fp64_F_after_K": float(hist["fp64"][K - 1]), "mixed_F_after_K": float(hist["mixed"][K - 1]),
        "fp64_iter_per_s": K / t64, "mixed_iter_per_s": K / tmx, "mixed_obs_per_s": scene.q * K / tmx,
        "profile": profile,
        "speedup_at_equal_cost_reduction": profile[-1]["speedup"],
        "speedup_tau": TAUS[-1],
        # the stricter reading: MIXED until it reaches the FP64 cost after K iterations
        "mixed_iterations_to_fp64_F_after_K": n_strict,
        "speedup_to_fp64_F_after_K": None if n_strict is None else t64 / seconds("mixed", n_strict),
    }


if __name__ == "__main__":
    main()
