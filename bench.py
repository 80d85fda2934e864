#!/usr/bin/env python3
"""Benchmark of the power-series bundle-adjustment hot path on one MI355X.

Workload (default): the city-shaped synthetic problem - 1,100 cameras,
780,000 landmarks, ~4.94M observations with heavy-tailed tracks (mean 6.3,
max 200), 1 px noise, 2% outliers at 20 px, Huber loss (delta 3 px); series
order m = 32; float32 storage.  Observations are produced on the GPU by the
library's own projection of the ground truth plus the generator's noise.

A step is one full LM iteration from the initial state (linearise both
orders, assemble, damped inverses, reduced right-hand side, 32 series
orders, back-substitution, trial cost and model decrease, accept / reject);
the state is reset to the initial one before each step so all steps do the
same work.  The step time comes from K steps timed as a whole; per-kernel
times come from HIP events that the library records around every launch in
a second run of the same K steps (those events add gaps between kernels, so
they stay out of the step time).

The main line runs on point records (the camera-frame point and IRLS weight
per observation, from which every pass rebuilds the Jacobian blocks), the
faster of the two record kinds per LM iteration; the same step over stored
Jacobian blocks is measured beside it (`stored_blocks`).  bfloat16 storage
exists for Jacobian blocks only, so `--precision bf16` runs stored blocks.

Printed JSON line: `value` is the series throughput in GB/s (algorithmic
bytes of the m series orders divided by their kernel time); `roofline`
refers to the dominant kernel; `cpu_baseline` is the float64 oracle's series
on a bounded sample, single-threaded; extra keys give the LM iteration time
and the time to the 1% cost tolerance in float64, float32 and bf16 storage.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "power-series RCS solve GB/s & LM iteration time to 1% cost tol, FP32 vs FP64, 1 GPU"
SJ = {"f64": 8, "f32": 4, "bf16": 2}
SX = {"f64": 8, "f32": 4, "bf16": 4}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c3.json")
KERNEL_SOURCES = ["paper_2204_12834_amd/csrc/solve.hip", "paper_2204_12834_amd/csrc/device_ops.hpp",
                  "paper_2204_12834_amd/csrc/common.hpp"]


def series_bytes(n_obs, n_lms, prec, records="jacobian", range_pass=None):
    """Algorithmic bytes of one series order, per pass (dual-order design):
    landmark pass reads each observation record and camera index once and each
    V^-1 once, writes s; camera pass reads each record, landmark index and the
    gathered s once per observation.  A record is the 24 Jacobian scalars, or
    the 4 scalars (P, sqrt(w)) of a point record.  With the range-staged
    camera pass (range_pass = (non-empty groups, observed landmarks)) the
    camera pass reads s once per landmark as stored (4 scalars) instead of
    once per observation, and writes 9 sums per (camera, range) group."""
    sj, sx = SJ[prec], SX[prec]
    rec = 24 * sj if records == "jacobian" else 4 * sx
    lm = n_obs * (rec + 4) + n_lms * (6 * sx + 3 * sx)
    if range_pass is None:
        cam = n_obs * (rec + 4 + 3 * sx)
    else:
        groups, nseg = range_pass
        cam = n_obs * (rec + 4) + nseg * 4 * sx + groups * 9 * sx
    return lm, cam


def range_groups(scene, R):
    """(non-empty (camera, landmark range) groups, observed landmarks) of the
    camera-major order with R ranges over the observed landmarks."""
    import numpy as np
    observed = np.bincount(scene.obs_lm, minlength=scene.n_lms) > 0
    rank = np.cumsum(observed) - observed
    nseg = int(observed.sum())
    spr = max(1, -(-max(nseg, 1) // R))
    key = scene.obs_cam.astype(np.int64) * R + rank[scene.obs_lm] // spr
    return int(np.unique(key).size), nseg


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


class FileScene:
    """A problem read from a BAL file: observations and initial state as given."""

    def __init__(self, path):
        from paper_2204_12834_amd import bal
        p = bal.read(path)
        self.name = f"bal file {p.name}"
        self.n_cams, self.n_lms, self.n_obs = p.n_cams, p.n_lms, p.n_obs
        self.obs_cam, self.obs_lm, self.obs_xy = p.obs_cam, p.obs_lm, p.obs_xy
        self.cams0, self.lms0 = p.cams, p.lms


def make_scene(workload, huber=0.0):
    from paper_2204_12834_amd import synth
    if workload.startswith("bal:"):
        return FileScene(workload[4:]), (huber or None)
    if workload == "c3":
        return synth.config("c3"), 3.0
    if workload == "c3-angle-axis-x0":  # the earlier initial state (synth._perturb)
        return synth.config("c3", x0="angle-axis"), 3.0
    if workload == "c3s":  # reduced city for quick checks
        return synth.city_scene(n_cams=300, n_lms=60000, seed=0, name="c3s"), 3.0
    if workload == "c2":
        return synth.config("c2"), None
    if workload in ("c1", "c5"):  # LM runs on these shapes (--tau-only)
        return synth.config(workload), None
    raise SystemExit(f"unknown workload {workload}")


def pin_one_core():
    """Pins this process to one core of those it may use; returns its index."""
    try:
        cpu = min(os.sched_getaffinity(0))
        os.sched_setaffinity(0, {cpu})
        return cpu
    except (AttributeError, OSError):
        return None


def host_text(cores_used=1):
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        model = "unknown"
    return f"{cores_used} of {os.cpu_count()} cores, {model}"


# --------------------------------------------------------------- CPU leg ----

def cpu_baseline_child(workload, m, sample_lms, huber=0.0, gpu_precision="f32", gpu_records="jacobian"):
    """Oracle (float64 NumPy) series on a landmark subset, single thread,
    pinned to one core."""
    import numpy as np
    import oracle
    from oracle import camera, lm as olm, schur
    cpu = pin_one_core()
    scene, delta = make_scene(workload, huber)
    sample_lms = min(sample_lms, scene.n_lms)
    keep = scene.obs_lm < sample_lms
    oc, ol = scene.obs_cam[keep], scene.obs_lm[keep]
    cams0, lms0 = scene.cams0, scene.lms0[:sample_lms]
    if isinstance(scene, FileScene):
        obs = scene.obs_xy[keep]
    else:
        obs = camera.project(scene.cams_gt, scene.lms_gt[:sample_lms], oc, ol) + scene.noise[keep]
    F, r, Jp, Jl = olm.linearize(cams0, lms0, oc, ol, obs, delta)
    from oracle import normal
    U, V, bp, bl = normal.assemble(Jp, Jl, r, oc, ol, scene.n_cams, sample_lms)
    dp, dl = normal.damping_diagonals(U, V)
    Ul, Vl = normal.damp(U, V, 1e-4, dp, dl)
    Uinv, Vinv = normal.block_inverse(Ul), normal.block_inverse(Vl)
    bt = schur.reduced_rhs(Jp, Jl, oc, ol, bp, bl, Vinv)
    t0 = time.perf_counter()
    schur.power_series(Jp, Jl, oc, ol, Uinv, Vinv, bt, m, 0.0)
    dt = time.perf_counter() - t0
    n_keep = int(keep.sum())
    lmb, camb = series_bytes(n_keep, sample_lms, gpu_precision, gpu_records)
    lmb64, camb64 = series_bytes(n_keep, sample_lms, "f64")
    out = {"value": m * (lmb + camb) / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": f"{workload}: landmarks 0..{sample_lms - 1} ({n_keep} observations, all "
                     f"{scene.n_cams} cameras), oracle power series m={m} in float64, {dt:.1f} s on one pinned "
                     f"core; GB/s counted with the same byte formula as the GPU line ({gpu_precision} "
                     f"{gpu_records} records)",
           "seconds": dt, "value_f64_formula": m * (lmb64 + camb64) / dt / 1e9, "pinned_cpu": cpu,
           "host": host_text()}
    print(json.dumps(out))


def run_cpu_baseline(workload, m, sample_lms, huber=0.0, precision="f32", records="jacobian"):
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--workload", workload, "--m", str(m),
           "--sample-lms", str(sample_lms), "--huber", str(huber), "--precision", precision, "--records", records]
    return _oracle_child(cmd, 900)


def _oracle_child(cmd, timeout):
    env = dict(os.environ, OMP_NUM_THREADS="1", MKL_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    # the child's progress lines go straight to our stderr
    res = subprocess.run(cmd, env=env, stdout=subprocess.PIPE, text=True, timeout=timeout)
    if res.returncode != 0:
        print(f"[bench] oracle child failed with status {res.returncode}", file=sys.stderr)
        return None
    return json.loads(res.stdout.strip().splitlines()[-1])


def oracle_lm_child(workload, m, iters, huber=0.0):
    """The oracle's LM loop (Sec. 5.1 settings, series order m) from x0 on
    one pinned core: per-iteration costs and cumulative seconds (the first
    linearisation included).  iters = 0 runs to termination."""
    import oracle
    from oracle import camera, lm as olm
    cpu = pin_one_core()
    scene, delta = make_scene(workload, huber)
    if isinstance(scene, FileScene):
        obs = scene.obs_xy
    else:
        obs = camera.project(scene.cams_gt, scene.lms_gt, scene.obs_cam, scene.obs_lm) + scene.noise
    opts = olm.LMOptions(m=m, huber_delta=delta, max_iters=iters if iters > 0 else 50)
    rows = []
    t0 = time.perf_counter()

    def cb(it, cams_new, lms_new):
        rows.append({"cost": it.cost, "cost_new": it.cost_new, "accepted": bool(it.accepted), "gain": it.gain,
                     "lambda": it.lam, "stop_order": it.stop_order, "t_s": time.perf_counter() - t0})
        print(f"[oracle-lm] {workload} iteration {len(rows)}: F {it.cost:.6e} -> {it.cost_new:.6e} "
              f"{'accepted' if it.accepted else 'rejected'} at {rows[-1]['t_s']:.1f} s", file=sys.stderr, flush=True)

    print(f"[oracle-lm] {workload} scene and observations ready at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)

    def progress(stage):
        print(f"[oracle-lm] {workload} iteration {len(rows) + 1}: {stage} at {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)

    res = olm.lm(scene.cams0, scene.lms0, scene.obs_cam, scene.obs_lm, obs, opts, callback=cb, progress=progress)
    print(json.dumps({"workload": workload, "m": m, "iterations": rows, "converged": bool(res.converged),
                      "ran_to_termination": iters <= 0 or res.converged or len(rows) < iters,
                      "pinned_cpu": cpu, "host": host_text()}))


# --------------------------------------------------------------- GPU leg ----

def gpu_setup(scene, delta, precision, dev, records="jacobian", lm_ranges=0):
    import torch
    from paper_2204_12834_amd.solver import Problem, project
    if isinstance(scene, FileScene):
        obs = torch.as_tensor(scene.obs_xy, dtype=torch.float64, device=dev)
    else:
        obs = project(scene.obs_cam, scene.obs_lm, scene.cams_gt, scene.lms_gt, device=dev)
        obs += torch.as_tensor(scene.noise, device=dev)
    prob = Problem(scene.obs_cam, scene.obs_lm, obs, scene.n_cams, scene.n_lms, precision=precision,
                   loss="huber" if delta else "l2", huber_delta=delta or 0.0, device=dev, records=records,
                   lm_ranges=lm_ranges)
    cams0 = torch.as_tensor(scene.cams0, dtype=torch.float64, device=dev)
    lms0 = torch.as_tensor(scene.lms0, dtype=torch.float64, device=dev)
    return prob, cams0, lms0, obs


def stream_probe(dev, nbytes=1 << 32):
    """Achievable HBM bandwidth of the library's plain streaming kernels
    (read-only, copy and write-only, 4 GiB, best over a few grid sizes)."""
    import ctypes
    import torch
    from paper_2204_12834_amd import _lib
    lib = _lib.load()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = {}
    for kind, name, moved in [(0, "read", nbytes), (1, "copy", 2 * nbytes), (2, "write", nbytes)]:
        best = 0.0
        for blocks in [512, 768, 1024, 2048, 4096, 8192, 16384]:
            for _ in range(2):
                _lib.check("poba_probe", lib.poba_probe(kind, ctypes.c_void_p(src.data_ptr()),
                                                        ctypes.c_void_p(dst.data_ptr()), nbytes, blocks, s))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                lib.poba_probe(kind, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                               blocks, s)
            e1.record()
            torch.cuda.synchronize()
            gbs = 5 * moved / (e0.elapsed_time(e1) / 1e3) / 1e9
            if gbs > best:
                best, out[name + "_blocks"] = gbs, blocks
        out[name + "_GBps"] = round(best, 1)
    del src, dst
    torch.cuda.empty_cache()
    return out


def lm_run(prob, cams0, lms0, opts, max_iters):
    """LM loop to termination with one event after every iteration; returns
    [(cost after the iteration, seconds since the start, state)]."""
    import torch
    from paper_2204_12834_amd._lib import PobaLMState
    from paper_2204_12834_amd.solver import read_lm_state
    dev = cams0.device
    cams, lms = cams0.clone(), lms0.clone()
    st = prob.lm_init(opts)
    size = st.numel()
    hist = torch.zeros(max_iters, size, dtype=torch.uint8, device=dev)
    start = torch.cuda.Event(enable_timing=True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(max_iters)]
    torch.cuda.synchronize()
    start.record()
    for i in range(max_iters):
        prob.lm_step(cams, lms, st, opts)
        hist[i].copy_(st)
        evs[i].record()
    torch.cuda.synchronize()
    states = [read_lm_state(hist[i]) for i in range(max_iters)]
    times = [start.elapsed_time(e) / 1e3 for e in evs]
    out = []
    for s, t in zip(states, times):
        if s["iteration"] == 0:
            break
        out.append((s["cost"], t, s))
        if s["done"]:
            break
    return out


def measure_steps(prob, cams0, lms0, scene, args, precision, records):
    """Times args.steps LM iterations from x0 (state reset before each), then
    runs as many again with the library's per-kernel event timing (whose event
    records add gaps between kernels, so the step time comes from the first,
    untimed-per-kernel run); returns the step time, the per-class kernel times,
    the series throughput and the roofline of the dominant series kernel."""
    import torch
    from paper_2204_12834_amd.solver import LMOptions
    cams, lms = cams0.clone(), lms0.clone()
    opts = LMOptions(m=args.m, eps=0.0, func_tol=0.0, max_iters=1 << 30)
    st = prob.lm_init(opts)

    def step():
        cams.copy_(cams0)
        lms.copy_(lms0)
        prob.lm_init(opts, state=st)
        prob.lm_step(cams, lms, st, opts)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # the same steps again with per-kernel event timing
    prob.profile(True)
    prob.profile_read()
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = prob.profile_read()
    prob.profile(False)
    print(f"[bench] {precision} {records}: {args.steps} steps, {ms_per_step:.3f} ms/step; per step: "
          + ", ".join(f"{k} {v[0] / args.steps:.3f} ms ({v[1] // args.steps})" for k, v in prof.items()),
          file=sys.stderr, flush=True)
    N, nl = scene.n_obs, scene.n_lms
    rp = None
    if records == "point" and prob.get_tuning("range_lds"):
        rp = range_groups(scene, prob.get_tuning("lm_ranges"))
    lmb, camb = series_bytes(N, nl, precision, records, rp)
    k = args.steps
    # one landmark pass, camera pass and finish per order (the reduced
    # right-hand side is timed apart)
    t_lm, n_lm = prof["landmark_pass"][0] / 1e3, prof["landmark_pass"][1]
    t_cam, n_cam = prof["camera_pass"][0] / 1e3, prof["camera_pass"][1]
    t_fin, n_fin = prof["camera_finish"][0] / 1e3, prof["camera_finish"][1]
    avg_lm, avg_cam = t_lm / n_lm, t_cam / n_cam
    avg_fin = t_fin / n_fin if n_fin else 0.0
    series_time = k * args.m * (avg_lm + avg_cam + avg_fin)
    value = k * args.m * (lmb + camb) / series_time / 1e9
    dom = "landmark_pass" if t_lm >= t_cam else "camera_pass"
    dom_bytes = lmb if dom == "landmark_pass" else camb
    dom_avg = avg_lm if dom == "landmark_pass" else avg_cam
    achieved = dom_bytes / dom_avg / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        key = f"{args.workload}_{precision}_{dom}" + ("" if records == "jacobian" else "_point")
        if tr.get("source_hash") == kernel_source_hash() and key in tr.get("bytes_per_launch", {}):
            traffic = tr["bytes_per_launch"][key]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "bytes_per_launch": dom_bytes, "avg_launch_ms": round(dom_avg * 1e3, 4)}
    phases = {name: round(v[0] / k, 4) for name, v in prof.items()}
    return {"ms_per_step": round(ms_per_step, 4), "prof": prof, "value": round(value, 1), "roofline": roofline,
            "phases": phases, "series_us_per_order": round(1e6 * (avg_lm + avg_cam + avg_fin), 2),
            "series_bytes_per_order": lmb + camb, "records": records,
            "camera_pass": "range-staged" if rp else "per-piece gather"}


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_batched(args, dev):
    """256 independent ring problems of uneven size (20-200 cameras,
    2k-40k landmarks, log-uniform; tracks 2-8), float32, m = 16: one LM
    iteration of all problems per step, as (a) the batched handle with the
    autotuned launch shape, eagerly and (b) as one captured graph launch,
    against (c) the batched handle with the default shape and (d) one handle
    and launch sequence per problem.  Tuning and capture are outside the
    timed regions."""
    import numpy as np
    import torch
    from paper_2204_12834_amd import autotune, synth
    from paper_2204_12834_amd.solver import LMOptions, Problem, project
    m = 16 if args.m == 32 else args.m
    prec = args.precision
    t_gen = time.perf_counter()
    scenes = synth.config("c4")
    cat, co, lo = synth.concat_scenes(scenes, name="c4")
    print(f"[bench] c4: {len(scenes)} problems, {cat.n_cams} cams, {cat.n_lms} lms, {cat.n_obs} obs "
          f"({time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    obs = project(cat.obs_cam, cat.obs_lm, cat.cams_gt, cat.lms_gt, device=dev)
    obs += torch.as_tensor(cat.noise, device=dev)
    oc = torch.as_tensor(cat.obs_cam, device=dev)
    ol = torch.as_tensor(cat.obs_lm, device=dev)
    cams0 = torch.as_tensor(cat.cams0, dtype=torch.float64, device=dev)
    lms0 = torch.as_tensor(cat.lms0, dtype=torch.float64, device=dev)
    opts = LMOptions(m=m, eps=0.0, func_tol=0.0, max_iters=1 << 30)

    def make(ps):
        return Problem(oc, ol, obs, cat.n_cams, cat.n_lms, precision=prec, piece_size=ps, device=dev,
                       prob_cam_off=co, prob_lm_off=lo)

    if args.graph_only:
        # only the captured LM step with the default shape, for a kernel trace
        prob = make(autotune.DEFAULT["piece_size"])
        prob.linearize(cams0, lms0)
        autotune.apply(prob, autotune.DEFAULT)
        cams, lms = cams0.clone(), lms0.clone()
        st = prob.lm_init(opts)
        graph = prob.lm_graph(cams, lms, st, 1, opts)
        times = []
        for i in range(args.warmup + args.steps):
            cams.copy_(cams0)
            lms.copy_(lms0)
            prob.lm_init(opts, state=st)
            torch.cuda.synchronize()
            e0, e1 = _events()
            e0.record()
            graph.launch()
            e1.record()
            torch.cuda.synchronize()
            if i >= args.warmup:
                times.append(e0.elapsed_time(e1))
        graph.close()
        print(json.dumps({"mode": "c4 graph only", "graph_ms": [round(t, 4) for t in times],
                          "warmup": args.warmup, "steps": args.steps, "m": m}), flush=True)
        return 0
    t_tune = time.perf_counter()
    cfg, prob = autotune.tune(make, prec, cat.n_obs, cat.n_lms, cams0, lms0,
                              log=lambda s: print(s, file=sys.stderr, flush=True))
    t_tune = time.perf_counter() - t_tune
    print(f"[bench] tuned in {t_tune:.1f} s: {cfg.get('piece_size')}/{cfg.get('tiles_per_wave')}/"
          f"{cfg.get('lds_camera')}", file=sys.stderr, flush=True)
    cams, lms = cams0.clone(), lms0.clone()
    st = prob.lm_init(opts)

    def reset(pr, c, l, s_):
        c.copy_(cams0)
        l.copy_(lms0)
        pr.lm_init(opts, state=s_)

    def timed(fn, pre, k):
        for _ in range(args.warmup):
            pre()
            fn()
        tot = 0.0
        for _ in range(k):
            pre()
            e0, e1 = _events()
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            tot += e0.elapsed_time(e1)
        return tot / k

    k = args.steps
    eager_ms = timed(lambda: prob.lm_step(cams, lms, st, opts), lambda: reset(prob, cams, lms, st), k)
    # series bytes and kernel times of the tuned batched step
    reset(prob, cams, lms, st)
    prob.profile(True)
    prob.profile_read()
    prob.lm_step(cams, lms, st, opts)
    prof = prob.profile_read()
    prob.profile(False)
    graph = prob.lm_graph(cams, lms, st, 1, opts)
    graph_ms = timed(graph.launch, lambda: reset(prob, cams, lms, st), k)
    graph.close()
    del prob
    torch.cuda.empty_cache()
    plain = make(autotune.DEFAULT["piece_size"])
    plain.linearize(cams0, lms0)
    autotune.apply(plain, autotune.DEFAULT)
    pst = plain.lm_init(opts)
    default_ms = timed(lambda: plain.lm_step(cams, lms, pst, opts), lambda: reset(plain, cams, lms, pst), k)
    del plain
    torch.cuda.empty_cache()
    # one handle and one launch sequence per problem
    solo = []
    for j, sc in enumerate(scenes):
        a, b_ = int(co[j]), int(co[j + 1])
        la, lb = int(lo[j]), int(lo[j + 1])
        sel = (oc >= a) & (oc < b_)
        pj = Problem(oc[sel] - a, ol[sel] - la, obs[sel], b_ - a, lb - la, precision=prec, device=dev)
        cj, lj = cams0[a:b_].clone(), lms0[la:lb].clone()
        solo.append((pj, cj, lj, pj.lm_init(opts), a, b_, la, lb))

    def solo_reset():
        for pj, cj, lj, sj, a, b_, la, lb in solo:
            cj.copy_(cams0[a:b_])
            lj.copy_(lms0[la:lb])
            pj.lm_init(opts, state=sj)

    def solo_step():
        for pj, cj, lj, sj, *_ in solo:
            pj.lm_step(cj, lj, sj, opts)

    solo_ms = timed(solo_step, solo_reset, max(2, k // 2))
    lmb = camb = 0
    for sc in scenes:
        a_, b2 = series_bytes(sc.n_obs, sc.n_lms, prec)
        lmb += a_
        camb += b2
    t_series = (prof["landmark_pass"][0] + prof["camera_pass"][0] + prof["camera_finish"][0]) / 1e3
    n_ord = max(prof["landmark_pass"][1], 1)
    value = n_ord * (lmb + camb) / t_series / 1e9
    line = {
        "metric": "batched LM iteration time and series GB/s, 256 sub-problems, 1 GPU",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": k, "warmup": args.warmup,
        "ms_per_step": round(graph_ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": f"c4: {len(scenes)} ring problems, {cat.n_cams} cameras, {cat.n_lms} landmarks, "
                               f"{cat.n_obs} observations, m={m}, {prec}, one LM iteration of every problem per step",
                   "n_problems": len(scenes), "n_obs": cat.n_obs, "m": m, "precision": prec},
        "lm_step_ms": {"batched_graph_tuned": round(graph_ms, 3), "batched_eager_tuned": round(eager_ms, 3),
                       "batched_eager_default_shape": round(default_ms, 3),
                       "one_handle_per_problem": round(solo_ms, 3)},
        "speedup_graph_vs_per_problem": round(solo_ms / graph_ms, 2),
        "tuned": {kk: cfg[kk] for kk in ("piece_size", "tiles_per_wave", "lds_camera", "us_per_order", "spread",
                                        "default_us_per_order", "default_spread", "candidates", "cached")
                  if kk in cfg},
        "tune_seconds": round(t_tune, 1),
        "phase_ms_per_step": {name: round(v[0], 4) for name, v in prof.items()},
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_adjoint(args, dev):
    """Differentiable damped step: 200 cameras, 50,000 landmarks (ring, tracks
    2-8), float32, lambda = 1, m = 32: forward (linearise + power solve) and
    backward (adjoint power solve + gradients of the observations and
    intrinsics) through the autograd Function."""
    import numpy as np
    import torch
    from paper_2204_12834_amd import synth
    from paper_2204_12834_amd.autograd import damped_step
    from paper_2204_12834_amd.solver import Problem, project
    s = synth.config("c5")
    obs = project(s.obs_cam, s.obs_lm, s.cams_gt, s.lms_gt, device=dev) + torch.as_tensor(s.noise, device=dev)
    prob = Problem(s.obs_cam, s.obs_lm, obs, s.n_cams, s.n_lms, precision=args.precision, device=dev)
    rng = np.random.default_rng(1)
    gp = torch.as_tensor(rng.normal(size=(s.n_cams, 9)), device=dev)
    gl = torch.as_tensor(rng.normal(size=(s.n_lms, 3)), device=dev)
    extr = torch.as_tensor(s.cams0[:, :6].copy(), device=dev)
    lms = torch.as_tensor(s.lms0, device=dev)
    intr0 = torch.as_tensor(s.cams0[:, 6:9].copy(), device=dev)

    def run():
        o = obs.clone().requires_grad_(True)
        intr = intr0.clone().requires_grad_(True)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        dxc, dxl = damped_step(prob, o, intr, extr, lms, 1.0, 32)
        e1.record()
        loss = (dxc * gp).sum() + (dxl * gl).sum()
        g_o, g_i = torch.autograd.grad(loss, [o, intr])
        e2.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), e1.elapsed_time(e2)

    for _ in range(args.warmup):
        run()
    f = b = 0.0
    for _ in range(args.steps):
        tf, tb = run()
        f += tf
        b += tb
    f /= args.steps
    b /= args.steps
    line = {"metric": "differentiable damped step: forward + backward time, 1 GPU", "value": round(f + b, 4),
            "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(f + b, 4),
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
            "data": "synthetic",
            "config": {"workload": f"c5: {s.n_cams} cameras, {s.n_lms} landmarks, {s.n_obs} observations, "
                                   f"lambda=1, m=32, {args.precision}", "n_obs": s.n_obs},
            "forward_ms": round(f, 4), "backward_ms": round(b, 4)}
    print(json.dumps(line), flush=True)
    return 0


def bench_pcg(args, dev):
    """Fig. 2 comparison: preconditioned CG on the reduced camera system at
    the first LM linearisation points of the workload (the trajectory of the
    power-series LM with the Sec. 5.1 settings).  At each point: the power
    series (order args.m, stop rule eps = 0.01) and its reduced residual
    |S x + b~| / |b~|; then CG with the Schur-Jacobi preconditioner and with
    the power-series preconditioner S~(m) for m in 0, 1, 2, 4, run to that
    same residual (equal accuracy), with their iteration counts and times;
    and a run of each to 1e-10 whose CG coefficients give the Lanczos
    estimate of kappa(M^-1 S)."""
    import numpy as np
    import torch
    from paper_2204_12834_amd.solver import LMOptions, read_lm_state, read_solve_info

    def kappa(co, k):
        # Ritz values of the k-step Lanczos matrix (diagonal 1/a_j + b_{j-1}/a_{j-1},
        # off-diagonal sqrt(b_j)/a_j)
        a, b = co[:k, 0, 0], co[:k - 1, 0, 1]
        T = np.diag(1.0 / a)
        T[1:, 1:] += np.diag(b / a[:-1])
        off = np.sqrt(b) / a[:-1]
        T += np.diag(off, 1) + np.diag(off, -1)
        ev = np.linalg.eigvalsh(T)
        return float(ev[-1] / ev[0])

    scene, delta = make_scene(args.workload, args.huber)
    prob, cams0, lms0, _ = gpu_setup(scene, delta, args.precision, dev, args.records)
    opts = LMOptions(m=args.m)
    cams, lms = cams0.clone(), lms0.clone()
    st = prob.lm_init(opts)
    precs = [("schur_jacobi", 0)] + [("power", m) for m in (0, 1, 2, 4)]
    rows = []
    for it in range(args.pcg_points):
        lam = read_lm_state(st)["lambda"]
        prob.linearize(cams, lms)
        row = {"lm_iteration": it, "lambda": lam}
        e0, e1 = _events()
        for _ in range(2):  # warm, then timed
            e0.record()
            dxc, _, info = prob.power_solve(lam, args.m, 0.01)
            e1.record()
            torch.cuda.synchronize()
        si = read_solve_info(info)
        res = prob.solve_residual(dxc).item()
        row["series"] = {"ms": round(e0.elapsed_time(e1), 3), "order": si["stop_order"], "rel_residual": res}
        for name, m in precs:
            key = name if name != "power" else f"power_m{m}"
            out = {}
            for tol, tag in [(res, "equal_accuracy"), (1e-10, "tight")]:
                e0.record()
                dxc, _, pinfo, co = prob.pcg_solve(lam, name, m, tol, 2000, coeffs=True)
                e1.record()
                torch.cuda.synchronize()
                k = pinfo[0]["iterations"]
                d = {"iterations": k, "ms": round(e0.elapsed_time(e1), 3), "converged": pinfo[0]["converged"],
                     "rel_residual": prob.solve_residual(dxc).item()}
                if tag == "tight" and k > 1:
                    d["kappa_estimate"] = round(kappa(co.cpu().numpy(), k), 3)
                out[tag] = d
            row[key] = out
        rows.append(row)
        print(f"[pcg] point {it}: lambda {lam:.2e}, series {row['series']}, "
              + ", ".join(f"{k} {row[k]['equal_accuracy']['iterations']} it {row[k]['equal_accuracy']['ms']} ms"
                          for k in row if k.startswith(("schur", "power"))), file=sys.stderr, flush=True)
        prob.lm_step(cams, lms, st, opts)
    # per-iteration phases of one Schur-Jacobi solve at the last point
    prob.profile(True)
    prob.profile_read()
    _, _, pinfo, _ = prob.pcg_solve(read_lm_state(st)["lambda"], "schur_jacobi", 0, 1e-10, 200)
    prof = prob.profile_read()
    prob.profile(False)
    n_it = max(pinfo[0]["iterations"], 1)
    cg_iter_ms = sum(v[0] for v in prof.values()) / n_it
    # the float64 product S p per iteration: landmark part (records, camera words, V and the
    # damping diagonal in float64, s written in float64) and camera part (records, landmark
    # indices, the float64 s gathered per observation)
    rec = 24 * SJ[args.precision] if args.records == "jacobian" else 4 * SX[args.precision]
    nl_obs = int(np.count_nonzero(np.bincount(scene.obs_lm, minlength=scene.n_lms)))
    s_apply = {}
    for name, nbytes in [("landmark_pass", scene.n_obs * (rec + 4) + nl_obs * (6 + 3 + 4) * 8),
                         ("camera_pass", scene.n_obs * (rec + 4 + 3 * 8))]:
        t, n = prof[name]
        if n:
            gbs = nbytes / (t / n / 1e3) / 1e9
            s_apply[name] = {"bytes_per_launch": nbytes, "avg_launch_ms": round(t / n, 4), "achieved": round(gbs, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    mean = lambda key: float(np.mean([r[key]["equal_accuracy"]["ms"] for r in rows]))
    line = {"metric": "PCG on the reduced camera system vs the power series: solve time at equal accuracy "
                      "(Schur-Jacobi PCG), 1 GPU",
            "value": round(mean("schur_jacobi"), 3), "unit": "ms", "n_gpus": 1, "steps": args.pcg_points,
            "warmup": 1, "ms_per_step": round(mean("schur_jacobi"), 3), "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
            "data": "file" if isinstance(scene, FileScene) else "synthetic",
            "config": {"workload": f"{scene.name}: {scene.n_cams} cameras, {scene.n_lms} landmarks, "
                                   f"{scene.n_obs} observations, {args.precision} "
                                   f"{'Jacobian blocks' if args.records == 'jacobian' else 'point records'}, "
                                   f"first {args.pcg_points} LM linearisation points, series m={args.m} eps=0.01",
                       "records": args.records},
            "series_ms_mean": round(float(np.mean([r["series"]["ms"] for r in rows])), 3),
            "mean_ms_equal_accuracy": {k: round(mean(k), 3) for k in rows[0] if k.startswith(("schur", "power"))},
            "sj_iteration_ms": round(cg_iter_ms, 4),
            "sj_phases_ms_per_iteration": {k: round(v[0] / n_it, 4) for k, v in prof.items() if v[1]},
            "s_apply_roofline": s_apply,
            "points": rows}
    print(json.dumps(line), flush=True)
    return 0


def bench_post(args, dev):
    """Sec. 5.3 on the GPU: LM with the clustered step of PoST (clusters of at
    most 100 cameras, a new seeded draw of clusters per iteration, or a pool
    of draws used in turn) against the LM with the power series of the whole
    problem, from the same x0 with the Sec. 5.1 settings and series order
    args.m.  Wall time per iteration (the clustering and relabelling run on
    the host inside it), time and iterations to the 1% cost tolerance."""
    import numpy as np
    import torch
    from paper_2204_12834_amd.post import PoST
    from paper_2204_12834_amd.solver import LMOptions

    scene, delta = make_scene(args.workload, args.huber)
    opts = LMOptions(m=args.m)
    prob, cams0, lms0, obs = gpu_setup(scene, delta, args.precision, dev, args.records, args.lm_ranges)
    lm_run(prob, cams0, lms0, LMOptions(m=args.m, max_iters=2), 2)  # warm
    poba = lm_run(prob, cams0, lms0, opts, 50)
    f0 = prob.linearize(cams0, lms0).item()
    del prob
    torch.cuda.empty_cache()
    runs = {"poba": [(c, t) for c, t, _ in poba]}
    detail = {}
    for draws in ([0] + [args.post_draws] if args.post_draws else [0]):
        t_setup = time.perf_counter()
        p = PoST(scene.obs_cam, scene.obs_lm, obs, scene.n_cams, scene.n_lms, max_cluster=args.post_cluster,
                 seed=1, draws=draws, precision=args.precision, loss="huber" if delta else "l2",
                 huber_delta=delta or 0.0, records=args.records, device=dev)
        if draws:
            for it in range(draws):
                p.clustered(it)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t_setup
        cams, lms = cams0.clone(), lms0.clone()
        times = []
        t0 = time.perf_counter()
        states = p.lm(cams, lms, opts, callback=lambda it, s: times.append(time.perf_counter() - t0))
        name = f"post_draws{draws}" if draws else "post"
        runs[name] = [(s["cost"], t) for s, t in zip(states, times)]
        c = p.clustered(0)
        sizes = np.bincount(c.cluster)
        # one iteration's parts, timed apart at the final state
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cl, k = p.graph.cluster(args.post_cluster, 12345)
        t2 = time.perf_counter()
        p.graph.layout(cl, k)
        t3 = time.perf_counter()
        p.whole.linearize(cams, lms)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        _, _, _, c_step = p.step(cams, lms, 1e-4, args.m, 0.01, iteration=0)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        # one series at the final state, timed per kernel: the clustered (batched) handle against the whole one
        series = {}
        for key, hp in [("whole", p.whole), ("clustered", c_step.problem)]:
            hp.profile(True)
            hp.profile_read()
            hp.power_solve(1e-4, args.m, 0.0)
            pr = hp.profile_read()
            hp.profile(False)
            per = sum(pr[k][0] / pr[k][1] for k in ("landmark_pass", "camera_pass", "camera_finish") if pr[k][1])
            series[key] = {"us_per_order": round(1e3 * per, 2)}
            if args.records == "jacobian":
                nbytes = sum(series_bytes(scene.n_obs, hp.n_lms, args.precision, "jacobian"))
                gbs = nbytes / (per / 1e3) / 1e9
                series[key].update({"bytes_per_order": nbytes, "GBps": round(gbs, 1),
                                    "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)})
        detail[name] = {"series": series, "setup_s": round(t_setup, 3), "clusters": int(c.n_clusters),
                        "cluster_size_min_mean_max": [int(sizes.min()), round(float(sizes.mean()), 1),
                                                      int(sizes.max())],
                        "cluster_ms": round(1e3 * (t2 - t1), 2), "layout_ms": round(1e3 * (t3 - t2), 2),
                        "linearize_ms": round(1e3 * (t4 - t3), 2),
                        "step_ms" + ("" if draws else "_incl_new_handle"): round(1e3 * (t5 - t4), 2)}
        print(f"[post] {name}: {len(states)} iterations, {times[-1]:.3f} s, final cost {states[-1]['cost']:.6e}, "
              f"{detail[name]}", file=sys.stderr, flush=True)
        p.close()
        del p
        torch.cuda.empty_cache()
    fstar = min(min(c for c, _ in r) for r in runs.values())
    ftau = fstar + 0.01 * (f0 - fstar)
    out = {}
    for name, r in runs.items():
        hit = next(((i + 1, t) for i, (c, t) in enumerate(r) if c <= ftau), None)
        out[name] = {"iterations": len(r), "seconds": round(r[-1][1], 4), "final_cost": r[-1][0],
                     "ms_per_iteration": round(1e3 * r[-1][1] / len(r), 3),
                     "iters_to_1pct": hit[0] if hit else None, "t_1pct_s": round(hit[1], 4) if hit else None}
    line = {"metric": "PoST on the GPU: LM time to 1% cost tol with per-cluster power series vs the whole-problem "
                      "series, 1 GPU", "value": out["post"]["t_1pct_s"], "unit": "s", "n_gpus": 1,
            "steps": out["post"]["iterations"], "warmup": 0, "ms_per_step": out["post"]["ms_per_iteration"],
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
            "data": "file" if isinstance(scene, FileScene) else "synthetic",
            "config": {"workload": f"{scene.name}: {scene.n_cams} cameras, {scene.n_lms} landmarks, "
                                   f"{scene.n_obs} observations, {args.precision} "
                                   f"{'Jacobian blocks' if args.records == 'jacobian' else 'point records'}, "
                                   f"clusters of at most {args.post_cluster} cameras, m={args.m}, eps=0.01",
                       "records": args.records},
            "f0": f0, "f_star": fstar, "f_tau": ftau, "runs": out, "post_detail": detail}
    print(json.dumps(line), flush=True)
    return 0


def lm_trace_rows(out, n, lambda0):
    """The first n iterations of an lm_run: the damping each step used, the
    trial cost, gain, acceptance and series order, the cost after the
    iteration and the time since the start."""
    rows = []
    lam = lambda0
    for i, (c, t, st) in enumerate(out[:n]):
        rows.append({"iteration": i + 1, "lambda_used": lam, "cost_trial": st["cost_new"], "gain": st["gain"],
                     "model_decrease": st["model_decrease"], "accepted": st["accepted"],
                     "stop_order": st["stop_order"], "cost_after": c, "t_ms": round(1e3 * t, 3)})
        lam = st["lambda"]
    return rows


def tau_runs(args, scene, delta, dev):
    """LM to termination (Sec. 5.1 settings) from x0 for every precision,
    record kind and series order asked for; f* is the best final cost over
    all of them, f_tau = f* + 0.01 (f0 - f*) (Sec. 5, performance profiles),
    and T_1% the time of the first iteration whose cost is at or below it."""
    import numpy as np
    import torch
    from paper_2204_12834_amd.solver import LMOptions
    precisions = [p for p in args.tau_precisions.split(",") if p]
    ms = [int(v) for v in (args.tau_m or str(args.m)).split(",")]
    records = ["jacobian"] + ([] if args.no_point else ["point"])
    runs, steps_at_x0, traces = {}, {}, {}
    for m in ms:
        for rec in records:
            for prec in precisions:
                if rec == "point" and prec == "bf16":
                    continue
                name = prec if rec == "jacobian" else f"{prec}_point"
                if len(ms) > 1:
                    name += f"_m{m}"
                p2, c0, l0, _ = gpu_setup(scene, delta, prec, dev, rec)
                # the damped step at x0 (lambda0, fixed order) for the precision comparison
                p2.linearize(c0, l0)
                dxc, dxl, _ = p2.power_solve(1e-4, m, 0.0)
                steps_at_x0[name] = (dxc.cpu().numpy(), dxl.cpu().numpy(), m)
                o2 = LMOptions(m=m)  # Sec. 5.1 settings, series order m
                runs[name] = lm_run(p2, c0, l0, o2, 50)
                traces[name] = lm_trace_rows(runs[name], args.trace_iters, o2.lambda0)
                print(f"[bench] LM {name}: {len(runs[name])} iterations, final cost {runs[name][-1][0]:.6e}",
                      file=sys.stderr, flush=True)
                del p2
                torch.cuda.empty_cache()
    # F(x0) from a plain linearisation
    p3, c0, l0, _ = gpu_setup(scene, delta, "f64", dev)
    f0 = p3.linearize(c0, l0).item()
    del p3
    fstar = min(min(c for c, _, _ in out) for out in runs.values())
    ftau = fstar + 0.01 * (f0 - fstar)
    tau = {}
    for name, out in runs.items():
        hit = [t for c, t, _ in out if c <= ftau]
        k = next((i + 1 for i, (c, _, _) in enumerate(out) if c <= ftau), None)
        tau[name] = {"t_1pct_s": round(hit[0], 4) if hit else None, "iterations": len(out),
                     "final_cost": out[-1][0], "lm_iter_ms": round(1e3 * out[-1][1] / len(out), 3),
                     "iters_to_1pct": k,
                     "ms_per_iter_to_1pct": round(1e3 * hit[0] / k, 3) if hit else None,
                     "accepted": sum(1 for _, _, st in out if st["accepted"]),
                     "converged": out[-1][2]["converged"]}
    prec_err = {}
    for name, (c_, l_, m) in steps_at_x0.items():
        ref = next((v for k_, v in steps_at_x0.items() if v[2] == m and k_.split("_")[0] == "f64"
                    and "point" not in k_), None)
        if ref is None or ref[0] is c_:
            continue
        prec_err[name] = {"dx_cams": float(np.linalg.norm(c_ - ref[0]) / np.linalg.norm(ref[0])),
                          "dx_lms": float(np.linalg.norm(l_ - ref[1]) / np.linalg.norm(ref[1]))}
    return {"f0": f0, "f_star": fstar, "f_tau": ftau, "time_to_1pct": tau, "step_error_vs_f64_at_x0": prec_err,
            "lm_trace": traces}


def bench_tau(args, dev):
    """Time to the 1% cost tolerance only (and, if asked, the oracle's LM on
    one pinned core beside it): one JSON line."""
    t_gen = time.perf_counter()
    scene, delta = make_scene(args.workload, args.huber)
    print(f"[bench] scene {scene.name}: {scene.n_cams} cams, {scene.n_lms} lms, {scene.n_obs} obs "
          f"({time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)
    res = tau_runs(args, scene, delta, dev)
    line = {"metric": "LM time to 1% cost tolerance", "workload": scene.name, "n_cams": scene.n_cams,
            "n_lms": scene.n_lms, "n_obs": scene.n_obs, "huber_delta": delta}
    line.update(res)
    if args.oracle_lm >= 0:
        m = int((args.tau_m or str(args.m)).split(",")[0])
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-lm-child", "--workload", args.workload, "--m",
               str(m), "--oracle-lm", str(args.oracle_lm), "--huber", str(args.huber)]
        orc = _oracle_child(cmd, 3000)
        if orc is not None:
            ftau = res["f_tau"]
            rows = orc["iterations"]
            cost_after = [r["cost_new"] if r["accepted"] else r["cost"] for r in rows]
            hit = next((i for i, c in enumerate(cost_after) if c <= ftau), None)
            orc["t_1pct_s"] = round(rows[hit]["t_s"], 3) if hit is not None else None
            gpu = res["time_to_1pct"].get("f64") or res["time_to_1pct"].get(f"f64_m{m}") or {}
            if hit is None and rows and gpu.get("iters_to_1pct"):
                # fewer oracle iterations than the GPU float64 run needed: extrapolate
                per = (rows[-1]["t_s"] - rows[0]["t_s"]) / max(len(rows) - 1, 1) if len(rows) > 1 else rows[0]["t_s"]
                orc["t_1pct_extrapolated_s"] = round(rows[0]["t_s"] + per * (gpu["iters_to_1pct"] - 1), 3)
                orc["extrapolation"] = (f"first oracle iteration plus the mean of the timed ones times the "
                                        f"{gpu['iters_to_1pct']} iterations the GPU float64 run took to f_tau")
            line["oracle_lm"] = orc
    print(json.dumps(line), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3",
                    help="c3 (default), c2, c3s, c4, c5, or bal:PATH for a problem in the BAL text format")
    ap.add_argument("--huber", type=float, default=0.0, help="Huber delta in pixels for a bal: workload (0: squared loss)")
    ap.add_argument("--precision", default="f32", choices=["f64", "f32", "bf16"])
    ap.add_argument("--records", default=None, choices=["jacobian", "point"],
                    help="per-observation records: Jacobian blocks, or camera-frame points the passes rebuild them "
                         "from (default: point records for the main line, Jacobian blocks for bf16 and for the "
                         "other modes)")
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--sample-lms", type=int, default=600000,
                    help="landmarks of the scene the CPU oracle's series runs on (about 10-20 s of CPU work)")
    ap.add_argument("--tpw", type=int, default=0, help="landmark tiles per wavefront (0: library default)")
    ap.add_argument("--lm-ranges", type=int, default=0,
                    help="landmark ranges of the camera-major order (0: automatic, else 1 or a multiple of 8)")
    ap.add_argument("--lds-camera", type=int, default=-1,
                    help="1/0: landmark pass reads the camera vector from LDS / from L2 (-1: library default)")
    ap.add_argument("--sweep-tpw", default="", help="comma list: time the series for each and exit")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tau", action="store_true", help="skip the time-to-tolerance LM runs")
    ap.add_argument("--no-alt", action="store_true",
                    help="main line: skip the same step with the other record kind")
    ap.add_argument("--no-point", action="store_true",
                    help="skip the point-record runs of the time-to-tolerance part (implies --no-alt)")
    ap.add_argument("--pcg", action="store_true",
                    help="compare CG on the reduced camera system (Schur-Jacobi and power-series "
                         "preconditioners) with the power series at the first LM points, and exit")
    ap.add_argument("--pcg-points", type=int, default=5, help="LM linearisation points of the --pcg comparison")
    ap.add_argument("--post", action="store_true",
                    help="compare the LM of PoST (clustered reduced camera system) with the whole-problem LM, and exit")
    ap.add_argument("--post-cluster", type=int, default=100, help="largest camera cluster of --post")
    ap.add_argument("--post-draws", type=int, default=4,
                    help="--post also runs with this many cluster draws used in turn (0: only new draws)")
    ap.add_argument("--tau-only", action="store_true",
                    help="only the time-to-tolerance LM runs on the workload (c1, c2, c3, c5, bal:PATH), then exit")
    ap.add_argument("--tau-m", default="", help="comma list of series orders for the LM runs (default: --m)")
    ap.add_argument("--tau-precisions", default="f64,f32,bf16", help="comma list of precisions for the LM runs")
    ap.add_argument("--trace-iters", type=int, default=5, help="LM iterations listed per run in lm_trace")
    ap.add_argument("--oracle-lm", type=int, default=-1,
                    help="with --tau-only: also time the oracle's LM on one pinned core for this many "
                         "iterations (0: to termination; -1: not at all)")
    ap.add_argument("--graph-only", action="store_true",
                    help="with --workload c4: only time the captured LM step (default shape), for kernel traces")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--oracle-lm-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.records is None:
        main_line = not (args.tau_only or args.workload in ("c4", "c5") or args.pcg or args.post
                         or args.sweep_tpw or args.cpu_baseline_child or args.oracle_lm_child)
        args.records = "point" if main_line and args.precision != "bf16" else "jacobian"
    if args.no_point:
        args.no_alt = True

    if args.cpu_baseline_child:
        cpu_baseline_child(args.workload, args.m, args.sample_lms, args.huber, args.precision, args.records)
        return 0
    if args.oracle_lm_child:
        oracle_lm_child(args.workload, args.m, args.oracle_lm, args.huber)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the library has no multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2204_12834_amd.solver import LMOptions

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.tau_only:
        return bench_tau(args, dev)
    if args.workload == "c4":
        return bench_batched(args, dev)
    if args.workload == "c5":
        return bench_adjoint(args, dev)
    if args.pcg:
        return bench_pcg(args, dev)
    if args.post:
        return bench_post(args, dev)
    t_gen = time.perf_counter()
    scene, delta = make_scene(args.workload, args.huber)
    print(f"[bench] scene {scene.name}: {scene.n_cams} cams, {scene.n_lms} lms, {scene.n_obs} obs "
          f"({time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)

    prob, cams0, lms0, obs = gpu_setup(scene, delta, args.precision, dev, args.records, args.lm_ranges)
    if args.tpw:
        prob.set_tuning("tiles_per_wave", args.tpw)
    if args.lds_camera >= 0:
        prob.set_tuning("lds_camera", args.lds_camera)
    if args.sweep_tpw:
        prob.linearize(cams0, lms0)
        for tpw in [int(x) for x in args.sweep_tpw.split(",")]:
            prob.set_tuning("tiles_per_wave", tpw)
            prob.power_solve(1e-4, args.m, 0.0)
            torch.cuda.synchronize()
            prob.profile(True)
            prob.profile_read()
            for _ in range(3):
                prob.power_solve(1e-4, args.m, 0.0)
            torch.cuda.synchronize()
            pr = prob.profile_read()
            prob.profile(False)
            print(f"[sweep] tpw={tpw}: " + ", ".join(f"{k} {v[0] / max(v[1], 1) * 1e3:.1f} us x{v[1] // 3}"
                                                    for k, v in pr.items() if v[1]), file=sys.stderr, flush=True)
        return 0
    res = measure_steps(prob, cams0, lms0, scene, args, args.precision, args.records)
    ms_per_step, prof, value, roofline, phases = (res[k] for k in ("ms_per_step", "prof", "value", "roofline",
                                                                  "phases"))
    N, nl, nc = scene.n_obs, scene.n_lms, scene.n_cams
    achieved = roofline["achieved"]
    del prob
    torch.cuda.empty_cache()

    alt = None
    other = "jacobian" if args.records == "point" else ("point" if args.precision != "bf16" else None)
    if other is not None and not args.no_alt:
        # the same step with the other record kind
        p2, c2, l2, _ = gpu_setup(scene, delta, args.precision, dev, other)
        alt = measure_steps(p2, c2, l2, scene, args, args.precision, other)
        alt.pop("prof")
        del p2
        torch.cuda.empty_cache()

    probe = stream_probe(dev)
    print(f"[bench] probe: {probe}", file=sys.stderr, flush=True)

    extra = {}
    if not args.no_tau:
        extra = tau_runs(args, scene, delta, dev)
    if alt is not None:
        extra["stored_blocks" if other == "jacobian" else "point_records"] = alt

    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_baseline(args.workload, args.m, args.sample_lms, args.huber, args.precision, args.records)

    if isinstance(scene, FileScene):
        loss_text = f"Huber delta {delta:g} px, " if delta else ""
    else:
        loss_text = "Huber delta 3 px, 2% outliers, " if delta else ""
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "file" if isinstance(scene, FileScene) else "synthetic",
        "config": {"workload": f"{scene.name}: {nc} cameras, {nl} landmarks, {N} observations, "
                               f"{loss_text}m={args.m}, "
                               f"{args.precision} {'Jacobian blocks' if args.records == 'jacobian' else 'point records'}"
                               f", one LM iteration per step",
                   "n_cams": nc, "n_lms": nl, "n_obs": N, "m": args.m, "precision": args.precision,
                   "records": args.records},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phase_ms_per_step": phases,
        "measured_read_GBps": probe["read_GBps"],
        "measured_copy_GBps": probe["copy_GBps"],
        "measured_write_GBps": probe["write_GBps"],
        "dominant_vs_measured_read": round(achieved / probe["read_GBps"], 4),
    }
    line.update(extra)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
