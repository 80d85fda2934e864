"""Launch-shape autotuner for the series kernels.

A measurement loop over the launch parameters that change only the
floating-point summation order, never the result beyond it:

  piece_size      observations per camera-pass work item (set at creation)
  tiles_per_wave  64-observation landmark tiles walked by one wavefront (the
                  landmark pass that reads the camera vector from L2)
  lds_camera      landmark pass reads the camera vector from LDS or L2

Each candidate is timed on the problem itself: the median of ten solves of
eight series orders, each timed with the library's own events.  A candidate
replaces the default only if its median beats the default's by more than
both spreads (the distance from median to the slower quartile of each) and
by at least 2%, so that noise never picks a shape.  The choice is kept in a
JSON cache keyed by (device architecture, precision, observation count
bucket, mean track length bucket), so later problems of the same shape skip
the search.  The cache file is `POBA_TUNE_CACHE` or ~/.cache/poba/tune.json.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

PIECE_SIZES = (256, 512, 1024, 2048)
TILES_PER_WAVE = (1, 2, 4, 8)
LDS_CAMERA = (1, 0)
DEFAULT = {"piece_size": 1024, "tiles_per_wave": 4, "lds_camera": 1}


def cache_path() -> str:
    return os.environ.get("POBA_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "poba", "tune.json"))


def shape_key(precision: str, n_obs: int, n_lms: int, arch: str | None = None) -> str:
    if arch is None:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    nb = int(round(math.log2(max(n_obs, 1))))
    track = n_obs / max(n_lms, 1)
    tb = int(round(2.0 * math.log2(max(track, 1.0))))
    return f"{arch}|{precision}|N2^{nb}|t{tb}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store_cache(cache: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_orders(problem, lam: float = 1e-2, orders: int = 8, reps: int = 10) -> list:
    """Microseconds per series order (landmark pass + camera pass + finish) of
    `reps` solves of `orders` orders, sorted; the problem must be linearised."""
    problem.power_solve(lam, 1, 0.0)  # warm-up
    out = []
    for _ in range(reps):
        problem.profile(True)
        problem.power_solve(lam, orders, 0.0)
        prof = problem.profile_read()
        problem.profile(False)
        t = prof["landmark_pass"][0] + prof["camera_pass"][0] + prof["camera_finish"][0]
        n = max(prof["landmark_pass"][1], 1)
        out.append(1e3 * t / n)
    return sorted(out)


def summary(samples) -> tuple:
    """(median, spread): spread is the slower quartile minus the median."""
    xs = sorted(samples)
    n = len(xs)
    med = 0.5 * (xs[(n - 1) // 2] + xs[n // 2])
    q3 = xs[min(n - 1, (3 * n) // 4)]
    return med, max(q3 - med, 0.0)


def beats(cand, default, min_gain: float = 0.02) -> bool:
    """A candidate (median, spread) is kept over the default only when it is
    faster by more than both spreads and by at least min_gain."""
    return cand[0] + cand[1] + default[1] < default[0] and cand[0] < (1.0 - min_gain) * default[0]


def apply(problem, config: dict) -> None:
    problem.set_tuning("tiles_per_wave", int(config["tiles_per_wave"]))
    problem.set_tuning("lds_camera", int(config["lds_camera"]))


def tune(make_problem, precision: str, n_obs: int, n_lms: int, cams: torch.Tensor, lms: torch.Tensor,
         piece_sizes=PIECE_SIZES, tiles=TILES_PER_WAVE, lds=LDS_CAMERA, cache: str | None = None,
         force: bool = False, log=None, timer=time_orders, arch: str | None = None) -> tuple[dict, object]:
    """Returns (config, problem): the best configuration for this shape and a
    handle created and tuned with it.  make_problem(piece_size) builds a
    handle; it is linearised at (cams, lms) here.  timer(problem) returns the
    per-order samples of the applied configuration."""
    key = shape_key(precision, n_obs, n_lms, arch)
    table = load_cache(cache)
    if not force and key in table:
        cfg = table[key]
        prob = make_problem(int(cfg["piece_size"]))
        prob.linearize(cams, lms)
        apply(prob, cfg)
        return dict(cfg, cached=True), prob
    t0 = time.time()
    results = []
    default = None
    best = None
    for ps in piece_sizes:
        prob = make_problem(ps)
        prob.linearize(cams, lms)
        for tpw in tiles:
            for lc in lds:
                cfg = {"piece_size": ps, "tiles_per_wave": tpw, "lds_camera": lc}
                apply(prob, cfg)
                med, spread = summary(timer(prob))
                results.append(dict(cfg, us_per_order=round(med, 2), spread=round(spread, 2)))
                if log:
                    log(f"[tune] {cfg} {med:.1f} us/order (+{spread:.1f})")
                if cfg == DEFAULT:
                    default = (med, spread, cfg)
                if best is None or med < best[0]:
                    best = (med, spread, cfg)
        del prob
        if torch.cuda.is_available():
            torch.cuda.empty_cache()
    choice = best
    if default is not None and best[2] != DEFAULT and not beats(best[:2], default[:2]):
        choice = default
    med, spread, cfg = choice
    entry = dict(cfg, us_per_order=round(med, 2), spread=round(spread, 2), candidates=len(results),
                 tune_seconds=round(time.time() - t0, 2))
    if default is not None:
        entry["default_us_per_order"] = round(default[0], 2)
        entry["default_spread"] = round(default[1], 2)
    table[key] = entry
    store_cache(table, cache)
    prob = make_problem(int(cfg["piece_size"]))
    prob.linearize(cams, lms)
    apply(prob, cfg)
    return dict(entry, cached=False, all=results), prob
