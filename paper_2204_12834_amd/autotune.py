"""Launch-shape autotuner for the series kernels.

A measurement loop over the launch parameters that change only the
floating-point summation order, never the result beyond it:

  piece_size      observations per camera-pass work item (set at creation)
  tiles_per_wave  64-observation landmark tiles walked by one wavefront (the
                  landmark pass that reads the camera vector from L2)
  lds_camera      landmark pass reads the camera vector from LDS or L2

Each candidate is timed on the problem itself (a few series orders with the
library's own event timing, best of several repetitions) and the fastest is
kept in a JSON cache keyed by (device architecture, precision, observation
count bucket, mean track length bucket), so later problems of the same shape
skip the search.  The cache file is `POBA_TUNE_CACHE` or
~/.cache/poba/tune.json.
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


def time_orders(problem, lam: float = 1e-2, orders: int = 8, reps: int = 3) -> float:
    """Microseconds per series order (landmark pass + camera pass + finish),
    best of `reps` solves of `orders` orders; the problem must be linearised."""
    best = math.inf
    problem.power_solve(lam, 1, 0.0)  # warm-up
    for _ in range(reps):
        problem.profile(True)
        problem.power_solve(lam, orders, 0.0)
        prof = problem.profile_read()
        problem.profile(False)
        t = prof["landmark_pass"][0] + prof["camera_pass"][0] + prof["camera_finish"][0]
        n = max(prof["landmark_pass"][1], 1)
        best = min(best, 1e3 * t / n)
    return best


def apply(problem, config: dict) -> None:
    problem.set_tuning("tiles_per_wave", int(config["tiles_per_wave"]))
    problem.set_tuning("lds_camera", int(config["lds_camera"]))


def tune(make_problem, precision: str, n_obs: int, n_lms: int, cams: torch.Tensor, lms: torch.Tensor,
         piece_sizes=PIECE_SIZES, tiles=TILES_PER_WAVE, lds=LDS_CAMERA, cache: str | None = None,
         force: bool = False, log=None) -> tuple[dict, object]:
    """Returns (config, problem): the best configuration for this shape and a
    handle created and tuned with it.  make_problem(piece_size) builds a
    handle; it is linearised at (cams, lms) here."""
    key = shape_key(precision, n_obs, n_lms)
    table = load_cache(cache)
    if not force and key in table:
        cfg = table[key]
        prob = make_problem(int(cfg["piece_size"]))
        prob.linearize(cams, lms)
        apply(prob, cfg)
        return dict(cfg, cached=True), prob
    t0 = time.time()
    results = []
    best = None
    for ps in piece_sizes:
        prob = make_problem(ps)
        prob.linearize(cams, lms)
        for tpw in tiles:
            for lc in lds:
                cfg = {"piece_size": ps, "tiles_per_wave": tpw, "lds_camera": lc}
                apply(prob, cfg)
                us = time_orders(prob)
                results.append(dict(cfg, us_per_order=round(us, 2)))
                if log:
                    log(f"[tune] {cfg} {us:.1f} us/order")
                if best is None or us < best[0]:
                    best = (us, cfg)
        del prob
        torch.cuda.empty_cache()
    us, cfg = best
    entry = dict(cfg, us_per_order=round(us, 2), candidates=len(results), tune_seconds=round(time.time() - t0, 2))
    table[key] = entry
    store_cache(table, cache)
    prob = make_problem(int(cfg["piece_size"]))
    prob.linearize(cams, lms)
    apply(prob, cfg)
    return dict(entry, cached=False, all=results), prob
