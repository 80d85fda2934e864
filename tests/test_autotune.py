"""Host logic of the launch-shape autotuner: cache keys, the cache file, and
the choice among candidates (with an injected timer, so no GPU is needed)."""
import json

import pytest

from paper_2204_12834_amd import autotune


class FakeProblem:
    """Records the launch parameters applied to it."""

    def __init__(self, piece_size):
        self.piece_size = piece_size
        self.tuning = {}
        self.linearized = 0

    def linearize(self, cams, lms):
        self.linearized += 1

    def set_tuning(self, key, value):
        self.tuning[key] = value

    def config(self):
        return {"piece_size": self.piece_size, "tiles_per_wave": self.tuning["tiles_per_wave"],
                "lds_camera": self.tuning["lds_camera"]}


def timer_from(table, spread=0.5):
    """Samples around table[config] (microseconds per order), default 100."""

    def timer(prob):
        med = table.get(tuple(sorted(prob.config().items())), 100.0)
        return [med - spread, med - spread / 2, med, med, med + spread / 2, med + spread]

    return timer


def key(**cfg):
    return tuple(sorted(cfg.items()))


def _tune(tmp_path, timer, **kw):
    made = []

    def make(ps):
        made.append(FakeProblem(ps))
        return made[-1]

    cfg, prob = autotune.tune(make, "f32", 1 << 20, 1 << 17, None, None, cache=str(tmp_path / "tune.json"),
                              timer=timer, arch="gfx950", **kw)
    return cfg, prob, made


def test_shape_key_buckets():
    k = autotune.shape_key("f32", 4_936_708, 780_000, arch="gfx950")
    assert k == "gfx950|f32|N2^22|t5"
    # same buckets for nearby sizes, different ones across a factor of two
    assert autotune.shape_key("f32", 5_000_000, 790_000, arch="gfx950") == k
    assert autotune.shape_key("f32", 10_000_000, 780_000, arch="gfx950") != k
    assert autotune.shape_key("f64", 4_936_708, 780_000, arch="gfx950") != k
    assert autotune.shape_key("f32", 0, 0, arch="gfx950") == "gfx950|f32|N2^0|t0"


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    autotune.store_cache({"a": {"piece_size": 512}}, path)
    assert autotune.load_cache(path) == {"a": {"piece_size": 512}}
    with open(path, "w") as f:
        f.write("{not json")
    assert autotune.load_cache(path) == {}


def test_summary_and_margin():
    med, spread = autotune.summary([5.0, 1.0, 3.0, 2.0, 4.0])
    assert med == 3.0 and spread == 1.0
    assert autotune.summary([2.0, 4.0]) == (3.0, 1.0)
    assert autotune.beats((90.0, 1.0), (100.0, 1.0))
    assert not autotune.beats((99.0, 0.1), (100.0, 0.1))     # under 2%
    assert not autotune.beats((95.0, 3.0), (100.0, 3.0))     # within the spreads


def test_clear_winner_is_chosen_and_cached(tmp_path):
    table = {key(piece_size=512, tiles_per_wave=8, lds_camera=0): 70.0}
    cfg, prob, made = _tune(tmp_path, timer_from(table))
    assert (cfg["piece_size"], cfg["tiles_per_wave"], cfg["lds_camera"]) == (512, 8, 0)
    assert cfg["cached"] is False and cfg["candidates"] == 32
    assert prob.config() == {"piece_size": 512, "tiles_per_wave": 8, "lds_camera": 0}
    assert prob.linearized == 1
    stored = json.load(open(tmp_path / "tune.json"))
    assert stored["gfx950|f32|N2^20|t6"]["piece_size"] == 512
    # a second call takes the cache without timing anything
    def no_timer(prob):
        raise AssertionError("timed a cached shape")
    cfg2, prob2, made2 = _tune(tmp_path, no_timer)
    assert cfg2["cached"] is True and len(made2) == 1
    assert prob2.config() == prob.config()


def test_noise_keeps_the_default(tmp_path):
    # the fastest candidate is 1% ahead: not enough to leave the default
    table = {key(piece_size=2048, tiles_per_wave=1, lds_camera=0): 99.0}
    cfg, prob, _ = _tune(tmp_path, timer_from(table))
    d = autotune.DEFAULT
    assert (cfg["piece_size"], cfg["tiles_per_wave"], cfg["lds_camera"]) == (
        d["piece_size"], d["tiles_per_wave"], d["lds_camera"])
    assert prob.config() == d


def test_wide_spread_keeps_the_default(tmp_path):
    table = {key(piece_size=256, tiles_per_wave=2, lds_camera=1): 95.0}
    cfg, _, _ = _tune(tmp_path, timer_from(table, spread=8.0))
    assert cfg["piece_size"] == autotune.DEFAULT["piece_size"]


def test_force_retunes(tmp_path):
    table = {key(piece_size=256, tiles_per_wave=1, lds_camera=1): 50.0}
    _tune(tmp_path, timer_from(table))
    table2 = {key(piece_size=2048, tiles_per_wave=2, lds_camera=0): 40.0}
    cfg, _, _ = _tune(tmp_path, timer_from(table2), force=True)
    assert (cfg["piece_size"], cfg["tiles_per_wave"]) == (2048, 2)
