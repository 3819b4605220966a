"""Host-side check of the autotuner's search (coordinate descent with
repeated passes) against a synthetic cost, with the device parts replaced."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1404_0076_amd import autotune  # noqa: E402

SPACE = [("a", (0, 1, 2)), ("b", (0, 1, 2))]


class FakeHandle:
    def __init__(self):
        self.cfg = None

    def set_config(self, **cfg):
        self.cfg = dict(cfg)

    def set_order(self, order):
        pass

    def free(self):
        pass


def run(cost, passes, monkeypatch, invalid=()):
    h = FakeHandle()
    monkeypatch.setattr(autotune, "batch_load", lambda *a, **k: h)
    monkeypatch.setattr(autotune, "key_for", lambda nl, sp: "k")

    def valid(hh, cfg):
        hh.set_config(**cfg)
        return (cfg["a"], cfg["b"]) not in invalid

    monkeypatch.setattr(autotune, "_valid", valid)
    timed = []

    def time_it(hh, reps):
        timed.append((hh.cfg["a"], hh.cfg["b"]))
        return cost[(hh.cfg["a"], hh.cfg["b"])]

    monkeypatch.setattr(autotune, "_time", time_it)
    best = autotune.tune(None, [None, None], 0, 0, space=SPACE, cache=None, passes=passes)
    return best, timed


def test_second_pass_leaves_a_first_pass_local_optimum(monkeypatch):
    # from (0, 0): knob a settles at 0 (b = 0), knob b then moves to 2; only
    # a second pass over a finds (2, 2), the best point
    cost = {(a, b): 10.0 for a in range(3) for b in range(3)}
    cost[(0, 0)] = 5.0
    cost[(0, 2)] = 4.0
    cost[(2, 2)] = 1.0
    one, _ = run(cost, 1, monkeypatch)
    assert one["config"] == {"a": 0, "b": 2} and one["seconds"] == 4.0
    two, timed = run(cost, 2, monkeypatch)
    assert two["config"] == {"a": 2, "b": 2} and two["seconds"] == 1.0
    assert len(timed) == len(set(timed))  # a configuration is timed once


def test_invalid_configurations_are_skipped(monkeypatch):
    cost = {(a, b): float(10 - a - b) for a in range(3) for b in range(3)}
    best, timed = run(cost, 2, monkeypatch, invalid={(2, 0), (2, 1), (2, 2)})
    assert best["config"] == {"a": 1, "b": 2}
    assert all(a != 2 for a, _ in timed)
