"""Launch-shape autotuner for the net engines.

For a given workload (a list of nets, reduced by one launch), searches the
launch configuration one knob at a time (coordinate descent from the library
defaults, in the order of the space: each value of a knob is timed with the
others held, the fastest kept): engine width (lanes per net engine), engine
variant, cap on resident engines, LDS frontier tile, one-wave threshold, and
for a single net the multi-workgroup engine's thresholds.  Results are cached
in a JSON file keyed by the device name, a signature of the workload and the
searched space, so a tuned configuration is reused across runs;
``python -m paper_1404_0076_amd.autotune`` writes the tuned table for the
benchmark workloads (``TUNED``), which ``bench.py`` reads.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import batch_load

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")
TUNED = os.path.join(HERE, "tuned.json")

# the searched knobs, in search order (inet_config fields; 0 = library default)
BATCH_SPACE: List[Tuple[str, Tuple[int, ...]]] = [
    ("wg_size", (1024, 512, 256, 64)),
    ("engine", (3, 4, 2)),
    ("max_resident", (0, 256, 128, 64, 32, 16)),
    ("qcap", (0, 1024, 2048, 8192)),
    ("solo_max", (64, 32, 128, 256)),
]
SINGLE_SPACE: List[Tuple[str, Tuple[int, ...]]] = [
    ("wg_size", (1024, 512, 256)),
    ("grid", (0, -1, 64, 32, 16)),
    ("grid_hi", (2048, 1024, 512, 256, 4096)),
    ("grid_lo", (1024, 512, 256, 2048)),
    ("grid_ppw", (0, 256, 512, 128, 64, 2048)),
    ("qcap", (0, 2048, 8192)),
    ("solo_max", (64, 32, 128)),
]

def workload_signature(net_list: Sequence) -> str:
    h = hashlib.sha256()
    for n in net_list:
        h.update(np.ascontiguousarray(n.label).tobytes())
        h.update(np.ascontiguousarray(n.port).tobytes())
        h.update(np.ascontiguousarray(n.eq_lhs).tobytes())
        h.update(np.ascontiguousarray(n.eq_rhs).tobytes())
    return h.hexdigest()[:16]


def space_signature(space) -> str:
    return ";".join(f"{k}={'-'.join(map(str, v))}" for k, v in space)


def _time(h, reps: int) -> float:
    import torch
    h.reset()
    h.reduce_async()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        h.reset()
        h.reduce_async()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _valid(h, cfg) -> bool:
    """The configuration is accepted and its results are complete."""
    from . import InetError
    try:
        h.set_config(**cfg)
        h.reset()
        rs = h.reduce()
    except InetError:
        return False
    return all(r.status >= 0 for r in rs)


def _load_table(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path, key, value):
    table = _load_table(path)
    table[key] = value
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_signature() -> str:
    """The device a tuned entry holds for: ISA and compute-unit count (the
    marketing name is not reported the same way on every host and under
    every tool)."""
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{p.gcnArchName.split(':')[0]}x{p.multi_processor_count}"


def key_for(net_list, space) -> str:
    return f"{device_signature()}/{workload_signature(net_list)}/{len(net_list)}/{space_signature(space)}"


def lookup(net_list, space, path: str = TUNED) -> Optional[Dict]:
    """The tuned entry for this workload and space on this device, if any."""
    return _load_table(path).get(key_for(net_list, space))


def tune(rules, net_list: Sequence, agent_caps, name_caps, order=None, reps: int = 2,
         space=None, cache: Optional[str] = CACHE, verbose: bool = False,
         passes: int = 2) -> Dict:
    """Best configuration for this workload: {"config": {...}, "seconds",
    "trials"}; ``config`` holds every searched knob (set_config keywords).
    Coordinate descent: one knob at a time over its values, the others held at
    their best so far, repeated over all knobs up to ``passes`` times (a pass
    that changes nothing ends the search; a configuration is timed once)."""
    if space is None:
        space = BATCH_SPACE if len(net_list) > 1 else SINGLE_SPACE
    key = key_for(net_list, space)
    if cache:
        hit = _load_table(cache).get(key)
        if hit:
            return hit
    h = batch_load(rules, net_list, agent_caps=agent_caps, name_caps=name_caps)
    if order is not None:
        h.set_order(order)
    cur = {k: vals[0] for k, vals in space}
    trials = []
    best_t = None
    for _ in range(max(1, passes)):
        before = dict(cur)
        for k, vals in space:
            best_v = cur[k]
            for v in vals:
                cfg = dict(cur, **{k: v})
                if any(t["config"] == cfg for t in trials):
                    t = next(t["seconds"] for t in trials if t["config"] == cfg)
                elif not _valid(h, cfg):
                    continue
                else:
                    t = _time(h, reps)
                    trials.append({"config": cfg, "seconds": t})
                    if verbose:
                        print("autotune", trials[-1], flush=True)
                if best_t is None or t < best_t:
                    best_t, best_v = t, v
            cur[k] = best_v
        if cur == before:
            break
    h.free()
    best = {"config": cur, "seconds": best_t, "trials": trials}
    if cache:
        _store(cache, key, best)
    return best


def main():
    """Tune the benchmark's workloads on this GPU and write TUNED."""
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import bench
    import paper_1404_0076_amd as P
    from . import nets
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TUNED)
    ap.add_argument("--only", default="", help="comma-separated workload names")
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    A = nets.arith_rules()
    work = {"batch": (A, nets.config4_batch(seed=0)),
            "addtree": (A, [nets.config1_add_tree(0)]),
            "mul": (A, [nets.config2_mul(0)]),
            "fib27": (A, [nets.config3_fib(27)]),
            "algae27": (nets.algae_rules(), [nets.algae_net(27)]),
            "ackermann": (nets.ackermann_rules(), [nets.ackermann_net(3, 7)])}
    only = [w for w in args.only.split(",") if w]
    for name, (R, net_list) in work.items():
        if only and name not in only:
            continue
        space = BATCH_SPACE if len(net_list) > 1 else SINGLE_SPACE
        print("tuning", name, flush=True)
        ua, un, steps, _ = bench.size_batch(P, R, net_list, 1024)
        order = np.argsort(-steps, kind="stable").astype(np.int32)
        best = tune(R, net_list, ua + 64, un + 64, order=order, reps=args.reps, space=space,
                    cache=None, verbose=True)
        best["workload"] = name
        _store(args.out, key_for(net_list, space), best)
        print("tuned", name, best["config"], best["seconds"], flush=True)


if __name__ == "__main__":
    main()
