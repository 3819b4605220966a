"""Launch-shape autotuner for the net engines.

For a given workload (a list of nets), times the batched reduction for each
engine width (lanes per net engine, which also fixes the LDS frontier tile),
each engine variant and a few caps on resident engines, and keeps the fastest.
Results are cached in a JSON file keyed by the device name and a signature of
the workload, so a tuned configuration is reused across runs.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, Optional, Sequence

import numpy as np

from . import batch_load

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
WIDTHS = (64, 128, 256, 512, 1024)
ENGINES = (2, 3, 4)  # rule-uniform, rules compiled in, and that with atomic append
# (engine 1 is never faster)
# caps on resident engines: as many as fit, one per compute unit, or fewer
# (a batch whose time is one net's critical path runs that path a little
# faster with fewer engines beside it, as long as the others still finish
# within it)
RESIDENTS = (0, 64, 128, 256)


def workload_signature(net_list: Sequence) -> str:
    h = hashlib.sha256()
    for n in net_list:
        h.update(np.ascontiguousarray(n.label).tobytes())
        h.update(np.ascontiguousarray(n.port).tobytes())
        h.update(np.ascontiguousarray(n.eq_lhs).tobytes())
        h.update(np.ascontiguousarray(n.eq_rhs).tobytes())
    return h.hexdigest()[:16]


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


def tune(rules, net_list: Sequence, agent_caps, name_caps, order=None, reps: int = 2,
         widths=WIDTHS, engines=ENGINES, residents=RESIDENTS, cache: Optional[str] = CACHE,
         verbose: bool = False) -> Dict:
    """Best {"wg_size", "engine", "max_resident", "seconds"} for this workload."""
    import torch
    dev = torch.cuda.get_device_name(0)
    key = (f"{dev}/{workload_signature(net_list)}/{len(net_list)}/"
           f"{'-'.join(map(str, widths))}/{'-'.join(map(str, engines))}/{'-'.join(map(str, residents))}")
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            return table[key]
    else:
        table = {}
    h = batch_load(rules, net_list, agent_caps=agent_caps, name_caps=name_caps)
    if order is not None:
        h.set_order(order)
    best = None
    trials = []
    for wg in widths:
        for eng in engines:
            for res in residents:
                h.set_config(wg_size=wg, engine=eng, max_resident=res)
                t = _time(h, reps)
                trials.append({"wg_size": wg, "engine": eng, "max_resident": res, "seconds": t})
                if verbose:
                    print("autotune", trials[-1], flush=True)
                if best is None or t < best["seconds"]:
                    best = dict(trials[-1])
    h.free()
    best["trials"] = trials
    if cache:
        table[key] = best
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1)
        os.replace(tmp, cache)
    return best
