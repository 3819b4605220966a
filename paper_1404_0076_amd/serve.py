"""Continuous-batching driver over the C-ABI server (inet_server_*).

Requests (nets) arrive at given times.  The loop admits every arrived request
for which the server has a free slot and enough free device bytes (uploads go
on a separate stream, so they overlap the running round), launches a round
(every resident net advances by at most ``round_steps`` parallel steps),
harvests the nets that finished, and records each request's latency
(completion minus arrival, queueing included).  A request that ran out of its
capacities is resubmitted with larger ones.

``serve`` runs that loop here (it can keep every normal form, for checks);
``serve_native`` runs the same loop inside the library (inet_server_run),
with the request pool resident on the device and each round's admissions
installed by one launch, which is what the served measurements use.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import ENOMEM, OK, STUCK, Server


@dataclasses.dataclass
class Served:
    index: int
    arrival: float
    done: float
    status: int
    interactions: int
    steps: int
    nf: Optional[np.ndarray] = None
    per_rule: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class ServeReport:
    served: List[Served]
    wall: float
    rounds: int
    max_resident: int
    retries: int

    @property
    def interactions(self) -> int:
        return int(sum(s.interactions for s in self.served))

    def latency_ms(self, q: float) -> float:
        lat = np.array([s.latency for s in self.served]) * 1e3
        return float(np.percentile(lat, q)) if len(lat) else float("nan")


def serve(rules, pool: Sequence, arrivals: np.ndarray, pick: Sequence[int],
          caps: Optional[Sequence] = None, max_slots: int = 4096,
          workspace_bytes: int = 8 << 30, round_steps: int = 256, wg_size: int = 0,
          keep_results: bool = False, time_limit: float = 600.0,
          server: Optional[Server] = None) -> ServeReport:
    """Serve ``pool[pick[i]]`` arriving at ``arrivals[i]`` seconds (relative
    to the start).  ``caps[j] = (agent_cap, name_cap)`` for pool entry j, or
    None for the library defaults (4x growth, retried x8 on ENOMEM)."""
    import torch

    srv = server or Server(rules, max_slots, workspace_bytes)
    srv.set_config(wg_size=wg_size)
    compute = torch.cuda.current_stream()
    upload = torch.cuda.Stream()
    queue = collections.deque((float(arrivals[i]), int(pick[i]), None) for i in range(len(pick)))
    inflight: Dict[int, tuple] = {}
    served: List[Served] = []
    rounds = retries = max_res = 0
    t0 = time.perf_counter()

    def cap_of(j, boost):
        if caps is None:
            n = pool[j]
            a = max(1024, 16 * n.n_agents + 4096)
            return (a * boost, 4 * a * boost)
        a, m = caps[j]
        return (int(a) * boost, int(m) * boost)

    def admit(now):
        while queue and queue[0][0] <= now:
            arr, j, boost = queue[0]
            a, m = cap_of(j, boost or 1)
            t = srv.submit(pool[j], agent_cap=a, name_cap=m, stream=upload)
            if t is None:
                return
            queue.popleft()
            inflight[t] = (arr, j, boost or 1)

    while queue or inflight:
        now = time.perf_counter() - t0
        if now > time_limit:
            raise RuntimeError("serving did not finish within the time limit")
        admit(now)
        if not inflight:
            if queue:
                time.sleep(max(0.0, min(queue[0][0] - now, 0.01)))
            continue
        srv.step(round_steps, stream=compute)
        rounds += 1
        # arrivals during the round are admitted on the upload stream
        admit(time.perf_counter() - t0)
        max_res = max(max_res, len(inflight))
        for t in srv.poll(stream=compute):
            done = time.perf_counter() - t0
            arr, j, boost = inflight.pop(t)
            res, nf = srv.result(t, stream_out=keep_results)
            if res.status == ENOMEM:
                srv.release(t)
                retries += 1
                queue.appendleft((arr, j, boost * 8))
                continue
            pr = srv.per_rule(t) if keep_results else None
            served.append(Served(j, arr, done, res.status, res.interactions, res.steps, nf, pr))
            srv.release(t)
    wall = time.perf_counter() - t0
    if server is None:
        srv.free()
    return ServeReport(served, wall, rounds, max_res, retries)


def serve_native(rules, pool: Sequence, arrivals: np.ndarray, pick: Sequence[int],
                 caps: Optional[Sequence] = None, max_slots: int = 4096,
                 workspace_bytes: int = 8 << 30, round_steps: int = 256, wg_size: int = 0,
                 time_limit: float = 600.0, server: Optional[Server] = None,
                 per_rule: bool = False, want_nf=None, **config) -> ServeReport:
    """The serving loop of ``serve`` run by the library (inet_server_run).
    Results carry counters; with ``per_rule`` also the per-rule counts, and
    the normal forms of the requests flagged in ``want_nf``.  ``config``:
    further server configuration (``max_resident`` and the inet_config keys,
    e.g. ``round_scale``)."""
    import torch

    srv = server or Server(rules, max_slots, workspace_bytes)
    srv.set_config(wg_size=wg_size, **config)
    out = srv.run(pool, arrivals, pick, caps=caps, round_steps=round_steps,
                  time_limit=time_limit, stream=torch.cuda.current_stream(), per_rule=per_rule,
                  want_nf=want_nf)
    served = [Served(int(pick[i]), float(arrivals[i]), float(out["done"][i]), int(out["status"][i]),
                     int(out["interactions"][i]), int(out["steps"][i]),
                     out["nf"][i] if want_nf is not None else None,
                     out["per_rule"][i] if per_rule else None)
              for i in range(len(pick))]
    if server is None:
        srv.free()
    return ServeReport(served, out["wall"], out["rounds"], out["max_resident"], out["retries"])
