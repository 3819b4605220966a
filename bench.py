#!/usr/bin/env python3
"""Benchmark: interactions/s of the MI355X interaction-net evaluator.

A step is one pass of the whole hot path over one batch of synthetic input:
restore the loaded nets (device to device), reduce every net to normal form
(int/com step loop, pointer jumping), with the inputs resident in HBM.

Default workload: 4096 independent nets (Add trees, Mul, Fib; lognormal sizes,
seed 0) reduced by one persistent launch; the same line carries the plain
single-net evaluator on the three single-net workloads (single_net_configs) and
the served stream at two arrival rates (served).  --workload
mul|fib|addtree|ackermann|algae times one net instead, --workload serve one
served rate.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "interactions/sec (single net vs batched/served) + p50/p99 net latency, 1 MI355X"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ["paper_1404_0076_amd/csrc/device.h", "paper_1404_0076_amd/csrc/kernels.hip",
                  "paper_1404_0076_amd/csrc/inet_internal.h", "paper_1404_0076_amd/csrc/jit.cpp"]


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(workload_key: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (profiles/*_hbm.txt), if one was taken with the current kernel sources on
    this workload (else None)."""
    import glob
    want = kernel_sources_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm.txt"))):
        meta = {}
        for line in open(path):
            if line.startswith("# ") and ":" in line:
                k, v = line[2:].split(":", 1)
                meta[k.strip()] = v.strip()
        if meta.get("kernel_sources_sha256") != want or meta.get("workload_key") != workload_key:
            continue
        try:
            return float(meta["traffic_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    return None


def kernel_name(engine: int, wg: int) -> str:
    """Name of the reduce kernel as the profiler lists it."""
    return f"inet_static_{wg}" if engine >= 3 else "k_reduce"


def size_batch(P, R, net_list, wg, engine=0):
    """Find exact heap needs (agents and name cells are deterministic: they
    depend only on the per-rule counts) by reducing once with growing caps."""
    n = len(net_list)
    acap = np.array([max(1024, 16 * x.n_agents + 4096) for x in net_list], dtype=np.int64)
    ncap = 4 * acap
    used_a = np.zeros(n, np.int64)
    used_n = np.zeros(n, np.int64)
    steps = np.zeros(n, np.int64)
    inter = np.zeros(n, np.int64)
    pending = list(range(n))
    for _ in range(8):
        if not pending:
            break
        h = P.batch_load(R, [net_list[i] for i in pending], agent_caps=acap[pending],
                         name_caps=ncap[pending])
        h.set_config(wg_size=wg, engine=engine)
        rs = h.reduce()
        h.free()
        again = []
        for j, i in enumerate(pending):
            r = rs[j]
            if r.status == P.ENOMEM:
                acap[i] *= 8
                ncap[i] *= 8
                again.append(i)
            elif r.status in (P.OK, P.STUCK):
                used_a[i], used_n[i] = r.agents_used, r.names_used
                steps[i], inter[i] = r.steps, r.interactions
            else:
                raise RuntimeError(f"net {i}: status {r.status}")
        pending = again
    if pending:
        raise RuntimeError(f"{len(pending)} nets did not fit")
    return used_a, used_n, steps, inter


def cpu_baseline(R, net_list, seconds):
    import oracle
    t0 = time.perf_counter()
    tot = 0
    k = 0
    while k < len(net_list) and time.perf_counter() - t0 < seconds:
        r = oracle.reduce(R, net_list[k])
        tot += r.interactions
        k += 1
    dt = time.perf_counter() - t0
    return {"value": tot / dt, "unit": "interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"first {k} of {len(net_list)} nets in launch order, {tot} interactions, "
                      f"{dt:.1f} s, single thread"}


_POOL_JOB = None  # (rules, nets) shared with forked workers


def _oracle_share(k, workers):
    import oracle
    R, net_list = _POOL_JOB
    return [(i, int(oracle.reduce(R, net_list[i]).interactions))
            for i in range(k, len(net_list), workers)]


def oracle_parallel(R, net_list, what="nets"):
    """The oracle over every net of ``net_list`` in independent processes, one
    per host core of this GPU's share (at most 16).  Runs before anything
    touches the GPU, so the workers are plain forks of a process without a GPU
    context.  Returns (baseline record, per-net interaction counts)."""
    import multiprocessing as mp
    global _POOL_JOB
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    workers = max(1, min(16, cores))
    _POOL_JOB = (R, net_list)
    counts = np.zeros(len(net_list), np.int64)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        for part in pool.starmap(_oracle_share, [(k, workers) for k in range(workers)]):
            for i, c in part:
                counts[i] = c
    dt = time.perf_counter() - t0
    _POOL_JOB = None
    tot = int(counts.sum())
    rec = {"value": tot / dt, "unit": "interactions/s", "cores": workers, "kind": "oracle",
           "sample": f"all {len(net_list)} {what}, {tot} interactions, {dt:.2f} s, "
                     f"{workers} processes (nets dealt round-robin)"}
    return rec, counts


def cpu_baseline_parallel(R, net_list):
    return oracle_parallel(R, net_list)[0]


def measure_served(P, R, pool, caps, ref_counts, rate, duration, round_steps=256, wg=0,
                   loop="native", round_scale=0):
    """Serve a Poisson stream (rate nets/s for duration s, seed 3) of requests
    drawn from ``pool`` with replacement (seed 4).  Latency = completion -
    arrival (queueing included); sustained rate = completed interactions over
    the loop's wall time.  The served interaction total is checked against
    ``ref_counts`` (per pool net) for the picked entries."""
    from paper_1404_0076_amd.serve import serve
    arrivals = nets_mod().poisson_arrivals(3, rate, duration)
    rng = np.random.Generator(np.random.PCG64(4))
    pick = rng.integers(0, len(pool), len(arrivals))
    log(f"serving {len(arrivals)} requests at {rate:g}/s")
    import torch
    if loop == "native":
        srv = P.Server(R, 8192, 48 << 30)
        srv.set_config(wg_size=wg, round_scale=round_scale)
        # a short untimed run first: the load-time compilation of the engine
        # for this launch shape would otherwise stall the first round while
        # arrivals queue up
        srv.run(pool, np.zeros(64), np.arange(64) % len(pool), caps=caps,
                round_steps=round_steps, time_limit=60.0, stream=torch.cuda.current_stream())
        res = srv.run(pool, arrivals, pick, caps=caps, round_steps=round_steps, time_limit=900.0,
                      stream=torch.cuda.current_stream())
        srv.free()
        status, inter_done = res["status"], res["interactions"].astype(np.int64)
        lat = (res["done"] - arrivals) * 1e3
        rounds, wall, max_res = res["rounds"], res["wall"], res["max_resident"]
    else:
        rep = serve(R, pool, arrivals, pick, caps=caps, max_slots=8192, workspace_bytes=48 << 30,
                    round_steps=round_steps, wg_size=wg)
        status = np.array([x.status for x in rep.served])
        inter_done = np.array([x.interactions for x in rep.served], dtype=np.int64)
        lat = np.array([x.latency for x in rep.served]) * 1e3
        rounds, wall, max_res = rep.rounds, rep.wall, rep.max_resident
    bad = int(np.sum((status != P.OK) & (status != P.STUCK)))
    if bad:
        raise RuntimeError(f"{bad} requests failed")
    total = int(inter_done.sum())
    want = int(ref_counts[pick].sum())
    if total != want:
        raise RuntimeError(f"served {total} interactions, the reference counts give {want}")
    return {"rate": rate, "duration_s": duration, "requests": int(len(arrivals)),
            "interactions": total, "sustained": total / wall, "offered": total / duration,
            "wall_s": wall, "rounds": int(rounds), "max_resident": int(max_res),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "loop": loop}


def nets_mod():
    from paper_1404_0076_amd import nets
    return nets


def served_pool(P, R, nets, pool_size, wg=64, pool=None):
    """The request pool and its exact capacities (one sizing pass)."""
    if pool is None:
        pool = nets.config5_pool(seed=2, n_nets=pool_size)
    log(f"sizing pool of {len(pool)}")
    used_a, used_n, steps, inter = size_batch(P, R, pool, wg)
    caps = list(zip(used_a + 64, used_n + 64))
    return pool, caps, inter


def bench_serve(args, P, R, nets, torch, pool_ref=None, pool=None):
    """Served workload: Poisson arrivals of nets drawn from the batch mix."""
    pool, caps, inter = served_pool(P, R, nets, args.pool, args.wg or 64, pool)
    ref, checked = inter, "the sizing pass"
    if pool_ref is not None:
        ref, checked = pool_ref[1], "the oracle"
    rec = measure_served(P, R, pool, caps, ref, args.rate, args.duration, args.round_steps,
                         args.wg, args.serve_loop, args.round_scale)
    out = {
        "metric": METRIC, "value": rec["sustained"], "unit": "interactions/s",
        "n_gpus": 1, "steps": rec["rounds"], "warmup": 0,
        "ms_per_step": rec["wall_s"] * 1e3 / max(1, rec["rounds"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"served: Poisson arrivals at {args.rate:g} nets/s for {args.duration:g} s "
                               f"from a pool of {len(pool)} nets (batch mix, seed 2)",
                   "round_steps": args.round_steps, "round_scale": args.round_scale,
                   "requests": rec["requests"],
                   "loop": args.serve_loop},
        "latency_ms": rec["latency_ms"],
        "offered_interactions_per_s": rec["offered"],
        "rounds": rec["rounds"], "max_resident": rec["max_resident"], "wall_s": rec["wall_s"],
        "interactions_checked_against": checked,
    }
    if pool_ref is not None:
        out["cpu_baseline"] = pool_ref[0]
    print(json.dumps(out), flush=True)


def time_single(P, R, net, wg=1024, reps=3, engine=0, **cfg):
    """The plain single-net evaluator on one net: exact capacities from a
    sizing pass, then ``reps`` timed restore + reduce runs.  Returns
    interactions/s over the wall time, the reduce kernel's mean time (HIP
    events on the launch stream) and the algorithmic-byte roofline fraction.
    ``cfg``: further launch tunables (the multi-workgroup engine's thresholds)."""
    import torch
    ua, un, st, it = size_batch(P, R, [net], wg, engine)
    hs = P.batch_load(R, [net], agent_caps=ua + 64, name_caps=un + 64)
    hs.set_config(wg_size=wg, engine=engine, **cfg)
    hs.reset(); hs.reduce_async(); torch.cuda.synchronize()
    kms = []
    t1 = time.perf_counter()
    for _ in range(reps):
        hs.reset()
        hs.reduce_async()
        kms.append(hs.last_kernel_ms())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / reps
    rs = hs.results()
    assert rs[0].interactions == int(it[0]), "interaction count changed between runs"
    alg = float(np.dot(hs.per_rule(0).astype(np.float64), hs.rule_bytes().astype(np.float64)))
    kmean = float(np.mean(kms))
    used = hs.get_config()
    hs.free()
    return {"value": float(it[0]) / dt, "ms": dt * 1000, "kernel_ms": kmean, "steps": int(st[0]),
            "interactions": int(it[0]), "wg_size": used["wg_size"], "engine": used["engine"],
            "max_frontier": int(rs[0].max_frontier),
            "config": {k: used[k] for k in P.CONFIG_KEYS if used[k]},
            "roofline_frac": alg / (kmean * 1e-3) / 1e9 / HBM_PEAK_GBS}


def bench_pipeline(args, P, R, net_list, workload, used_a, used_n, inter, steps, torch):
    """The paper's own evaluation loop (inet_reduce_pipeline) on the same nets,
    for comparison with the net engines (an ablation, not the headline)."""
    # the loop allocates every slot of an iteration before filtering, so give
    # it room beyond the engines' exact heap needs
    h = P.batch_load(R, net_list, agent_caps=used_a + 64, name_caps=used_n + 64)
    for _ in range(args.warmup):
        h.reset()
        h.reduce_pipeline()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h.reset()
        rs = h.reduce_pipeline()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bad = [i for i, r in enumerate(rs) if r.status not in (P.OK, P.STUCK)]
    if bad:
        raise RuntimeError(f"{len(bad)} nets failed, e.g. net {bad[0]} status {rs[bad[0]].status}")
    total = int(sum(r.interactions for r in rs))
    assert total == int(inter.sum()), "the pipeline's interaction count differs from the engine's"
    out = {
        "metric": METRIC, "value": total * args.steps / wall, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": dict(workload, evaluator="paper pipeline (dummies, filter, sort-based com)",
                       interactions_per_step=total),
        "iterations": int(max(r.steps for r in rs)), "engine_steps": int(steps.max()),
    }
    h.free()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch",
                    choices=["batch", "mul", "fib", "addtree", "serve", "ackermann", "algae"])
    ap.add_argument("--ack-m", type=int, default=3)
    ap.add_argument("--ack-n", type=int, default=7)
    ap.add_argument("--algae-n", type=int, default=27)
    ap.add_argument("--rate", type=float, default=1.0e4, help="serve: Poisson arrival rate (nets/s)")
    ap.add_argument("--duration", type=float, default=10.0, help="serve: seconds of arrivals")
    ap.add_argument("--pool", type=int, default=65536, help="serve: request pool size")
    ap.add_argument("--round-steps", type=int, default=256, help="serve: step budget per round")
    ap.add_argument("--round-scale", type=int, default=8,
                    help="serve: a round's budget grows with the running nets per engine, up to "
                         "this factor (inet_config.round_scale; 0: fixed rounds)")
    ap.add_argument("--serve-loop", default="native", choices=["native", "python"],
                    help="serve: the library's serving loop or the Python driver")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n-nets", type=int, default=4096)
    ap.add_argument("--fib-n", type=int, default=27)
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--max-resident", type=int, default=-1,
                    help="cap on simultaneously resident net engines (0: as many as fit; "
                         "default: one per compute unit for a batch)")
    ap.add_argument("--engine", type=int, default=0,
                    help="0 default, 1 interpreter, 2 rule-uniform, 3 rules compiled in at load time, "
                         "4 the same with per-lane atomic append")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the launch configuration now (cached) instead of reading the "
                         "tuned table (paper_1404_0076_amd/tuned.json)")
    ap.add_argument("--no-tuned", action="store_true",
                    help="use the library defaults, not the tuned table")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-net side measurements (Add tree, Mul, Fib(27))")
    ap.add_argument("--no-serve", action="store_true",
                    help="batch line: skip the served measurements")
    ap.add_argument("--serve-rates", default="1e4,1e5",
                    help="batch line: served arrival rates (nets/s), comma-separated")
    ap.add_argument("--serve-duration", type=float, default=10.0,
                    help="batch line: seconds of arrivals per served rate")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay measurement")
    ap.add_argument("--pipeline", action="store_true",
                    help="time the paper's own evaluation loop (ablation) instead of the engine")
    ap.add_argument("--print-kernel-hash", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (to scale HBM counters) and exit")
    args = ap.parse_args()
    if args.print_kernel_hash:
        print(kernel_sources_hash())
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (the nets of a "
              "batch are independent, so each GPU would reduce its own share of them)",
              file=sys.stderr)
        sys.exit(2)

    par_baseline = None
    pool_ref = None  # (oracle record, per-net interaction counts) of the served pool
    pool_nets = None
    want_serve = args.workload == "serve" or (args.workload == "batch" and not args.no_serve)
    if want_serve and not args.copy_calibration:
        from paper_1404_0076_amd import nets as _nets
        log(f"building the served pool ({args.pool} nets)")
        pool_nets = _nets.config5_pool(seed=2, n_nets=args.pool)
    if not args.no_cpu_baseline and not args.copy_calibration:
        # the oracle on all host cores, before the GPU is initialised
        from paper_1404_0076_amd import nets as _nets
        if args.workload == "batch":
            log("cpu baseline (parallel)")
            par_baseline = cpu_baseline_parallel(_nets.arith_rules(),
                                                 _nets.config4_batch(seed=args.seed, n_nets=args.n_nets))
        if want_serve:
            log("oracle over the served pool (parallel)")
            pool_ref = oracle_parallel(_nets.arith_rules(), pool_nets, what="pool nets")

    import torch

    import paper_1404_0076_amd as P
    from paper_1404_0076_amd import nets

    torch.cuda.set_device(0)
    if args.copy_calibration:
        x = torch.ones(args.copy_calibration, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration, "reps": 3}), flush=True)
        return
    R = nets.arith_rules()
    if args.workload == "ackermann":
        R = nets.ackermann_rules()
    elif args.workload == "algae":
        R = nets.algae_rules()
    if args.workload == "serve":
        return bench_serve(args, P, R, nets, torch, pool_ref, pool_nets)
    if args.workload == "batch":
        net_list = nets.config4_batch(seed=args.seed, n_nets=args.n_nets)
        workload = {"workload": f"batch of {args.n_nets} nets (Add tree / Mul / Fib mix, "
                                f"lognormal sizes median 2e3 interactions, seed {args.seed})",
                    "n_nets": args.n_nets, "seed": args.seed}
    elif args.workload == "mul":
        net_list = [nets.config2_mul(args.seed)]
        m = net_list[0].meta
        workload = {"workload": f"single net Mul(S^{m['a']} Z, S^{m['b']} Z), seed {args.seed}"}
    elif args.workload == "fib":
        net_list = [nets.config3_fib(args.fib_n)]
        workload = {"workload": f"single net Fib(S^{args.fib_n} Z)"}
    elif args.workload == "ackermann":
        net_list = [nets.ackermann_net(args.ack_m, args.ack_n)]
        workload = {"workload": f"single net Ackermann({args.ack_m},{args.ack_n}) "
                                f"(benchmark program of Section 4.1, our rules)"}
    elif args.workload == "algae":
        net_list = [nets.algae_net(args.algae_n)]
        workload = {"workload": f"single net algae L-System, generation {args.algae_n} "
                                f"(benchmark program of Section 4.1, our rules)"}
    else:
        net_list = [nets.config1_add_tree(args.seed)]
        workload = {"workload": f"single net: balanced Add tree over 1024 numerals in [0,256), "
                                f"seed {args.seed}"}
    # 1024-lane engines: all waves step together while a frontier is wide,
    # wave 0 alone (no barriers) while it is narrow
    wg = args.wg or 1024
    if args.max_resident < 0:
        # batch: one engine per compute unit (the longest net's engine then has
        # its CU to itself; the other engines still finish the rest within its
        # critical path); single nets: not applicable
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        args.max_resident = n_cu if len(net_list) > 1 else 0
    log(f"sizing {len(net_list)} nets (wg {wg})")
    used_a, used_n, steps, inter = size_batch(P, R, net_list, wg, args.engine)
    order = np.argsort(-steps, kind="stable").astype(np.int32)  # longest critical path first
    engine = args.engine
    extra = {}  # further tunables (LDS tile, one-wave threshold, multi-workgroup engine)
    tuned = None
    if not (args.wg or args.engine or args.no_tuned) or args.autotune:
        # the launch configuration the autotuner picked for this workload on
        # this device: from the committed table, or tuned now (--autotune)
        from paper_1404_0076_amd import autotune
        space = autotune.BATCH_SPACE if len(net_list) > 1 else autotune.SINGLE_SPACE
        best = (autotune.tune(R, net_list, used_a + 64, used_n + 64, order=order, space=space)
                if args.autotune else autotune.lookup(net_list, space))
        if best:
            tuned = dict(best["config"])
            cfg = dict(tuned)
            wg = cfg.pop("wg_size", wg) or wg
            engine = cfg.pop("engine", engine)
            if "max_resident" in cfg:
                args.max_resident = cfg.pop("max_resident")
            extra = cfg
            log(f"tuned: {tuned}")
        else:
            log("no tuned entry for this workload and device: library defaults")
    if args.pipeline:
        return bench_pipeline(args, P, R, net_list, workload, used_a, used_n, inter, steps, torch)
    h = P.batch_load(R, net_list, agent_caps=used_a + 64, name_caps=used_n + 64)
    h.set_config(wg_size=wg, engine=engine, max_resident=args.max_resident, **extra)
    h.set_order(order)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        h.reset()
        h.reduce_async()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        h.reset()
        ev[k][1].record(stream)
        h.reduce_async()
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rs = h.results()
    bad = [i for i, r in enumerate(rs) if r.status not in (P.OK, P.STUCK)]
    if bad:
        raise RuntimeError(f"{len(bad)} nets failed, e.g. net {bad[0]} status {rs[bad[0]].status}")
    total = int(sum(r.interactions for r in rs))
    assert total == int(inter.sum()), "interaction count changed between runs"
    kern_ms = np.array([ev[k][1].elapsed_time(ev[k][2]) for k in range(args.steps)])
    reset_ms = np.array([ev[k][0].elapsed_time(ev[k][1]) for k in range(args.steps)])
    ms_per_step = wall * 1000.0 / args.steps
    value = total * args.steps / wall
    # algorithmic bytes: per-rule counts x bytes per interaction of each rule
    rb = h.rule_bytes().astype(np.float64)
    alg = 0.0
    for i in range(len(net_list)):
        alg += float(np.dot(h.per_rule(i).astype(np.float64), rb))
    kmean = float(kern_ms.mean())
    wkey = f"{args.workload}/{args.n_nets}/{args.seed}/wg{wg}/engine{h.get_config()['engine']}"
    if any(extra.values()):
        wkey += "/" + ",".join(f"{k}{v}" for k, v in sorted(extra.items()) if v)
    achieved = alg / (kmean * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "interactions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic", "config": dict(workload, wg_size=wg, engine=h.get_config()["engine"],
                                            max_resident=args.max_resident,
                                            interactions_per_step=total,
                                            tuned=tuned is not None,
                                            **{k: v for k, v in extra.items() if v}),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counter_traffic(wkey),
                     "kernel": kernel_name(h.get_config()["engine"], wg), "kernel_ms": kmean,
                     "algorithmic_bytes": alg, "workload_key": wkey},
        "reset_ms": float(reset_ms.mean()),
        "max_steps_per_net": int(steps.max()),
    }
    if not args.no_graph:
        # the same step (restore + reduce + jump) captured once as a HIP graph
        # and replayed: the whole batch as one graph launch per step
        h.graph_capture()
        h.graph_launch(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            h.graph_launch(stream)
        torch.cuda.synchronize()
        gwall = time.perf_counter() - t0
        gtot = int(sum(r.interactions for r in h.results()))
        assert gtot == total, "graph replay changed the interaction count"
        out["graph"] = {"value": gtot * args.steps / gwall, "ms_per_step": gwall * 1e3 / args.steps}
    h.free()
    if args.workload == "batch" and not args.no_single:
        # the plain single-net evaluator on the same GPU: the three single-net
        # workloads (Add tree seed 0, Mul seed 0, Fib(27))
        singles = {}
        for key, net, what in (
                ("addtree", nets.config1_add_tree(0), "balanced Add tree over 1024 numerals in [0,256), seed 0"),
                ("mul", nets.config2_mul(0), None),
                ("fib27", nets.config3_fib(27), "Fib(S^27 Z)")):
            if what is None:
                what = f"Mul(S^{net.meta['a']} Z, S^{net.meta['b']} Z), seed 0"
            log(f"single net {key}")
            best = None
            if not args.no_tuned:
                from paper_1404_0076_amd import autotune
                best = autotune.lookup([net], autotune.SINGLE_SPACE)
            cfg = dict(best["config"]) if best else {}
            wg1 = cfg.pop("wg_size", 1024) or 1024
            rec = time_single(P, R, net, wg=wg1, **cfg)
            rec["workload"] = what
            rec["tuned"] = best is not None
            singles[key] = rec
        out["single_net_configs"] = singles
        out["single_net"] = dict(singles["mul"])
    if args.workload == "batch" and not args.no_serve:
        pool, caps, inter_pool = served_pool(P, R, nets, args.pool, pool=pool_nets)
        ref = inter_pool if pool_ref is None else pool_ref[1]
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        out["served"] = {
            "workload": f"Poisson arrivals from a pool of {len(pool)} nets (batch mix, seed 2), "
                        f"native serving loop, {args.round_steps} steps per round "
                        f"(up to {max(1, args.round_scale)}x under load)",
            "interactions_checked_against": "the sizing pass" if pool_ref is None else "the oracle",
            "rates": [measure_served(P, R, pool, caps, ref, rate, args.serve_duration,
                                     args.round_steps, round_scale=args.round_scale)
                      for rate in rates]}
        if pool_ref is not None:
            out["served"]["cpu_baseline"] = pool_ref[0]
    if not args.no_cpu_baseline:
        ordered = [net_list[i] for i in order] if args.workload == "batch" else net_list
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(R, ordered, args.cpu_seconds)
    if par_baseline is not None:
        out["cpu_baseline_parallel"] = par_baseline
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
