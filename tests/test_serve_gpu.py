"""GPU: hipGraph replay of a batched step, and continuous batching -- every
served result equals the oracle's and the result of the same net reduced
alone, whatever else was resident."""

import numpy as np
import pytest

import oracle
import paper_1404_0076_amd as P
from paper_1404_0076_amd import nets
from paper_1404_0076_amd.serve import serve, serve_native

from closed_forms import fib_count, mul_count, small_exprs, tree_count
from gpu_util import assert_same, oracle_run

pytestmark = pytest.mark.gpu
R = nets.arith_rules()


def say(*a):
    print(*a, flush=True)


def pool_net_count(net) -> int:
    m = net.meta
    if m["family"] == "mul":
        return mul_count(m["a"], m["b"])
    if m["family"] == "fib":
        return fib_count(m["n"])
    return tree_count(m["values"])


def _pool():
    pool = [n for _, n in small_exprs(60, 12, 5, 100_000)]
    pool += [nets.fib_net(n) for n in (3, 7, 10, 12)] + [nets.mul_net(a, b) for a, b in
                                                         ((3, 4), (20, 31), (0, 5), (40, 2))]
    pool += [nets.config1_add_tree(s, 32, 20) for s in range(4)]
    pool += [nets.parse_net(nets.ARITH_SIG, "<r | S(r) = Z>")]
    return pool


def test_graph_replay_matches_eager():
    import torch
    batch = [n for _, n in small_exprs(30, 12, 5, 50_000)] + [nets.fib_net(9), nets.mul_net(11, 13)]
    refs = [oracle_run(R, n) for n in batch]
    caps = [n.n_agents + 4 * r.interactions + 1024 for n, r in zip(batch, refs)]
    h = P.batch_load(R, batch, agent_caps=caps, name_caps=[4 * c for c in caps])
    h.set_config(wg_size=64)
    h.graph_capture()
    for rep in range(3):
        say("graph replay", rep)
        h.graph_launch()
        rs = h.results()
        for i in range(len(batch)):
            assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"replay {rep} net {i}")
        # eager work of the program between replays
        h.reset()
        h.reduce()
        x = torch.ones(1 << 20, device="cuda").sum().item()
        assert x == float(1 << 20)
    h.free()


def test_served_equals_alone_and_oracle():
    pool = _pool()
    refs = [oracle_run(R, n) for n in pool]
    caps = [(n.n_agents + 4 * r.interactions + 1024, 4 * (n.n_agents + 4 * r.interactions + 1024))
            for n, r in zip(pool, refs)]
    rng = np.random.Generator(np.random.PCG64(3))
    pick = rng.integers(0, len(pool), 400)
    arrivals = np.cumsum(rng.exponential(1.0 / 20000.0, len(pick)))
    say("serving", len(pick), "requests")
    rep = serve(R, pool, arrivals, pick, caps=caps, max_slots=64, workspace_bytes=1 << 30,
                round_steps=16, keep_results=True)
    assert len(rep.served) == len(pick)
    assert rep.rounds > 1
    for s in rep.served:
        assert_same((P.Result(s.status, refs[s.index].n_stuck, s.interactions, s.steps, 0, 0, 0, 0),
                     s.nf, s.per_rule), refs[s.index], f"served net {s.index}")
    # the same nets alone, through the single-net path
    for j in sorted(set(int(p) for p in pick))[:20]:
        res, nf, pr = P.reduce_net(R, pool[j])
        served_j = next(s for s in rep.served if s.index == j)
        assert np.array_equal(nf, served_j.nf) and res.interactions == served_j.interactions
        assert res.steps == served_j.steps


def test_admission_by_free_bytes_and_retry():
    pool = [n for _, n in small_exprs(12, 12, 5, 20_000, min_count=2_000)]
    refs = [oracle_run(R, n) for n in pool]
    srv = P.Server(R, 8, 64 << 20)
    free0 = srv.stats()["free_bytes"]
    need = max(srv.net_bytes(n, n.n_agents + 4 * r.interactions + 1024,
                             4 * (n.n_agents + 4 * r.interactions + 1024)) for n, r in zip(pool, refs))
    assert need < free0
    # too-small capacities: every net first fails with ENOMEM and is retried
    caps = [(n.n_agents + 8, n.n_names + 8) for n in pool]
    pick = np.arange(len(pool))
    rep = serve(R, pool, np.zeros(len(pool)), pick, caps=caps, round_steps=64, keep_results=True,
                server=srv)
    assert rep.retries >= 1
    for s in rep.served:
        assert s.status == P.OK
        assert np.array_equal(s.nf, refs[s.index].nf) and s.interactions == refs[s.index].interactions
    assert srv.stats()["free_bytes"] == free0 and srv.stats()["running"] == 0
    srv.free()


def test_native_loop_matches_oracle():
    # the library's own serving loop: every request's status and interaction
    # count equal the oracle's and its step count the same net's reduced
    # alone, on a server that is reused for a second run
    pool = _pool()
    refs = [oracle.reduce(R, n) for n in pool]
    alone = [P.reduce_net(R, n)[0].steps for n in pool]
    caps = [(n.n_agents + 4 * r.interactions + 1024, 4 * (n.n_agents + 4 * r.interactions + 1024))
            for n, r in zip(pool, refs)]
    rng = np.random.Generator(np.random.PCG64(11))
    srv = P.Server(R, 64, 1 << 30)
    free0 = srv.stats()["free_bytes"]
    for run in range(2):
        pick = rng.integers(0, len(pool), 600)
        arrivals = np.cumsum(rng.exponential(1.0 / 30000.0, len(pick)))
        say("native serving", run, len(pick), "requests")
        rep = serve_native(R, pool, arrivals, pick, caps=caps, round_steps=16, server=srv)
        assert len(rep.served) == len(pick) and rep.rounds > 1
        for s in rep.served:
            ref = refs[s.index]
            assert s.status == ref.status and s.interactions == ref.interactions, s.index
            assert s.steps == alone[s.index], s.index
            assert s.done >= s.arrival
        assert srv.stats()["free_bytes"] == free0 and srv.stats()["running"] == 0
    srv.free()


def test_native_loop_with_scaled_rounds():
    # rounds whose budget grows with the running nets per engine (4 engines
    # for up to 64 running nets): the same results, fewer rounds
    pool = _pool()
    refs = [oracle.reduce(R, n) for n in pool]
    alone = [P.reduce_net(R, n)[0].steps for n in pool]
    caps = [(n.n_agents + 4 * r.interactions + 1024, 4 * (n.n_agents + 4 * r.interactions + 1024))
            for n, r in zip(pool, refs)]
    rng = np.random.Generator(np.random.PCG64(12))
    pick = rng.integers(0, len(pool), 600)
    arrivals = np.zeros(len(pick))
    rounds = {}
    for scale in (0, 8):
        srv = P.Server(R, 64, 1 << 30)
        say("native serving, round scale", scale)
        rep = serve_native(R, pool, arrivals, pick, caps=caps, round_steps=16, server=srv,
                           max_resident=4, round_scale=scale)
        assert len(rep.served) == len(pick)
        for s in rep.served:
            ref = refs[s.index]
            assert s.status == ref.status and s.interactions == ref.interactions, s.index
            assert s.steps == alone[s.index], s.index
        rounds[scale] = rep.rounds
        srv.free()
    assert rounds[8] < rounds[0]


def test_native_loop_retries_out_of_memory():
    pool = [n for _, n in small_exprs(12, 12, 5, 20_000, min_count=2_000)]
    refs = [oracle_run(R, n) for n in pool]
    caps = [(n.n_agents + 8, n.n_names + 8) for n in pool]
    pick = np.arange(len(pool))
    say("native retries", len(pool))
    rep = serve_native(R, pool, np.zeros(len(pool)), pick, caps=caps, max_slots=8,
                       workspace_bytes=256 << 20, round_steps=64)
    assert rep.retries >= 1
    for s in rep.served:
        assert s.status == P.OK and s.interactions == refs[s.index].interactions


def test_server_rejects_when_full():
    srv = P.Server(R, 2, 16 << 20)
    net = nets.fib_net(8)
    t1 = srv.submit(net, agent_cap=4096, name_cap=16384)
    t2 = srv.submit(net, agent_cap=4096, name_cap=16384)
    assert t1 is not None and t2 is not None
    assert srv.submit(net, agent_cap=4096, name_cap=16384) is None  # no free slot
    big = srv.net_bytes(net, agent_cap=1 << 22, name_cap=1 << 22)
    assert big > srv.stats()["free_bytes"]
    done = []
    while len(done) < 2:
        srv.step(1000)
        done += srv.poll()
    for t in done:
        res, nf = srv.result(t)
        assert res.status == P.OK and oracle.decode_nat(nf, 0, 1) == 34
        srv.release(t)
    assert srv.stats()["free_slots"] == 2
    srv.free()


def test_autotune_picks_a_valid_shape(tmp_path):
    from paper_1404_0076_amd import autotune
    batch = [n for _, n in small_exprs(24, 12, 5, 50_000)]
    refs = [oracle_run(R, n) for n in batch]
    caps = [n.n_agents + 4 * r.interactions + 1024 for n, r in zip(batch, refs)]
    cache = str(tmp_path / "tune.json")
    space = [("wg_size", (64, 256)), ("engine", (3, 4)), ("max_resident", (0, 64)),
             ("qcap", (0, 1024)), ("solo_max", (64, 32))]
    best = autotune.tune(R, batch, caps, [4 * c for c in caps], reps=1, space=space, cache=cache)
    cfg = best["config"]
    for k, vals in space:
        assert cfg[k] in vals
    assert 1 <= len(best["trials"]) <= sum(len(v) for _, v in space)
    again = autotune.tune(R, batch, caps, [4 * c for c in caps], space=space, cache=cache)
    assert again["config"] == cfg  # from the cache
    # the tuned shape still gives the oracle's results
    h = P.batch_load(R, batch, agent_caps=caps, name_caps=[4 * c for c in caps])
    h.set_config(**cfg)
    rs = h.reduce()
    for i in range(len(batch)):
        assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"tuned net {i}")
    h.free()
