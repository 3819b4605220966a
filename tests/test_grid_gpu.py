"""GPU: the multi-workgroup engine of one net (workgroup 0 steps the net alone
while it is narrow; wider steps are shared by several workgroups with a
barrier between steps) against the oracle, bit-exact; the pointer-jumping
pass on long name chains; the barrier's give-up."""
import sys

import numpy as np
import pytest

import oracle
import paper_1404_0076_amd as P
from paper_1404_0076_amd import nets

from closed_forms import (algae_count, algae_per_rule, fib_count, mul_count, small_exprs,
                          tree_count)
from gpu_util import assert_same, oracle_run

pytestmark = pytest.mark.gpu
R = nets.arith_rules()
EMPTY = 0x7FFFFFFF

# thresholds low enough that the small nets below take shared steps: more
# than 64 active pairs hands the net over, 32 or fewer hands it back, and a
# shared step gives each workgroup about 48 pairs
FORCED = dict(grid_lo=32, grid_hi=64, grid_ppw=48)
ALWAYS = dict(grid_lo=1, grid_hi=1, grid_ppw=16)  # every step with two or more pairs is shared
# the smallest LDS tile: a workgroup's new pairs of a shared step overflow it,
# so the pairs past it go to the global queue and the tiles are flushed
# behind them before the next step
TILE = dict(grid_lo=32, grid_hi=64, grid_ppw=48, qcap=64)
ONE_WG = dict(grid=-1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu(rules, net, **kw):
    return P.reduce_net(rules, net, **kw)


def grid_used(rules, net, **kw):
    """Reduce once on a handle and report the largest frontier (to check
    that the forced thresholds were crossed)."""
    h = P.load(rules, net, agent_cap=max(4 * net.n_agents + 4096, 1 << 16), name_cap=1 << 20)
    h.set_config(**kw)
    res = h.reduce()[0]
    h.free()
    return res


SMALL_NETS = [nets.mul_net(30, 41), nets.fib_net(12), nets.config1_add_tree(3, 64, 30),
              nets.mul_net(120, 90), nets.fib_net(16),
              nets.parse_net(nets.ARITH_SIG, "<r, q | S(r) = Z, Add(q, y) = Fib(y)>")]


@pytest.mark.parametrize("cfg", [FORCED, ALWAYS, TILE], ids=["forced", "always", "tile"])
@pytest.mark.parametrize("wg", [256, 1024])
def test_grid_small_nets(cfg, wg):
    for net in SMALL_NETS + [n for _, n in small_exprs(8, 12, 5, 400_000)]:
        say("grid", cfg, wg, net.meta.get("family"))
        assert_same(gpu(R, net, wg_size=wg, **cfg), oracle_run(R, net), f"grid {cfg}")
    assert grid_used(R, nets.mul_net(120, 90), wg_size=wg, **cfg).max_frontier > 64


@pytest.mark.parametrize("cfg", [FORCED, ALWAYS, ONE_WG, TILE], ids=["forced", "always", "one", "tile"])
def test_grid_steps_equal_oracle_rounds(cfg):
    # a shared step reduces exactly the active pairs present after com has
    # run to closure, like a one-workgroup step: maximal parallel rounds
    for net in (nets.fib_net(10), nets.mul_net(40, 31), nets.config1_add_tree(1, 64, 20)):
        res, _, _ = gpu(R, net, **cfg)
        ref = oracle.reduce(R, net, schedule="rounds")
        say("rounds", cfg, res.steps, ref.rounds)
        assert res.steps == ref.rounds


def test_grid_other_rule_tables():
    from test_parity_gpu import OTHER_TABLES
    for name, sig, texts, cases in OTHER_TABLES:
        rules = nets.parse_rules(sig, texts)
        for net in cases:
            ref = oracle_run(rules, net)
            say("grid table", name, net.n_agents)
            for cfg in (FORCED, ALWAYS):
                assert_same(gpu(rules, net, **cfg), ref, f"{name} {cfg}")


def test_grid_resume_after_step_limit():
    net = nets.mul_net(60, 47)
    ref = oracle_run(R, net)
    h = P.load(R, net, agent_cap=1 << 16, name_cap=1 << 18)
    h.set_config(**FORCED)
    steps = 0
    for i in range(10000):
        res = h.reduce(max_steps=5)[0]
        if res.status != P.ELIMIT:
            break
        assert res.steps == steps + 5
        steps = res.steps
    assert res.status == P.OK and i > 3
    assert_same((res, h.readback(0), h.per_rule(0)), ref, "grid resume")
    h.free()


def test_grid_out_of_memory_reported():
    net = nets.mul_net(60, 60)
    h = P.load(R, net, agent_cap=net.n_agents + 600, name_cap=net.n_names + 600)
    h.set_config(**ALWAYS)
    res = h.reduce()[0]
    assert res.status == P.ENOMEM
    h.free()


def test_grid_barrier_gives_up():
    # a give-up of one microsecond without progress: the workgroups waiting
    # while workgroup 0 links and steps the net alone give up at once (its
    # first progress mark comes after 1024 steps); the kernel still ends and
    # the net reports INET_ETIMEDOUT
    net = nets.config1_add_tree(0, 1024, 64)
    h = P.load(R, net, agent_cap=1 << 20, name_cap=1 << 21)
    h.set_config(timeout_us=1)
    res = h.reduce()[0]
    assert res.status == P.ETIMEDOUT
    # the same handle, reset, with the default give-up: the oracle's result
    h.set_config()
    h.reset()
    res = h.reduce()[0]
    assert_same((res, h.readback(0), h.per_rule(0)), oracle_run(R, net), "after give-up")
    h.free()


# ---------------------------------------------------------------------------
# pointer jumping: long chains of name-to-name equations


def chain_sig():
    sig = nets.Signature(["A", "B", "C"], [1, 0, 0])
    return sig, nets.parse_rules(sig, ["A(r) = B -> r = C"])


def long_chain_net(length, free):
    """<r[, y] | A(r) = x0, x0 = x1, ..., x(L-1) = B | y>: a chain of L names
    from the active side to an agent or to a free name."""
    sig, _ = chain_sig()
    nb = nets.NetBuilder(sig)
    r = nb.name()
    y = nb.name() if free else None
    xs = [nb.name() for _ in range(length)]
    nb.eq(nb.agent("A", r), xs[0])
    for i in range(length - 1):
        nb.eq(xs[i], xs[i + 1])
    nb.eq(xs[-1], y if free else nb.agent("B"))
    return nb.build(family="chain", length=length, free=free)


def assert_one_hop(cells):
    """Every cell holding a name points at a name whose own cell is empty:
    every chain is one hop long after the pass."""
    c = np.asarray(cells, np.int64)
    named = c < 0
    tgt = -1 - c[named]
    assert np.all(c[tgt] == EMPTY), "a chain longer than one hop is left"


@pytest.mark.parametrize("length", [1000, 100_000])
@pytest.mark.parametrize("free", [False, True], ids=["agent", "free"])
@pytest.mark.parametrize("cfg", [{}, ONE_WG], ids=["grid", "one"])
def test_long_chains(length, free, cfg):
    _, rules = chain_sig()
    net = long_chain_net(length, free)
    ref = oracle_run(rules, net)
    say("long chain", length, free, cfg)
    h = P.load(rules, net, agent_cap=1 << 12, name_cap=length + 1024)
    h.set_config(**cfg)
    res = h.reduce()[0]
    assert_same((res, h.readback(0), h.per_rule(0)), ref, f"chain {length}")
    cells = h.cells(0)
    assert len(cells) == res.names_used
    assert_one_hop(cells)
    h.free()


def nested_add_net(length):
    """Add(r1, r0) = Z, Add(r2, r1) = Z, ..., Add(rL, r(L-1)) = Z, rL = S(Z):
    all L pairs are active at once, and their Add><Z links r(i-1) = ri form
    one chain of L names within a single step."""
    nb = nets.NetBuilder(nets.ARITH_SIG)
    rs = [nb.name() for _ in range(length + 1)]
    for i in range(length):
        nb.eq(nb.agent("Add", rs[i + 1], rs[i]), nb.agent("Z"))
    nb.eq(rs[length], nb.numeral(1))
    return nb.build(family="nested-add", length=length)


@pytest.mark.parametrize("length", [1000, 100_000])
@pytest.mark.parametrize("cfg", [{}, ONE_WG, ALWAYS], ids=["grid", "one", "always"])
def test_chain_within_one_step(length, cfg):
    net = nested_add_net(length)
    ref = oracle_run(R, net)
    say("one-step chain", length, cfg)
    h = P.load(R, net, agent_cap=2 * length + 4096, name_cap=2 * length + 4096)
    h.set_config(**cfg)
    res = h.reduce()[0]
    nf = h.readback(0)
    assert res.steps == 1 and res.interactions == length
    assert oracle.decode_nat(nf, 0, 1) == 1
    assert_same((res, nf, h.per_rule(0)), ref, f"nested add {length}")
    # the chain r0 -> r1 -> ... -> S(Z) parked in the cells is one hop after the pass
    assert_one_hop(h.cells(0))
    h.free()


def test_jump_in_batch_engines():
    # the batch kernel compresses each net's chains with its own workgroup
    _, crules = chain_sig()
    batch = [nested_add_net(n) for n in (10, 1000, 30_000)]
    refs = [oracle_run(R, n) for n in batch]
    for wg in (64, 1024):
        say("batch jump", wg)
        h = P.batch_load(R, batch, agent_caps=[2 * n.n_agents + 4096 for n in batch],
                         name_caps=[2 * n.n_names + 4096 for n in batch])
        h.set_config(wg_size=wg)
        rs = h.reduce()
        for i in range(len(batch)):
            assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"batch jump {i}")
            assert_one_hop(h.cells(i))
        h.free()


# ---------------------------------------------------------------------------
# full-size single nets through the multi-workgroup engine


@pytest.mark.slow
@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("cfg", [{}, FORCED, TILE,
                                 dict(grid=16, grid_lo=2048, grid_hi=2048, grid_ppw=128, qcap=8192)],
                         ids=["default", "forced", "tile", "g16-even"])
def test_grid_config2_mul_full(seed, cfg):
    net = nets.config2_mul(seed)
    a, b = net.meta["a"], net.meta["b"]
    say("grid config2", seed, a, b, cfg)
    g = gpu(R, net, agent_cap=a * b + 4 * (a + b) + 4096, name_cap=4 * a * b + 8 * (a + b) + 4096,
            **cfg)
    assert g[0].interactions == mul_count(a, b)
    assert_same(g, oracle_run(R, net), f"grid config2 seed {seed}")


@pytest.mark.slow
def test_grid_hand_offs_see_every_wave_s_stores():
    # regression: with 16 workgroups and equal hand-off thresholds, Mul hands
    # the net between workgroup 0 and the shared steps hundreds of times; once every wave's stores of an
    # epoch were not waited for before the workgroup barrier, a hand-off
    # could read queue entries another workgroup had not yet made visible
    net = nets.config2_mul(0)
    a, b = net.meta["a"], net.meta["b"]
    h = P.load(R, net, agent_cap=a * b + 4 * (a + b) + 4096, name_cap=4 * a * b + 8 * (a + b) + 4096)
    h.set_config(grid=16, grid_lo=2048, grid_hi=2048, grid_ppw=128, qcap=8192)
    for k in range(8):
        h.reset()
        res = h.reduce()[0]
        say("hand-offs", k, res.status, res.interactions)
        assert res.status == P.OK and res.n_stuck == 0 and res.interactions == mul_count(a, b)
    h.free()


# the single-net workloads at full size, each in the launch shape the
# benchmark takes from the tuned table on this device
TUNED_SINGLES = {
    "addtree": lambda: (R, nets.config1_add_tree(0)),
    "mul": lambda: (R, nets.config2_mul(0)),
    "fib27": lambda: (R, nets.config3_fib(27)),
    "algae27": lambda: (nets.algae_rules(), nets.algae_net(27)),
    "ackermann": lambda: (nets.ackermann_rules(), nets.ackermann_net(3, 7)),
}


@pytest.mark.slow
@pytest.mark.parametrize("which", list(TUNED_SINGLES))
def test_tuned_single_net_shapes(which):
    from paper_1404_0076_amd import autotune
    rules, net = TUNED_SINGLES[which]()
    best = autotune.lookup([net], autotune.SINGLE_SPACE)
    if best is None:
        pytest.skip("no tuned entry for this device")
    cfg = dict(best["config"])
    wg = cfg.pop("wg_size", 1024) or 1024
    say("tuned single", which, wg, cfg)
    g = gpu(rules, net, wg_size=wg, agent_cap=1 << 25, name_cap=1 << 26, **cfg)
    assert_same(g, oracle_run(rules, net), f"tuned single {which}")


@pytest.mark.slow
@pytest.mark.parametrize("cfg", [{}, FORCED], ids=["default", "forced"])
def test_grid_fib27_and_add_tree(cfg):
    net = nets.fib_net(27)
    say("grid fib 27", cfg)
    g = gpu(R, net, agent_cap=4 * fib_count(27), name_cap=8 * fib_count(27), **cfg)
    assert g[0].interactions == fib_count(27)
    assert_same(g, oracle_run(R, net), "grid fib 27")
    net = nets.config1_add_tree(0)
    say("grid add tree", cfg)
    g = gpu(R, net, agent_cap=1 << 20, name_cap=1 << 22, **cfg)
    assert g[0].interactions == tree_count(net.meta["values"])
    assert_same(g, oracle_run(R, net), "grid add tree")


# 64 workgroups of 512 lanes, full chunks, so the heap reservation is taken
# once per workgroup
ALGAE_512 = dict(wg_size=512, grid=64, grid_lo=256, grid_hi=1024, grid_ppw=256, qcap=8192)


@pytest.mark.slow
@pytest.mark.parametrize("cfg", [{}, FORCED, ONE_WG, TILE, ALGAE_512],
                         ids=["default", "forced", "one", "tile", "wg512"])
def test_grid_algae_27(cfg):
    rules = nets.algae_rules()
    net = nets.algae_net(27)
    say("grid algae 27", cfg)
    res, nf, pr = g = gpu(rules, net, **cfg)
    assert res.interactions == algae_count(27)
    assert tuple(int(c) for c in pr) == algae_per_rule(27)
    assert_same(g, oracle_run(rules, net), "grid algae 27")


@pytest.mark.slow
def test_grid_ackermann_3_7():
    rules = nets.ackermann_rules()
    net = nets.ackermann_net(3, 7)
    for cfg in ({}, FORCED):
        say("grid ackermann 3 7", cfg)
        assert_same(gpu(rules, net, **cfg), oracle_run(rules, net), f"A(3,7) {cfg}")


# ---------------------------------------------------------------------------
# the available-parallelism trace (active pairs per parallel step)


@pytest.mark.parametrize("cfg", [{}, ONE_WG, FORCED, dict(engine=2), dict(wg_size=64)],
                         ids=["grid", "one", "forced", "engine2", "wave"])
def test_parallelism_trace(cfg):
    for rules, net in ((R, nets.mul_net(40, 31)), (R, nets.fib_net(12)),
                       (nets.algae_rules(), nets.algae_net(14)),
                       (R, nets.parse_net(nets.ARITH_SIG, "<r, q | S(r) = Z, Add(q, y) = Fib(y)>"))):
        ref = oracle_run(rules, net)
        rounds = oracle.reduce(rules, net, schedule="rounds").rounds
        say("trace", cfg, net.meta.get("family"))
        tr = P.parallelism(rules, net, **cfg)
        res = gpu(rules, net, **cfg)[0]
        # one entry per parallel step (maximal rounds when no pair is left
        # without a rule: the oracle's rounds count reductions only), every
        # step reduces a pair, and every active pair is reduced once (or kept
        # as a residual)
        assert len(tr) == res.steps
        if ref.n_stuck == 0:
            assert res.steps == rounds
        assert np.all(tr > 0)
        assert int(tr.sum()) == ref.interactions + ref.n_stuck
        assert int(tr.max()) == res.max_frontier


def test_parallelism_of_the_algae_system():
    # generation n of A -> AB, B -> A: the widest step of our encoding is set
    # by the string lengths, a Fibonacci sequence; the trace grows with n
    rules = nets.algae_rules()
    peaks = [int(P.parallelism(rules, nets.algae_net(n)).max()) for n in (10, 14, 18)]
    assert peaks[0] < peaks[1] < peaks[2]
