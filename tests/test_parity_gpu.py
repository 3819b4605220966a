"""GPU parity: the HIP evaluator (through the C ABI) against the CPU oracle,
element by element on the canonical normal-form stream, the interaction
count and the per-rule histogram (all integers: bit-exact)."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1404_0076_amd as P
from paper_1404_0076_amd import nets

from closed_forms import expr_count, fib_count, mul_count, small_exprs, tree_count
from gpu_util import assert_same, oracle_run

pytestmark = pytest.mark.gpu
R = nets.arith_rules()
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu(rules, net, wg=0, **kw):
    return P.reduce_net(rules, net, wg_size=wg, **kw)


def test_paper_examples():
    for case in json.load(open(GOLDEN))["cases"]:
        say("paper example", case["net"])
        rules = nets.add_rules()
        net = nets.parse_net(nets.ARITH_SIG, case["net"])
        res, nf, pr = gpu(rules, net)
        assert res.status == P.OK
        assert nf.tolist() == case["nf"]
        assert res.interactions == case["interactions"]
        assert_same((res, nf, pr), oracle_run(rules, net), case["net"])
        if "rounds" in case:
            assert res.steps == case["rounds"]


RESIDUALS = os.path.join(os.path.dirname(__file__), "golden", "residuals_and_cycles.json")


@pytest.mark.parametrize("engine", [0, 1, 2, 4])
def test_residuals_and_cycles(engine):
    # residual equations in the order and orientation worked out by hand, and
    # name cycles left out of the stream
    for case in json.load(open(RESIDUALS))["cases"]:
        say("residuals", engine, case["net"])
        net = nets.parse_net(nets.ARITH_SIG, case["net"])
        res, nf, pr = g = gpu(R, net, engine=engine)
        assert res.status == case["status"] and res.interactions == case["interactions"]
        assert res.n_stuck == case["n_stuck"]
        assert nf.tolist() == case["nf"]
        assert_same(g, oracle_run(R, net), case["net"])


SMALL = [
    "<r | Add(Z, r) = S(Z)>", "<r | Add(S(Z), r) = Z>", "<r | Mul(Z, r) = Z>",
    "<p, q | Dup(p, q) = Z>", "< | Era = Z>", "<r | Fib(r) = Z>", "<r | Fib2(r) = Z>",
    "< | Era = S(Z)>", "<p, q | Dup(p, q) = S(Z)>", "<r | Fib(r) = S(Z)>",
    "<r | Fib2(r) = S(Z)>", "<r | Mul(Z, r) = S(Z)>", "<r | S(r) = Z>", "<r | S(Z) = Add(Z, r)>",
    "<r, y | Add(y, r) = S(S(Z))>", "<r | Add(b, r) = a, Mul(S(Z), a) = S(Z), Fib(b) = S(Z)>",
]


@pytest.mark.parametrize("text", SMALL)
def test_small_nets(text):
    say("small", text)
    net = nets.parse_net(nets.ARITH_SIG, text)
    assert_same(gpu(R, net), oracle_run(R, net), text)


def test_chains():
    sig = nets.Signature(names=["A", "B", "C"], arity=[1, 0, 0])
    rules = nets.parse_rules(sig, ["A(r) = B -> r = C"])
    for length in (1, 2, 5, 40):
        links = ", ".join(f"x{i} = x{i+1}" for i in range(length - 1))
        for end in ("B", "y"):
            text = f"<r | A(r) = x0, {links + ', ' if links else ''}x{length - 1} = {end}>"
            say("chain", length, end)
            net = nets.parse_net(sig, text)
            assert_same(gpu(rules, net), oracle_run(rules, net), text)


def test_closed_loop():
    sig = nets.Signature(names=["P", "Q"], arity=[1, 1])
    rules = nets.parse_rules(sig, ["P(a) = Q(b) -> a = b"])
    net = nets.parse_net(sig, "< | P(x) = Q(x)>")
    res, nf, pr = gpu(rules, net)
    assert res.status == P.OK and res.interactions == 1 and nf.tolist() == [0, 0]


@pytest.mark.parametrize("a,b", [(0, 0), (1, 1), (3, 5), (17, 4), (40, 25), (120, 90)])
def test_mul(a, b):
    say("mul", a, b)
    net = nets.mul_net(a, b)
    g = gpu(R, net)
    assert g[0].interactions == mul_count(a, b)
    assert_same(g, oracle_run(R, net), f"mul {a} {b}")


@pytest.mark.parametrize("n", [0, 1, 2, 5, 9, 14])
def test_fib(n):
    say("fib", n)
    net = nets.fib_net(n)
    g = gpu(R, net)
    assert g[0].interactions == fib_count(n)
    assert_same(g, oracle_run(R, net), f"fib {n}")


EXPRS = small_exprs(30, 12, 5, 3_000_000)
MID = small_exprs(1, 12, 6, 20_000, min_count=5_000)[0][1]


@pytest.mark.parametrize("seed,net", EXPRS, ids=[str(s) for s, _ in EXPRS])
def test_random_expressions(seed, net):
    say("expr", seed, expr_count(net.meta["expr"]))
    assert_same(gpu(R, net), oracle_run(R, net), f"expr {seed}")


# rule tables other than arithmetic: the chain example of Section 3.6, a rule
# that wires its two arguments together, and a rule with five link equations
# (four argument links and an active pair between two new agents)
CHAIN_SIG = nets.Signature(["A", "B", "C"], [1, 0, 0])
LOOP_SIG = nets.Signature(["P", "Q"], [1, 1])
WIDE_SIG = nets.Signature(["P", "Q", "E", "F"], [2, 2, 0, 0])
WIDE_RULES = ["P(a, b) = Q(c, d) -> a = E, b = F, c = E, d = F, E = F", "E = F ->"]


def wide_net(k):
    # k pairs joined through names: x(i+1) links pair i to pair i+1, so every
    # pair's F meets the next pair's E after com; 3k - 1 interactions
    iface = ["x0"] + [f"r{i}, s{i}" for i in range(k)] + [f"x{k}"]
    eqs = [f"P(x{i}, r{i}) = Q(s{i}, x{i + 1})" for i in range(k)]
    return nets.parse_net(WIDE_SIG, f"<{', '.join(iface)} | {', '.join(eqs)}>")


def chain_net(length, free=False):
    links = "".join(f"x{i} = x{i + 1}, " for i in range(length - 1))
    end = "y" if free else "B"
    iface = "r, y" if free else "r"
    return nets.parse_net(CHAIN_SIG, f"<{iface} | A(r) = x0, {links}x{length - 1} = {end}>")


# rules whose right-hand side keeps x = C[x] (a fresh name parked at the top
# of an equation, its other occurrence inside C), next to ordinary links
CYCLE_SIG = nets.Signature(["P", "Q", "S", "Z", "D"], [1, 1, 1, 0, 2])
CYCLE_RULES = ["P(a) = Q(b) -> a = b, x = S(x)", "D(p, q) = Z -> p = Z, q = Z",
               "P(a) = Z -> y = D(y, a)"]


def cycle_net(k):
    # k rule applications of each kind, the results joined through names
    eqs, iface = [], []
    for i in range(k):
        eqs += [f"P(r{i}) = Q(s{i})", f"P(u{i}) = Z", f"D(v{i}, w{i}) = Z"]
        iface += [f"r{i}", f"s{i}", f"u{i}", f"v{i}", f"w{i}"]
    return nets.parse_net(CYCLE_SIG, f"<{', '.join(iface)} | {', '.join(eqs)}>")


OTHER_TABLES = [
    ("cycle", CYCLE_SIG, CYCLE_RULES, [cycle_net(1), cycle_net(5), cycle_net(200)]),
    ("chain", CHAIN_SIG, ["A(r) = B -> r = C"],
     [chain_net(1), chain_net(5), chain_net(40), chain_net(3, free=True)]),
    ("loop", LOOP_SIG, ["P(a) = Q(b) -> a = b"],
     [nets.parse_net(LOOP_SIG, "< | P(x) = Q(x)>"), nets.parse_net(LOOP_SIG, "<r, s | P(r) = Q(s)>")]),
    ("wide", WIDE_SIG, WIDE_RULES, [wide_net(1), wide_net(7), wide_net(300)]),
]


@pytest.mark.parametrize("engine", [1, 2, 3, 4])
@pytest.mark.parametrize("wg", [64, 1024])
def test_engines_agree(engine, wg):
    # every engine (per-lane interpreter, rule-uniform, rules compiled in at
    # load time, and that with per-lane atomic reservations) gives the
    # oracle's normal form, count and histogram
    for net in (nets.mul_net(30, 41), nets.fib_net(12), nets.config1_add_tree(3, 64, 30), MID,
                nets.parse_net(nets.ARITH_SIG, "<r, q | S(r) = Z, Add(q, y) = Fib(y)>")):
        say("engine", engine, wg, net.meta.get("family"))
        assert_same(gpu(R, net, wg=wg, engine=engine), oracle_run(R, net), f"engine {engine}")


@pytest.mark.parametrize("engine", [1, 2, 3, 4])
@pytest.mark.parametrize("name,sig,texts,cases", OTHER_TABLES, ids=[t[0] for t in OTHER_TABLES])
def test_other_rule_tables(engine, name, sig, texts, cases):
    rules = nets.parse_rules(sig, texts)
    for net in cases:
        ref = oracle_run(rules, net)
        say("table", name, engine, net.n_agents, ref.interactions)
        for wg in (64, 256):
            assert_same(gpu(rules, net, wg=wg, engine=engine), ref, f"{name} engine {engine}")
    if name == "wide":
        assert oracle_run(rules, wide_net(7)).interactions == 3 * 7 - 1


@pytest.mark.parametrize("engine", [1, 2, 3, 4])
def test_batch_engines_agree(engine):
    batch = [n for _, n in small_exprs(12, 12, 5, 200_000)] + \
            [nets.mul_net(5, 7), nets.fib_net(9), nets.config1_add_tree(2, 16, 12),
             nets.parse_net(nets.ARITH_SIG, "<r | S(r) = Z>")]
    refs = [oracle_run(R, net) for net in batch]
    caps = [net.n_agents + 4 * r.interactions + 1024 for net, r in zip(batch, refs)]
    say("batch engine", engine)
    h = P.batch_load(R, batch, agent_caps=caps, name_caps=[4 * c for c in caps])
    h.set_config(wg_size=64, engine=engine)
    assert h.get_config()["engine"] == engine
    rs = h.reduce()
    for i in range(len(batch)):
        assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"net {i}")
    h.free()


@pytest.mark.parametrize("wg", [64, 128, 256, 512, 1024])
def test_launch_shapes_agree(wg):
    # uniform confluence: the launch geometry changes the schedule only
    for net in (nets.mul_net(30, 41), nets.fib_net(12), nets.config1_add_tree(3, 64, 30),
                MID):
        say("shape", wg, net.meta.get("family"))
        assert_same(gpu(R, net, wg=wg), oracle_run(R, net), f"wg {wg}")


@pytest.mark.parametrize("engine", [0, 4])
def test_steps_equal_oracle_rounds(engine):
    # one GPU step reduces every active pair present after com has run to
    # closure: exactly the oracle's maximal parallel rounds
    for net in (nets.fib_net(10), nets.mul_net(12, 9), nets.config1_add_tree(1, 32, 20)):
        res, _, _ = gpu(R, net, engine=engine)
        ref = oracle.reduce(R, net, schedule="rounds")
        say("rounds", res.steps, ref.rounds)
        assert res.steps == ref.rounds


def test_stuck_residuals():
    for text in ("<r | S(r) = Z>", "<r, q | S(r) = Z, Add(q, y) = Fib(y)>"):
        say("stuck", text)
        net = nets.parse_net(nets.ARITH_SIG, text)
        g = gpu(R, net)
        assert g[0].status == P.STUCK
        assert_same(g, oracle_run(R, net), text)


def test_resume_after_step_limit():
    net = nets.fib_net(11)
    ref = oracle_run(R, net)
    h = P.load(R, net, agent_cap=1 << 16, name_cap=1 << 18)
    steps = 0
    for i in range(10000):
        res = h.reduce(max_steps=7)[0]
        if res.status != P.ELIMIT:
            break
        assert res.steps == steps + 7
        steps = res.steps
    assert res.status == P.OK
    assert_same((res, h.readback(0), h.per_rule(0)), ref, "resume")
    h.free()


@pytest.mark.parametrize("engine", [0, 4])
def test_out_of_memory_reported(engine):
    net = nets.mul_net(30, 30)
    h = P.load(R, net, agent_cap=net.n_agents + 8, name_cap=net.n_names + 8)
    h.set_config(engine=engine)
    res = h.reduce()[0]
    assert res.status == P.ENOMEM
    h.free()


def test_out_of_memory_in_a_wide_step_leaves_the_engine_usable():
    """An error found in a step that all waves of a 1024-lane engine share
    (the Add tree's first steps hold about 1,000 pairs, each making a fresh
    name cell, against a name heap 16 cells larger than the net) ends that
    net with ENOMEM; the one resident engine then takes the next nets, which
    must still match the oracle (every wave left the error step alike)."""
    wide = nets.config1_add_tree(0)
    others = [nets.mul_net(30, 41), nets.fib_net(12), nets.config1_add_tree(3, 64, 30)]
    refs = [oracle_run(R, n) for n in others]
    caps = [max(4 * n.n_agents + 4096, 1 << 16) for n in [wide] + others]
    ncaps = [wide.n_names + 16] + [4 * c for c in caps[1:]]
    h = P.batch_load(R, [wide] + others, agent_caps=caps, name_caps=ncaps)
    h.set_config(wg_size=1024, max_resident=1)
    rs = h.reduce()
    say("wide step out of memory", rs[0].status, rs[0].steps, rs[0].max_frontier)
    assert rs[0].status == P.ENOMEM and rs[0].max_frontier > 64
    for i, ref in enumerate(refs, 1):
        assert_same((rs[i], h.readback(i), h.per_rule(i)), ref, f"net {i} after the error")
    h.free()


def test_reset_repeats_exactly():
    net = MID
    ref = oracle_run(R, net)
    h = P.load(R, net, agent_cap=1 << 16, name_cap=1 << 18)
    for rep in range(3):
        h.reset()
        res = h.reduce()[0]
        assert_same((res, h.readback(0), h.per_rule(0)), ref, f"rep {rep}")
    h.free()


def test_batch_matches_single_and_oracle():
    batch = [n for _, n in small_exprs(40, 12, 5, 200_000)] + \
            [nets.mul_net(a, b) for a, b in ((5, 7), (0, 3), (9, 0))] + \
            [nets.fib_net(n) for n in (0, 3, 8, 11)] + \
            [nets.config1_add_tree(s, 16, 12) for s in range(4)] + \
            [nets.parse_net(nets.ARITH_SIG, "<r | S(r) = Z>")]
    refs = [oracle_run(R, net) for net in batch]
    caps = [net.n_agents + 4 * r.interactions + 1024 for net, r in zip(batch, refs)]
    for wg in (64, 256):
        say("batch", len(batch), "wg", wg)
        h = P.batch_load(R, batch, agent_caps=caps, name_caps=[4 * c for c in caps])
        h.set_config(wg_size=wg)
        rs = h.reduce()
        for i, net in enumerate(batch):
            assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"net {i}")
        h.free()


@pytest.mark.slow
@pytest.mark.parametrize("seed", range(5))
def test_config1_add_tree_full(seed):
    net = nets.config1_add_tree(seed)
    say("config1", seed, net.n_agents)
    g = gpu(R, net, agent_cap=1 << 20, name_cap=1 << 22)
    assert g[0].interactions == tree_count(net.meta["values"])
    assert_same(g, oracle_run(R, net), f"config1 seed {seed}")


@pytest.mark.slow
@pytest.mark.parametrize("seed", range(5))
def test_config2_mul_full(seed):
    net = nets.config2_mul(seed)
    a, b = net.meta["a"], net.meta["b"]
    say("config2", seed, a, b)
    g = gpu(R, net, agent_cap=a * b + 4 * (a + b) + 4096, name_cap=4 * a * b + 8 * (a + b) + 4096)
    assert g[0].interactions == mul_count(a, b)
    assert_same(g, oracle_run(R, net), f"config2 seed {seed}")


@pytest.mark.slow
@pytest.mark.parametrize("n", [20, 23, 25, 27])
def test_config3_fib_full(n):
    say("config3", n)
    net = nets.fib_net(n)
    g = gpu(R, net, agent_cap=4 * fib_count(n), name_cap=8 * fib_count(n))
    assert g[0].interactions == fib_count(n)
    assert_same(g, oracle_run(R, net), f"fib {n}")


@pytest.mark.slow
def test_config4_batch_full():
    """The 4096-net batch (seed 0): 1024-lane engines, one resident engine per
    compute unit, longest critical path first, heaps sized exactly, eagerly
    and by HIP-graph replay; then in the launch configuration the benchmark
    times (the tuned shape); every net against the oracle."""
    import torch
    batch = nets.config4_batch(seed=0)
    say("config4 oracle", len(batch))
    refs = [oracle_run(R, net) for net in batch]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    # sizing run: generous heaps (a rule makes at most 3 agents beyond the
    # pair's two slots and at most 8 fresh names)
    caps = [net.n_agents + 3 * r.interactions + 64 for net, r in zip(batch, refs)]
    ncaps = [net.n_names + 8 * r.interactions + 64 for net, r in zip(batch, refs)]
    say("config4 sizing run, resident", n_cu)
    h = P.batch_load(R, batch, agent_caps=caps, name_caps=ncaps)
    h.set_config(wg_size=1024, max_resident=n_cu)
    rs = h.reduce()
    used_a = np.array([r.agents_used for r in rs], np.int64)
    used_n = np.array([r.names_used for r in rs], np.int64)
    steps = np.array([r.steps for r in rs], np.int64)
    for i, net in enumerate(batch):
        assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"net {i}")
    h.free()
    say("config4 exact heaps, longest first")
    h = P.batch_load(R, batch, agent_caps=used_a + 64, name_caps=used_n + 64)
    h.set_config(wg_size=1024, max_resident=n_cu)
    h.set_order(np.argsort(-steps, kind="stable").astype(np.int32))
    h.reset()
    rs = h.reduce()
    for i in range(len(batch)):
        assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"exact heaps net {i}")
    say("config4 graph replay")
    h.graph_capture()
    for rep in range(2):
        h.graph_launch()
        torch.cuda.synchronize()
        rs = h.results()
        for i in range(len(batch)):
            assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"graph {rep} net {i}")
    h.free()
    # the shape the benchmark takes from the tuned table on this device
    from paper_1404_0076_amd import autotune
    best = autotune.lookup(batch, autotune.BATCH_SPACE)
    if best is None:
        say("config4: no tuned entry for this device")
        return
    say("config4 tuned shape", best["config"])
    h = P.batch_load(R, batch, agent_caps=used_a + 64, name_caps=used_n + 64)
    h.set_config(**best["config"])
    h.set_order(np.argsort(-steps, kind="stable").astype(np.int32))
    rs = h.reduce()
    for i in range(len(batch)):
        assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"tuned shape net {i}")
    h.free()
