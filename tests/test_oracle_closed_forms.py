"""Oracle pinned to closed forms derived by hand from the rule texts
(tests/closed_forms.py) and to Python integer arithmetic for the values."""
import numpy as np
import pytest

import oracle
from paper_1404_0076_amd import nets

from closed_forms import (add_count, expr_count, expr_value, fib_count, fib_value, mul_count,
                          mul_per_rule, rhs_agent_counts, small_exprs, tree_count)

EXPRS = small_exprs(40, 10, 4, 300_000)

R = nets.arith_rules()
RULE_NAMES = ["Add><S", "Add><Z", "Mul><S", "Mul><Z", "Dup><S", "Dup><Z", "Era><S",
              "Era><Z", "Fib><Z", "Fib><S", "Fib2><Z", "Fib2><S"]


def _nat(res):
    return oracle.decode_nat(res.nf, nets.Z, nets.S)


@pytest.mark.parametrize("a,b", [(0, 0), (1, 0), (0, 1), (3, 5), (17, 4), (200, 31)])
def test_add(a, b):
    res = oracle.reduce(R, nets.add_net(a, b))
    assert res.status == oracle.OK
    assert res.interactions == add_count(a, b)
    assert _nat(res) == a + b


@pytest.mark.parametrize("a,b", [(0, 0), (1, 1), (2, 3), (3, 2), (7, 11), (40, 25), (120, 90)])
def test_mul(a, b):
    res = oracle.reduce(R, nets.mul_net(a, b))
    assert res.status == oracle.OK
    assert res.interactions == mul_count(a, b)
    assert _nat(res) == a * b
    hist = {RULE_NAMES[i]: int(c) for i, c in enumerate(res.per_rule)}
    assert hist == mul_per_rule(a, b)


@pytest.mark.parametrize("n", list(range(0, 13)) + [18])
def test_fib(n):
    res = oracle.reduce(R, nets.fib_net(n))
    assert res.status == oracle.OK
    assert res.interactions == fib_count(n)
    assert _nat(res) == fib_value(n)


def test_fib_config_sizes():
    # the four Fibonacci workload sizes
    assert [fib_count(n) for n in nets.FIB_CONFIG_NS] == [138336, 624526, 1702178, 4632088]
    assert [fib_value(n) for n in nets.FIB_CONFIG_NS] == [10946, 46368, 121393, 317811]


@pytest.mark.parametrize("k", [0, 1, 5, 40])
def test_dup_era(k):
    d = nets.NetBuilder(nets.ARITH_SIG)
    p, q = d.name(), d.name()
    d.eq(d.agent(nets.DUP, p, q), d.numeral(k))
    res = oracle.reduce(R, d.build())
    assert res.interactions == k + 1
    assert res.nf.tolist() == [2] + [nets.S] * k + [nets.Z] + [nets.S] * k + [nets.Z] + [0]
    e = nets.NetBuilder(nets.ARITH_SIG)
    e.eq(e.agent(nets.ERA), e.numeral(k))
    res = oracle.reduce(R, e.build())
    assert res.interactions == k + 1 and res.nf.tolist() == [0, 0]


@pytest.mark.parametrize("seed,leaves,vmax", [(0, 2, 5), (1, 8, 9), (2, 64, 30), (3, 256, 12)])
def test_add_tree(seed, leaves, vmax):
    net = nets.config1_add_tree(seed, n_leaves=leaves, vmax=vmax)
    vals = net.meta["values"]
    res = oracle.reduce(R, net)
    assert res.status == oracle.OK
    assert res.interactions == tree_count(vals)
    assert _nat(res) == sum(vals)


@pytest.mark.parametrize("seed,net", EXPRS, ids=[str(s) for s, _ in EXPRS])
def test_random_expressions(seed, net):
    e = net.meta["expr"]
    res = oracle.reduce(R, net)
    assert res.status == oracle.OK
    assert res.interactions == expr_count(e)
    assert _nat(res) == expr_value(e)


@pytest.mark.parametrize("net", [nets.fib_net(9), nets.mul_net(6, 7),
                                 small_exprs(1, 10, 4, 5000, min_count=500)[0][1]],
                         ids=["fib9", "mul6x7", "expr"])
def test_live_agent_balance(net):
    # every int removes its two agents and adds the agents of its right-hand
    # side, so live agents = initial + sum_r count_r * (|RHS_r| - 2)
    res = oracle.reduce(R, net)
    grow = np.asarray(rhs_agent_counts(nets.ARITH_RULE_TEXTS)) - 2
    assert res.final_live_agents == net.n_agents + int(np.dot(res.per_rule.astype(np.int64), grow))


@pytest.mark.slow
def test_config_sizes_full():
    net = nets.config1_add_tree(0)
    res = oracle.reduce(R, net)
    assert res.interactions == tree_count(net.meta["values"])
    assert _nat(res) == sum(net.meta["values"])
    net = nets.config2_mul(0)
    a, b = net.meta["a"], net.meta["b"]
    res = oracle.reduce(R, net)
    assert res.interactions == mul_count(a, b) and _nat(res) == a * b
