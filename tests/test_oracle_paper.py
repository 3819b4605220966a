"""Oracle pinned to the paper's worked examples, its chain cases, the
single-rule instances of the arithmetic system and input validation."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1404_0076_amd import nets

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")
RULE_NAMES = ["Add><S", "Add><Z", "Mul><S", "Mul><Z", "Dup><S", "Dup><Z", "Era><S",
              "Era><Z", "Fib><Z", "Fib><S", "Fib2><Z", "Fib2><S"]


def _rules(which):
    return nets.add_rules() if which == "add" else nets.arith_rules()


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["net"])
@pytest.mark.parametrize("schedule", ["fifo", "lifo", "rounds", "random"])
def test_paper_worked_examples(case, schedule):
    rules = _rules(case["rules"])
    net = nets.parse_net(nets.ARITH_SIG, case["net"])
    res = oracle.reduce(rules, net, schedule=schedule, seed=7)
    assert res.status == oracle.OK
    assert res.nf.tolist() == case["nf"]
    assert res.interactions == case["interactions"]
    hist = {RULE_NAMES[i]: int(c) for i, c in enumerate(res.per_rule) if c}
    assert hist == case["per_rule"]
    if "col" in case:
        assert res.n_col == case["col"]
    if "rounds" in case and schedule == "rounds":
        assert res.rounds == case["rounds"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["net"])
def test_equations_are_symmetric(case):
    # t = s is the same equation as s = t (Section 2.2): swap every side
    net = nets.parse_net(nets.ARITH_SIG, case["net"])
    flipped = nets.Net(net.label, net.port, net.eq_rhs.copy(), net.eq_lhs.copy(), net.n_names)
    res = oracle.reduce(_rules(case["rules"]), flipped)
    assert res.nf.tolist() == case["nf"] and res.interactions == case["interactions"]


def test_paper_example_parallel_step_commutes():
    # the remark after the 1 + (0 + 1) example: the step with the zero commutes
    # with the other two, so exactly three int orders exist, one outcome
    case = _cases()[1]
    res = oracle.reduce(_rules("add"), nets.parse_net(nets.ARITH_SIG, case["net"]),
                        schedule="enumerate")
    assert res.status == oracle.OK
    assert res.n_schedules == case["schedules"]
    assert res.n_outcomes == 1


def test_eager_sub_col_matches_paper_trace():
    # Section 2.2 Example 2 applies col eagerly between the two ints
    case = _cases()[0]
    res = oracle.reduce(_rules("add"), nets.parse_net(nets.ARITH_SIG, case["net"]), eager=True)
    assert res.nf.tolist() == case["nf"] and res.n_col == 2 and res.interactions == 2


# chain cases of Section 3.6: {A = x, x = y, y = B} needs two com steps before
# the active pair A = B exists; {A = x1, ..., xi = y} with y free stays a chain
CHAIN_SIG = nets.Signature(names=["A", "B", "C"], arity=[1, 0, 0])
CHAIN_RULES = ["A(r) = B -> r = C"]


@pytest.mark.parametrize("length", [1, 2, 3, 7])
def test_chain_yields_active_pair(length):
    links = ", ".join(f"x{i} = x{i+1}" for i in range(length - 1))
    text = f"<r | A(r) = x0, {links + ', ' if links else ''}x{length - 1} = B>"
    net = nets.parse_net(CHAIN_SIG, text)
    rules = nets.parse_rules(CHAIN_SIG, CHAIN_RULES)
    for sched in ("fifo", "lifo", "rounds"):
        res = oracle.reduce(rules, net, schedule=sched)
        assert res.status == oracle.OK
        assert res.interactions == 1
        assert res.nf.tolist() == [1, 2, 0]  # <C | >
        assert res.n_com == length  # one com per name of the chain
        if sched == "rounds":
            assert res.rounds == 1


@pytest.mark.parametrize("length", [1, 3, 6])
def test_chain_to_free_name_reads_back(length):
    links = ", ".join(f"x{i} = x{i+1}" for i in range(length - 1))
    text = f"<r, y | A(r) = x0, {links + ', ' if links else ''}x{length - 1} = y>"
    net = nets.parse_net(CHAIN_SIG, text)
    rules = nets.parse_rules(CHAIN_SIG, CHAIN_RULES)
    res = oracle.reduce(rules, net)
    assert res.status == oracle.OK and res.interactions == 0
    # interface (r, y): r is free inside A, y reads back as A(r)
    assert res.nf.tolist() == [2, -1, 0, -1, 0]


@pytest.mark.parametrize("rule,net_text,nf", [
    ("Add><S", "<r | Add(Z, r) = S(Z)>", [1, 1, 0, 0]),
    ("Add><Z", "<r | Add(S(Z), r) = Z>", [1, 1, 0, 0]),
    ("Mul><Z", "<r | Mul(Z, r) = Z>", [1, 0, 0]),
    ("Dup><Z", "<p, q | Dup(p, q) = Z>", [2, 0, 0, 0]),
    ("Era><Z", "< | Era = Z>", [0, 0]),
    ("Fib><Z", "<r | Fib(r) = Z>", [1, 1, 0, 0]),
    ("Fib2><Z", "<r | Fib2(r) = Z>", [1, 1, 0, 0]),
    ("Era><S", "< | Era = S(Z)>", [0, 0]),
    ("Dup><S", "<p, q | Dup(p, q) = S(Z)>", [2, 1, 0, 1, 0, 0]),
    ("Fib><S", "<r | Fib(r) = S(Z)>", [1, 1, 0, 0]),
    ("Fib2><S", "<r | Fib2(r) = S(Z)>", [1, 1, 1, 0, 0]),
    ("Mul><S", "<r | Mul(Z, r) = S(Z)>", [1, 0, 0]),
])
def test_each_rule_smallest_instance(rule, net_text, nf):
    res = oracle.reduce(nets.arith_rules(), nets.parse_net(nets.ARITH_SIG, net_text))
    assert res.status == oracle.OK
    assert res.nf.tolist() == nf
    assert res.per_rule[RULE_NAMES.index(rule)] >= 1


def test_stuck_pair_is_residual():
    # no rule for S><Z: the pair stays as a residual equation, oriented by the
    # name-erased encoding (Z sorts before S(..)), and is not counted
    res = oracle.reduce(nets.arith_rules(), nets.parse_net(nets.ARITH_SIG, "<r | S(r) = Z>"))
    assert res.status == oracle.STUCK
    assert res.interactions == 0 and res.n_stuck == 1
    assert res.nf.tolist() == [1, -1, 1, 0, 1, -1]


def test_closed_loop_dropped():
    # A(x) = B with A(r) = B -> r = C would leave C; here the rule wires the
    # two arguments together and the loop x = x disappears
    sig = nets.Signature(names=["P", "Q"], arity=[1, 1])
    rules = nets.parse_rules(sig, ["P(a) = Q(b) -> a = b"])
    net = nets.parse_net(sig, "< | P(x) = Q(x)>")
    res = oracle.reduce(rules, net)
    assert res.status == oracle.OK and res.interactions == 1 and res.n_loops == 1
    assert res.nf.tolist() == [0, 0]


def _net(label, port, eql, eqr, n_names):
    return nets.Net(np.asarray(label, np.int32), np.asarray(port, np.int32).reshape(-1, 2),
                    np.asarray(eql, np.int32), np.asarray(eqr, np.int32), n_names)


@pytest.mark.parametrize("bad", [
    _net([1, 0], [[-1, 0], [0, 0]], [0], [-1], 1),          # name used 3 times
    _net([1, 0], [[1, 0], [0, 0]], [0, 1], [-1, -2], 2),    # agent 1 referenced twice
    _net([1, 0], [[-1, 0], [0, 0]], [0], [-2], 2),          # agent 1 never referenced
    _net([9], [[0, 0]], [0], [-1], 1),                      # label out of range
    _net([1, 1], [[1, 0], [0, 0]], [-1], [-2], 2),          # cyclic nesting S(S(...))
    _net([0], [[0, 0]], [0], [-5], 1),                      # name id out of range
])
def test_invalid_nets_rejected(bad):
    res = oracle.reduce(nets.arith_rules(), bad)
    assert res.status == oracle.EINVAL


@pytest.mark.parametrize("texts", [
    ["Add(y,r) = S(x) -> Add(y,y) = x, r = S(w)"],           # argument used twice, x.. w once
    ["Add(y,r) = S(x) -> r = S(x)", "Add(a,b) = S(c) -> a = S(c), b = Z"],  # duplicate pair
    ["Add(y,r) = S(x) -> r = S(w), x = y"],                   # bound name used once
])
def test_invalid_rules_rejected(texts):
    rules = nets.parse_rules(nets.ARITH_SIG, texts)
    res = oracle.reduce(rules, nets.add_net(1, 1))
    assert res.status == oracle.EINVAL


def test_self_pair_rule_rejected():
    sig = nets.Signature(names=["A"], arity=[0])
    rules = nets.parse_rules(sig, ["A = A ->"])
    res = oracle.reduce(rules, nets.parse_net(sig, "< | A = A>"))
    assert res.status == oracle.EINVAL


def test_empty_net():
    res = oracle.reduce(nets.arith_rules(), _net(np.zeros(0), np.zeros((0, 2)), [], [], 0))
    assert res.status == oracle.OK and res.nf.tolist() == [0, 0] and res.interactions == 0
