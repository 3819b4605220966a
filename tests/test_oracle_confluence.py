"""Uniform confluence (Proposition 2.1.1) and Theorem 1 of Section 2.2,
checked on the oracle: every order of the int steps reaches the same normal
form, interaction count and per-rule histogram; deferring sub/col to the end
changes nothing."""
import pytest

import oracle
from paper_1404_0076_amd import nets

R = nets.arith_rules()

TINY = [
    "<r | Add(y, r) = S(Z), Add(S(Z), y) = Z>",
    "<r | Mul(S(Z), r) = S(S(Z))>",
    "<r | Mul(S(S(Z)), r) = S(Z)>",
    "<p, q | Dup(p, q) = S(S(Z))>",
    "<r | Fib(r) = S(S(Z))>",
    "<r | Add(y, r) = S(S(Z)), Add(z, y) = S(Z), Add(Z, z) = Z>",
    "<r | Add(b, r) = a, Mul(S(Z), a) = S(Z), Fib(b) = S(Z)>",
]


@pytest.mark.parametrize("text", TINY)
def test_every_schedule_same_outcome(text):
    net = nets.parse_net(nets.ARITH_SIG, text)
    res = oracle.reduce(R, net, schedule="enumerate", max_interactions=300000)
    assert res.status == oracle.OK, res.status
    assert res.n_outcomes == 1
    assert res.n_schedules >= 1
    ref = oracle.reduce(R, net)
    assert res.nf.tolist() == ref.nf.tolist() and res.interactions == ref.interactions


@pytest.mark.parametrize("seed", range(12))
def test_random_expr_enumerated(seed):
    net = nets.random_expr_net(seed, budget=4, max_num=2, fib_budget=0)
    ref = oracle.reduce(R, net)
    if ref.interactions > 14:
        pytest.skip("too many interleavings to enumerate")
    res = oracle.reduce(R, net, schedule="enumerate", max_interactions=300000)
    assert res.status == oracle.OK and res.n_outcomes == 1
    assert res.nf.tolist() == ref.nf.tolist()


@pytest.mark.parametrize("seed", range(10))
def test_schedules_agree(seed):
    net = nets.random_expr_net(seed, budget=12, max_num=5)
    outs = []
    for sched, s in [("fifo", 0), ("lifo", 0), ("rounds", 0), ("random", 1), ("random", 99)]:
        for eager in (False, True):
            r = oracle.reduce(R, net, schedule=sched, seed=s, eager=eager)
            assert r.status == oracle.OK
            outs.append((r.nf.tolist(), r.interactions, r.per_rule.tolist()))
    assert all(o == outs[0] for o in outs)


def test_rounds_bounded_by_work():
    # a maximal parallel schedule needs at most one round per interaction and
    # at least one; Fib's critical path grows with its value
    for n in (3, 6, 9):
        r = oracle.reduce(R, nets.fib_net(n), schedule="rounds")
        assert 1 <= r.rounds <= r.interactions
    r1 = oracle.reduce(R, nets.fib_net(12), schedule="rounds").rounds
    r2 = oracle.reduce(R, nets.fib_net(14), schedule="rounds").rounds
    assert r2 > r1
