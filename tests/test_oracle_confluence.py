"""Uniform confluence (Proposition 2.1.1) and Theorem 1 of Section 2.2,
checked on the oracle: every order of the int steps reaches the same normal
form, interaction count and per-rule histogram; deferring sub/col to the end
changes nothing."""
import pytest

import oracle
from paper_1404_0076_amd import nets

from closed_forms import small_exprs

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


TINY_EXPRS = small_exprs(12, 4, 2, 12, min_count=2, fib_budget=0)
MID_EXPRS = small_exprs(10, 12, 5, 50_000, min_count=100)


@pytest.mark.parametrize("seed,net", TINY_EXPRS, ids=[str(s) for s, _ in TINY_EXPRS])
def test_random_expr_enumerated(seed, net):
    ref = oracle.reduce(R, net)
    res = oracle.reduce(R, net, schedule="enumerate", max_interactions=300000)
    assert res.status == oracle.OK and res.n_outcomes == 1
    assert res.nf.tolist() == ref.nf.tolist()


@pytest.mark.parametrize("seed,net", MID_EXPRS, ids=[str(s) for s, _ in MID_EXPRS])
def test_schedules_agree(seed, net):
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
