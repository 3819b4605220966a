"""Oracle pinned on the benchmark programs of Section 4.1 (our encodings of
Ackermann's function and of the algae L-System): values by the definition of
Ackermann's function and by plain string rewriting, interaction histograms by
recurrences derived by hand from the rule texts (tests/closed_forms.py)."""
import pytest

import oracle
from paper_1404_0076_amd import nets

from closed_forms import (ack_count, ack_per_rule, ack_value, algae_count, algae_per_rule,
                          algae_string, decode_letters)

ACK = nets.ackermann_rules()
ALGAE = nets.algae_rules()
CAT, LA, LB = (nets.ALGAE_SIG.label(s) for s in ("Cat", "La", "Lb"))


def test_ackermann_definition():
    # the reference values themselves: A(1, n) = n + 2, A(2, n) = 2n + 3,
    # A(3, n) = 2^(n+3) - 3
    for n in range(8):
        assert ack_value(0, n) == n + 1
        assert ack_value(1, n) == n + 2
        assert ack_value(2, n) == 2 * n + 3
        assert ack_value(3, n) == 2 ** (n + 3) - 3


@pytest.mark.parametrize("m,n", [(0, 0), (0, 5), (1, 0), (1, 3), (2, 0), (2, 2), (2, 3), (3, 0),
                                 (3, 1), (3, 2), (3, 3), (3, 5)])
def test_ackermann(m, n):
    res = oracle.reduce(ACK, nets.ackermann_net(m, n))
    assert res.status == oracle.OK
    assert oracle.decode_nat(res.nf, 0, 1) == ack_value(m, n)
    assert tuple(int(c) for c in res.per_rule) == ack_per_rule(m, n)
    assert res.interactions == ack_count(m, n)


@pytest.mark.parametrize("n", list(range(0, 13)))
def test_algae(n):
    res = oracle.reduce(ALGAE, nets.algae_net(n))
    assert res.status == oracle.OK
    assert decode_letters(res.nf, CAT, {LA: "a", LB: "b"}) == algae_string(n)
    assert tuple(int(c) for c in res.per_rule) == algae_per_rule(n)
    assert res.interactions == algae_count(n)


def test_algae_lengths_are_fibonacci():
    # |generation n| = F(n+2) with F(1) = F(2) = 1
    f = [0, 1, 1]
    while len(f) < 20:
        f.append(f[-1] + f[-2])
    for n in range(15):
        assert len(algae_string(n)) == f[n + 2]


@pytest.mark.parametrize("rules,net", [(ACK, nets.ackermann_net(2, 3)), (ACK, nets.ackermann_net(3, 2)),
                                       (ALGAE, nets.algae_net(9))])
def test_programs_schedule_independent(rules, net):
    ref = oracle.reduce(rules, net)
    for sched in ("lifo", "random", "rounds"):
        for eager in (False, True):
            res = oracle.reduce(rules, net, schedule=sched, seed=5, eager=eager)
            assert res.nf.tolist() == ref.nf.tolist()
            assert res.interactions == ref.interactions
            assert res.per_rule.tolist() == ref.per_rule.tolist()


def test_paper_sizes():
    # Ackermann(3,7) and L-System(27) as timed in Section 4.1, with our rules
    assert ack_count(3, 7) == 1_388_937
    assert algae_count(27) == 2_692_506


def test_paper_sizes_full():
    res = oracle.reduce(ACK, nets.ackermann_net(3, 7))
    assert res.status == oracle.OK and res.interactions == ack_count(3, 7)
    assert oracle.decode_nat(res.nf, 0, 1) == 1021
    res = oracle.reduce(ALGAE, nets.algae_net(27))
    assert res.status == oracle.OK and res.interactions == algae_count(27)
    assert tuple(int(c) for c in res.per_rule) == algae_per_rule(27)
    assert decode_letters(res.nf, CAT, {LA: "a", LB: "b"}) == algae_string(27)
