"""GPU parity on the benchmark programs of Section 4.1 (our encodings of
Ackermann's function and of the algae L-System): the HIP evaluator against
the oracle, bit-exact, plus the values and histograms of the hand-derived
recurrences at the paper's sizes."""
import sys

import numpy as np
import pytest

import oracle
import paper_1404_0076_amd as P
from paper_1404_0076_amd import nets

from closed_forms import (ack_count, ack_per_rule, ack_value, algae_count, algae_per_rule,
                          algae_string, decode_letters)
from gpu_util import assert_same, oracle_run

pytestmark = pytest.mark.gpu
ACK = nets.ackermann_rules()
ALGAE = nets.algae_rules()
CAT, LA, LB = (nets.ALGAE_SIG.label(s) for s in ("Cat", "La", "Lb"))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("engine", [0, 1, 2, 4])
def test_ackermann(engine):
    for m, n in [(0, 0), (1, 3), (2, 3), (3, 0), (3, 3), (3, 5)]:
        net = nets.ackermann_net(m, n)
        say("ackermann", m, n, "engine", engine)
        for wg in (64, 1024):
            assert_same(P.reduce_net(ACK, net, wg_size=wg, engine=engine), oracle_run(ACK, net),
                        f"A({m},{n}) wg {wg}")


@pytest.mark.parametrize("engine", [0, 1, 2, 4])
def test_algae(engine):
    for n in (0, 1, 2, 5, 10, 14):
        net = nets.algae_net(n)
        say("algae", n, "engine", engine)
        for wg in (64, 1024):
            assert_same(P.reduce_net(ALGAE, net, wg_size=wg, engine=engine),
                        oracle_run(ALGAE, net), f"algae {n} wg {wg}")


def test_programs_batched():
    for rules, batch in ((ACK, [nets.ackermann_net(m, n) for m in range(4) for n in range(5)]),
                         (ALGAE, [nets.algae_net(n) for n in range(16)])):
        refs = [oracle_run(rules, net) for net in batch]
        caps = [net.n_agents + 4 * r.interactions + 1024 for net, r in zip(batch, refs)]
        say("batch", len(batch))
        h = P.batch_load(rules, batch, agent_caps=caps, name_caps=[4 * c for c in caps])
        h.set_config(wg_size=64)
        rs = h.reduce()
        for i in range(len(batch)):
            assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"net {i}")
        h.free()


@pytest.mark.slow
def test_ackermann_3_7_full():
    net = nets.ackermann_net(3, 7)
    say("ackermann 3 7")
    res, nf, pr = g = P.reduce_net(ACK, net)
    assert res.interactions == ack_count(3, 7)
    assert tuple(int(c) for c in pr) == ack_per_rule(3, 7)
    assert oracle.decode_nat(nf, 0, 1) == ack_value(3, 7) == 1021
    assert_same(g, oracle_run(ACK, net), "A(3,7)")


@pytest.mark.slow
def test_algae_27_full():
    net = nets.algae_net(27)
    say("algae 27")
    res, nf, pr = g = P.reduce_net(ALGAE, net)
    assert res.interactions == algae_count(27)
    assert tuple(int(c) for c in pr) == algae_per_rule(27)
    assert decode_letters(nf, CAT, {LA: "a", LB: "b"}) == algae_string(27)
    assert_same(g, oracle_run(ALGAE, net), "algae 27")


@pytest.mark.parametrize("engine", [0, 2, 4])
def test_wide_frontier_single_wave(engine):
    # a one-wave engine (64 lanes) whose frontier far outgrows its LDS tile
    # (512 pairs): the overflow goes through the net's global queue
    for rules, net in ((ALGAE, nets.algae_net(18)),
                       (nets.arith_rules(), nets.config1_add_tree(1, 2048, 8))):
        ref = oracle_run(rules, net)
        say("wide", net.meta.get("family"), "engine", engine)
        res, nf, pr = g = P.reduce_net(rules, net, wg_size=64, engine=engine)
        assert res.max_frontier > 512
        assert_same(g, ref, f"{net.meta.get('family')} wg 64")
