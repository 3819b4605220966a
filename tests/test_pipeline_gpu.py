"""GPU: the paper's own evaluation loop (dummies, filter, sort-based com;
inet_reduce_pipeline), kept as an ablation, gives the oracle's normal forms,
interaction counts and per-rule histograms on the same nets."""
import sys

import numpy as np
import pytest

import paper_1404_0076_amd as P
from paper_1404_0076_amd import nets

from closed_forms import small_exprs
from gpu_util import assert_same, oracle_run

pytestmark = pytest.mark.gpu
R = nets.arith_rules()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pipeline(rules, net, cap=1 << 16):
    h = P.load(rules, net, agent_cap=max(cap, 4 * net.n_agents + 4096),
               name_cap=4 * max(cap, 4 * net.n_agents + 4096))
    res = h.reduce_pipeline()[0]
    out = (res, h.readback(0) if res.status in (P.OK, P.STUCK) else np.zeros(0, np.int32),
           h.per_rule(0))
    h.free()
    return out


CASES = ["<r | Add(Z, r) = S(Z)>", "<r | Add(S(S(Z)), r) = S(Z)>", "<p, q | Dup(p, q) = S(S(Z))>",
         "< | Era = S(Z)>", "<r | S(r) = Z>", "<r, q | S(r) = Z, Add(q, y) = Fib(y)>"]


@pytest.mark.parametrize("text", CASES)
def test_small(text):
    net = nets.parse_net(nets.ARITH_SIG, text)
    say("pipeline", text)
    assert_same(pipeline(R, net), oracle_run(R, net), text)


def test_programs():
    for net in (nets.mul_net(12, 9), nets.fib_net(9), nets.config1_add_tree(2, 16, 10)):
        say("pipeline", net.meta.get("family"))
        assert_same(pipeline(R, net), oracle_run(R, net), net.meta.get("family"))
    for seed, net in small_exprs(10, 12, 5, 50_000):
        assert_same(pipeline(R, net), oracle_run(R, net), f"expr {seed}")


def test_chains_need_one_iteration_per_name():
    # {A = x0, x0 = x1, ..., B}: com keyed on one name per equation merges one
    # link of the chain per iteration before the active pair A = B exists
    sig = nets.Signature(["A", "B", "C"], [1, 0, 0])
    rules = nets.parse_rules(sig, ["A(r) = B -> r = C"])
    for length in (1, 4, 12):
        links = "".join(f"x{i} = x{i + 1}, " for i in range(length - 1))
        net = nets.parse_net(sig, f"<r | A(r) = x0, {links}x{length - 1} = B>")
        say("chain", length)
        res, nf, pr = out = pipeline(rules, net)
        assert_same(out, oracle_run(rules, net), f"chain {length}")
        assert res.steps >= 2


def test_batch_and_reset():
    batch = [nets.mul_net(5, 7), nets.fib_net(7), nets.parse_net(nets.ARITH_SIG, "<r | S(r) = Z>")]
    refs = [oracle_run(R, n) for n in batch]
    h = P.batch_load(R, batch, agent_caps=[1 << 14] * 3, name_caps=[1 << 16] * 3)
    for rep in range(2):
        h.reset()
        rs = h.reduce_pipeline()
        for i in range(len(batch)):
            assert_same((rs[i], h.readback(i), h.per_rule(i)), refs[i], f"net {i} rep {rep}")
    h.free()
