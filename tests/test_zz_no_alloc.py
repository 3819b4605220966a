"""GPU: inet_reduce_noalloc, the entry point that allocates no device memory
(every array inside the library's static device array), against the
allocating entry points (inet_load + inet_reduce + inet_readback) on the same
nets, and against the oracle: two calls in a row, the second on a smaller
net, so that what the first call left in the shared array cannot leak into
the second."""
import sys

import numpy as np
import pytest

import paper_1404_0076_amd as P
from paper_1404_0076_amd import nets

from gpu_util import oracle_run

pytestmark = pytest.mark.gpu
R = nets.arith_rules()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def allocating(rules, net, agent_cap, name_cap):
    h = P.load(rules, net, agent_cap=agent_cap, name_cap=name_cap)
    res = h.reduce()[0]
    nf = h.readback(0) if res.status in (P.OK, P.STUCK) else None
    h.free()
    return res, nf


def check_pair(rules, net, agent_cap, name_cap, what):
    res, nf, rc = P.reduce_noalloc(rules, net, agent_cap=agent_cap, name_cap=name_cap)
    ref, ref_nf = allocating(rules, net, agent_cap, name_cap)
    oref = oracle_run(rules, net)
    say(what, res.status, res.interactions, res.steps)
    assert rc == res.status == ref.status == oref.status, what
    assert res.interactions == ref.interactions == oref.interactions, what
    assert res.steps == ref.steps, what
    assert res.agents_used == ref.agents_used and res.names_used == ref.names_used, what
    assert res.n_stuck == ref.n_stuck == oref.n_stuck, what
    assert np.array_equal(nf, ref_nf) and np.array_equal(nf, oref.nf), what


def test_two_calls_in_a_row_second_smaller():
    big = nets.mul_net(40, 31)
    small = nets.fib_net(9)
    check_pair(R, big, 1 << 16, 1 << 18, "first call, Mul(40,31)")
    check_pair(R, small, 1 << 12, 1 << 14, "second call, Fib(9)")
    # and once more in the other order, with a residual net last
    check_pair(R, nets.config1_add_tree(2, 64, 20), 1 << 15, 1 << 17, "add tree")
    check_pair(R, nets.parse_net(nets.ARITH_SIG, "<r, q | S(r) = Z, Add(q, y) = Fib(y)>"),
               1024, 4096, "stuck net")


def test_step_limit_and_too_large():
    net = nets.fib_net(11)
    res, nf, rc = P.reduce_noalloc(R, net, agent_cap=1 << 14, name_cap=1 << 16, max_steps=5)
    assert rc == P.ELIMIT and res.steps == 5 and nf is None
    # a workspace beyond the static array is refused before anything runs
    with pytest.raises(P.InetError) as e:
        P.reduce_noalloc(R, net, agent_cap=P.NOALLOC_SCRATCH_BYTES // 16 + 1, name_cap=1 << 16)
    assert e.value.status == P.ENOMEM
    # the array is still usable afterwards
    check_pair(R, nets.mul_net(7, 9), 1 << 12, 1 << 14, "after refusal")
