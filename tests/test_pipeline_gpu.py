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


# ---------------------------------------------------------------------------
# the ablation's own device primitives against numpy


def test_reduce_by_key_paper_example():
    # Section 3.5: reduce by key on {2,0,3,3,3,7,5,5} with addition as the
    # fold and equality of neighbours as the predicate gives {2,0,9,7,10}
    import torch
    x = [2, 0, 3, 3, 3, 7, 5, 5]
    keys = torch.tensor(x, dtype=torch.int32, device="cuda")
    vals = torch.tensor(x, dtype=torch.int64, device="cuda")
    ko, vo = P.prim.reduce_by_key(keys, vals, op=0)
    assert vo.cpu().tolist() == [2, 0, 9, 7, 10]
    assert ko.cpu().tolist() == [2, 0, 3, 7, 5]


def _runs(keys):
    """numpy reference: start index of every run of equal adjacent keys"""
    k = np.asarray(keys)
    return np.flatnonzero(np.r_[True, k[1:] != k[:-1]]) if len(k) else np.zeros(0, np.int64)


@pytest.mark.parametrize("n", [0, 1, 7, 2047, 2048, 2049, 100_003, 3_000_001])
def test_primitives_match_numpy(n):
    import torch
    rng = np.random.Generator(np.random.PCG64(n + 5))
    say("primitives", n)
    # inclusive sum (uint64, wrapping)
    x = rng.integers(0, 1 << 62, n, dtype=np.int64)
    got = P.prim.scan(torch.from_numpy(x).cuda()).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, np.cumsum(x.view(np.uint64), dtype=np.uint64))
    # compaction of everything but the dummy ~0
    y = rng.integers(0, 50, n, dtype=np.int64)
    y[rng.random(n) < 0.4] = -1
    got = P.prim.select(torch.from_numpy(y).cuda(), -1).cpu().numpy()
    assert np.array_equal(got, y[y != -1])
    # stable sort by 32-bit key (few distinct keys, high bits set, values record the input order)
    keys = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    keys[rng.random(n) < 0.5] = 0x80000003
    vals = np.arange(n, dtype=np.int64)
    kt, vt = torch.from_numpy(keys.view(np.int32)).cuda(), torch.from_numpy(vals).cuda()
    P.prim.sort_pairs(kt, vt)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(kt.cpu().numpy().view(np.uint32), keys[order])
    assert np.array_equal(vt.cpu().numpy(), vals[order])
    # reduce by key: runs of a sorted key array folded by sum
    rk = np.sort(rng.integers(0, max(1, n // 3 + 1), n)).astype(np.int32)
    rv = rng.integers(0, 1000, n, dtype=np.int64)
    ko, vo = P.prim.reduce_by_key(torch.from_numpy(rk).cuda(), torch.from_numpy(rv).cuda(), op=0)
    heads = _runs(rk)
    assert np.array_equal(ko.cpu().numpy(), rk[heads])
    assert np.array_equal(vo.cpu().numpy(), np.add.reduceat(rv, heads) if n else rv[:0])


def test_reduce_by_key_merges_equations():
    # op 1: (x, t) and (x, s) sharing the variable x give the equation (s, t)
    import torch
    def eq(l, r):
        return (l & 0xFFFFFFFF) | ((r & 0xFFFFFFFF) << 32)
    keys = torch.tensor([4, 4, 9, 11, 11], dtype=torch.int32, device="cuda")
    packed = np.array([eq(-5, 17), eq(-5, 23), eq(-10, 3), eq(-12, -3), eq(-12, 40)], np.uint64)
    vals = torch.from_numpy(packed.view(np.int64)).cuda()
    ko, vo = P.prim.reduce_by_key(keys, vals, op=1)
    got = [(int(v) & 0xFFFFFFFF, (int(v) >> 32) & 0xFFFFFFFF) for v in vo.cpu().numpy().view(np.uint64)]
    to_i = lambda u: u - (1 << 32) if u >= 1 << 31 else u  # noqa: E731
    assert ko.cpu().tolist() == [4, 9, 11]
    assert [(to_i(a), to_i(b)) for a, b in got] == [(23, 17), (-10, 3), (40, -3)]
