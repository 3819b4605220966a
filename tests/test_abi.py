"""C-ABI library: loads on the CPU, exports every declared symbol, and its
host logic (rule compiler, net validation, workspace sizing) behaves; no
device call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1404_0076_amd as P
from paper_1404_0076_amd import nets

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "inet.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(inet_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert sorted(P.EXPORTS) == names


def test_strerror_covers_codes():
    for code in (P.OK, P.STUCK, P.EINVAL, P.ENOMEM, P.ELIMIT, P.ERANGE, P.EAGAIN, P.EHIP, P.ENOSYS):
        assert P.strerror(code) != "unknown status"
    assert P.strerror(12345) == "unknown status"


def test_rule_templates_after_folding():
    info = P.rules_check(nets.arith_rules())
    # agents of each right-hand side are kept; bound names that only connect a
    # top-level equation with a nested port are folded away (sub/com inside
    # the rule), leaving wires and the links that touch a rule argument
    assert info["n_new"].tolist() == [2, 0, 3, 2, 3, 2, 1, 0, 2, 1, 2, 5]
    assert info["n_fresh"].tolist() == [1, 0, 2, 0, 2, 0, 0, 0, 0, 0, 0, 2]
    assert info["n_links"].tolist() == [2, 1, 2, 2, 3, 2, 1, 0, 1, 1, 1, 2]
    assert info["bytes"].tolist() == [68, 32, 88, 48, 88, 48, 32, 16, 40, 40, 40, 96]


# a right-hand side that keeps x = C[x]: folding cannot move C into the other
# occurrence of x (it is inside C), so the equation stays as a link whose name
# side is a fresh name
CYCLE_SIG = nets.Signature(["P", "Q", "S", "Z", "D"], [1, 1, 1, 0, 2])
CYCLE_RULES = ["P(a) = Q(b) -> a = b, x = S(x)", "D(p, q) = Z -> p = Z, q = Z",
               "P(a) = Z -> y = D(y, a)"]


def test_cycle_rule_keeps_fresh_link():
    rules = nets.parse_rules(CYCLE_SIG, CYCLE_RULES)
    info = P.rules_check(rules)
    assert info["n_new"].tolist() == [1, 2, 1]
    assert info["n_fresh"].tolist() == [1, 0, 1]
    assert info["n_links"].tolist() == [2, 2, 1]
    rc, nbytes, log = P.jit_build(rules, "gfx950")
    assert rc == P.OK, log


@pytest.mark.parametrize("texts", [
    ["Add(y,r) = S(x) -> Add(y,y) = x, r = S(w)"],
    ["Add(y,r) = S(x) -> r = S(x)", "Add(a,b) = S(c) -> a = S(c), b = Z"],
    ["Add(y,r) = S(x) -> r = S(w), x = y"],
])
def test_invalid_rules_rejected(texts):
    with pytest.raises(P.InetError) as e:
        P.rules_check(nets.parse_rules(nets.ARITH_SIG, texts))
    assert e.value.status == P.EINVAL


def test_rule_limits():
    # a right-hand side with more than 8 agents is refused
    big = "Era = S(x) -> Era = x, " + ", ".join(f"Era = S(S(S(Z)))" for _ in range(3))
    with pytest.raises(P.InetError):
        P.rules_check(nets.parse_rules(nets.ARITH_SIG, [big]))


def _try_load(net, rules=None):
    """inet_batch_load with a dummy device pointer and no bytes: validation
    runs entirely on the host, a valid net then stops at ENOMEM."""
    rules = rules or nets.arith_rules()
    R = P.RulesArg(rules)
    label, port, a_off, eql, eqr, e_off, n_names = nets.pack([net])
    arrs = [P._arr(x, t) for x, t in ((label, np.int32), (port, np.int32), (a_off, np.int64),
                                     (eql, np.int32), (eqr, np.int32), (e_off, np.int64),
                                     (n_names, np.int32))]
    h = ctypes.c_void_p()
    return P.library().inet_batch_load(R.ptr, 1, *(a.ctypes.data for a in arrs), None, None,
                                       ctypes.c_void_p(256), 0, None, ctypes.byref(h))


def _net(label, port, eql, eqr, n_names):
    return nets.Net(np.asarray(label, np.int32), np.asarray(port, np.int32).reshape(-1, 2),
                    np.asarray(eql, np.int32), np.asarray(eqr, np.int32), n_names)


@pytest.mark.parametrize("bad", [
    _net([1, 0], [[-1, 0], [0, 0]], [0], [-1], 1),
    _net([1, 0], [[1, 0], [0, 0]], [0, 1], [-1, -2], 2),
    _net([1, 0], [[-1, 0], [0, 0]], [0], [-2], 2),
    _net([9], [[0, 0]], [0], [-1], 1),
    _net([1, 1], [[1, 0], [0, 0]], [-1], [-2], 2),
    _net([0], [[0, 0]], [0], [-5], 1),
])
def test_invalid_nets_rejected_on_host(bad):
    assert _try_load(bad) == P.EINVAL


@pytest.mark.parametrize("net", [nets.fib_net(5), nets.mul_net(3, 4), nets.config1_add_tree(0, 16, 9),
                                 nets.parse_net(nets.ARITH_SIG, "<r | S(r) = Z>")])
def test_valid_nets_pass_validation(net):
    assert _try_load(net) == P.ENOMEM


def test_workspace_grows_with_caps():
    R = nets.arith_rules()
    a = P.workspace_bytes(R, [10], [1], [1], [1000], [1000])
    b = P.workspace_bytes(R, [10], [1], [1], [100000], [1000])
    c = P.workspace_bytes(R, [10], [1], [1], [100000], [100000])
    assert a < b < c
    two = P.workspace_bytes(R, [10, 10], [1, 1], [1, 1], [1000, 1000], [1000, 1000])
    assert two > a


def test_rule_specialised_engine_builds_on_host():
    # the engine with the rule table compiled in is built by hipRTC on the
    # host; no device is needed to produce its code object
    rc, nbytes, log = P.jit_build(nets.arith_rules(), "gfx950")
    assert rc == P.OK, log
    assert nbytes > 1000
    # a table with a rule whose right-hand side has no equations still builds
    sig = nets.Signature(["A", "B"], [0, 0])
    rc, nbytes, log = P.jit_build(nets.parse_rules(sig, ["A = B ->"]), "gfx950")
    assert rc == P.OK, log
    rc, _, _ = P.jit_build(nets.arith_rules(), "")
    assert rc == P.ENOSYS
