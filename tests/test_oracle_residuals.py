"""Oracle pinned on normal forms that keep residual equations or name cycles:
the stream conventions (orientation and order of residuals, cycles left out of
the stream and counted) against streams derived by hand in
tests/golden/residuals_and_cycles.json, under every schedule."""
import json
import os

import pytest

import oracle
from paper_1404_0076_amd import nets

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "residuals_and_cycles.json")


def cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def case_holds(case, lib=None, schedule="fifo", eager=False):
    net = nets.parse_net(nets.ARITH_SIG, case["net"])
    r = oracle.reduce(nets.arith_rules(), net, schedule=schedule, seed=5, eager=eager, lib=lib)
    return (r.nf.tolist() == case["nf"] and r.status == case["status"]
            and r.interactions == case["interactions"] and r.n_stuck == case["n_stuck"]
            and r.n_cycles == case["n_cycles"] and r.n_loops == case["n_loops"])


@pytest.mark.parametrize("case", cases(), ids=lambda c: c["net"])
@pytest.mark.parametrize("schedule", ["fifo", "lifo", "rounds", "random"])
@pytest.mark.parametrize("eager", [False, True])
def test_residuals_and_cycles(case, schedule, eager):
    assert case_holds(case, schedule=schedule, eager=eager)


def test_residual_order_independent_of_input_order():
    # the same residuals listed in every rotation give one stream
    case = cases()[0]
    inner = case["net"].split("|", 1)[1].rstrip(">").split(",")
    eqs = [e.strip() for e in inner]
    for k in range(len(eqs)):
        text = "<p | " + ", ".join(eqs[k:] + eqs[:k]) + ">"
        r = oracle.reduce(nets.arith_rules(), nets.parse_net(nets.ARITH_SIG, text))
        assert r.nf.tolist() == case["nf"], text
