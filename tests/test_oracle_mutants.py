"""Planted mistakes in the oracle (built on the CPU with -DORC_MUTANT=k) must
each be caught by the pins: a transposed operand, a lost orientation swap, a
dropped right-hand-side equation, com counted as an interaction, residuals
oriented larger side first, residuals sorted by their right sides first, and
name cycles not counted."""
import os
import subprocess
import sys

import pytest

import oracle
from paper_1404_0076_amd import nets

from closed_forms import expr_count, expr_value, fib_count, mul_count, small_exprs

R = nets.arith_rules()


def _pins_hold(lib):
    checks = []
    for a, b in [(2, 3), (3, 1)]:
        r = oracle.reduce(R, nets.mul_net(a, b), lib=lib)
        checks.append(r.status == 0 and r.interactions == mul_count(a, b)
                      and oracle.decode_nat(r.nf, 0, 1) == a * b)
    r = oracle.reduce(R, nets.fib_net(6), lib=lib)
    checks.append(r.status == 0 and r.interactions == fib_count(6))
    for seed, net in small_exprs(4, 8, 3, 20_000, min_count=20):
        r = oracle.reduce(R, net, lib=lib)
        e = net.meta["expr"]
        checks.append(r.status == 0 and r.interactions == expr_count(e)
                      and oracle.decode_nat(r.nf, 0, 1) == expr_value(e))
    r = oracle.reduce(nets.add_rules(), nets.parse_net(nets.ARITH_SIG, "<r | Add(Z, r) = S(Z)>"),
                      lib=lib)
    checks.append(r.nf.tolist() == [1, 1, 0, 0] and r.interactions == 2)
    # equations are symmetric (Section 2.2): the same example written S(Z) = Add(Z, r)
    r = oracle.reduce(nets.add_rules(), nets.parse_net(nets.ARITH_SIG, "<r | S(Z) = Add(Z, r)>"),
                      lib=lib)
    checks.append(r.nf.tolist() == [1, 1, 0, 0] and r.interactions == 2)
    # stream conventions: residual orientation and order, cycles counted
    import test_oracle_residuals as tr
    checks += [tr.case_holds(c, lib=lib) for c in tr.cases()]
    return all(checks)


def test_correct_oracle_passes_pins():
    assert _pins_hold(oracle._load())


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5, 6, 7])
def test_mutant_caught(mutant, tmp_path):
    # a planted mistake may also corrupt the oracle's state and crash it: the
    # pins run in a child process, and a crash counts as caught
    path = oracle.build(out=str(tmp_path / f"liboracle_m{mutant}.so"),
                        defines=[f"ORC_MUTANT={mutant}"])
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys; sys.path[:0] = [%r, %r]; import oracle, test_oracle_mutants as t; "
            "sys.exit(0 if t._pins_hold(oracle.load_library(%r)) else 3)"
            % (here, os.path.dirname(here), path))
    rc = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=300).returncode
    assert rc != 0
