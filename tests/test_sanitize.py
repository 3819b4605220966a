"""The host side under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the rule compiler, net validation and read-back of the evaluator
(linked with host-only stand-ins for the kernel launchers), and the oracle,
built with -fsanitize=address,undefined and run on valid, invalid and
scrambled inputs.  Any report fails the run (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1404_0076_amd import nets

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1404_0076_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")


def _cases():
    """(rules, net, kind) triples: the workload rule tables on valid nets,
    finished heaps, scrambled heaps, and invalid rule tables and nets."""
    A = nets.arith_rules()
    out = []
    for net in (nets.mul_net(5, 7), nets.fib_net(6), nets.config1_add_tree(1, 16, 6),
                nets.random_expr_net(3, 12, 4), nets.parse_net(nets.ARITH_SIG, "<r | S(r) = Z>"),
                nets.parse_net(nets.ARITH_SIG, "<r | Add(Z, r) = S(Z)>")):
        for kind in (0, 1, 2):
            out.append((A, net, kind))
    out.append((nets.ackermann_rules(), nets.ackermann_net(2, 2), 1))
    out.append((nets.algae_rules(), nets.algae_net(5), 1))
    sig = nets.Signature(["P", "Q", "S", "Z", "D"], [1, 1, 1, 0, 2])
    cyc = nets.parse_rules(sig, ["P(a) = Q(b) -> a = b, x = S(x)", "D(p, q) = Z -> p = Z, q = Z"])
    out.append((cyc, nets.parse_net(sig, "<r, s | P(r) = Q(s)>"), 1))
    # invalid nets: a name three times, an agent attached twice, a ref out of range
    bad = nets.parse_net(nets.ARITH_SIG, "<r | Add(x, r) = x>")
    twice = nets.Net(bad.label.copy(), bad.port.copy(), np.array([-1, -1], np.int32),
                     np.array([0, 0], np.int32), bad.n_names)
    out.append((A, twice, 0))
    oob = nets.Net(bad.label.copy(), bad.port.copy(), np.array([-1], np.int32),
                   np.array([7], np.int32), bad.n_names)
    out.append((A, oob, 0))
    # an invalid rule table: a right-hand side referring past its names
    broken = nets.RuleTable(A.sig, list(A.texts), A.lhs.copy(), A.rhs_off.copy(), A.rhs.copy())
    broken.rhs[-1] = 999
    out.append((broken, nets.mul_net(2, 2), 0))
    return out


def _write(path, cases):
    words = [len(cases)]
    for rules, net, kind in cases:
        words += [rules.sig.n_symbols] + list(rules.arity_array())
        words += [rules.n_rules] + list(np.asarray(rules.lhs).reshape(-1))
        words += list(rules.rhs_off) + list(rules.rhs)
        words += [net.n_agents] + list(net.label) + list(np.asarray(net.port).reshape(-1))
        words += [net.n_eqs] + list(net.eq_lhs) + list(net.eq_rhs) + [net.n_names, kind]
    np.asarray(words, dtype=np.int32).tofile(path)


@pytest.fixture(scope="module")
def cases_file(tmp_path_factory):
    cases = _cases()
    path = str(tmp_path_factory.mktemp("san") / "cases.bin")
    _write(path, cases)
    return path, len(cases)


def _run(exe, arg):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([exe, arg], capture_output=True, text=True, timeout=600, env=env)


def test_host_runtime_under_sanitizers(cases_file, tmp_path):
    path, n = cases_file
    exe = str(tmp_path / "host_checks")
    srcs = [os.path.join(HERE, "host_checks.cpp"), os.path.join(HERE, "device_stubs.cpp")] + \
        [os.path.join(CSRC, f) for f in ("rules.cpp", "readback.cpp", "runtime.cpp")]
    cmd = ["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", exe,
           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64"]
    subprocess.check_call(cmd)
    r = _run(exe, path)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.strip().splitlines()
    assert len(lines) == n
    # the valid workload nets validate and read back; the invalid ones are refused
    first = [ln for ln in lines if " net 0 " in ln]
    assert len(first) >= 15
    assert lines[-3].split()[7] == "-1" and lines[-2].split()[7] == "-1"  # the invalid nets
    assert lines[-1].split()[3] == "-1"                                    # the broken rule table


def test_oracle_under_sanitizers(cases_file, tmp_path):
    path, n = cases_file
    exe = str(tmp_path / "oracle_checks")
    cmd = ["gcc", "-std=c99", *SAN, "-I", os.path.join(ROOT, "oracle"),
           os.path.join(HERE, "oracle_checks.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe]
    subprocess.check_call(cmd)
    r = _run(exe, path)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert len(r.stdout.strip().splitlines()) >= 5 * n
