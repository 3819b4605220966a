"""CPU oracle for the lightweight interaction calculus -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain C,
sequential, literal term rewriting; see that file for what each part follows)
through ctypes and shares no code with the GPU evaluator.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

FIFO, LIFO, RANDOM, ROUNDS, ENUMERATE = 0, 1, 2, 3, 4
EAGER = 0x100
SCHEDULES = {"fifo": FIFO, "lifo": LIFO, "random": RANDOM, "rounds": ROUNDS,
             "enumerate": ENUMERATE}
OK, STUCK, EINVAL, ENOMEM, ELIMIT, ERANGE = 0, 1, -1, -2, -3, -4


def build(force: bool = False, out: str = LIB_PATH, defines=()) -> str:
    """Compile oracle.c with gcc into ``out`` (in-tree by default)."""
    src = os.path.join(HERE, "oracle.c")
    hdr = os.path.join(HERE, "oracle.h")
    newest = max(os.path.getmtime(src), os.path.getmtime(hdr))
    if force or defines or not os.path.exists(out) or os.path.getmtime(out) < newest:
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-Wno-unused-parameter",
               "-shared", "-fPIC"] + [f"-D{d}" for d in defines] + ["-o", tmp, src]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


class _Input(ctypes.Structure):
    _fields_ = [
        ("n_symbols", ctypes.c_int32), ("arity", ctypes.c_void_p),
        ("n_rules", ctypes.c_int32), ("rule_lhs", ctypes.c_void_p),
        ("rhs_off", ctypes.c_void_p), ("rhs", ctypes.c_void_p),
        ("n_agents", ctypes.c_int32), ("label", ctypes.c_void_p), ("port", ctypes.c_void_p),
        ("n_eqs", ctypes.c_int32), ("eq_lhs", ctypes.c_void_p), ("eq_rhs", ctypes.c_void_p),
        ("n_names", ctypes.c_int32),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("n_iface", ctypes.c_int32), ("n_stuck", ctypes.c_int32),
        ("n_cycles", ctypes.c_int32), ("n_loops", ctypes.c_int32), ("n_outcomes", ctypes.c_int32),
        ("interactions", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
        ("n_com", ctypes.c_uint64), ("n_sub", ctypes.c_uint64), ("n_col", ctypes.c_uint64),
        ("max_live_agents", ctypes.c_uint64), ("final_live_agents", ctypes.c_uint64),
        ("n_schedules", ctypes.c_uint64), ("nf_len", ctypes.c_int64),
    ]


_lib = None


def load_library(path: str):
    lib = ctypes.CDLL(path)
    lib.orc_reduce.restype = ctypes.c_int
    lib.orc_reduce.argtypes = [ctypes.POINTER(_Input), ctypes.c_int, ctypes.c_uint64,
                               ctypes.c_uint64, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                               ctypes.POINTER(_Result)]
    lib.orc_free.restype = None
    lib.orc_free.argtypes = [ctypes.c_void_p]
    lib.orc_version.restype = ctypes.c_char_p
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load_library(LIB_PATH)
    return _lib


@dataclasses.dataclass
class OracleResult:
    status: int
    interactions: int
    per_rule: np.ndarray
    nf: np.ndarray
    rounds: int
    n_iface: int
    n_stuck: int
    n_cycles: int
    n_loops: int
    n_com: int
    n_sub: int
    n_col: int
    max_live_agents: int
    final_live_agents: int
    n_outcomes: int
    n_schedules: int


def _c(a, dtype=np.int32):
    return np.ascontiguousarray(a, dtype=dtype)


def reduce(rules, net, schedule="fifo", seed: int = 0, eager: bool = False,
           max_interactions: int = 0, lib=None) -> OracleResult:
    """Reduce ``net`` (nets.Net) under ``rules`` (nets.RuleTable) to normal form."""
    lib = lib or _load()
    arity = _c(rules.arity_array())
    lhs = _c(rules.lhs)
    off = _c(rules.rhs_off)
    rhs = _c(rules.rhs if rules.rhs.size else np.zeros(1, np.int32))
    label = _c(net.label if net.n_agents else np.zeros(1, np.int32))
    port = _c(net.port if net.n_agents else np.zeros((1, 2), np.int32))
    eql = _c(net.eq_lhs if net.n_eqs else np.zeros(1, np.int32))
    eqr = _c(net.eq_rhs if net.n_eqs else np.zeros(1, np.int32))
    inp = _Input(rules.sig.n_symbols, arity.ctypes.data, rules.n_rules, lhs.ctypes.data,
                 off.ctypes.data, rhs.ctypes.data, net.n_agents, label.ctypes.data,
                 port.ctypes.data, net.n_eqs, eql.ctypes.data, eqr.ctypes.data, net.n_names)
    sched = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    if eager:
        sched |= EAGER
    per_rule = np.zeros(max(1, rules.n_rules), dtype=np.uint64)
    res = _Result()
    ptr = ctypes.POINTER(ctypes.c_int32)()
    rc = lib.orc_reduce(ctypes.byref(inp), sched, seed, max_interactions, per_rule.ctypes.data,
                        ctypes.byref(ptr), ctypes.byref(res))
    nf = np.zeros(0, np.int32)
    if ptr:
        n = int(res.nf_len)
        if n > 0:
            nf = np.ctypeslib.as_array(ptr, shape=(n,)).copy()
        lib.orc_free(ptr)
    return OracleResult(
        status=int(rc), interactions=int(res.interactions), per_rule=per_rule[:rules.n_rules].copy(),
        nf=nf,
        rounds=int(res.rounds), n_iface=int(res.n_iface), n_stuck=int(res.n_stuck),
        n_cycles=int(res.n_cycles), n_loops=int(res.n_loops), n_com=int(res.n_com),
        n_sub=int(res.n_sub), n_col=int(res.n_col), max_live_agents=int(res.max_live_agents),
        final_live_agents=int(res.final_live_agents), n_outcomes=int(res.n_outcomes),
        n_schedules=int(res.n_schedules))


def decode_nat(nf: np.ndarray, z_label: int, s_label: int) -> Optional[int]:
    """If the stream is one interface term S^k Z with no residuals, return k."""
    if len(nf) < 3 or nf[0] != 1:
        return None
    k = 0
    i = 1
    while i < len(nf) and nf[i] == s_label:
        k += 1
        i += 1
    if i < len(nf) and nf[i] == z_label and i + 1 < len(nf) and nf[i + 1] == 0 and i + 2 == len(nf):
        return k
    return None


def version() -> str:
    return _load().orc_version().decode()
