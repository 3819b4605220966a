"""MI355X evaluator for the lightweight interaction calculus.

Thin ctypes binding of ``libinet.so`` (C ABI in ``include/inet.h``): argument
marshalling only.  Device memory and streams come from PyTorch; every step of
the reduction runs in the library's HIP kernels.  There is no fallback: if the
library is missing or no GPU is present, calls fail loudly.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

from . import nets  # noqa: F401  (re-exported for convenience)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinet.so")

OK, STUCK, EINVAL, ENOMEM, ELIMIT, ERANGE, EAGAIN, EHIP, ENOSYS, EINTERNAL = 0, 1, -1, -2, -3, -4, -5, -6, -7, -8
ETIMEDOUT = -9

EXPORTS = [
    "inet_workspace_bytes", "inet_load", "inet_batch_load", "inet_set_config", "inet_get_config",
    "inet_set_order", "inet_reduce_async", "inet_results", "inet_reduce", "inet_reset",
    "inet_readback", "inet_per_rule", "inet_rule_bytes", "inet_num_nets", "inet_free",
    "inet_strerror", "inet_last_kernel_ms", "inet_rules_check", "inet_graph_capture",
    "inet_graph_launch", "inet_server_create", "inet_server_set_config", "inet_server_net_bytes",
    "inet_server_submit", "inet_server_step", "inet_server_poll", "inet_server_result",
    "inet_server_per_rule", "inet_server_release", "inet_server_stats", "inet_server_free",
    "inet_jit_build", "inet_server_run", "inet_reduce_pipeline", "inet_cells", "inet_set_trace",
    "inet_prim_scan", "inet_prim_select", "inet_prim_sort_pairs", "inet_prim_reduce_by_key",
    "inet_reduce_noalloc",
]


class InetError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class _Rules(ctypes.Structure):
    _fields_ = [("n_symbols", ctypes.c_int32), ("arity", ctypes.c_void_p),
                ("n_rules", ctypes.c_int32), ("rule_lhs", ctypes.c_void_p),
                ("rhs_off", ctypes.c_void_p), ("rhs", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_stuck", ctypes.c_int32),
                ("interactions", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("agents_used", ctypes.c_int64), ("names_used", ctypes.c_int64),
                ("max_frontier", ctypes.c_int32), ("loops", ctypes.c_int32)]


class _Config(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("jump", ctypes.c_int32),
                ("max_resident", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("solo_max", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("grid_lo", ctypes.c_int32), ("grid_hi", ctypes.c_int32),
                ("grid_ppw", ctypes.c_int32), ("timeout_us", ctypes.c_int32),
                ("qcap", ctypes.c_int32), ("round_scale", ctypes.c_int32)]


# tunables of inet_config beyond wg_size / jump / max_resident / engine (all
# 0 = the library's default; grid -1 keeps a single net on one workgroup)
CONFIG_KEYS = ("solo_max", "grid", "grid_lo", "grid_hi", "grid_ppw", "timeout_us", "qcap",
               "round_scale")


def _config(wg_size, jump, max_resident, engine, extra) -> "_Config":
    bad = set(extra) - set(CONFIG_KEYS)
    if bad:
        raise TypeError(f"unknown configuration keys {sorted(bad)}")
    return _Config(wg_size, 1 if jump else 0, max_resident, engine,
                   *[int(extra.get(k, 0)) for k in CONFIG_KEYS])


_lib = None

_P = ctypes.c_void_p
_I32, _I64, _U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64


def library():
    """Load libinet.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1404_0076_amd/build.py first")
        lib = ctypes.CDLL(LIB_PATH)
        sig = {
            "inet_workspace_bytes": [_P, _I32, _P, _P, _P, _P, _P, _P],
            "inet_load": [_P, _P, _P, _I32, _P, _P, _I32, _I32, _I64, _I64, _P, ctypes.c_size_t, _P, _P],
            "inet_batch_load": [_P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P, _P],
            "inet_set_config": [_P, _P], "inet_get_config": [_P, _P], "inet_set_order": [_P, _P],
            "inet_reduce_async": [_P, _P, _U64], "inet_results": [_P, _P, _P],
            "inet_reduce": [_P, _P, _U64, _P], "inet_reset": [_P, _P],
            "inet_readback": [_P, _I32, _P, _I64, _P], "inet_per_rule": [_P, _I32, _P, _I32],
            "inet_cells": [_P, _I32, _P, _I64, _P], "inet_set_trace": [_P, _I32, _P, _I64],
            "inet_prim_scan": [_P, _P, _I64, _P], "inet_prim_select": [_P, _P, _I64, _U64, _P, _P],
            "inet_prim_sort_pairs": [_P, _P, _I64, _P],
            "inet_prim_reduce_by_key": [_P, _P, _I64, _P, _P, _I32, _P, _P],
            "inet_reduce_noalloc": [_P, _P, _P, _I32, _P, _P, _I32, _I32, _I64, _I64, _U64, _P, _P,
                                    _P, _I64, _P],
            "inet_rule_bytes": [_P, _P, _I32], "inet_num_nets": [_P],
            "inet_rules_check": [_P, _P, _P, _P, _P, _I32],
            "inet_jit_build": [_P, ctypes.c_char_p, _P, _P, ctypes.c_size_t],
            "inet_graph_capture": [_P, _U64], "inet_graph_launch": [_P, _P],
            "inet_server_create": [_P, _I32, _P, ctypes.c_size_t, _P],
            "inet_server_set_config": [_P, _P],
            "inet_server_net_bytes": [_P, _I32, _I32, _I32, _I64, _I64, _P],
            "inet_server_submit": [_P, _P, _P, _I32, _P, _P, _I32, _I32, _I64, _I64, _P, _P],
            "inet_server_step": [_P, _P, ctypes.c_uint32],
            "inet_server_poll": [_P, _P, _P, _I32, _P],
            "inet_server_result": [_P, _I64, _P, _P, _I64, _P],
            "inet_server_per_rule": [_P, _I64, _P, _I32],
            "inet_server_release": [_P, _I64], "inet_server_stats": [_P, _P, _P, _P],
            "inet_reduce_pipeline": [_P, _P, _U64],
            "inet_server_run": [_P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I64, _P, _P,
                                ctypes.c_uint32, ctypes.c_double, _P, _P, _P, _P, _P, _P, _P],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib.inet_free.argtypes = [_P]
        lib.inet_free.restype = None
        lib.inet_server_free.argtypes = [_P]
        lib.inet_server_free.restype = None
        lib.inet_strerror.argtypes = [ctypes.c_int]
        lib.inet_strerror.restype = ctypes.c_char_p
        lib.inet_last_kernel_ms.argtypes = [_P]
        lib.inet_last_kernel_ms.restype = ctypes.c_float
        _lib = lib
    return _lib


def strerror(status: int) -> str:
    return library().inet_strerror(int(status)).decode()


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.size == 0:
        a = np.zeros(1, dtype=dtype)
    return a


class RulesArg:
    """Keeps the numpy arrays alive for the duration of a call."""

    def __init__(self, rules):
        self.arity = _arr(rules.arity_array(), np.int32)
        self.lhs = _arr(rules.lhs, np.int32)
        self.off = _arr(rules.rhs_off, np.int32)
        self.rhs = _arr(rules.rhs, np.int32)
        self.n_rules = rules.n_rules
        self.s = _Rules(rules.sig.n_symbols, self.arity.ctypes.data, rules.n_rules,
                        self.lhs.ctypes.data, self.off.ctypes.data, self.rhs.ctypes.data)

    @property
    def ptr(self):
        return ctypes.byref(self.s)


@dataclasses.dataclass
class Result:
    status: int
    n_stuck: int
    interactions: int
    steps: int
    agents_used: int
    names_used: int
    max_frontier: int
    loops: int


def workspace_bytes(rules, n_agents, n_eqs, n_names, agent_cap=None, name_cap=None) -> int:
    R = RulesArg(rules)
    n = len(n_agents)
    na = _arr(n_agents, np.int64)
    ne = _arr(n_eqs, np.int64)
    nn = _arr(n_names, np.int32)
    ac = _arr(agent_cap if agent_cap is not None else np.zeros(n), np.int64)
    nc = _arr(name_cap if name_cap is not None else np.zeros(n), np.int64)
    out = ctypes.c_size_t(0)
    rc = library().inet_workspace_bytes(R.ptr, n, na.ctypes.data, ne.ctypes.data, nn.ctypes.data,
                                        ac.ctypes.data, nc.ctypes.data, ctypes.byref(out))
    if rc:
        raise InetError(rc, "inet_workspace_bytes")
    return int(out.value)


def rules_check(rules) -> dict:
    """Host-only compile of a rule table (inet_rules_check)."""
    R = RulesArg(rules)
    n = max(1, rules.n_rules)
    out = {k: np.zeros(n, np.int32) for k in ("n_new", "n_fresh", "n_links", "bytes")}
    rc = library().inet_rules_check(R.ptr, out["n_new"].ctypes.data, out["n_fresh"].ctypes.data,
                                    out["n_links"].ctypes.data, out["bytes"].ctypes.data, n)
    if rc:
        raise InetError(rc, "inet_rules_check")
    return {k: v[: rules.n_rules] for k, v in out.items()}


def jit_build(rules, arch: str = "gfx950"):
    """Host-only build of the rule-specialised engine (inet_jit_build):
    (status, code object bytes, compiler log)."""
    R = RulesArg(rules)
    n = ctypes.c_size_t(0)
    log = ctypes.create_string_buffer(8192)
    rc = library().inet_jit_build(R.ptr, arch.encode(), ctypes.byref(n), log, len(log))
    return rc, int(n.value), log.value.decode(errors="replace")


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream), stream


class Handle:
    """A loaded batch of nets (a single net is a batch of one)."""

    def __init__(self, ptr, workspace, rules, n_nets):
        self._h = ptr
        self.workspace = workspace  # torch tensor that owns the device memory
        self.rules = rules
        self.n_nets = n_nets

    def _check(self, rc, what):
        if rc not in (OK, STUCK):
            raise InetError(rc, what)
        return rc

    def set_config(self, wg_size: int = 0, jump: bool = True, max_resident: int = 0,
                   engine: int = 0, **extra):
        """Launch shape and tunables (inet_config); ``extra`` takes the keys
        of CONFIG_KEYS."""
        cfg = _config(wg_size, jump, max_resident, engine, extra)
        self._check(library().inet_set_config(self._h, ctypes.byref(cfg)), "inet_set_config")

    def get_config(self) -> dict:
        cfg = _Config()
        self._check(library().inet_get_config(self._h, ctypes.byref(cfg)), "inet_get_config")
        out = {"wg_size": cfg.wg_size, "jump": bool(cfg.jump), "max_resident": cfg.max_resident,
               "engine": cfg.engine}
        out.update({k: getattr(cfg, k) for k in CONFIG_KEYS})
        return out

    def set_trace(self, net: int = 0, buf=None):
        """Record the active pairs of each parallel step of ``net`` into the
        int32 device tensor ``buf`` (inet_set_trace); None turns it off."""
        import torch
        if buf is None:
            self._check(library().inet_set_trace(self._h, net, None, 0), "inet_set_trace")
            self._trace = None
            return
        assert buf.is_cuda and buf.dtype == torch.int32 and buf.is_contiguous()
        self._trace = buf
        self._check(library().inet_set_trace(self._h, net, ctypes.c_void_p(buf.data_ptr()),
                                             buf.numel()), "inet_set_trace")

    def cells(self, net: int = 0) -> np.ndarray:
        """The raw name cells of a finished net (inet_cells), after results()."""
        n = ctypes.c_int64(0)
        rc = library().inet_cells(self._h, net, None, 0, ctypes.byref(n))
        if rc not in (OK, ERANGE):
            raise InetError(rc, "inet_cells")
        buf = np.zeros(max(1, n.value), np.int32)
        self._check(library().inet_cells(self._h, net, buf.ctypes.data, buf.size, ctypes.byref(n)),
                    "inet_cells")
        return buf[: n.value]

    def set_order(self, order: Sequence[int]):
        o = _arr(order, np.int32)
        self._check(library().inet_set_order(self._h, o.ctypes.data), "inet_set_order")

    def reduce_async(self, max_steps: int = 0, stream=None):
        s, _ = _stream_handle(stream)
        self._check(library().inet_reduce_async(self._h, s, max_steps), "inet_reduce_async")

    def results(self, stream=None) -> List[Result]:
        s, _ = _stream_handle(stream)
        out = (_Result * self.n_nets)()
        self._check(library().inet_results(self._h, s, out), "inet_results")
        return [Result(r.status, r.n_stuck, r.interactions, r.steps, r.agents_used,
                       r.names_used, r.max_frontier, r.loops) for r in out]

    def reduce(self, max_steps: int = 0, stream=None) -> List[Result]:
        s, _ = _stream_handle(stream)
        out = (_Result * self.n_nets)()
        rc = library().inet_reduce(self._h, s, max_steps, out)
        if rc in (EINVAL, EHIP):
            raise InetError(rc, "inet_reduce")
        return [Result(r.status, r.n_stuck, r.interactions, r.steps, r.agents_used,
                       r.names_used, r.max_frontier, r.loops) for r in out]

    def reduce_pipeline(self, max_iterations: int = 0, stream=None) -> List[Result]:
        """The paper's own evaluation loop (inet_reduce_pipeline), for comparison."""
        s, _ = _stream_handle(stream)
        self._check(library().inet_reduce_pipeline(self._h, s, max_iterations), "inet_reduce_pipeline")
        return self.results(stream)

    def reset(self, stream=None):
        s, _ = _stream_handle(stream)
        self._check(library().inet_reset(self._h, s), "inet_reset")

    def readback(self, net: int = 0) -> np.ndarray:
        n = ctypes.c_int64(0)
        rc = library().inet_readback(self._h, net, None, 0, ctypes.byref(n))
        if rc != ERANGE:
            raise InetError(rc, "inet_readback")
        buf = np.zeros(max(1, n.value), dtype=np.int32)
        rc = library().inet_readback(self._h, net, buf.ctypes.data, buf.size, ctypes.byref(n))
        self._check(rc, "inet_readback")
        return buf[: n.value].copy()

    def per_rule(self, net: int = 0) -> np.ndarray:
        out = np.zeros(max(1, self.rules.n_rules), dtype=np.uint64)
        self._check(library().inet_per_rule(self._h, net, out.ctypes.data, out.size), "inet_per_rule")
        return out[: self.rules.n_rules]

    def rule_bytes(self) -> np.ndarray:
        out = np.zeros(max(1, self.rules.n_rules), dtype=np.int32)
        self._check(library().inet_rule_bytes(self._h, out.ctypes.data, out.size), "inet_rule_bytes")
        return out[: self.rules.n_rules]

    def graph_capture(self, max_steps: int = 0):
        """Capture restore + reduce as a HIP graph (inet_graph_capture)."""
        self._check(library().inet_graph_capture(self._h, max_steps), "inet_graph_capture")

    def graph_launch(self, stream=None):
        s, _ = _stream_handle(stream)
        self._check(library().inet_graph_launch(self._h, s), "inet_graph_launch")

    def last_kernel_ms(self) -> float:
        return float(library().inet_last_kernel_ms(self._h))

    def free(self):
        if self._h:
            library().inet_free(self._h)
            self._h = None
            self.workspace = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def batch_load(rules, net_list: Sequence["nets.Net"], agent_caps=None, name_caps=None,
               stream=None, device="cuda") -> Handle:
    """Load independent nets into one handle (inet_batch_load)."""
    import torch
    label, port, a_off, eql, eqr, e_off, n_names = nets.pack(net_list)
    n = len(net_list)
    ac = _arr(agent_caps if agent_caps is not None else np.zeros(n), np.int64)
    nc = _arr(name_caps if name_caps is not None else np.zeros(n), np.int64)
    nbytes = workspace_bytes(rules, np.diff(a_off), np.diff(e_off), n_names, ac, nc)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    s, _ = _stream_handle(stream)
    R = RulesArg(rules)
    la, po, ao = _arr(label, np.int32), _arr(port, np.int32), _arr(a_off, np.int64)
    el, er, eo, nn = _arr(eql, np.int32), _arr(eqr, np.int32), _arr(e_off, np.int64), _arr(n_names, np.int32)
    h = ctypes.c_void_p()
    rc = library().inet_batch_load(R.ptr, n, la.ctypes.data, po.ctypes.data, ao.ctypes.data,
                                   el.ctypes.data, er.ctypes.data, eo.ctypes.data, nn.ctypes.data,
                                   ac.ctypes.data, nc.ctypes.data, ctypes.c_void_p(ws.data_ptr()),
                                   nbytes, s, ctypes.byref(h))
    if rc:
        raise InetError(rc, "inet_batch_load")
    return Handle(h, ws, rules, n)


def load(rules, net: "nets.Net", agent_cap: int = 0, name_cap: int = 0, stream=None,
         device="cuda") -> Handle:
    """Load one net (inet_load)."""
    import torch
    nbytes = workspace_bytes(rules, [net.n_agents], [net.n_eqs], [net.n_names], [agent_cap],
                             [name_cap])
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    s, _ = _stream_handle(stream)
    R = RulesArg(rules)
    la, po = _arr(net.label, np.int32), _arr(net.port, np.int32)
    el, er = _arr(net.eq_lhs, np.int32), _arr(net.eq_rhs, np.int32)
    h = ctypes.c_void_p()
    rc = library().inet_load(R.ptr, la.ctypes.data, po.ctypes.data, net.n_agents, el.ctypes.data,
                             er.ctypes.data, net.n_eqs, net.n_names, agent_cap, name_cap,
                             ctypes.c_void_p(ws.data_ptr()), nbytes, s, ctypes.byref(h))
    if rc:
        raise InetError(rc, "inet_load")
    return Handle(h, ws, rules, 1)


def parallelism(rules, net, agent_cap: int = 0, name_cap: int = 0, max_steps: int = 1 << 22,
                **config) -> np.ndarray:
    """Active pairs reduced in each parallel step of ``net`` (the available
    parallelism of Section 4.1), from a reduction with inet_set_trace."""
    import torch
    agent_cap = agent_cap or max(4 * net.n_agents + 4096, 1 << 16)
    name_cap = name_cap or 4 * agent_cap
    h = load(rules, net, agent_cap=agent_cap, name_cap=name_cap)
    h.set_config(**config)
    buf = torch.zeros(max_steps, dtype=torch.int32, device="cuda")
    h.set_trace(0, buf)
    res = h.reduce()[0]
    if res.status not in (OK, STUCK):
        h.free()
        raise InetError(res.status, "parallelism")
    out = buf[: min(int(res.steps), max_steps)].cpu().numpy().copy()
    h.free()
    return out


def reduce_net(rules, net, agent_cap: int = 0, name_cap: int = 0, wg_size: int = 0,
               max_retries: int = 6, jump: bool = True, engine: int = 0, **extra):
    """Load, reduce and read back one net; on ENOMEM reload with 4x capacity.
    ``extra``: further configuration keys (CONFIG_KEYS).
    Returns (Result, normal-form stream, per-rule counts)."""
    agent_cap = agent_cap or max(4 * net.n_agents + 4096, 1 << 16)
    name_cap = name_cap or 4 * agent_cap
    for _ in range(max_retries):
        h = load(rules, net, agent_cap=agent_cap, name_cap=name_cap)
        h.set_config(wg_size=wg_size, jump=jump, engine=engine, **extra)
        res = h.reduce()[0]
        if res.status == ENOMEM:
            h.free()
            agent_cap *= 4
            name_cap *= 4
            continue
        nf = h.readback(0) if res.status in (OK, STUCK) else np.zeros(0, np.int32)
        pr = h.per_rule(0)
        h.free()
        return res, nf, pr
    raise InetError(ENOMEM, "reduce_net")


NOALLOC_SCRATCH_BYTES = 64 << 20  # INET_NOALLOC_SCRATCH_BYTES


def reduce_noalloc(rules, net, agent_cap: int = 0, name_cap: int = 0, max_steps: int = 0,
                   nf_words: int = 1 << 22, stream=None):
    """inet_reduce_noalloc: one net loaded, reduced and read back inside the
    library's static device array (no device allocation).  Returns (Result,
    normal-form stream or None, status)."""
    s, _ = _stream_handle(stream)
    R = RulesArg(rules)
    la, po = _arr(net.label, np.int32), _arr(net.port, np.int32)
    el, er = _arr(net.eq_lhs, np.int32), _arr(net.eq_rhs, np.int32)
    r = _Result()
    buf = np.zeros(max(1, nf_words), np.int32)
    n = ctypes.c_int64(0)
    rc = library().inet_reduce_noalloc(R.ptr, la.ctypes.data, po.ctypes.data, net.n_agents,
                                       el.ctypes.data, er.ctypes.data, net.n_eqs, net.n_names,
                                       agent_cap, name_cap, max_steps, s, ctypes.byref(r),
                                       buf.ctypes.data, buf.size, ctypes.byref(n))
    if rc not in (OK, STUCK, ELIMIT):
        raise InetError(rc, "inet_reduce_noalloc")
    res = _result(r)
    return res, (buf[: n.value].copy() if res.status in (OK, STUCK) else None), rc


def _result(r) -> Result:
    return Result(r.status, r.n_stuck, r.interactions, r.steps, r.agents_used, r.names_used,
                  r.max_frontier, r.loops)


class _ServeStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("max_resident", ctypes.c_int32),
                ("retries", ctypes.c_int32), ("wall_s", ctypes.c_double)]


class _ServeCapture(ctypes.Structure):
    _fields_ = [("per_rule", ctypes.c_void_p), ("want_nf", ctypes.c_void_p),
                ("nf_buf", ctypes.c_void_p), ("nf_cap", ctypes.c_int64),
                ("nf_pos", ctypes.c_void_p), ("nf_len", ctypes.c_void_p)]


class Server:
    """Continuous batching (inet_server_*): admit nets while others run."""

    def __init__(self, rules, max_slots: int, workspace_bytes: int, device="cuda"):
        import torch
        self.rules = rules
        self.R = RulesArg(rules)
        self.workspace = torch.empty(workspace_bytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        rc = library().inet_server_create(self.R.ptr, max_slots, ctypes.c_void_p(self.workspace.data_ptr()),
                                          workspace_bytes, ctypes.byref(h))
        if rc:
            raise InetError(rc, "inet_server_create")
        self._h = h
        self.max_slots = max_slots

    def set_config(self, wg_size: int = 0, jump: bool = True, max_resident: int = 0,
                   engine: int = 0, **extra):
        cfg = _config(wg_size, jump, max_resident, engine, extra)
        rc = library().inet_server_set_config(self._h, ctypes.byref(cfg))
        if rc:
            raise InetError(rc, "inet_server_set_config")

    def net_bytes(self, net, agent_cap=0, name_cap=0) -> int:
        out = ctypes.c_int64(0)
        rc = library().inet_server_net_bytes(self._h, net.n_agents, net.n_eqs, net.n_names, agent_cap,
                                             name_cap, ctypes.byref(out))
        if rc:
            raise InetError(rc, "inet_server_net_bytes")
        return int(out.value)

    def submit(self, net, agent_cap: int = 0, name_cap: int = 0, stream=None) -> Optional[int]:
        """Ticket, or None when there is no room (INET_EAGAIN)."""
        s, _ = _stream_handle(stream)
        la, po = _arr(net.label, np.int32), _arr(net.port, np.int32)
        el, er = _arr(net.eq_lhs, np.int32), _arr(net.eq_rhs, np.int32)
        t = ctypes.c_int64(0)
        rc = library().inet_server_submit(self._h, la.ctypes.data, po.ctypes.data, net.n_agents,
                                          el.ctypes.data, er.ctypes.data, net.n_eqs, net.n_names,
                                          agent_cap, name_cap, s, ctypes.byref(t))
        if rc == EAGAIN:
            return None
        if rc:
            raise InetError(rc, "inet_server_submit")
        return int(t.value)

    def run(self, pool, arrivals, pick, caps=None, round_steps: int = 256,
            time_limit: float = 600.0, stream=None, per_rule: bool = False,
            want_nf=None, nf_words: int = 1 << 24) -> dict:
        """The native serving loop (inet_server_run) over ``pool``: request i
        is ``pool[pick[i]]`` arriving ``arrivals[i]`` seconds after the start.
        ``caps[j] = (agent_cap, name_cap)`` or None for the defaults.  Returns
        per-request completion times, statuses, interaction counts and steps
        plus the loop's statistics; with ``per_rule`` also the per-rule counts
        of every request, and with ``want_nf`` (a boolean per request) the
        normal-form streams of the flagged requests (``nf[i]``, None for the
        others), read back within ``nf_words`` int32 words in all."""
        from .nets import pack
        s, _ = _stream_handle(stream)
        label, port, a_off, eql, eqr, e_off, n_names = pack(pool)
        label, port = _arr(label, np.int32), _arr(port, np.int32)
        eql, eqr = _arr(eql, np.int32), _arr(eqr, np.int32)
        a_off, e_off, n_names = _arr(a_off, np.int64), _arr(e_off, np.int64), _arr(n_names, np.int32)
        ac = nc = None
        if caps is not None:
            ac = _arr(np.asarray([c[0] for c in caps]), np.int64)
            nc = _arr(np.asarray([c[1] for c in caps]), np.int64)
        arr = _arr(np.asarray(arrivals, dtype=np.float64), np.float64)
        pk_ = _arr(np.asarray(pick), np.int32)
        n = len(arr)
        done = np.zeros(n, np.float64)
        status = np.zeros(n, np.int32)
        inter = np.zeros(n, np.uint64)
        steps = np.zeros(n, np.uint32)
        st = _ServeStats()
        ptr = lambda a: None if a is None else a.ctypes.data  # noqa: E731
        cap = None
        nr = max(1, self.rules.n_rules)
        pr = np.zeros((n, nr), np.uint64) if per_rule else None
        wnf = nf_buf = nf_pos = nf_len = None
        if want_nf is not None:
            wnf = _arr(np.asarray(want_nf, dtype=bool).astype(np.uint8), np.uint8)
            assert len(wnf) == n
            nf_buf = np.zeros(max(1, nf_words), np.int32)
            nf_pos = np.zeros(n, np.int64)
            nf_len = np.zeros(n, np.int64)
        if per_rule or want_nf is not None:
            cap = _ServeCapture(ptr(pr), ptr(wnf), ptr(nf_buf), 0 if nf_buf is None else nf_buf.size,
                                ptr(nf_pos), ptr(nf_len))
        rc = library().inet_server_run(
            self._h, len(pool), ptr(label), ptr(port), ptr(a_off), ptr(eql), ptr(eqr), ptr(e_off),
            ptr(n_names), ptr(ac), ptr(nc), n, ptr(arr), ptr(pk_), round_steps, time_limit, s,
            done.ctypes.data, status.ctypes.data, inter.ctypes.data, steps.ctypes.data,
            ctypes.byref(st), None if cap is None else ctypes.byref(cap))
        if rc:
            raise InetError(rc, "inet_server_run")
        out = {"done": done, "status": status, "interactions": inter, "steps": steps,
               "rounds": int(st.rounds), "max_resident": int(st.max_resident),
               "retries": int(st.retries), "wall": float(st.wall_s)}
        if per_rule:
            out["per_rule"] = pr[:, : self.rules.n_rules]
        if want_nf is not None:
            out["nf"] = [nf_buf[nf_pos[i]: nf_pos[i] + nf_len[i]].copy() if nf_pos[i] >= 0 else None
                         for i in range(n)]
        return out

    def step(self, max_steps: int, stream=None):
        s, _ = _stream_handle(stream)
        rc = library().inet_server_step(self._h, s, max_steps)
        if rc:
            raise InetError(rc, "inet_server_step")

    def poll(self, stream=None) -> List[int]:
        s, _ = _stream_handle(stream)
        out = []
        buf = np.zeros(1024, np.int64)
        while True:
            n = ctypes.c_int32(0)
            rc = library().inet_server_poll(self._h, s, buf.ctypes.data, buf.size, ctypes.byref(n))
            if rc:
                raise InetError(rc, "inet_server_poll")
            out.extend(int(x) for x in buf[: n.value])
            if n.value < buf.size:
                return out

    def result(self, ticket: int, stream_out: bool = True):
        r = _Result()
        if not stream_out:
            rc = library().inet_server_result(self._h, ticket, ctypes.byref(r), None, 0, None)
            return _result(r), None
        n = ctypes.c_int64(0)
        rc = library().inet_server_result(self._h, ticket, ctypes.byref(r), None, 0, ctypes.byref(n))
        res = _result(r)
        if rc != ERANGE:
            return res, None
        buf = np.zeros(max(1, n.value), np.int32)
        rc = library().inet_server_result(self._h, ticket, ctypes.byref(r), buf.ctypes.data, buf.size,
                                          ctypes.byref(n))
        if rc not in (OK, STUCK):
            raise InetError(rc, "inet_server_result")
        return res, buf[: n.value].copy()

    def per_rule(self, ticket: int) -> np.ndarray:
        out = np.zeros(max(1, self.rules.n_rules), np.uint64)
        rc = library().inet_server_per_rule(self._h, ticket, out.ctypes.data, out.size)
        if rc:
            raise InetError(rc, "inet_server_per_rule")
        return out[: self.rules.n_rules]

    def release(self, ticket: int):
        rc = library().inet_server_release(self._h, ticket)
        if rc:
            raise InetError(rc, "inet_server_release")

    def stats(self) -> dict:
        fb, fs, rn = ctypes.c_int64(0), ctypes.c_int32(0), ctypes.c_int32(0)
        library().inet_server_stats(self._h, ctypes.byref(fb), ctypes.byref(fs), ctypes.byref(rn))
        return {"free_bytes": int(fb.value), "free_slots": int(fs.value), "running": int(rn.value)}

    def free(self):
        if getattr(self, "_h", None):
            library().inet_server_free(self._h)
            self._h = None
            self.workspace = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class prim:
    """The ablation's device primitives (inet_prim_*) on torch device tensors:
    argument marshalling only."""

    @staticmethod
    def _ptr(t, dtype):
        import torch
        assert t.is_cuda and t.dtype == dtype and t.is_contiguous()
        return ctypes.c_void_p(t.data_ptr())

    @staticmethod
    def scan(x):
        """Inclusive prefix sum of an int64 tensor (as uint64, wrapping)."""
        import torch
        out = torch.empty_like(x)
        s, _ = _stream_handle(None)
        rc = library().inet_prim_scan(prim._ptr(x, torch.int64), prim._ptr(out, torch.int64),
                                      x.numel(), s)
        if rc:
            raise InetError(rc, "inet_prim_scan")
        return out

    @staticmethod
    def select(x, drop: int):
        """The elements of an int64 tensor that differ from ``drop`` (as
        uint64), in order."""
        import torch
        out = torch.empty_like(x)
        n = ctypes.c_int64(0)
        s, _ = _stream_handle(None)
        rc = library().inet_prim_select(prim._ptr(x, torch.int64), prim._ptr(out, torch.int64),
                                        x.numel(), int(drop) & ((1 << 64) - 1), ctypes.byref(n), s)
        if rc:
            raise InetError(rc, "inet_prim_select")
        return out[: n.value]

    @staticmethod
    def sort_pairs(keys, vals):
        """Stable sort of (int32 key as uint32, int64 value) pairs by key, in place."""
        import torch
        s, _ = _stream_handle(None)
        rc = library().inet_prim_sort_pairs(prim._ptr(keys, torch.int32), prim._ptr(vals, torch.int64),
                                            keys.numel(), s)
        if rc:
            raise InetError(rc, "inet_prim_sort_pairs")

    @staticmethod
    def reduce_by_key(keys, vals, op: int = 0):
        """Runs of equal adjacent keys folded (op 0: sum; 1: the merge of two
        equations sharing a variable).  Returns (keys, values) of the runs."""
        import torch
        ko = torch.empty_like(keys)
        vo = torch.empty_like(vals)
        n = ctypes.c_int64(0)
        s, _ = _stream_handle(None)
        rc = library().inet_prim_reduce_by_key(prim._ptr(keys, torch.int32), prim._ptr(vals, torch.int64),
                                               keys.numel(), prim._ptr(ko, torch.int32),
                                               prim._ptr(vo, torch.int64), op, ctypes.byref(n), s)
        if rc:
            raise InetError(rc, "inet_prim_reduce_by_key")
        return ko[: n.value], vo[: n.value]


def check_exports() -> List[str]:
    """Names from include/inet.h missing in the library (empty when complete)."""
    lib = library()
    return [n for n in EXPORTS if not hasattr(lib, n)]
