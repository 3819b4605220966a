"""Seeded synthetic inputs for the lightweight interaction calculus.

This module builds *inputs only*: a signature (symbols and their arities), rule
tables written in the calculus notation of the paper (Section 2.2, the
``alpha(x) = beta(y) -> Theta`` form), and nets as configurations
``<t | Delta>`` flattened into int32 arrays.  It performs no reduction and no
arithmetic of the method; both the GPU evaluator and the CPU oracle consume
the arrays it produces.

Flat net format (shared by every consumer):

* a *term ref* is an int32: ``r >= 0`` is agent ``r``; ``r < 0`` is name
  ``-1 - r``;
* ``label[n_agents]`` gives each agent's symbol, ``port[n_agents, 2]`` the refs
  attached to its auxiliary ports (entries at or beyond the arity are ignored
  and written as 0).  An agent ref in a port means that agent's principal port
  is attached there (a nested term ``alpha(..., beta(...), ...)``);
* ``eq_lhs[n_eqs]``, ``eq_rhs[n_eqs]`` are the two sides of each equation;
* names are ids in ``[0, n_names)``; a name occurring once in Delta belongs to
  the interface, which is ordered by ascending id.

Flat rule format: ``lhs[n_rules, 2]`` labels of the active pair; for rule ``k``
the words ``rhs[rhs_off[k]:rhs_off[k+1]]`` hold ``n_eq`` followed by the
equations of Theta, each as two prefix-encoded terms.  In a prefix-encoded term
a value ``>= 0`` is a label followed by its ``arity`` subterms and a value
``< 0`` is the name ``-1 - v``; inside a rule, names ``0 .. ar(alpha)-1`` are
alpha's auxiliary ports, the next ``ar(beta)`` names are beta's, and larger
names are bound names of Theta (replaced by fresh names at every use).
"""
from __future__ import annotations

import dataclasses
import math
import re
from typing import Dict, List, Sequence, Tuple

import numpy as np

MAX_ARITY = 2

# ---------------------------------------------------------------------------
# signature and rules
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Signature:
    names: List[str]
    arity: List[int]

    def label(self, sym: str) -> int:
        return self.names.index(sym)

    @property
    def n_symbols(self) -> int:
        return len(self.names)


@dataclasses.dataclass
class RuleTable:
    sig: Signature
    texts: List[str]
    lhs: np.ndarray  # int32 [n_rules, 2]
    rhs_off: np.ndarray  # int32 [n_rules + 1]
    rhs: np.ndarray  # int32 [rhs_off[-1]]

    @property
    def n_rules(self) -> int:
        return int(self.lhs.shape[0])

    def arity_array(self) -> np.ndarray:
        return np.asarray(self.sig.arity, dtype=np.int32)


_TOKEN = re.compile(r"\s*([A-Za-z_][A-Za-z_0-9']*|\(|\)|,|=|->|<|>|\|)")


def _tokenize(text: str) -> List[str]:
    pos, out = 0, []
    text = text.strip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m:
            raise ValueError(f"cannot parse {text[pos:]!r}")
        out.append(m.group(1))
        pos = m.end()
        while pos < len(text) and text[pos].isspace():
            pos += 1
    return out


class _TermParser:
    """Parses ``Sym(t, ...)`` / ``name`` terms; upper-case first letter = agent
    (the paper's convention of Section 3.3), lower-case = name."""

    def __init__(self, tokens: List[str]):
        self.t = tokens
        self.i = 0

    def peek(self):
        return self.t[self.i] if self.i < len(self.t) else None

    def take(self, expect=None):
        tok = self.peek()
        if tok is None or (expect is not None and tok != expect):
            raise ValueError(f"expected {expect!r}, got {tok!r}")
        self.i += 1
        return tok

    def term(self):
        tok = self.take()
        if tok[0].isupper():
            args = []
            if self.peek() == "(":
                self.take("(")
                if self.peek() != ")":
                    args.append(self.term())
                    while self.peek() == ",":
                        self.take(",")
                        args.append(self.term())
                self.take(")")
            return ("A", tok, args)
        if tok[0].islower() or tok[0] == "_":
            return ("N", tok)
        raise ValueError(f"bad term token {tok!r}")

    def equations(self, stop=None):
        eqs = []
        if self.peek() is None or self.peek() == stop:
            return eqs
        while True:
            lhs = self.term()
            self.take("=")
            rhs = self.term()
            eqs.append((lhs, rhs))
            if self.peek() == ",":
                self.take(",")
                continue
            return eqs


def parse_rules(sig: Signature, texts: Sequence[str]) -> RuleTable:
    """Rules as in the paper: ``Add(y,r) = S(x) -> Add(y,w) = x, r = S(w)``."""
    lhs_l, words, offs = [], [], [0]
    for text in texts:
        toks = _tokenize(text)
        p = _TermParser(toks)
        a = p.term()
        p.take("=")
        b = p.term()
        p.take("->")
        eqs = p.equations()
        if p.peek() is not None:
            raise ValueError(f"trailing tokens in rule {text!r}")
        if a[0] != "A" or b[0] != "A":
            raise ValueError(f"rule LHS must be an active pair: {text!r}")
        la, lb = sig.label(a[1]), sig.label(b[1])
        if len(a[2]) != sig.arity[la] or len(b[2]) != sig.arity[lb]:
            raise ValueError(f"arity mismatch in LHS of {text!r}")
        names: Dict[str, int] = {}
        for arg in list(a[2]) + list(b[2]):
            if arg[0] != "N" or arg[1] in names:
                raise ValueError(f"LHS arguments must be distinct names: {text!r}")
            names[arg[1]] = len(names)

        def enc(t, out):
            if t[0] == "N":
                if t[1] not in names:
                    names[t[1]] = len(names)
                out.append(-1 - names[t[1]])
            else:
                lab = sig.label(t[1])
                if len(t[2]) != sig.arity[lab]:
                    raise ValueError(f"arity mismatch for {t[1]} in {text!r}")
                out.append(lab)
                for s in t[2]:
                    enc(s, out)

        w = [len(eqs)]
        for l, r in eqs:
            enc(l, w)
            enc(r, w)
        lhs_l.append((la, lb))
        words.extend(w)
        offs.append(len(words))
    return RuleTable(
        sig=sig,
        texts=list(texts),
        lhs=np.asarray(lhs_l, dtype=np.int32).reshape(-1, 2),
        rhs_off=np.asarray(offs, dtype=np.int32),
        rhs=np.asarray(words, dtype=np.int32),
    )


# The arithmetic system used by every workload.  Port order: the first
# auxiliary port is the (non-principal) operand or copy, the result comes last;
# the principal port is the term itself.  Addition is the paper's pair of
# equations in Section 2.2 (Example 2); multiplication, duplication, erasure and
# Fibonacci are written in the same style for the synthetic workloads.
ARITH_SIG = Signature(
    names=["Z", "S", "Add", "Mul", "Dup", "Era", "Fib", "Fib2"],
    arity=[0, 1, 2, 2, 2, 0, 1, 1],
)
Z, S, ADD, MUL, DUP, ERA, FIB, FIB2 = range(8)

ADD_RULE_TEXTS = [
    "Add(y,r) = S(x) -> Add(y,w) = x, r = S(w)",
    "Add(y,r) = Z -> r = y",
]
ARITH_RULE_TEXTS = ADD_RULE_TEXTS + [
    "Mul(y,r) = S(x) -> Dup(y1,y2) = y, Add(w,r) = y1, Mul(y2,w) = x",
    "Mul(y,r) = Z -> Era = y, r = Z",
    "Dup(p,q) = S(x) -> p = S(x1), q = S(x2), Dup(x1,x2) = x",
    "Dup(p,q) = Z -> p = Z, q = Z",
    "Era = S(x) -> Era = x",
    "Era = Z ->",
    "Fib(r) = Z -> r = S(Z)",
    "Fib(r) = S(x) -> Fib2(r) = x",
    "Fib2(r) = Z -> r = S(Z)",
    "Fib2(r) = S(x) -> Dup(x1,x2) = x, Fib(a) = x1, Fib(b) = S(x2), Add(b,r) = a",
]


def arith_rules() -> RuleTable:
    return parse_rules(ARITH_SIG, ARITH_RULE_TEXTS)


def add_rules() -> RuleTable:
    return parse_rules(ARITH_SIG, ADD_RULE_TEXTS)


# The benchmark programs of Section 4.1 (Ackermann, an L-System), written in
# the same style; the paper does not print its encodings, so these are ours.
#
# Ackermann: A(n, r) with its principal port on the first argument m;
# A2(p, r) holds the predecessor p of m while the second argument is examined.
#   A(0, n) = n + 1;  A(m+1, 0) = A(m, 1);  A(m+1, n+1) = A(m, A(m+1, n)).
ACK_SIG = Signature(names=["Z", "S", "Dup", "A", "A2"], arity=[0, 1, 2, 2, 2])
ACK_RULE_TEXTS = [
    "A(n,r) = Z -> r = S(n)",
    "A(n,r) = S(p) -> A2(p,r) = n",
    "A2(p,r) = Z -> A(S(Z),r) = p",
    "A2(p,r) = S(q) -> Dup(p1,p2) = p, A(q,t) = S(p1), A(t,r) = p2",
    "Dup(a,b) = S(x) -> a = S(x1), b = S(x2), Dup(x1,x2) = x",
    "Dup(a,b) = Z -> a = Z, b = Z",
]

# Algae L-System (A -> AB, B -> A): GA(r) / GB(r) expand symbol A / B for the
# number of generations on their principal port; Cat joins two strings and
# La / Lb are the letters of the final generation.
ALGAE_SIG = Signature(names=["Z", "S", "Dup", "GA", "GB", "Cat", "La", "Lb"],
                      arity=[0, 1, 2, 1, 1, 2, 0, 0])
ALGAE_RULE_TEXTS = [
    "GA(r) = Z -> r = La",
    "GA(r) = S(k) -> Dup(k1,k2) = k, r = Cat(x,y), GA(x) = k1, GB(y) = k2",
    "GB(r) = Z -> r = Lb",
    "GB(r) = S(k) -> GA(r) = k",
    "Dup(a,b) = S(x) -> a = S(x1), b = S(x2), Dup(x1,x2) = x",
    "Dup(a,b) = Z -> a = Z, b = Z",
]


def ackermann_rules() -> RuleTable:
    return parse_rules(ACK_SIG, ACK_RULE_TEXTS)


def algae_rules() -> RuleTable:
    return parse_rules(ALGAE_SIG, ALGAE_RULE_TEXTS)


# ---------------------------------------------------------------------------
# nets
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Net:
    label: np.ndarray  # int32 [n_agents]
    port: np.ndarray  # int32 [n_agents, 2]
    eq_lhs: np.ndarray  # int32 [n_eqs]
    eq_rhs: np.ndarray  # int32 [n_eqs]
    n_names: int
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_agents(self) -> int:
        return int(self.label.shape[0])

    @property
    def n_eqs(self) -> int:
        return int(self.eq_lhs.shape[0])


def name_ref(k: int) -> int:
    return -1 - k


class NetBuilder:
    """Accumulates agents/equations in numpy chunks (numerals are built as
    whole blocks so that nets with 10^6 agents are cheap to generate)."""

    def __init__(self, sig: Signature):
        self.sig = sig
        self._labels: List[np.ndarray] = []
        self._ports: List[np.ndarray] = []
        self._n = 0
        self._eqs: List[Tuple[int, int]] = []
        self.n_names = 0

    def name(self) -> int:
        k = self.n_names
        self.n_names += 1
        return name_ref(k)

    def agent(self, sym, *args) -> int:
        lab = sym if isinstance(sym, (int, np.integer)) else self.sig.label(sym)
        if len(args) != self.sig.arity[lab]:
            raise ValueError("arity mismatch")
        p = list(args) + [0] * (MAX_ARITY - len(args))
        self._labels.append(np.asarray([lab], dtype=np.int32))
        self._ports.append(np.asarray([p], dtype=np.int32))
        self._n += 1
        return self._n - 1

    def numeral(self, k: int) -> int:
        """S^k Z as a block: Z first, then each S holds the previous agent."""
        base = self._n
        lab = np.full(k + 1, self.sig.label("S"), dtype=np.int32)
        lab[0] = self.sig.label("Z")
        prt = np.zeros((k + 1, 2), dtype=np.int32)
        prt[1:, 0] = np.arange(base, base + k, dtype=np.int32)
        self._labels.append(lab)
        self._ports.append(prt)
        self._n += k + 1
        return base + k

    def eq(self, t: int, u: int) -> None:
        self._eqs.append((int(t), int(u)))

    def build(self, **meta) -> Net:
        label = np.concatenate(self._labels) if self._labels else np.zeros(0, np.int32)
        port = np.concatenate(self._ports) if self._ports else np.zeros((0, 2), np.int32)
        e = np.asarray(self._eqs, dtype=np.int32).reshape(-1, 2)
        return Net(label=label, port=port.reshape(-1, 2), eq_lhs=e[:, 0].copy(),
                   eq_rhs=e[:, 1].copy(), n_names=self.n_names, meta=meta)


def parse_net(sig: Signature, text: str) -> Net:
    """``<r | Add(Z, r) = S(Z)>``: names are numbered by first appearance, the
    interface list before the bar is only a comment (the interface is derived:
    the names that occur once in Delta, ascending id)."""
    toks = _tokenize(text)
    p = _TermParser(toks)
    p.take("<")
    iface = []
    while p.peek() not in ("|", None):
        tok = p.take()
        if tok != ",":
            iface.append(tok)
    p.take("|")
    eqs = p.equations(stop=">")
    p.take(">")
    b = NetBuilder(sig)
    names: Dict[str, int] = {}
    for nm in iface:
        if nm not in names:
            names[nm] = -1 - len(names)

    def build(t):
        if t[0] == "N":
            if t[1] not in names:
                names[t[1]] = -1 - len(names)
            return names[t[1]]
        kids = [build(s) for s in t[2]]
        return b.agent(t[1], *kids)

    for l, r in eqs:
        b.eq(build(l), build(r))
    b.n_names = len(names)
    return b.build(text=text)


# ---------------------------------------------------------------------------
# workload families (all seeded with numpy PCG64)
# ---------------------------------------------------------------------------


def add_net(a: int, b: int) -> Net:
    """<r | Add(S^b Z, r) = S^a Z>."""
    nb = NetBuilder(ARITH_SIG)
    r = nb.name()
    y = nb.numeral(b)
    x = nb.numeral(a)
    nb.eq(nb.agent(ADD, y, r), x)
    return nb.build(family="add", a=a, b=b)


def mul_net(a: int, b: int) -> Net:
    """<r | Mul(S^b Z, r) = S^a Z>."""
    nb = NetBuilder(ARITH_SIG)
    r = nb.name()
    y = nb.numeral(b)
    x = nb.numeral(a)
    nb.eq(nb.agent(MUL, y, r), x)
    return nb.build(family="mul", a=a, b=b)


def fib_net(n: int) -> Net:
    """<r | Fib(r) = S^n Z>."""
    nb = NetBuilder(ARITH_SIG)
    r = nb.name()
    x = nb.numeral(n)
    nb.eq(nb.agent(FIB, r), x)
    return nb.build(family="fib", n=n)


def ackermann_net(m: int, n: int) -> Net:
    """<r | A(S^n Z, r) = S^m Z>: Ackermann(m, n)."""
    nb = NetBuilder(ACK_SIG)
    r = nb.name()
    y = nb.numeral(n)
    x = nb.numeral(m)
    nb.eq(nb.agent("A", y, r), x)
    return nb.build(family="ackermann", m=m, n=n)


def algae_net(n: int) -> Net:
    """<r | GA(r) = S^n Z>: generation n of the algae L-System from axiom A."""
    nb = NetBuilder(ALGAE_SIG)
    r = nb.name()
    x = nb.numeral(n)
    nb.eq(nb.agent("GA", r), x)
    return nb.build(family="algae", n=n)


def add_tree_net(values: Sequence[int]) -> Net:
    """Balanced binary tree of Add agents over numerals ``values`` (leaves in
    the given order, length a power of two).  Each internal node v becomes one
    equation ``Add(t_R, r_v) = t_L``: the left operand is the principal one,
    ``t_L``/``t_R`` are the leaf numerals or the children's result names, and
    the root's result name is the interface."""
    values = [int(v) for v in values]
    n = len(values)
    if n < 2 or n & (n - 1):
        raise ValueError("number of leaves must be a power of two >= 2")
    nb = NetBuilder(ARITH_SIG)
    root = nb.name()  # name 0 = interface
    level = [("leaf", v) for v in values]

    def materialise(item):
        return nb.numeral(item[1]) if item[0] == "leaf" else item[1]

    depth = int(math.log2(n))
    for d in range(depth):
        nxt = []
        for i in range(0, len(level), 2):
            left, right = level[i], level[i + 1]
            r = root if (d == depth - 1) else nb.name()
            tl = materialise(left)
            tr = materialise(right)
            nb.eq(nb.agent(ADD, tr, r), tl)
            nxt.append(("name", r))
        level = nxt
    return nb.build(family="addtree", values=values)


def config1_add_tree(seed: int = 0, n_leaves: int = 1024, vmax: int = 256) -> Net:
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = rng.integers(0, vmax, n_leaves)
    net = add_tree_net(vals)
    net.meta.update(config=1, seed=seed)
    return net


def config2_mul(seed: int = 0) -> Net:
    rng = np.random.Generator(np.random.PCG64(seed))
    a, b = (int(v) for v in rng.integers(500, 2001, 2))
    net = mul_net(a, b)
    net.meta.update(config=2, seed=seed)
    return net


FIB_CONFIG_NS = (20, 23, 25, 27)


def config3_fib(n: int = 27) -> Net:
    net = fib_net(n)
    net.meta.update(config=3)
    return net


def _size_to_net(family: int, s: float, rng: np.random.Generator) -> Net:
    """Shape a net of family 1 (Add tree), 2 (Mul) or 3 (Fib) whose amount of
    work is *roughly* ``s`` interactions.  Only coarse size proxies are used
    (tree volume, a*b, golden-ratio growth); exact counts come from the
    evaluators themselves."""
    if family == 1:
        d = int(min(10, max(1, round(math.log2(max(s, 2)) / 2))))
        m = max(1, int(round(2.0 * s / ((1 << d) * d))))
        vals = rng.integers(0, 2 * m, 1 << d)
        return add_tree_net(vals)
    if family == 2:
        a = max(1, int(round(math.sqrt(s / 2.0))))
        b = max(0, int(round(s / (2.0 * a + 1.0))))
        return mul_net(a, b)
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    n = int(max(0, min(40, round(math.log(max(s, 1.0) / 4.0) / math.log(phi)))))
    return fib_net(n)


def config4_batch(seed: int = 0, n_nets: int = 4096, median: float = 2000.0,
                  sigma: float = 1.75, smin: float = 16.0, smax: float = 1.0e6) -> List[Net]:
    """Independent nets drawn from the three families, sizes lognormal."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fam = rng.integers(1, 4, n_nets)
    size = np.clip(rng.lognormal(math.log(median), sigma, n_nets), smin, smax)
    nets = []
    for i in range(n_nets):
        net = _size_to_net(int(fam[i]), float(size[i]), rng)
        net.meta.update(config=4, seed=seed, index=i, target=float(size[i]))
        nets.append(net)
    return nets


def config5_pool(seed: int = 2, n_nets: int = 65536, **kw) -> List[Net]:
    return config4_batch(seed=seed, n_nets=n_nets, **kw)


def poisson_arrivals(seed: int, rate: float, duration: float) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream of the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rate * duration * 1.2 + 100)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, n))])
    return t[t < duration]


def random_expr_net(seed: int, budget: int = 12, max_num: int = 4,
                    ops=("Add", "Mul", "Fib"), fib_budget: int = 2, op_depth: int = 2) -> Net:
    """A random arithmetic expression over the ARITH system as one net:
    e ::= S^k Z | Add(e, e) | Mul(e, e) | Fib(e).  Sub-results are connected
    through names, so the net has several initial equations.  The expression
    tree is returned in ``meta["expr"]`` as nested tuples
    ``("num", k) | ("add", e1, e2) | ("mul", e1, e2) | ("fib", e)`` where e1 is
    the operand attached to the operator's principal port.  The top
    ``op_depth`` levels are always operators."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = NetBuilder(ARITH_SIG)
    root = nb.name()

    def gen(res_name: int, budget: int, depth: int = 0):
        if budget <= 0 or (depth >= op_depth and rng.random() < 0.3):
            k = int(rng.integers(0, max_num + 1))
            nb.eq(res_name, nb.numeral(k))
            return ("num", k)
        op = ops[int(rng.integers(0, len(ops)))]
        if op == "Fib":
            x = nb.name()
            nb.eq(nb.agent(FIB, res_name), x)
            return ("fib", gen(x, min(budget - 1, fib_budget), depth + 1))
        x = nb.name()
        y = nb.name()
        lab = ADD if op == "Add" else MUL
        nb.eq(nb.agent(lab, y, res_name), x)
        e1 = gen(x, budget - 2, depth + 1)
        e2 = gen(y, budget - 2, depth + 1)
        return (op.lower(), e1, e2)

    expr = gen(root, budget)
    return nb.build(family="expr", seed=seed, expr=expr)


def pack(nets: Sequence[Net]):
    """Concatenate nets for the batched entry points: per-net offsets into the
    packed agent and equation arrays (refs stay local to each net)."""
    a_off = np.zeros(len(nets) + 1, dtype=np.int64)
    e_off = np.zeros(len(nets) + 1, dtype=np.int64)
    for i, n in enumerate(nets):
        a_off[i + 1] = a_off[i] + n.n_agents
        e_off[i + 1] = e_off[i] + n.n_eqs
    label = np.concatenate([n.label for n in nets]).astype(np.int32)
    port = np.concatenate([n.port for n in nets]).astype(np.int32).reshape(-1, 2)
    eql = np.concatenate([n.eq_lhs for n in nets]).astype(np.int32)
    eqr = np.concatenate([n.eq_rhs for n in nets]).astype(np.int32)
    n_names = np.asarray([n.n_names for n in nets], dtype=np.int32)
    return label, port, a_off, eql, eqr, e_off, n_names
