"""Closed forms for the interaction counts and values of the arithmetic rule
system, derived by hand from the rule texts (independent of both evaluators).

Notation: a numeral S^k Z has value k.  Add(y,r) = x consumes x one S per
step: Add><S a times, then Add><Z once.  Mul(y,r) = x with x = S^a Z,
y = S^b Z fires Mul><S a times (each spawning a Dup of y and an Add of one
copy), the Dups copy b S's and one Z each, the Adds consume b S's each, the
final Mul><Z erases the last copy of y through b Era><S and one Era><Z.
Fib(r) = S^n Z computes fib(n) with fib(0) = fib(1) = 1.
"""
from __future__ import annotations

from functools import lru_cache


def add_count(a: int, b: int) -> int:
    return a + 1


def mul_count(a: int, b: int) -> int:
    return 2 * a * b + 3 * a + b + 2


def mul_per_rule(a: int, b: int) -> dict:
    return {"Add><S": a * b, "Add><Z": a, "Mul><S": a, "Mul><Z": 1, "Dup><S": a * b,
            "Dup><Z": a, "Era><S": b, "Era><Z": 1, "Fib><Z": 0, "Fib><S": 0,
            "Fib2><Z": 0, "Fib2><S": 0}


def fib_value(n: int) -> int:
    a, b = 1, 1  # fib(0), fib(1)
    for _ in range(n):
        a, b = b, a + b
    return a


@lru_cache(maxsize=None)
def fib_count(n: int) -> int:
    """T(0) = 1 (Fib><Z), T(1) = 2 (Fib><S, Fib2><Z); for n >= 2 Fib><S and
    Fib2><S (2), the Dup of S^(n-2) Z (n-1), then Fib(n-2) and Fib(n-1) and
    the Add consuming fib(n-2) (fib(n-2)+1)."""
    t = [1, 2]
    for k in range(2, n + 1):
        t.append(t[k - 1] + t[k - 2] + fib_value(k - 2) + k + 2)
    return t[n]


def tree_count(values) -> int:
    """Balanced Add tree, left operand principal: every internal node costs
    (sum of its left subtree) + 1."""
    values = list(values)
    total = 0
    level = values
    while len(level) > 1:
        nxt = []
        for i in range(0, len(level), 2):
            total += level[i] + 1
            nxt.append(level[i] + level[i + 1])
        level = nxt
    return total


def expr_value(e) -> int:
    if e[0] == "num":
        return e[1]
    if e[0] == "add":
        return expr_value(e[1]) + expr_value(e[2])
    if e[0] == "mul":
        return expr_value(e[1]) * expr_value(e[2])
    return fib_value(expr_value(e[1]))


def small_exprs(count: int, budget: int, max_num: int, limit: int, min_count: int = 1,
                **kw):
    """The first ``count`` seeds whose expression needs between min_count and
    limit interactions (values are checked first so huge ones are skipped
    without building their counts)."""
    from paper_1404_0076_amd import nets
    out = []
    seed = 0
    while len(out) < count and seed < 100000:
        net = nets.random_expr_net(seed, budget=budget, max_num=max_num, **kw)
        e = net.meta["expr"]
        if _bounded(e, limit):
            c = expr_count(e)
            if min_count <= c <= limit:
                out.append((seed, net))
        seed += 1
    return out


def _bounded(e, limit) -> bool:
    """True when every intermediate value is small enough to count cheaply."""
    if e[0] == "num":
        return True
    if not all(_bounded(s, limit) for s in e[1:]):
        return False
    v = expr_value(e)
    if e[0] == "fib":
        return expr_value(e[1]) <= 40
    return v <= limit


def expr_count(e) -> int:
    if e[0] == "num":
        return 0
    if e[0] == "fib":
        return expr_count(e[1]) + fib_count(expr_value(e[1]))
    c = expr_count(e[1]) + expr_count(e[2])
    v1, v2 = expr_value(e[1]), expr_value(e[2])
    if e[0] == "add":
        return c + add_count(v1, v2)
    return c + mul_count(v1, v2)


# number of agents in each rule's right-hand side (count of upper-case symbols
# in the rule text after the arrow), in ARITH_RULE_TEXTS order
def rhs_agent_counts(rule_texts) -> list:
    import re
    out = []
    for t in rule_texts:
        rhs = t.split("->", 1)[1]
        out.append(len(re.findall(r"\b[A-Z][A-Za-z0-9]*", rhs)))
    return out


# ---------------------------------------------------------------------------
# Benchmark programs of Section 4.1 (rule texts in nets.ACK_RULE_TEXTS and
# nets.ALGAE_RULE_TEXTS); histograms in rule order.


_ACK_ROWS: dict = {}


def ack_value(m: int, n: int) -> int:
    """Ackermann's function by its definition, A(0, n) = n + 1,
    A(m, 0) = A(m-1, 1), A(m, n) = A(m-1, A(m, n-1)), one row per m memoised."""
    if m == 0:
        return n + 1
    row = _ACK_ROWS.setdefault(m, [])
    while len(row) <= n:
        row.append(ack_value(m - 1, 1) if not row else ack_value(m - 1, row[-1]))
    return row[n]


@lru_cache(maxsize=None)
def ack_per_rule(m: int, n: int) -> tuple:
    """[A><Z, A><S, A2><Z, A2><S, Dup><S, Dup><Z] to reduce A(m, n):
    m = 0 fires A><Z once; m > 0 fires A><S, then n = 0 fires A2><Z and
    continues as A(m-1, 1), while n > 0 fires A2><S, copies S^(m-1) Z
    (m-1 Dup><S and one Dup><Z), and runs A(m, n-1) and A(m-1, A(m, n-1))."""
    if m == 0:
        return (1, 0, 0, 0, 0, 0)
    if n == 0:
        rest = ack_per_rule(m - 1, 1)
        return tuple(x + d for x, d in zip(rest, (0, 1, 1, 0, 0, 0)))
    inner = ack_per_rule(m, n - 1)
    outer = ack_per_rule(m - 1, ack_value(m, n - 1))
    return tuple(x + y + d for x, y, d in zip(inner, outer, (0, 1, 0, 1, m - 1, 1)))


def ack_count(m: int, n: int) -> int:
    return sum(ack_per_rule(m, n))


def algae_string(n: int) -> str:
    """Generation n of A -> AB, B -> A from the axiom A, by string rewriting."""
    s = "a"
    for _ in range(n):
        s = "".join("ab" if c == "a" else "a" for c in s)
    return s


@lru_cache(maxsize=None)
def _algae(sym: str, k: int) -> tuple:
    """[GA><Z, GA><S, GB><Z, GB><S, Dup><S, Dup><Z] to expand one symbol for
    k generations: GA><S copies S^(k-1) Z (k-1 Dup><S, one Dup><Z) and
    expands A and B for k-1; GB><S expands A for k-1."""
    if sym == "a":
        if k == 0:
            return (1, 0, 0, 0, 0, 0)
        a, b = _algae("a", k - 1), _algae("b", k - 1)
        return tuple(x + y + d for x, y, d in zip(a, b, (0, 1, 0, 0, k - 1, 1)))
    if k == 0:
        return (0, 0, 1, 0, 0, 0)
    return tuple(x + d for x, d in zip(_algae("a", k - 1), (0, 0, 0, 1, 0, 0)))


def algae_per_rule(n: int) -> tuple:
    return _algae("a", n)


def algae_count(n: int) -> int:
    return sum(algae_per_rule(n))


def decode_letters(nf, cat: int, letters: dict) -> str:
    """The single interface term of a normal-form stream (no residuals) read
    as a binary tree of ``cat`` nodes over nullary letter labels."""
    nf = [int(v) for v in nf]
    assert nf[0] == 1, "one interface term expected"
    out = []
    pos = 1
    pending = 1
    while pending:
        lab = nf[pos]
        pos += 1
        pending -= 1
        if lab == cat:
            pending += 2
        else:
            out.append(letters[lab])
    assert nf[pos:] == [0], "no residual equations expected"
    return "".join(out)
