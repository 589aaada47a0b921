"""Brute-force regular-expression membership, independent of the oracle.

It has its own tokenizer and parser for the same byte-level syntax (see
oracle/regex.py for the grammar) and decides membership straight from the
set semantics of regular expressions, with no automaton:

  M(e, i) = the set of j such that e matches x[i:j]
  M(sym S, i)   = {i+1} if x[i] in S
  M(e1 e2, i)   = union of M(e2, k) for k in M(e1, i)
  M(e1 | e2, i) = M(e1, i) | M(e2, i)
  M(e*, i)      = least fixed point of {i} | M(e, .) applied to it

and x is in L(e) iff len(x) in M(e, 0).  Memoized on (node, i), so it runs
in polynomial time where a backtracking matcher may take exponential time.
"""

from functools import lru_cache

_ESC = {"n": 10, "t": 9, "r": 13, "f": 12, "v": 11, "0": 0}


def _tokens(p: bytes):
    """Yield (kind, value) tokens: ('set', frozenset) for symbol classes,
    ('op', ch) for operators, ('rep', (m, hi)) for braces."""
    i, n = 0, len(p)
    out = []
    while i < n:
        ch = chr(p[i])
        if ch == "\\":
            v, i = _escape(p, i + 1)
            out.append(("set", v))
            continue
        if ch == ".":
            out.append(("set", frozenset(range(256))))
            i += 1
        elif ch == "[":
            v, i = _bracket(p, i + 1)
            out.append(("set", v))
        elif ch in "()|*+?":
            out.append(("op", ch))
            i += 1
        elif ch == "{":
            j = p.index(b"}", i)
            body = p[i + 1:j].decode()
            if "," in body:
                a, b = body.split(",", 1)
                rng = (int(a), None if b == "" else int(b))
            else:
                rng = (int(body), int(body))
            out.append(("rep", rng))
            i = j + 1
        else:
            out.append(("set", frozenset([p[i]])))
            i += 1
    return out


def _escape(p, i):
    ch = chr(p[i])
    if ch in _ESC:
        return frozenset([_ESC[ch]]), i + 1
    if ch == "d":
        return frozenset(range(48, 58)), i + 1
    if ch == "x":
        return frozenset([int(p[i + 1:i + 3], 16)]), i + 3
    return frozenset([p[i]]), i + 1


def _bracket(p, i):
    neg = p[i] == ord("^")
    if neg:
        i += 1
    members = set()
    start = i
    while not (p[i] == ord("]") and i > start):
        if p[i] == ord("\\"):
            lo, i = _escape(p, i + 1)
        else:
            lo, i = frozenset([p[i]]), i + 1
        if p[i] == ord("-") and p[i + 1] != ord("]"):
            if p[i + 1] == ord("\\"):
                hi, i = _escape(p, i + 2)
            else:
                hi, i = frozenset([p[i + 1]]), i + 2
            members |= set(range(min(lo), max(hi) + 1))
        else:
            members |= lo
    if neg:
        members = set(range(256)) - members
    return frozenset(members), i + 1


class _P:
    def __init__(self, toks):
        self.t = toks
        self.k = 0

    def peek(self):
        return self.t[self.k] if self.k < len(self.t) else (None, None)

    def expr(self):
        alts = [self.seq()]
        while self.peek() == ("op", "|"):
            self.k += 1
            alts.append(self.seq())
        return ("|", tuple(alts))

    def seq(self):
        items = []
        while self.peek()[0] is not None and self.peek() not in (("op", "|"), ("op", ")")):
            items.append(self.factor())
        return (".", tuple(items))

    def factor(self):
        kind, v = self.t[self.k]
        self.k += 1
        if kind == "set":
            node = ("s", v)
        elif v == "(":
            node = self.expr()
            assert self.t[self.k] == ("op", ")")
            self.k += 1
        else:
            raise ValueError("bad token %r" % (v,))
        while True:
            kind, v = self.peek()
            if kind == "op" and v in "*+?":
                self.k += 1
                node = {"*": ("*", node), "+": ("+", node), "?": ("?", node)}[v]
            elif kind == "rep":
                self.k += 1
                node = ("{", node, v[0], v[1])
            else:
                return node


def compile_brute(pattern: bytes):
    tree = _P(_tokens(bytes(pattern))).expr()

    def fullmatch(x: bytes) -> bool:
        n = len(x)

        @lru_cache(maxsize=None)
        def M(node, i):
            op = node[0]
            if op == "s":
                return frozenset([i + 1]) if i < n and x[i] in node[1] else frozenset()
            if op == "|":
                out = set()
                for a in node[1]:
                    out |= M(a, i)
                return frozenset(out)
            if op == ".":
                cur = {i}
                for a in node[1]:
                    nxt = set()
                    for k in cur:
                        nxt |= M(a, k)
                    cur = nxt
                return frozenset(cur)
            if op == "?":
                return frozenset({i}) | M(node[1], i)
            if op in "*+":
                reach, frontier = set(), {i}
                if op == "*":
                    reach.add(i)
                while frontier:
                    nxt = set()
                    for k in frontier:
                        nxt |= M(node[1], k)
                    frontier = nxt - reach
                    reach |= nxt
                return frozenset(reach)
            # bounded or unbounded repeat {m,hi}
            body, m, hi = node[1], node[2], node[3]
            cur = {i}
            for _ in range(m):
                nxt = set()
                for k in cur:
                    nxt |= M(body, k)
                cur = nxt
            if hi is None:
                return _star_from(cur, body)
            out = set(cur)
            for _ in range(hi - m):
                nxt = set()
                for k in cur:
                    nxt |= M(body, k)
                cur = nxt
                out |= cur
            return frozenset(out)

        def _star_from(start, body):
            reach, frontier = set(start), set(start)
            while frontier:
                nxt = set()
                for k in frontier:
                    nxt |= M(body, k)
                frontier = nxt - reach
                reach |= nxt
            return frozenset(reach)

        return n in M(tree, 0)

    return fullmatch
