"""Oracle: byte-level regular-expression parser.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use the oracle.

The paper fixes no concrete syntax (it takes the language as an RE or an NFA,
Sect. 3.1).  This parser accepts the following byte-level syntax:

* ``e1|e2`` alternation, juxtaposition for concatenation, ``( )`` grouping
  (``()`` is the empty string);
* postfix ``*``, ``+``, ``?``, ``{m}``, ``{m,}``, ``{m,n}`` (0 <= m <= n <= 1000);
* ``.`` any byte 0..255;
* ``[...]`` bracket classes with ranges ``a-z``, a leading ``^`` for the
  complement over all 256 bytes, and escapes inside; a ``]`` right after
  ``[`` or ``[^`` is a literal, and so is a ``-`` first or last;
* escapes ``\\n \\t \\r \\f \\v \\0 \\xHH \\d`` (``\\d`` = ``[0-9]``); a backslash
  before any other byte makes that byte a literal;
* every other byte stands for itself (``^``, ``$``, ``]`` and ``}`` included).

The result is a tree of tuples:

  ('sym', frozenset_of_bytes) | ('eps',) | ('cat', (n1, n2, ...)) |
  ('alt', (n1, n2, ...)) | ('star', n) | ('plus', n) | ('opt', n) |
  ('rep', n, m, hi)        # hi is None for {m,}
"""

from __future__ import annotations

MAX_REPEAT = 1000


class ParseError(ValueError):
    def __init__(self, msg: str, offset: int):
        super().__init__(f"{msg} at offset {offset}")
        self.offset = offset


_SIMPLE_ESC = {
    ord("n"): 10, ord("t"): 9, ord("r"): 13, ord("f"): 12, ord("v"): 11, ord("0"): 0,
}


class _Parser:
    def __init__(self, pattern: bytes):
        self.p = bytes(pattern)
        self.i = 0

    def peek(self):
        return self.p[self.i] if self.i < len(self.p) else None

    def take(self):
        c = self.peek()
        if c is None:
            raise ParseError("unexpected end of pattern", self.i)
        self.i += 1
        return c

    # alternation ---------------------------------------------------------
    def alt(self):
        branches = [self.concat()]
        while self.peek() == ord("|"):
            self.i += 1
            branches.append(self.concat())
        return branches[0] if len(branches) == 1 else ("alt", tuple(branches))

    def concat(self):
        items = []
        while self.peek() is not None and self.peek() not in (ord("|"), ord(")")):
            items.append(self.postfix())
        if not items:
            return ("eps",)
        return items[0] if len(items) == 1 else ("cat", tuple(items))

    def postfix(self):
        node = self.atom()
        while True:
            c = self.peek()
            if c == ord("*"):
                self.i += 1
                node = ("star", node)
            elif c == ord("+"):
                self.i += 1
                node = ("plus", node)
            elif c == ord("?"):
                self.i += 1
                node = ("opt", node)
            elif c == ord("{"):
                node = self.braces(node)
            else:
                return node

    def number(self):
        j = self.i
        while self.peek() is not None and ord("0") <= self.peek() <= ord("9"):
            self.i += 1
        if j == self.i:
            raise ParseError("expected a number", self.i)
        v = int(self.p[j:self.i])
        if v > MAX_REPEAT:
            raise ParseError("repeat count too large", j)
        return v

    def braces(self, node):
        at = self.i
        self.i += 1  # '{'
        m = self.number()
        hi = m
        if self.peek() == ord(","):
            self.i += 1
            hi = None if self.peek() == ord("}") else self.number()
        if self.peek() != ord("}"):
            raise ParseError("expected '}'", self.i)
        self.i += 1
        if hi is not None and hi < m:
            raise ParseError("bad repeat bounds", at)
        return ("rep", node, m, hi)

    # atoms ---------------------------------------------------------------
    def atom(self):
        at = self.i
        c = self.take()
        if c == ord("("):
            node = self.alt()
            if self.peek() != ord(")"):
                raise ParseError("missing ')'", self.i)
            self.i += 1
            return node
        if c == ord(")"):
            raise ParseError("unbalanced ')'", at)
        if c in (ord("*"), ord("+"), ord("?"), ord("{")):
            raise ParseError("nothing to repeat", at)
        if c == ord("."):
            return ("sym", frozenset(range(256)))
        if c == ord("["):
            return ("sym", self.bracket())
        if c == ord("\\"):
            return ("sym", self.escape())
        return ("sym", frozenset([c]))

    def escape(self):
        at = self.i - 1
        c = self.take()
        if c in _SIMPLE_ESC:
            return frozenset([_SIMPLE_ESC[c]])
        if c == ord("d"):
            return frozenset(range(ord("0"), ord("9") + 1))
        if c == ord("x"):
            h = self.p[self.i:self.i + 2]
            if len(h) != 2 or any(ch not in b"0123456789abcdefABCDEF" for ch in h):
                raise ParseError("bad \\x escape", at)
            self.i += 2
            return frozenset([int(h, 16)])
        return frozenset([c])

    def class_byte(self):
        c = self.take()
        if c == ord("\\"):
            s = self.escape()
            return s
        return frozenset([c])

    def bracket(self):
        at = self.i - 1
        neg = False
        if self.peek() == ord("^"):
            neg = True
            self.i += 1
        members = set()
        first = True
        while True:
            c = self.peek()
            if c is None:
                raise ParseError("missing ']'", at)
            if c == ord("]") and not first:
                self.i += 1
                break
            first = False
            lo = self.class_byte()
            if (self.peek() == ord("-") and self.i + 1 < len(self.p)
                    and self.p[self.i + 1] != ord("]")):
                self.i += 1
                hi = self.class_byte()
                if len(lo) != 1 or len(hi) != 1:
                    raise ParseError("bad range", self.i)
                a, b = next(iter(lo)), next(iter(hi))
                if b < a:
                    raise ParseError("bad range", self.i)
                members.update(range(a, b + 1))
            else:
                members.update(lo)
        if neg:
            members = set(range(256)) - members
        return frozenset(members)


def parse(pattern: bytes):
    """Parse ``pattern`` (bytes) into the tuple tree described above."""
    if isinstance(pattern, str):
        pattern = pattern.encode("latin-1")
    ps = _Parser(pattern)
    node = ps.alt()
    if ps.i != len(ps.p):
        raise ParseError("unbalanced ')'", ps.i)
    return node
