"""Oracle: automaton constructions of the paper, written plainly.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use the oracle.

Everything here works on the full byte alphabet 0..255 with sparse transition
maps (a missing entry means "no move").  Nothing is blocked, fused or reordered
beyond the definitions cited at each function.

Automaton records
-----------------
NFA   : ``n`` states 0..n-1 with initial state 0 (the paper's q0), ``delta[q]``
        a dict byte -> frozenset of successors (the relation rho), ``final`` a
        frozenset (F).
DFA   : ``n`` states with initial state 0, ``delta[s]`` a dict byte -> state,
        ``final`` a frozenset.  Used for the subset DFA, the minimal DFA and
        also for the RI-DFA transition graph, whose moves are deterministic.
RIDFA : a DFA plus ``content[p]`` (the frozenset of NFA states that the state
        p stands for, Sect. 3.1) and ``initial[q]`` = the id of the singleton
        state {q} for every NFA state q.
"""

from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field

from .regex import parse


@dataclass
class NFA:
    n: int
    delta: list            # list of dict[int, frozenset[int]]
    final: frozenset

    def moves(self, q: int, b: int) -> frozenset:
        return self.delta[q].get(b, frozenset())


@dataclass
class DFA:
    n: int
    delta: list            # list of dict[int, int]
    final: frozenset


@dataclass
class RIDFA:
    n: int
    delta: list            # list of dict[int, int]
    final: frozenset       # F^RID: states whose content meets F
    content: list          # list of frozenset[int] (NFA states)
    initial: list          # initial[q] = id of the singleton {q}
    index: dict = field(default_factory=dict)   # content -> id


# ---------------------------------------------------------------------------
# RE -> position NFA (McNaughton-Yamada / Glushkov), Sect. 4.1
# ---------------------------------------------------------------------------

def _expand(node):
    """Rewrite bounded repeats into plain operators.

    e{m}    -> e e ... e (m copies)
    e{m,}   -> e ... e e*            (m copies, then a star)
    e{m,n}  -> e ... e (e (e (...)?)?)?   (m copies, then n-m nested options)
    Every copy is a separate subtree, so its positions are distinct.
    """
    kind = node[0]
    if kind in ("sym", "eps"):
        return node
    if kind in ("cat", "alt"):
        return (kind, tuple(_expand(c) for c in node[1]))
    if kind in ("star", "plus", "opt"):
        return (kind, _expand(node[1]))
    assert kind == "rep"
    body, m, hi = _expand(node[1]), node[2], node[3]
    parts = [body] * m
    if hi is None:
        parts.append(("star", body))
    elif hi > m:
        tail = ("opt", body)
        for _ in range(hi - m - 1):
            tail = ("opt", ("cat", (body, tail)))
        parts.append(tail)
    if not parts:
        return ("eps",)
    return parts[0] if len(parts) == 1 else ("cat", tuple(parts))


def position_nfa(pattern: bytes) -> NFA:
    """Position automaton of an RE: state 0 is q0, states 1..m are the symbol
    occurrences (positions) numbered left to right in the expanded expression.

    rho(0, b) = {p in first(E) : b in sym(p)},
    rho(p, b) = {p' in follow(p) : b in sym(p')},
    F = last(E), plus 0 when E is nullable.
    """
    tree = _expand(parse(pattern))
    syms = [None]                 # syms[p] = frozenset of bytes, p >= 1
    follow = [set()]

    def walk(node):
        kind = node[0]
        if kind == "sym":
            syms.append(node[1])
            follow.append(set())
            p = len(syms) - 1
            return False, {p}, {p}
        if kind == "eps":
            return True, set(), set()
        if kind == "cat":
            nullable, first, last = True, set(), set()
            for child in node[1]:
                n2, f2, l2 = walk(child)
                for x in last:
                    follow[x] |= f2
                first = first | f2 if nullable else first
                last = l2 | last if n2 else l2
                nullable = nullable and n2
            return nullable, first, last
        if kind == "alt":
            nullable, first, last = False, set(), set()
            for child in node[1]:
                n2, f2, l2 = walk(child)
                nullable |= n2
                first |= f2
                last |= l2
            return nullable, first, last
        n1, f1, l1 = walk(node[1])
        if kind in ("star", "plus"):
            for x in l1:
                follow[x] |= f1
        if kind == "plus":
            return n1, f1, l1
        return True, f1, l1       # star, opt

    nullable, first, last = walk(tree)
    m = len(syms) - 1
    delta = []
    for q in range(m + 1):
        succ = first if q == 0 else follow[q]
        d = {}
        for p in succ:
            for b in syms[p]:
                d.setdefault(b, set()).add(p)
        delta.append({b: frozenset(s) for b, s in d.items()})
    final = set(last)
    if nullable:
        final.add(0)
    return NFA(m + 1, delta, frozenset(final))


def nfa_from_edges(n: int, edges, final, alphabet: bytes = None) -> NFA:
    """Build an NFA from (q, symbols, q') triples, e.g. the paper's drawings.

    ``symbols`` is a bytes/str of symbols, or None for the whole ``alphabet``
    (the paper's label Sigma)."""
    delta = [dict() for _ in range(n)]
    for q, syms, r in edges:
        if syms is None:
            syms = alphabet
        if isinstance(syms, str):
            syms = syms.encode()
        for b in syms:
            delta[q].setdefault(b, set()).add(r)
    delta = [{b: frozenset(s) for b, s in d.items()} for d in delta]
    return NFA(n, delta, frozenset(final))


def trim(nfa: NFA) -> NFA:
    """Keep the states that are reachable from 0 and can reach F, renumbered
    in increasing order of their old numbers (so 0 stays 0).  When 0 itself
    cannot reach F the language is empty and the result has no states."""
    fwd = {0}
    work = [0]
    while work:
        q = work.pop()
        for succ in nfa.delta[q].values():
            for r in succ:
                if r not in fwd:
                    fwd.add(r)
                    work.append(r)
    pred = [set() for _ in range(nfa.n)]
    for q in range(nfa.n):
        for succ in nfa.delta[q].values():
            for r in succ:
                pred[r].add(q)
    bwd = set(nfa.final)
    work = list(nfa.final)
    while work:
        r = work.pop()
        for q in pred[r]:
            if q not in bwd:
                bwd.add(q)
                work.append(q)
    keep = sorted(fwd & bwd)
    if 0 not in keep:
        return NFA(0, [], frozenset())
    new = {q: i for i, q in enumerate(keep)}
    delta = []
    for q in keep:
        d = {}
        for b, succ in nfa.delta[q].items():
            s = frozenset(new[r] for r in succ if r in new)
            if s:
                d[b] = s
        delta.append(d)
    return NFA(len(keep), delta, frozenset(new[q] for q in nfa.final if q in new))


def nfa_step(nfa: NFA, S, b: int) -> frozenset:
    """rho(S, b): union of the moves of the states in S on b."""
    out = set()
    for q in S:
        out |= nfa.moves(q, b)
    return frozenset(out)


# ---------------------------------------------------------------------------
# NFA -> DFA powerset construction and Moore minimization
# ---------------------------------------------------------------------------

def _successor_map(nfa: NFA, S) -> dict:
    """For a subset S, the dict b -> rho(S, b) over the bytes with a move."""
    acc = {}
    for q in S:
        for b, succ in nfa.delta[q].items():
            acc.setdefault(b, set()).update(succ)
    return {b: frozenset(s) for b, s in acc.items()}


def subset_dfa(nfa: NFA):
    """Powerset DFA from {0} (textbook construction).  Returns (dfa, subsets),
    where subsets[s] is the NFA-state set of DFA state s.  The empty set is
    never created: a missing move stands for it."""
    if nfa.n == 0:
        return DFA(0, [], frozenset()), []
    start = frozenset([0])
    subsets = [start]
    index = {start: 0}
    delta = [None]
    work = deque([0])
    while work:
        s = work.popleft()
        d = {}
        for b, T in _successor_map(nfa, subsets[s]).items():
            if T not in index:
                index[T] = len(subsets)
                subsets.append(T)
                delta.append(None)
                work.append(index[T])
            d[b] = index[T]
        delta[s] = d
    final = frozenset(s for s, S in enumerate(subsets) if S & nfa.final)
    return DFA(len(subsets), delta, final), subsets


def moore_partition(n: int, delta, final) -> list:
    """Nerode (language-equivalence) classes of a deterministic transition
    graph with states 0..n-1, completed by an implicit dead state.

    Moore's refinement: start from {final, non-final}; split classes by the
    class of the successor on every byte until nothing changes.  A missing
    move goes to the dead state, so a move into the dead state's class and a
    missing move are the same and are left out of the signature.
    Returns cls[0..n] where cls[n] is the dead state's class.
    """
    dead = n
    cls = [1 if s in final else 0 for s in range(n)] + [0]
    while True:
        sigs = {}
        new = []
        for s in range(n + 1):
            moves = delta[s] if s < n else {}
            sig = (cls[s], frozenset((b, cls[t]) for b, t in moves.items()
                                     if cls[t] != cls[dead]))
            new.append(sigs.setdefault(sig, len(sigs)))
        if len(sigs) == len(set(cls)):
            return new
        cls = new


def minimize(dfa: DFA) -> DFA:
    """Minimal DFA, trimmed (no dead state) and canonically numbered.

    Canonical numbering: breadth-first from the initial class, scanning the
    bytes 0..255 in ascending order at each state, ids given on first
    discovery.  The result is unique for the language, so any two correct
    constructions agree id for id.  An empty language gives 0 states."""
    if dfa.n == 0:
        return DFA(0, [], frozenset())
    cls = moore_partition(dfa.n, dfa.delta, dfa.final)
    dead = cls[dfa.n]
    if cls[0] == dead:
        return DFA(0, [], frozenset())
    rep = {}
    for s in range(dfa.n):
        rep.setdefault(cls[s], s)
    ids = {cls[0]: 0}
    order = [cls[0]]
    k = 0
    while k < len(order):
        c = order[k]
        k += 1
        s = rep[c]
        for b in range(256):
            t = dfa.delta[s].get(b)
            if t is None or cls[t] == dead:
                continue
            if cls[t] not in ids:
                ids[cls[t]] = len(order)
                order.append(cls[t])
    delta = []
    for c in order:
        s = rep[c]
        delta.append({b: ids[cls[t]] for b, t in dfa.delta[s].items() if cls[t] != dead})
    final = frozenset(ids[c] for c in order if rep[c] in dfa.final)
    return DFA(len(order), delta, final)


def min_dfa_of(nfa: NFA) -> DFA:
    return minimize(subset_dfa(nfa)[0])


# ---------------------------------------------------------------------------
# RI-DFA, Sect. 3.1
# ---------------------------------------------------------------------------

def ri_dfa(nfa: NFA) -> RIDFA:
    """Reduced-interface DFA B = (P, Sigma, delta^B, I^B, F^B) of an NFA.

    The powerset construction is applied |Q_N| times, from {q0}, then {q1},
    and so on; each pass adds only the states and moves not yet present.
    P is the union of all passes, I^B the singletons, and F^B the states
    whose content holds a final NFA state.  delta^B is partial: an empty
    successor means the move is undefined."""
    content = []
    index = {}
    delta = []

    def add(S):
        index[S] = len(content)
        content.append(S)
        delta.append(None)
        return index[S]

    for q in range(nfa.n):
        S = frozenset([q])
        if S in index:
            continue
        work = deque([add(S)])
        while work:
            p = work.popleft()
            d = {}
            for b, T in _successor_map(nfa, content[p]).items():
                if T not in index:
                    work.append(add(T))
                d[b] = index[T]
            delta[p] = d
    final = frozenset(p for p, S in enumerate(content) if S & nfa.final)
    initial = [index[frozenset([q])] for q in range(nfa.n)]
    return RIDFA(len(content), delta, final, content, initial, index)


# ---------------------------------------------------------------------------
# Interface reduction by downgrading with delegation, Sect. 3.4
# ---------------------------------------------------------------------------

@dataclass
class Reduction:
    classes: list          # Nerode class of every RI-DFA state
    rep: list              # rep[q] = NFA state whose singleton is the delegate of {q}
    kept: list             # NFA states q whose singleton stays initial (rep[q] == q)


def interface_reduction(B: RIDFA) -> Reduction:
    """Nerode classes of B (its moves are deterministic from every state,
    initial ones included); in each class of initial singletons the one with
    the lowest NFA index stays initial and the others delegate to it.  The
    transition graph is left unchanged."""
    cls = moore_partition(B.n, B.delta, B.final)[: B.n]
    rep = []
    first = {}
    for q, p in enumerate(B.initial):
        first.setdefault(cls[p], q)
        rep.append(first[cls[p]])
    kept = [q for q in range(len(rep)) if rep[q] == q]
    return Reduction(cls, rep, kept)


def if_fun(B: RIDFA, plas) -> frozenset:
    """if(PLAS): the singleton states {q} of every q in the content of some
    state of PLAS (Sect. 3.2).  Returned as RI-DFA state ids."""
    out = set()
    for p in plas:
        for q in B.content[p]:
            out.add(B.initial[q])
    return frozenset(out)


def if_min_fun(B: RIDFA, red: Reduction, plas) -> frozenset:
    """if_min(PLAS): every singleton of if(PLAS) that is still initial, or its
    delegate when it was downgraded (Sect. 3.4)."""
    out = set()
    for p in plas:
        for q in B.content[p]:
            out.add(B.initial[red.rep[q]])
    return frozenset(out)


def quotient_nfa(nfa: NFA, red: Reduction) -> NFA:
    """N' = N / ==, where q == q' iff their singletons are Nerode-equivalent
    in B, i.e. q and q' have the same right language.  Class ids follow the
    lowest member, so the class of q0 is 0.  Merging states with equal right
    languages keeps the language of the NFA."""
    ids = {r: i for i, r in enumerate(sorted(set(red.rep)))}
    cid = [ids[red.rep[q]] for q in range(nfa.n)]
    delta = [dict() for _ in ids]
    for q in range(nfa.n):
        d = delta[cid[q]]
        for b, succ in nfa.delta[q].items():
            d.setdefault(b, set()).update(cid[r] for r in succ)
    delta = [{b: frozenset(s) for b, s in d.items()} for d in delta]
    final = frozenset(cid[q] for q in nfa.final)
    return NFA(len(ids), delta, final)


# ---------------------------------------------------------------------------
# everything the tests need for one expression
# ---------------------------------------------------------------------------

@dataclass
class Built:
    nfa: NFA               # trimmed position NFA N
    dfa: DFA               # minimal, trimmed, canonically numbered DFA
    B: RIDFA               # RI-DFA of N (Sect. 3.1)
    red: Reduction         # interface reduction of B (Sect. 3.4)
    nfa_q: NFA             # quotient NFA N'
    Bq: RIDFA              # RI-DFA of N'


def build_from_nfa(nfa: NFA) -> Built:
    nfa = trim(nfa)
    dfa = min_dfa_of(nfa)
    B = ri_dfa(nfa)
    red = interface_reduction(B)
    nq = quotient_nfa(nfa, red)
    Bq = ri_dfa(nq)
    return Built(nfa, dfa, B, red, nq, Bq)


def build(pattern: bytes) -> Built:
    return build_from_nfa(position_nfa(pattern))
