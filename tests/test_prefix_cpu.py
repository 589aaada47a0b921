"""Host construction of the transformation automaton of the starts (no GPU).

The warm-up's first bytes are read by an automaton whose state after a word
u is the vector of the states every start reaches on u.  ri_build expands
every word of up to ``prefix_depth`` bytes; its state count must be the number
of distinct such vectors, counted here by a breadth-first search over the
oracle's automata: B' = RI-DFA(N') with the singletons of N' as starts
(Sect. 3.4), and the minimal DFA with every state as a start.  State ids
differ between the two constructions, the number of distinct vectors does
not.
"""

import numpy as np
import pytest

import oracle
from workloads import gen

ri = pytest.importorskip("paper_2412_14975_amd")

CAP = 65535            # the builder's state cap
WORK = 1 << 27         # and its budget for states x classes x starts
MAX_DEPTH = 64


def dense(delta, n):
    """[n + 1][256] successor table; row n is the dead state."""
    t = np.full((n + 1, 256), n, dtype=np.int32)
    for s in range(n):
        for b, d in delta[s].items():
            t[s, b] = d
    return t


def levels(delta, n, starts):
    """Sizes of the union of the vectors of all words of length <= d, for
    d = 0, 1, ... until no new vector appears (or 64)."""
    t = dense(delta, n)
    cols = {}
    for b in range(256):                       # one representative per byte class
        cols.setdefault(t[:, b].tobytes(), b)
    reps = list(cols.values())
    root = np.array(starts, dtype=np.int32)
    seen = {root.tobytes()}
    level = [root]
    sizes = [1]
    for _ in range(MAX_DEPTH):
        nxt = {}
        for v in level:
            for b in reps:
                w = t[v, b]
                nxt.setdefault(w.tobytes(), w)
        level = list(nxt.values())
        seen.update(nxt)
        sizes.append(len(seen))
    return sizes, len(reps)


def expected(sizes, K, L):
    cap = min(CAP, WORK // (K * L))
    depth = 0
    for d in range(1, len(sizes)):
        if sizes[d] > cap:
            break
        depth = d
    return depth, sizes[depth]


@pytest.mark.parametrize("pattern", [b"(ab|c)*d", gen.regexp_family(3), b"(a|b)*a(a|b)(a|b)",
                                     b"(foo|bar|ba[rz]q)*x?", b"([a-c]{2,4}-)*[0-9]"])
def test_prefix_state_count_small(pattern):
    b = oracle.build(pattern)
    h = ri.ri_build(pattern)
    try:
        info = ri.ri_info(h)
    finally:
        ri.ri_free(h)
    Bq = b.Bq
    starts = [Bq.initial[q] for q in range(b.nfa_q.n)]
    sizes, K = levels(Bq.delta, Bq.n, starts)
    assert info["starts"][0] == len(starts)
    assert (info["prefix_depth"][0], info["prefix_states"][0]) == expected(sizes, K, len(starts))
    d = b.dfa
    sizes, K = levels(d.delta, d.n, list(range(d.n)))
    assert (info["prefix_depth"][1], info["prefix_states"][1]) == expected(sizes, K, d.n)


def test_prefix_log_grammar():
    """The log-lines grammar (227 starts, 22 classes): the budget allows
    2^27 / (22 * 227) = 26877 states, reached between depths 25 and 26."""
    rx = gen.c3_regex()
    b = oracle.build(rx)
    Bq = b.Bq
    starts = [Bq.initial[q] for q in range(b.nfa_q.n)]
    t = dense(Bq.delta, Bq.n)
    cols = {}
    for x in range(256):
        cols.setdefault(t[:, x].tobytes(), x)
    reps = list(cols.values())
    assert (len(starts), len(reps)) == (227, 22)
    seen = set()
    root = np.array(starts, dtype=np.int32)
    seen.add(root.tobytes())
    level = [root]
    sizes = [1]
    for _ in range(26):
        nxt = {}
        for v in level:
            for x in reps:
                w = t[v, x]
                nxt.setdefault(w.tobytes(), w)
        level = list(nxt.values())
        seen.update(nxt)
        sizes.append(len(seen))
    h = ri.ri_build(rx)
    try:
        info = ri.ri_info(h)
    finally:
        ri.ri_free(h)
    assert sizes[25] <= (1 << 27) // (22 * 227) < sizes[26]
    assert (info["prefix_depth"][0], info["prefix_states"][0]) == (25, sizes[25])


def test_prefix_option():
    rec = ri.Recognizer(b"(ab|c)*d")
    try:
        assert rec.get_option("prefix") == 1
        rec.set_option("prefix", 0)
        assert rec.get_option("prefix") == 0
        with pytest.raises(ri.RIError):
            rec.set_option("prefix", 2)
    finally:
        rec.close()
