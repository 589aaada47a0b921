"""Pins of the oracle against closed forms, Python's ``re`` and the
invariants of Lemma 1 / Th. 1.  None of these recomputes the oracle's own
formulas: each checks a fact fixed by the mathematics or by an independent
library routine."""

import itertools
import re

import numpy as np
import pytest

import oracle
from oracle import automata as A
from oracle import recognize as R
from workloads import gen

from brute_re import compile_brute


def small_pattern(rng, alphabet: bytes, depth: int, maxpos: int = 40) -> bytes:
    """Draw random expressions until the position NFA has at most ``maxpos``
    states (nested repeats can blow a depth-3 expression up to hundreds of
    positions and the powerset DFA up to 10^5 states)."""
    while True:
        p = gen.random_regex(rng, alphabet, depth)
        if A.position_nfa(p).n <= maxpos:
            return p


def strings(alphabet: bytes, maxlen: int):
    for L in range(maxlen + 1):
        for t in itertools.product(alphabet, repeat=L):
            yield bytes(t)


# ---------------------------------------------------------------------------
# regexp family (a|b)*a(a|b)^k, Tab. 1
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", range(0, 8))
def test_regexp_family_min_dfa_has_2_pow_k_plus_1_states(k):
    b = oracle.build(gen.regexp_family(k))
    assert b.dfa.n == 2 ** (k + 1)
    # the position NFA has 2k+4 states; the right-language classes of the
    # positions are k+2 (the classic minimal NFA of the family)
    assert b.nfa.n == 2 * k + 4
    assert b.nfa_q.n == k + 2
    assert len(b.red.kept) == k + 2


@pytest.mark.parametrize("k", [0, 1, 3, 5])
def test_regexp_family_membership_closed_form(k):
    b = oracle.build(gen.regexp_family(k))
    for s in strings(b"ab", 9):
        want = len(s) >= k + 1 and s[len(s) - k - 1] == ord("a")
        assert R.serial(b.dfa, s)[0] == want, s


def test_tiny_workload_derived_sizes():
    """C1 = (a|b)*a(a|b)^3: positions 0..9; right-language classes
    {0,1,2},{3},{4,5},{6,7},{8,9}; the RI-DFA of the quotient has the 16
    subsets containing [0] plus the 4 other singletons."""
    b = oracle.build(gen.c1_regex())
    assert b.nfa.n == 10
    assert b.red.rep == [0, 0, 0, 3, 4, 4, 6, 6, 8, 8]
    assert b.nfa_q.n == 5
    assert b.Bq.n == 20
    assert sum(1 for c in b.Bq.content if 0 in c) == 16
    acc, fin = R.serial(b.dfa, b"bbbabab")
    assert acc is True
    assert R.serial(b.dfa, b"bbbbbab")[0] is False


def test_tiny_workload_transition_closed_form():
    """Equal chunks of length m >= 4: the all-states DFA makes 16 complete
    runs per chunk after the first (the DFA of the family is complete), RID
    makes one full run from [0] plus 3+2+1+0 moves from the other starts."""
    b = oracle.build(gen.c1_regex())
    rng = gen.PCG(5)
    for c, m in ((2, 4), (4, 16), (8, 33)):
        x = gen.random_text(rng, b"ab", c * m)
        bounds = [i * m for i in range(c + 1)]
        assert R.csdpa(b.dfa, x, bounds)["transitions"] == m + (c - 1) * 16 * m
        assert R.rid(b.Bq, x, bounds)["transitions"] == m + (c - 1) * (m + 6)


# ---------------------------------------------------------------------------
# language of the construction against Python's re (a backtracking matcher)
# ---------------------------------------------------------------------------

def _check_against_re(pattern: bytes, alphabet: bytes, maxlen: int, re_maxlen: int = 5):
    """Membership of every string up to ``maxlen`` against the set-semantics
    matcher of tests/brute_re.py, and up to ``re_maxlen`` also against
    Python's backtracking ``re`` (which can take exponential time)."""
    b = oracle.build(pattern)
    rx = re.compile(pattern, re.DOTALL)
    brute = compile_brute(pattern)
    t = R.dense_table(b.dfa.n, b.dfa.delta)
    for s in strings(alphabet, maxlen):
        got = R.serial(b.dfa, s, t)[0] if b.dfa.n else False
        assert got == brute(s), (pattern, s)
        if len(s) <= re_maxlen:
            assert got == (rx.fullmatch(s) is not None), (pattern, s)


@pytest.mark.parametrize("seed", range(120))
def test_exhaustive_binary_alphabet(seed):
    rng = gen.PCG(1000 + seed)
    pattern = small_pattern(rng, b"ab", int(rng.integers(1, 4)))
    _check_against_re(pattern, b"ab", 10)


@pytest.mark.parametrize("seed", range(40))
def test_exhaustive_ternary_alphabet(seed):
    rng = gen.PCG(5000 + seed)
    pattern = small_pattern(rng, b"abc", int(rng.integers(1, 4)))
    _check_against_re(pattern, b"abc", 10)


@pytest.mark.parametrize("pattern,alphabet,maxlen", [
    (b"a{2,4}b?", b"ab", 7), (b"(ab|a)*b{1,}", b"ab", 8), (b"[^a]c.a", b"abc", 5),
    (b"(a|)(b|)c{0}", b"abc", 4), (b"()", b"ab", 3), (b"a\\.b", b"a.b", 4),
    (b"[a-c]{0,2}[b-c]+", b"abcd", 5), (b"\\x61\\d", b"a1x", 3),
])
def test_syntax_corner_cases(pattern, alphabet, maxlen):
    _check_against_re(pattern, alphabet, maxlen)


def test_empty_language_and_empty_text():
    b = oracle.build(b"a[^\\x00-\\xff]b")
    assert b.nfa.n == 0 and b.dfa.n == 0
    assert R.serial(b.dfa, b"") == (False, -1)
    assert R.serial(b.dfa, b"ab") == (False, -1)
    e = oracle.build(b"()")
    assert R.serial(e.dfa, b"") == (True, 0)
    assert R.serial(e.dfa, b"a") == (False, -1)


@pytest.mark.parametrize("bad", [b"(a", b"a)", b"*a", b"a{3,2}", b"[ab", b"a{x}", b"\\x4"])
def test_parse_errors(bad):
    with pytest.raises(oracle.ParseError):
        oracle.parse(bad)


# ---------------------------------------------------------------------------
# minimal DFA: state identity = residual language, canonical numbering
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(25))
def test_final_state_identifies_the_residual_language(seed):
    """Two strings end in the same minimal-DFA state iff no suffix tells them
    apart (Myhill-Nerode), checked with the brute-force matcher.  Patterns
    over {a,b} treat every other byte alike, so 'c' stands for all of them;
    in a minimal DFA with n live states plus the dead one, two states are
    told apart by some word of length <= n - 1 (Moore's bound)."""
    rng = gen.PCG(9000 + seed)
    while True:        # redraw until the DFA is small enough for the suffix check
        pattern = small_pattern(rng, b"ab", 2)
        b = oracle.build(pattern)
        if 1 <= b.dfa.n <= 7:
            break
    brute = compile_brute(pattern)
    words = list(strings(b"ab", 4))
    suffixes = list(strings(b"abc", max(b.dfa.n - 1, 1)))
    sig = {w: tuple(brute(w + z) for z in suffixes) for w in words}
    fin = {w: R.serial(b.dfa, w)[1] for w in words}
    for w in words:
        assert (fin[w] == -1) == (not any(sig[w])), (pattern, w)
    live = [w for w in words if fin[w] != -1]
    for w1 in live:
        for w2 in live:
            assert (fin[w1] == fin[w2]) == (sig[w1] == sig[w2]), (pattern, w1, w2)


@pytest.mark.parametrize("seed", range(10))
def test_canonical_numbering_is_bfs_order(seed):
    rng = gen.PCG(300 + seed)
    b = oracle.build(small_pattern(rng, b"abc", 3))
    d = b.dfa
    if d.n == 0:
        return
    seen, order = {0}, [0]
    for s in order:
        for byte in range(256):
            t = d.delta[s].get(byte)
            if t is not None and t not in seen:
                seen.add(t)
                order.append(t)
    assert order == list(range(d.n))


# ---------------------------------------------------------------------------
# interface reduction = right-language equivalence of NFA states
# ---------------------------------------------------------------------------

def _right_language_dfa(nfa, q):
    """Minimal DFA of L_N(q): re-root the NFA at q (swap q and 0)."""
    perm = list(range(nfa.n))
    perm[0], perm[q] = q, 0
    delta = [None] * nfa.n
    for s in range(nfa.n):
        delta[perm[s]] = {b: frozenset(perm[r] for r in succ) for b, succ in nfa.delta[s].items()}
    final = frozenset(perm[s] for s in nfa.final)
    d = A.minimize(A.subset_dfa(A.NFA(nfa.n, delta, final))[0])
    return (d.n, tuple(tuple(sorted(x.items())) for x in d.delta), d.final)


@pytest.mark.parametrize("seed", range(30))
def test_reduction_classes_are_right_language_classes(seed):
    rng = gen.PCG(700 + seed)
    b = oracle.build(small_pattern(rng, b"ab", 3))
    nfa = b.nfa
    if nfa.n == 0:
        return
    lang = [_right_language_dfa(nfa, q) for q in range(nfa.n)]
    for q in range(nfa.n):
        for r in range(nfa.n):
            assert (b.red.rep[q] == b.red.rep[r]) == (lang[q] == lang[r])
    # the quotient has no two equivalent singletons left (Th. 2's bound is met)
    red2 = A.interface_reduction(b.Bq)
    assert red2.rep == list(range(b.nfa_q.n))


# ---------------------------------------------------------------------------
# Th. 1 and Lemma 1 on random chunkings
# ---------------------------------------------------------------------------

def _random_bounds(rng, n, c):
    if n == 0:
        return [0, 0]
    c = max(1, min(c, n))
    cuts = sorted(rng.choice(np.arange(1, n), size=c - 1, replace=False).tolist()) if c > 1 else []
    return [0] + cuts + [n]


@pytest.mark.parametrize("seed", range(40))
def test_chunked_devices_agree_with_serial_and_lemma1(seed):
    rng = gen.PCG(2000 + seed)
    alphabet = b"abc"[: int(rng.integers(2, 4))]
    b = oracle.build(small_pattern(rng, alphabet, int(rng.integers(1, 4))))
    if b.nfa.n == 0:
        return
    kept = [b.B.initial[q] for q in b.red.kept]
    for trial in range(6):
        n = int(rng.integers(1, 40))
        x = gen.random_text(rng, alphabet, n)
        want, fin = R.serial(b.dfa, x)
        for c in sorted({1, 2, 3, n, int(rng.integers(1, n + 1))}):
            bounds = _random_bounds(rng, n, c)
            r_dfa = R.csdpa(b.dfa, x, bounds)
            r_b = R.rid(b.B, x, bounds)
            r_min = R.rid(b.B, x, bounds, starts=kept,
                          iface=lambda plas: A.if_min_fun(b.B, b.red, plas))
            r_q = R.rid(b.Bq, x, bounds)
            assert r_dfa["accept"] == r_b["accept"] == r_min["accept"] == r_q["accept"] == want
            # Lemma 1 at every boundary, for B (over N) and B' (over N')
            for i in range(len(bounds) - 1):
                prefix = x[: bounds[i + 1]]
                assert R.nst(b.B, r_b["plas"][i]) == R.nfa_reach(b.nfa, {0}, prefix)
                assert R.nst(b.Bq, r_q["plas"][i]) == R.nfa_reach(b.nfa_q, {0}, prefix)
            # the DFA device's PLAS_c is the serial final state
            assert r_dfa["plas"][-1] == (frozenset([fin]) if fin >= 0 else frozenset())


@pytest.mark.parametrize("n", [1, 2, 5, 17])
def test_every_chunk_count_tiny_workload(n):
    b = oracle.build(gen.c1_regex())
    rng = gen.PCG(n)
    x = gen.random_text(rng, b"ab", n)
    want = R.serial(b.dfa, x)[0]
    for c in range(1, n + 1):
        bounds = R.even_bounds(n, c)
        assert R.rid(b.Bq, x, bounds)["accept"] == want
        assert R.csdpa(b.dfa, x, bounds)["accept"] == want


def test_even_bounds():
    assert R.even_bounds(10, 3) == [0, 3, 6, 10]
    assert R.even_bounds(3, 8) == [0, 1, 2, 3]
    assert R.even_bounds(0, 4) == [0, 0]


# ---------------------------------------------------------------------------
# NFA simulation (nfa_step, nfa_reach) and CSDPA with the NFA chunk automaton
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(30))
def test_nfa_simulation_against_brute_force(seed):
    """Acceptance by simulating the position NFA with nfa_step from {q0}
    equals set-semantics membership on every string up to length 8."""
    rng = gen.PCG(7000 + seed)
    alphabet = b"abc"[: 2 + seed % 2]
    pattern = small_pattern(rng, alphabet, int(rng.integers(1, 4)))
    nfa = A.trim(A.position_nfa(pattern))
    brute = compile_brute(pattern)
    for s in strings(alphabet, 8 if len(alphabet) == 2 else 6):
        S = frozenset([0]) if nfa.n else frozenset()
        for b in s:
            S = A.nfa_step(nfa, S, b)
        assert bool(S & nfa.final) == brute(s), (pattern, s)


@pytest.mark.parametrize("seed", range(20))
def test_nfa_csdpa_is_chunk_invariant(seed):
    """The composed chunk relations give rho(q0, x) for every chunking (the
    NFA analogue of Lemma 1), so acceptance equals the minimal DFA's."""
    rng = gen.PCG(8000 + seed)
    alphabet = b"abcd"[: 2 + seed % 3]
    pattern = small_pattern(rng, alphabet, int(rng.integers(1, 4)))
    b = oracle.build(pattern)
    for n in (1, 7, 60, 257):
        x = gen.random_text(rng, alphabet, n)
        whole = R.nfa_reach(b.nfa, [0], x) if b.nfa.n else frozenset()
        want = R.serial(b.dfa, x)[0]
        for c in (1, 2, 5, n):
            cuts = sorted(set([0, n] + [int(v) for v in rng.integers(1, max(2, n), size=c - 1)]))
            res = R.nfa_csdpa(b.nfa, x, cuts)
            assert res["S"] == whole, (pattern, n, cuts)
            assert res["accept"] == want
