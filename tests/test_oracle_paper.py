"""Pins of the oracle against the paper's worked examples (Figs. 1-5).

Every expected value here is printed in the paper (fixtures under
tests/golden/, each with its citation); nothing is computed by the oracle
first and copied back.
"""

import json
import os

import pytest

import oracle
from oracle import automata as A
from oracle import recognize as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def nfa_of(spec, alphabet):
    edges = [(q, None if s == "*" else s, r) for q, s, r in spec["edges"]]
    return A.nfa_from_edges(spec["states"], edges, spec["final"], alphabet.encode())


def syms(s, alphabet):
    return (alphabet if s == "*" else s).encode()


def fs(x):
    return frozenset(x)


# ---------------------------------------------------------------------------
# Fig. 1 / Fig. 3 / Fig. 4
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def fig1():
    g = load("fig1_fig3_fig4.json")
    nfa = nfa_of(g["nfa"], g["alphabet"])
    return g, nfa, oracle.build_from_nfa(nfa)


def test_fig1_min_dfa_is_the_drawn_powerset_dfa(fig1):
    g, nfa, built = fig1
    dfa, subsets = A.subset_dfa(built.nfa)
    exp = g["min_dfa"]
    assert {fs(s) for s in subsets} == {fs(s) for s in exp["states"]}
    idx = {S: i for i, S in enumerate(subsets)}
    want = {}
    for src, sy, dst in exp["edges"]:
        for b in syms(sy, g["alphabet"]):
            want[(fs(src), b)] = fs(dst)
    got = {(S, b): subsets[t] for S in subsets for b, t in dfa.delta[idx[S]].items()}
    assert got == want
    assert {subsets[s] for s in dfa.final} == {fs(s) for s in exp["final"]}
    # the drawn DFA is minimal: minimization keeps its 4 states
    assert built.dfa.n == len(exp["states"])


def test_fig3_ridfa_construction(fig1):
    g, nfa, built = fig1
    B = built.B
    exp = g["ridfa"]
    assert {c for c in B.content} == {fs(s) for s in exp["states"]}
    assert len(B.content) == len(exp["states"])
    assert [B.content[p] for p in B.initial] == [fs(s) for s in exp["initial"]]
    assert {B.content[p] for p in B.final} == {fs(s) for s in exp["final"]}
    want = {}
    for src, sy, dst in exp["edges"]:
        for b in syms(sy, g["alphabet"]):
            want[(fs(src), b)] = fs(dst)
    got = {(B.content[p], b): B.content[t] for p in range(B.n) for b, t in B.delta[p].items()}
    assert got == want


def test_fig1_transition_counts(fig1):
    g, nfa, built = fig1
    x, bounds, T = g["text"].encode(), g["bounds"], g["transitions"]
    assert R.csdpa(built.dfa, x, bounds)["transitions"] == T["dfa"]
    assert R.nfa_csdpa_transitions(built.nfa, x, bounds) == T["nfa"]
    assert R.rid(built.B, x, bounds)["transitions"] == T["rid"]
    # serial operation makes exactly n transitions (Sect. 2)
    assert R.csdpa(built.dfa, x, [0, len(x)])["transitions"] == T["serial"] == len(x)


def test_fig4_rid_join(fig1):
    g, nfa, built = fig1
    B, exp = built.B, g["fig4"]
    res = R.rid(B, g["text"].encode(), g["bounds"])
    C = B.content
    lam1 = {C[p]: C[r] for p, r in res["lambdas"][0].items()}
    lam2 = {C[p]: C[r] for p, r in res["lambdas"][1].items()}
    assert lam1 == {fs(a): fs(b) for a, b in exp["lambda1"]}
    assert lam2 == {fs(a): fs(b) for a, b in exp["lambda2"]}
    assert {C[p] for p in res["plas"][0]} == {fs(s) for s in exp["plas1"]}
    assert {C[p] for p in A.if_fun(B, res["plas"][0])} == {fs(s) for s in exp["if_plas1"]}
    assert {C[p] for p in res["pis"][1]} == {fs(s) for s in exp["pis2"]}
    assert {C[p] for p in res["plas"][1]} == {fs(s) for s in exp["plas2"]}
    assert res["accept"] is exp["accept"]


def test_fig1_nfa_step_gives_the_drawn_ridfa_moves(fig1):
    """The RI-DFA of Fig. 3 is drawn with its contents: the move of a state S
    on b leads to rho(S, b) (empty = no edge).  nfa_step must give exactly
    the drawn targets for every drawn state and every symbol."""
    g, nfa, built = fig1
    exp = g["ridfa"]
    want = {}
    for src, sy, dst in exp["edges"]:
        for b in syms(sy, g["alphabet"]):
            want[(fs(src), b)] = fs(dst)
    for S in exp["states"]:
        for b in g["alphabet"].encode():
            assert A.nfa_step(built.nfa, fs(S), b) == want.get((fs(S), b), frozenset()), (S, chr(b))
    # and on sets that are not RI-DFA states: the union of the singleton moves
    assert A.nfa_step(built.nfa, fs([1, 2]), ord("b")) == fs([0, 1, 2])
    assert A.nfa_step(built.nfa, frozenset(), ord("a")) == frozenset()


def test_fig4_nfa_chunk_relations(fig1):
    """NFA as chunk automaton on aab.cab (Fig. 1): lambda_i(q) = rho(q, y_i).
    The RI-DFA runs of Fig. 4 start at the singletons, so their end-state
    contents are these sets: chunk 1 from q0 gives {0, 2}, chunk 2 gives
    {0, 2} from q0 and from q1 and nothing from q2; the composed set after
    chunk 2 is PLAS_2's content {0, 2}, which meets F = {2}."""
    g, nfa, built = fig1
    exp = g["fig4"]
    res = R.nfa_csdpa(built.nfa, g["text"].encode(), g["bounds"])
    assert res["lambdas"][0] == {0: fs(exp["lambda1"][0][1])}
    lam2 = {fs([q]): S for q, S in res["lambdas"][1].items() if S}
    assert lam2 == {fs(a): fs(b) for a, b in exp["lambda2"]}
    assert res["lambdas"][1][2] == frozenset()
    assert res["S"] == fs(exp["plas2"][0])
    assert res["accept"] is exp["accept"]


# ---------------------------------------------------------------------------
# Fig. 2
# ---------------------------------------------------------------------------

def test_fig2_csdpa_with_dfa():
    g = load("fig2.json")
    d = g["dfa"]
    delta = [dict() for _ in range(d["states"])]
    for q, s, r in d["edges"]:
        for b in s.encode():
            delta[q][b] = r
    dfa = A.DFA(d["states"], delta, frozenset(d["final"]))
    # the drawn DFA is the minimal DFA of the figure's expression
    m = oracle.build(g["regex"].encode()).dfa
    assert m.n == dfa.n and m.final == dfa.final and m.delta == dfa.delta
    res = R.csdpa(dfa, g["text"].encode(), g["bounds"])
    x = g["text"].encode()
    b = g["bounds"]
    # full mapping tables as printed (chunk 1's table lists every state)
    t = R.dense_table(dfa.n, dfa.delta)
    for key, (lo, hi) in (("lambda1", (b[0], b[1])), ("lambda2", (b[1], b[2]))):
        for q, r in g[key]:
            assert R.run(t, q, x, lo, hi)[0] == r
    assert res["pis"][0] == fs(g["pis1"])
    assert res["plas"][0] == fs(g["plas1"])
    assert res["pis"][1] == fs(g["pis2"])
    assert res["plas"][1] == fs(g["plas2"])
    assert res["accept"] is g["accept"]
    assert res["transitions"] == g["transitions"]


# ---------------------------------------------------------------------------
# Fig. 5 (interface minimization)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def fig5():
    g = load("fig5.json")
    nfa = nfa_of(g["nfa"], g["alphabet"])
    return g, oracle.build_from_nfa(nfa)


def test_fig5_ridfa_states_and_edges(fig5):
    g, built = fig5
    B = built.B
    names = {k: fs(v) for k, v in g["ridfa"]["names"].items()}
    assert set(B.content) == set(names.values())
    want = {}
    for src, sy, dst in g["ridfa"]["edges"]:
        for b in syms(sy, g["alphabet"]):
            want[(names[src], b)] = names[dst]
    got = {(B.content[p], b): B.content[t] for p in range(B.n) for b, t in B.delta[p].items()}
    assert got == want


def test_fig5_nerode_classes_and_delegation(fig5):
    g, built = fig5
    B, red = built.B, built.red
    names = {k: fs(v) for k, v in g["ridfa"]["names"].items()}
    pid = {v: B.index[v] for v in names.values()}
    classes = {}
    for k, v in names.items():
        classes.setdefault(red.classes[pid[v]], set()).add(k)
    nontriv = sorted(sorted(c) for c in classes.values() if len(c) > 1)
    assert nontriv == sorted(sorted(c) for c in g["nerode_nontrivial"])
    kept = {k for k, v in names.items() if B.index[v] in [B.initial[q] for q in red.kept]}
    assert kept == set(g["initial_after_reduction"])
    for down, dlg in g["delegates"].items():
        q = next(iter(names[down]))
        assert frozenset([red.rep[q]]) == names[dlg]


def test_fig5_runs_and_join(fig5):
    g, built = fig5
    B, red = built.B, built.red
    names = {k: fs(v) for k, v in g["ridfa"]["names"].items()}
    t = R.dense_table(B.n, B.delta)
    for start, word, path in g["runs"]:
        p = B.index[names[start]]
        seen = []
        for ch in word.encode():
            p = B.delta[p].get(ch)
            if p is None:
                break
            seen.append(B.content[p])
        assert seen == [names[s] for s in path]
    kept = [B.initial[q] for q in red.kept]
    res = R.rid(B, g["text"].encode(), g["bounds"], starts=kept,
                iface=lambda plas: A.if_min_fun(B, red, plas))
    assert {B.content[p] for p in res["plas"][0]} == {names[s] for s in g["plas1"]}
    assert ({B.content[p] for p in A.if_min_fun(B, red, res["plas"][0])}
            == {names[s] for s in g["if_min_plas1"]})
    assert {B.content[p] for p in res["plas"][1]} == {names[s] for s in g["plas2"]}
    assert res["accept"] is g["accept"]
    # the downgraded start's run is the one that RID_min no longer makes
    full = R.rid(B, g["text"].encode(), g["bounds"])
    assert full["transitions"] - res["transitions"] == 3


def test_fig5_quotient_is_fig1_nfa(fig5):
    """Merging 1 and 3 (the initial-state class alpha) gives Fig. 1's NFA."""
    g, built = fig5
    g1 = load(g["quotient_isomorphic_to"])
    n1 = A.trim(nfa_of(g1["nfa"], g1["alphabet"]))
    nq = built.nfa_q
    assert nq.n == n1.n
    # class ids follow the lowest member: [0]={0}, [1]={1,3}, [2]={2}
    assert nq.delta == n1.delta and nq.final == n1.final
