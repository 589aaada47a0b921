"""Oracle: serial recognizer and literal chunked simulators (Sects. 2 and 3.2).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use the oracle.

Result of recognition
---------------------
``accept``      x is in L (Th. 1: the chunked device and the serial one agree).
``final_state`` the state of the minimal, trimmed, canonically numbered DFA
                after reading x, or -1 when the run dies.  It is unique for
                (L, x), so two correct implementations agree bit for bit.

Chunk boundaries
----------------
``bounds`` is a list 0 = b_0 < b_1 < ... < b_c = n; chunk i is
x[b_{i-1}:b_i].  The paper asks only for non-empty chunks; ``even_bounds``
gives floor(i*n/c) with c clamped to n.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .automata import DFA, NFA, RIDFA, nfa_step

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "scan.c"), os.path.join(_HERE, "csdpa.c")]
_LIB = os.path.join(_HERE, "_scan.so")
_lib = None


def build_scan_library(force: bool = False) -> str:
    """Compile scan.c and csdpa.c with gcc into oracle/_scan.so."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


def _scanlib():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_scan_library())
        lib.oracle_scan.restype = ctypes.c_int32
        lib.oracle_scan.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_threaded_reach.restype = ctypes.c_int
        lib.oracle_threaded_reach.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
        _lib = lib
    return _lib


def dense_table(n: int, delta) -> np.ndarray:
    """[n][256] int32 table, -1 for an undefined move."""
    t = np.full((max(n, 1), 256), -1, dtype=np.int32)
    for s in range(n):
        for b, r in delta[s].items():
            t[s, b] = r
    return t


def run(table: np.ndarray, start: int, text: np.ndarray, begin: int, end: int):
    """One deterministic run over text[begin:end] from ``start``.
    Returns (end_state or -1, transitions made)."""
    text = _as_u8(text)
    k = ctypes.c_int64(0)
    s = _scanlib().oracle_scan(table.ctypes.data, int(start), text.ctypes.data,
                               int(begin), int(end), ctypes.byref(k))
    return int(s), int(k.value)


def serial(dfa: DFA, text, table: np.ndarray = None):
    """Serial operation (Sect. 2): one run of the minimal DFA over the whole
    text from its initial state.  Returns (accept, final_state)."""
    text = _as_u8(text)
    if dfa.n == 0:
        return False, -1
    if table is None:
        table = dense_table(dfa.n, dfa.delta)
    s, _ = run(table, 0, text, 0, len(text))
    return (s >= 0 and s in dfa.final), s


def even_bounds(n: int, c: int):
    c = max(1, min(c, n)) if n > 0 else 1
    return [(i * n) // c for i in range(c + 1)]


def _as_u8(text):
    if isinstance(text, (bytes, bytearray)):
        return np.frombuffer(bytes(text), dtype=np.uint8)
    return np.ascontiguousarray(text, dtype=np.uint8)


# ---------------------------------------------------------------------------
# CSDPA with a deterministic chunk automaton, Sect. 2 (Fig. 2)
# ---------------------------------------------------------------------------

def csdpa(dfa: DFA, text, bounds, table: np.ndarray = None):
    """Chunk automata A_i with I_1 = {q0} and I_i = Q for i >= 2.

    lambda_i maps each start q with delta(q, y_i) defined to that state;
    PIS_i is the set of such q; PLAS_1 = lambda_1(PIS_1) and
    PLAS_i = lambda_i(PLAS_{i-1} & PIS_i); accept iff PLAS_c meets F.
    ``transitions`` counts every move made by every run (failing moves
    count zero)."""
    x = _as_u8(text)
    if table is None:
        table = dense_table(dfa.n, dfa.delta)
    lambdas, pis, plas = [], [], []
    T = 0
    prev = None
    for i in range(len(bounds) - 1):
        starts = [0] if i == 0 else list(range(dfa.n))
        if dfa.n == 0:
            starts = []
        lam = {}
        for q in starts:
            r, k = run(table, q, x, bounds[i], bounds[i + 1])
            T += k
            if r >= 0:
                lam[q] = r
        P = frozenset(lam)
        L = frozenset(lam[q] for q in (P if i == 0 else (prev & P)))
        lambdas.append(lam)
        pis.append(P)
        plas.append(L)
        prev = L
    accept = bool(prev & dfa.final) if prev is not None else False
    return dict(lambdas=lambdas, pis=pis, plas=plas, accept=accept, transitions=T)


# ---------------------------------------------------------------------------
# RID with an RI-DFA chunk automaton, Sect. 3.2 (Fig. 4) and Sect. 3.4
# ---------------------------------------------------------------------------

def rid(B: RIDFA, text, bounds, starts=None, iface=None, table: np.ndarray = None):
    """Reduced-interface device.

    ``starts`` is the interface I (RI-DFA state ids), by default all
    singletons I^B; ``iface`` maps a PLAS to a set of initial states, by
    default the interface function ``if`` (Sect. 3.2).  For B_min pass the
    kept singletons and ``if_min`` (Sect. 3.4).

    PIS_1 = {p0}, PLAS_1 = lambda_1(PIS_1);
    PLAS_i = lambda_i(iface(PLAS_{i-1}) & PIS_i) for i >= 2, where PIS_i are
    the starts whose run over y_i is defined; accept iff PLAS_c meets F^RID."""
    from .automata import if_fun
    x = _as_u8(text)
    if table is None:
        table = dense_table(B.n, B.delta)
    if starts is None:
        starts = list(B.initial)
    if iface is None:
        def iface(plas):
            return if_fun(B, plas)
    lambdas, pis, plas = [], [], []
    T = 0
    prev = None
    p0 = B.initial[0] if B.initial else None
    for i in range(len(bounds) - 1):
        S = [p0] if i == 0 else list(starts)
        if p0 is None:
            S = []
        lam = {}
        for p in S:
            r, k = run(table, p, x, bounds[i], bounds[i + 1])
            T += k
            if r >= 0:
                lam[p] = r
        P = frozenset(lam)
        L = frozenset(lam[p] for p in (P if i == 0 else (iface(prev) & P)))
        lambdas.append(lam)
        pis.append(P)
        plas.append(L)
        prev = L
    accept = bool(prev & B.final) if prev is not None else False
    return dict(lambdas=lambdas, pis=pis, plas=plas, accept=accept, transitions=T)


def nst(B: RIDFA, plas) -> frozenset:
    """Nst(PLAS): the union of the contents of the states of PLAS (Sect. 3.3)."""
    out = set()
    for p in plas:
        out |= B.content[p]
    return frozenset(out)


# ---------------------------------------------------------------------------
# NFA simulation (the right-hand side of Lemma 1) and the NFA-CSDPA count
# ---------------------------------------------------------------------------

def nfa_reach(nfa: NFA, S, text) -> frozenset:
    """rho(S, x) for a set S of NFA states (Sect. 3.3): one nfa_step per
    byte, stopping once the set is empty."""
    cur = frozenset(S)
    for b in _as_u8(text).tolist():
        cur = nfa_step(nfa, cur, b)
        if not cur:
            break
    return cur


def nfa_csdpa(nfa: NFA, text, bounds):
    """CSDPA with the NFA itself as chunk automaton (Sect. 2, the third
    device of Fig. 1): chunk 1 is run from {q0} only, every other chunk from
    every single NFA state q, and lambda_i(q) = rho(q, y_i) is a set of NFA
    states (empty when every path dies).  The chunk relations are composed
    left to right: S_1 = lambda_1(q0), S_i = union of lambda_i(q) over q in
    S_{i-1}; x is accepted iff S_c meets F, and S_c = rho(q0, x).
    Returns dict(lambdas, S, accept) with lambdas[i][q] a frozenset."""
    x = _as_u8(text)
    lambdas = []
    S = None
    for i in range(len(bounds) - 1):
        y = x[bounds[i]:bounds[i + 1]]
        starts = [0] if i == 0 else list(range(nfa.n))
        if nfa.n == 0:
            starts = []
        lam = {q: nfa_reach(nfa, [q], y) for q in starts}
        lambdas.append(lam)
        if i == 0:
            S = lam.get(0, frozenset())
        else:
            nxt = set()
            for q in S:
                nxt |= lam[q]
            S = frozenset(nxt)
    if S is None:
        S = frozenset()
    return dict(lambdas=lambdas, S=S, accept=bool(S & nfa.final))


def nfa_csdpa_transitions(nfa: NFA, text, bounds) -> int:
    """Transitions made by CSDPA with the NFA as chunk automaton: chunk 1 from
    {q0}, every other chunk from every single NFA state; each step counts the
    moves out of every active state (Fig. 1's count of 14)."""
    x = _as_u8(text).tolist()
    T = 0
    for i in range(len(bounds) - 1):
        starts = [0] if i == 0 else list(range(nfa.n))
        for q in starts:
            cur = {q}
            for b in x[bounds[i]:bounds[i + 1]]:
                nxt = set()
                for r in cur:
                    m = nfa.moves(r, b)
                    T += len(m)
                    nxt |= m
                cur = nxt
                if not cur:
                    break
    return T
