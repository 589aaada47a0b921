"""Oracle: the paper's CPU scheme, timed as a reported baseline.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use the oracle.

Chunked speculative recognition as the paper runs it in its experiments
(Sect. 4): c chunks, one thread per chunk for the reach phase (csdpa.c),
then the join done serially chunk after chunk, which the paper reports as
under 1 % of the time.  Two chunk automata:

* ``dfa``: the minimal DFA speculated from all of its states (Sect. 2,
  Fig. 2); the join composes the partial functions lambda_i.
* ``rid``: the RI-DFA B' of the quotient NFA (every interface start, i.e.
  every singleton of N'); the join carries the set of N' states,
  S_i = union of content(lambda_i(q)) over q in S_{i-1} (Sect. 3.2).
"""

from __future__ import annotations

import ctypes
import time

import numpy as np

from .recognize import _as_u8, _scanlib, dense_table, even_bounds


def threaded_reach(table: np.ndarray, starts, text, bounds):
    """maps[i][s] (int32, -1 = no run) and the transitions made, with one
    POSIX thread per chunk."""
    x = _as_u8(text)
    st = np.ascontiguousarray(starts, dtype=np.int32)
    b = np.ascontiguousarray(bounds, dtype=np.int64)
    c = len(b) - 1
    maps = np.full((c, max(1, len(st))), -1, dtype=np.int32)
    k = ctypes.c_int64(0)
    rc = _scanlib().oracle_threaded_reach(table.ctypes.data, st.ctypes.data, int(len(st)), x.ctypes.data,
                                          b.ctypes.data, int(c), maps.ctypes.data, ctypes.byref(k))
    if rc != 0:
        raise RuntimeError("could not start the chunk threads")
    return maps, int(k.value)


def csdpa_dfa(dfa, text, chunks: int, table: np.ndarray = None):
    """Returns dict(accept, final_state, transitions, seconds)."""
    if table is None:
        table = dense_table(dfa.n, dfa.delta)
    x = _as_u8(text)
    bounds = even_bounds(len(x), chunks)
    t0 = time.perf_counter()
    maps, T = threaded_reach(table, list(range(dfa.n)), x, bounds)
    s = int(maps[0, 0])
    for i in range(1, len(bounds) - 1):
        if s < 0:
            break
        s = int(maps[i, s])
    dt = time.perf_counter() - t0
    return dict(accept=bool(s >= 0 and s in dfa.final), final_state=s, transitions=T, seconds=dt)


def csdpa_rid(Bq, text, chunks: int, table: np.ndarray = None):
    """Returns dict(accept, S (frozenset of N' states), transitions, seconds)."""
    if table is None:
        table = dense_table(Bq.n, Bq.delta)
    x = _as_u8(text)
    bounds = even_bounds(len(x), chunks)
    L = len(Bq.initial)
    t0 = time.perf_counter()
    maps, T = threaded_reach(table, list(Bq.initial), x, bounds)
    e = int(maps[0, 0])
    S = set(Bq.content[e]) if e >= 0 else set()
    for i in range(1, len(bounds) - 1):
        nxt = set()
        for q in S:
            e = int(maps[i, q])
            if e >= 0:
                nxt |= Bq.content[e]
        S = nxt
        if not S:
            break
    dt = time.perf_counter() - t0
    # final states of N': q is final iff its singleton is in F^RID
    fin = {q for q in range(L) if Bq.initial[q] in Bq.final}
    return dict(accept=bool(S & fin), S=frozenset(S), transitions=T, seconds=dt)
