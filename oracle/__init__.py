"""Oracle for the reduced-interface recognizer (RID) of Borsotti, Breveglieri,
Crespi Reghizzi and Morzenti, "Minimizing speculation overhead in a parallel
recognizer for regular texts" (arXiv 2412.14975).

TEST INFRASTRUCTURE.  This package is a plain, slow, serial CPU reference.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything under ``oracle/``.
The product (``paper_2412_14975_amd``) never uses it and shares no code with
it; the two meet only at the seeded input generators in ``workloads/``.

Contents
--------
regex.py      byte-level RE parser (syntax documented there)
automata.py   position NFA (Sect. 4.1), powerset DFA, Moore minimization with
              canonical numbering, RI-DFA (Sect. 3.1), interface reduction by
              downgrading with delegation (Sect. 3.4), quotient NFA
recognize.py  serial recognizer (Sect. 2), CSDPA with a DFA (Sect. 2, Fig. 2),
              RID with an RI-DFA and ``if`` / ``if_min`` (Sects. 3.2, 3.4),
              NFA simulation (Lemma 1), CSDPA with the NFA as chunk automaton
              and transition counts (Fig. 1)
baseline.py   the paper's CPU scheme (one thread per chunk, serial join) for
              the minimal DFA and RID, timed as a reported baseline
scan.c        the plain serial table scan used by recognize.py
csdpa.c       the threaded reach phase used by baseline.py

Parity status: every function here is pinned by tests against the paper's
worked examples (Figs. 1-5), closed forms of the regexp family, Python's
``re`` on exhaustive short strings, and the invariants of Lemma 1 and Th. 1.
"""

from .regex import ParseError, parse  # noqa: F401
from .automata import (  # noqa: F401
    NFA, DFA, RIDFA, Built, build, build_from_nfa, position_nfa, nfa_from_edges, trim,
    subset_dfa, minimize, min_dfa_of, ri_dfa, interface_reduction, quotient_nfa,
    if_fun, if_min_fun, moore_partition, nfa_step,
)
from .recognize import (  # noqa: F401
    serial, csdpa, rid, nst, nfa_reach, nfa_csdpa, nfa_csdpa_transitions, even_bounds, dense_table,
    run, build_scan_library,
)
