"""Writes c5_serving.json: the oracle's (accept, final state) for every
request of the serving workload (64 keyword-union automata built from
``workloads.gen.c5_automaton(SERVE_SEED, i)``, 2000 requests from
``workloads.gen.c5_requests``), with each automaton's oracle sizes.

Each expected value is the oracle's serial recognizer (Sect. 2: the minimal
DFA run left to right over the whole text) with the canonical minimal-DFA
numbering.  Uses only ``oracle/`` and the input generators; one worker
process per automaton.

    python tests/golden/make_c5_goldens.py [--procs P]
"""

import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import gen  # noqa: E402

AUTOMATA = 64
REQUESTS = 2000


def one_automaton(k):
    rx, _ = gen.c5_automaton(gen.SERVE_SEED, k)
    kws_of = [gen.c5_automaton(gen.SERVE_SEED, j)[1] for j in range(AUTOMATA)]
    nfa = oracle.trim(oracle.position_nfa(rx))
    d = oracle.min_dfa_of(nfa)
    table = oracle.dense_table(d.n, d.delta)
    rows = []
    for i, kk, x in gen.c5_requests(REQUESTS, kws_of, keep={k}):
        acc, fin = oracle.serial(d, x, table)
        rows.append([i, kk, int(len(x)), int(acc), int(fin)])
    print(k, nfa.n, d.n, len(rows), flush=True)
    return k, dict(positions=nfa.n, min_dfa_states=d.n), rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=6)
    args = ap.parse_args()
    autos, reqs = {}, []
    with ProcessPoolExecutor(max_workers=args.procs) as ex:
        for k, info, rows in ex.map(one_automaton, range(AUTOMATA)):
            autos[k] = info
            reqs.extend(rows)
    reqs.sort()
    out = {"seed": gen.SERVE_SEED, "generator": "workloads.gen.c5_automaton / c5_requests",
           "automata": [autos[k] for k in range(AUTOMATA)],
           "columns": ["request", "automaton", "length", "accept", "final_state"],
           "requests": reqs}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_serving.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    main()
