"""Writes c4_regexes.json: the 16 expressions of the batched workload.

Candidates come from ``workloads.gen.c4_candidate(seed, i)`` for i = 0, 1, ...
in order; a candidate is kept when its trimmed position NFA has at most 200
states, its minimal DFA (computed by the oracle) has 10 to 2000 states, and
its language is infinite (an unbounded repeat of a body with a non-empty
text).  Uses only ``oracle/`` and the input generators.

    python tests/golden/make_c4_regexes.py
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import gen  # noqa: E402

SEED = 1
COUNT = 16
MAX_POSITIONS = 200


def main():
    kept = []
    i = 0
    while len(kept) < COUNT:
        rx, tree, alphabet = gen.c4_candidate(SEED, i)
        nfa = oracle.trim(oracle.position_nfa(rx))
        if nfa.n <= MAX_POSITIONS and gen.unbounded(tree):
            d = oracle.min_dfa_of(nfa)
            if 10 <= d.n <= 2000:
                kept.append({"index": i, "regex": rx.decode("latin-1"), "alphabet_size": len(alphabet),
                             "positions": nfa.n, "min_dfa_states": d.n})
                print(i, nfa.n, d.n, flush=True)
        i += 1
    out = {"seed": SEED, "generator": "workloads.gen.c4_candidate", "max_positions": MAX_POSITIONS,
           "min_dfa_range": [10, 2000], "expressions": kept}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_regexes.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
