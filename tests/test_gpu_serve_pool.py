"""GPU parity of the full-scale serving pool against the oracle.

The automata are the serving workload's own keyword unions
(``workloads.gen.c5_automaton(SERVE_SEED, i)``: interfaces up to about 16k
states, minimal DFAs up to about 25k states) and the requests are the
workload's own stream (``workloads.gen.c5_requests``).  The expected
(accept, final state) of every request was written by
``tests/golden/make_c5_goldens.py`` from the oracle alone (serial minimal-DFA
recognition, Sect. 2) into ``tests/golden/c5_serving.json``.  Here the
device-only fused batch and the continuous-batching serving loop must give
exactly those values, for RID and for the all-states DFA.
"""

import json
import os

import numpy as np
import pytest

from workloads import gen

torch = pytest.importorskip("torch")
ri = pytest.importorskip("paper_2412_14975_amd")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c5_serving.json")


@pytest.fixture(scope="module")
def pool():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ri.binding.lib()
    g = json.load(open(GOLDEN))
    autos = g["automata"]
    # the three largest automata (by positions, which bounds the interface),
    # the one with the largest minimal DFA, and the two smallest
    by_pos = sorted(range(len(autos)), key=lambda k: autos[k]["positions"])
    by_dfa = sorted(range(len(autos)), key=lambda k: autos[k]["min_dfa_states"])
    chosen = sorted(set(by_pos[-3:] + by_dfa[-1:] + by_pos[:2]))
    kws_of = [gen.c5_automaton(g["seed"], k)[1] for k in range(len(autos))]
    recs = {k: ri.Recognizer(gen.c5_automaton(g["seed"], k)[0]) for k in chosen}
    rows = {r[0]: r for r in g["requests"]}
    reqs = []
    for i, k, x in gen.c5_requests(len(g["requests"]), kws_of, seed=g["seed"], keep=set(chosen)):
        r = rows[i]
        assert r[1] == k and r[2] == len(x)
        reqs.append((i, k, x, (bool(r[3]), int(r[4]))))
    yield recs, reqs, autos
    for r in recs.values():
        r.close()


def test_pool_covers_the_largest_automata(pool):
    recs, reqs, autos = pool
    sizes = [recs[k].info()["interface_states"] for k in recs]
    assert max(sizes) > 14000
    assert max(recs[k].info()["min_dfa_states"] for k in recs) == max(a["min_dfa_states"] for a in autos)
    assert len(reqs) >= 100
    assert 0 < sum(w[0] for *_, w in reqs) < len(reqs)


@pytest.mark.parametrize("algo", ["rid", "dfa"])
def test_fused_batch_against_oracle(pool, algo):
    recs, reqs, _ = pool
    texts = [torch.from_numpy(x).to("cuda") for _, _, x, _ in reqs]
    b = ri.Batch([(recs[k], t, algo) for (_, k, _, _), t in zip(reqs, texts)], mode="fused")
    try:
        got = b.run().cpu().numpy()
        for (i, k, x, want), g in zip(reqs, got):
            assert (bool(g[0]), int(g[1])) == want, (i, k, len(x))
    finally:
        b.close()


@pytest.mark.parametrize("algo", ["rid", "dfa"])
def test_serving_loop_against_oracle(pool, algo):
    recs, reqs, _ = pool
    keys = sorted(recs)
    pos = {k: j for j, k in enumerate(keys)}
    rng = gen.PCG(31)
    t, schedule = 0.0, []
    for _, k, x, _ in reqs:
        t += float(rng.exponential(1 / 2000.0))
        schedule.append((t, pos[k], x))
    srv = ri.serve.Server([recs[k] for k in keys], algo=algo, slots=3)
    try:
        done, _ = ri.serve.run_open_loop(srv, schedule)
    finally:
        srv.close()
    assert sorted(d["id"] for d in done) == list(range(len(reqs)))
    by_id = {d["id"]: d for d in done}
    for j, (i, k, x, want) in enumerate(reqs):
        assert (by_id[j]["accept"], by_id[j]["final_state"]) == want, (i, k, len(x))


def test_largest_interface_single_calls(pool):
    """ri_recognize_ex and the queued call on the automaton with the largest
    interface, every algorithm, against the oracle's values."""
    recs, reqs, _ = pool
    big = max(recs, key=lambda k: recs[k].info()["interface_states"])
    mine = [(i, x, w) for i, k, x, w in reqs if k == big and len(x) > 0][:12]
    assert mine
    res = torch.full((len(mine), 2), -7, dtype=torch.int32, device="cuda")
    for j, (i, x, want) in enumerate(mine):
        t = torch.from_numpy(x).to("cuda")
        for algo in ("rid", "dfa", "subset"):
            got = recs[big].recognize(t, algo=algo)
            assert (got["accept"], got["final_state"]) == want, (i, algo)
        recs[big].recognize_async(t, res[j], algo="rid")
        torch.cuda.synchronize()
    for (i, x, want), g in zip(mine, res.cpu().numpy()):
        assert (bool(g[0]), int(g[1])) == want, i
