"""GPU tests of the serving loop (paper_2412_14975_amd.serve): requests over
a pool of resident keyword-union automata, arriving while others run, are
admitted by device footprint and batched; every result equals the oracle's
serial result and the result of recognizing the text alone, and the budget
is never exceeded.
"""

import numpy as np
import pytest

import oracle
from workloads import gen

torch = pytest.importorskip("torch")
ri = pytest.importorskip("paper_2412_14975_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ri.binding.lib()


@pytest.fixture(scope="module")
def pool():
    autos = [gen.c5_automaton(3, i, nkw) for i, nkw in enumerate((5, 12, 30, 8, 20, 40))]
    recs = [ri.Recognizer(rx) for rx, _ in autos]
    refs = []
    for rx, _ in autos:
        d = oracle.min_dfa_of(oracle.trim(oracle.position_nfa(rx)))
        refs.append((d, oracle.dense_table(d.n, d.delta)))
    yield autos, recs, refs
    for r in recs:
        r.close()


def requests(autos, seed, count, median=4096, cap=1 << 18):
    rng = gen.PCG(seed)
    out = []
    for i in range(count):
        k = int(rng.integers(0, len(autos)))
        n = gen.c5_length(rng, median=median, cap=cap) if i % 7 else 0
        out.append((k, gen.c5_text(rng, autos[k][1], n, plant=i % 2 == 0)))
    return out


@pytest.mark.parametrize("algo", ["rid", "dfa"])
def test_results_alone_and_in_the_mix(pool, algo):
    autos, recs, refs = pool
    reqs = requests(autos, 1, 160)
    rng = gen.PCG(2)
    t, schedule = 0.0, []
    for k, x in reqs:
        t += float(rng.exponential(1 / 4000.0))
        schedule.append((t, k, x))
    srv = ri.serve.Server(recs, algo=algo, slots=3)
    try:
        done, wall = ri.serve.run_open_loop(srv, schedule)
    finally:
        srv.close()
    assert len(done) == len(reqs) and sorted(d["id"] for d in done) == list(range(len(reqs)))
    assert srv.steps >= 2
    by_id = {d["id"]: d for d in done}
    accepted = 0
    for i, (k, x) in enumerate(reqs):
        want = oracle.serial(refs[k][0], x, refs[k][1])
        got = by_id[i]
        assert (got["accept"], got["final_state"]) == want, (i, k, len(x))
        if len(x):
            alone = recs[k].recognize(torch.from_numpy(x).to("cuda"), algo=algo)
            assert (alone["accept"], alone["final_state"]) == want
        assert got["latency"] >= 0
        accepted += want[0]
    assert 0 < accepted < len(reqs)


def test_admission_by_footprint(pool):
    """A budget that holds only a few requests at a time: the server admits
    while the footprints fit, and every request still completes correctly."""
    autos, recs, refs = pool
    reqs = requests(autos, 3, 60, median=1 << 15, cap=1 << 17)
    fps = [ri.ri_request_footprint(recs[k].handle, "rid", len(x)) for k, x in reqs]
    budget = 3 * max(fps)
    srv = ri.serve.Server(recs, algo="rid", slots=2, hbm_budget=budget)
    try:
        for k, x in reqs:
            srv.submit(k, x)
        done = srv.drain()
    finally:
        srv.close()
    assert srv.max_used <= budget
    assert srv.steps >= sum(fps) // budget      # in-flight footprint never exceeds the budget
    by_id = {d["id"]: d for d in done}
    for i, (k, x) in enumerate(reqs):
        assert (by_id[i]["accept"], by_id[i]["final_state"]) == oracle.serial(refs[k][0], x, refs[k][1])


def test_batch_update_reuses_the_plan(pool):
    """ri_batch_update re-plans a fused batch for other requests; results
    follow the new requests."""
    autos, recs, refs = pool
    a = requests(autos, 5, 20)
    b = requests(autos, 6, 35)
    ta = [torch.from_numpy(x).to("cuda") for _, x in a]
    tb = [torch.from_numpy(x).to("cuda") for _, x in b]
    batch = ri.Batch([(recs[k], t, "rid") for (k, _), t in zip(a, ta)], mode="fused")
    try:
        for reqs, texts in ((a, ta), (b, tb), (a, ta)):
            ri.ri_batch_update(batch.handle, [(recs[k].handle, t, "rid") for (k, _), t in zip(reqs, texts)])
            batch.count = len(reqs)
            batch.results = torch.zeros(2 * len(reqs), dtype=torch.int32, device="cuda")
            got = batch.run().cpu().numpy()
            for i, (k, x) in enumerate(reqs):
                assert (bool(got[i, 0]), int(got[i, 1])) == oracle.serial(refs[k][0], x, refs[k][1])
    finally:
        batch.close()
