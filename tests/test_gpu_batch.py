"""GPU parity of batches (include/ri.h, ri_batch_*): every text of a batch
gets exactly the oracle's serial result (accept, canonical final state) and
the result of recognizing it alone, whatever the mix of automata, algorithms,
lengths (0, ragged, multi-level join trees) and chunk sizes; graph replays
and autotuned plans give the same results.
"""

import json
import os

import numpy as np
import pytest

import oracle
from workloads import gen

torch = pytest.importorskip("torch")
ri = pytest.importorskip("paper_2412_14975_amd")

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ALGOS = ("rid", "dfa", "subset")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ri.binding.lib()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint8)).to("cuda")


class MinRef:
    """The oracle's minimal DFA of an expression and its serial recognizer."""

    def __init__(self, pattern):
        self.dfa = oracle.min_dfa_of(oracle.trim(oracle.position_nfa(pattern)))
        self.table = oracle.dense_table(self.dfa.n, self.dfa.delta)

    def serial(self, x):
        return oracle.serial(self.dfa, x, self.table)


def small_pattern(rng, alphabet, depth, maxpos=40):
    while True:
        p = gen.random_regex(rng, alphabet, depth)
        if oracle.position_nfa(p).n <= maxpos:
            return p


def mixed_requests(seed):
    """(pattern, text, algo) triples over several automata and lengths."""
    rng = gen.PCG(4242 + seed)
    pats = [gen.c1_regex(), b"ab*", b"a[^\\x00-\\xff]", b"()"]
    pats += [small_pattern(rng, b"abc"[: 2 + k % 2], 3) for k in range(3)]
    lengths = (0, 1, 15, 16, 17, 100, 1000, 4097, 65541, 300007)
    out = []
    for pi, p in enumerate(pats):
        for li, n in enumerate(lengths):
            if (pi + li) % 2:
                continue
            alpha = b"ab" if p in (gen.c1_regex(), b"ab*") else b"abcz"
            x = gen.random_text(rng, alpha, n)
            if p == gen.c1_regex() and n >= 4:
                x[-4:] = np.frombuffer(b"abab", np.uint8)
            out.append((p, x, ALGOS[(pi + li // 2) % 3]))
    return out


MODES = ("grouped", "fused", "queue")


def check_batch(reqs, chunk_bytes, refs, recs, launch="run", mode="auto"):
    texts = [dev(x) for _, x, _ in reqs]
    b = ri.Batch([(recs[p], t, a) for (p, _, a), t in zip(reqs, texts)], chunk_bytes=chunk_bytes, mode=mode)
    try:
        if launch == "run":
            runs = [b.run().cpu().numpy()]
        else:
            # replays of one captured graph, with eager work of the same batch
            # in between: every replay must give the same results
            b.capture()
            runs = []
            for rep in range(3):
                runs.append(b.launch().cpu().numpy())
                if rep == 0:
                    b.run()
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        for got in runs:
            for i, (p, x, a) in enumerate(reqs):
                want = refs[p].serial(x)
                assert (bool(got[i, 0]), int(got[i, 1])) == want, (p, len(x), a, chunk_bytes)
        for i, (p, x, a) in enumerate(reqs):
            want = refs[p].serial(x)
            if len(x) and i % 3 == 0:
                alone = recs[p].recognize(texts[i], algo=a)
                assert (alone["accept"], alone["final_state"]) == want
        return b.info()
    finally:
        b.close()


@pytest.fixture(scope="module")
def mixed():
    reqs = mixed_requests(0)
    refs, recs = {}, {}
    for p, _, _ in reqs:
        if p not in refs:
            refs[p] = MinRef(p)
            recs[p] = ri.Recognizer(p)
    yield reqs, refs, recs
    for r in recs.values():
        r.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("chunk_bytes", [0, 16, 48, 256, 4096])
def test_mixed_batch(mixed, chunk_bytes, mode):
    reqs, refs, recs = mixed
    info = check_batch(reqs, chunk_bytes, refs, recs, mode=mode)
    assert info["texts"] == len(reqs)
    assert info["bytes"] == sum(len(x) for _, x, _ in reqs)
    assert info["fused"] == (mode == "fused")


@pytest.mark.parametrize("mode", MODES)
def test_mixed_batch_graph(mixed, mode):
    reqs, refs, recs = mixed
    info = check_batch(reqs, 64, refs, recs, launch="graph", mode=mode)
    assert info["captured"] == 1


@pytest.mark.parametrize("mode", MODES)
def test_deep_join_trees(mode):
    """16-byte chunks: a 300 KB text has ~19k chunks, so the per-text join
    tree has three or more levels; texts of one chunk sit beside it."""
    p = gen.c1_regex()
    ref, rec = MinRef(p), ri.Recognizer(p)
    rng = gen.PCG(5)
    xs = [gen.random_text(rng, b"ab", n) for n in (300000, 1, 16, 17, 1024, 65536, 70000)]
    for x in xs[::2]:
        if len(x) >= 4:
            x[-4:] = np.frombuffer(b"abab", np.uint8)
    try:
        for algo in ALGOS:
            reqs = [(p, x, algo) for x in xs]
            b = ri.Batch([(rec, dev(x), algo) for x in xs], chunk_bytes=16, mode=mode)
            try:
                assert b.group(0)["join_levels"] >= 3
                got = b.run().cpu().numpy()
                for i, x in enumerate(xs):
                    assert (bool(got[i, 0]), int(got[i, 1])) == ref.serial(x), (algo, len(x))
            finally:
                b.close()
            del reqs
    finally:
        rec.close()


@pytest.mark.parametrize("mode", MODES)
def test_graph_replays_with_eager_work_between(mode):
    """Replay the captured graph several times; between replays the results
    are overwritten by eager torch work, and every replay must restore them."""
    p = gen.c1_regex()
    ref, rec = MinRef(p), ri.Recognizer(p)
    rng = gen.PCG(9)
    xs = [gen.random_text(rng, b"ab", n) for n in (5000, 70001, 12345, 1 << 18)]
    xs[0][-4:] = np.frombuffer(b"abab", np.uint8)
    want = [ref.serial(x) for x in xs]
    texts = [dev(x) for x in xs]
    b = ri.Batch([(rec, t, a) for t, a in zip(texts, ("rid", "dfa", "rid", "subset"))], chunk_bytes=256, mode=mode)
    try:
        b.capture()
        for rep in range(4):
            b.results.fill_(-7)
            torch.cuda.synchronize()
            got = b.launch().cpu().numpy()
            assert [(bool(a), int(f)) for a, f in got] == want, rep
            scratch = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
            float(scratch)
    finally:
        b.close()
        rec.close()


@pytest.mark.parametrize("mode", MODES)
def test_batch_autotune_keeps_results(mode):
    rx, motifs = gen.c2_regex_and_motifs(2)
    ref = MinRef(rx)
    rng = gen.PCG(3)
    xs = []
    for k in range(12):
        x, rej = gen.c2_texts(100 + k, n=int(rng.integers(1 << 10, 1 << 20)) // 16 * 16 + k, motifs=motifs)
        xs.append(x if k % 2 == 0 else rej)
    rec = ri.Recognizer(rx)
    texts = [dev(x) for x in xs]
    b = ri.Batch([(rec, t, ("rid", "dfa")[i % 2]) for i, t in enumerate(texts)], mode=mode)
    try:
        tun = b.autotune()
        assert tun["trials"] >= 6 and tun["best_ms"] > 0
        for g in range(b.info()["groups"]):
            assert b.group(g)["tuned_ms"] > 0
        got = b.run().cpu().numpy()
        for i, x in enumerate(xs):
            assert (bool(got[i, 0]), int(got[i, 1])) == ref.serial(x)
    finally:
        b.close()
        rec.close()


def test_batch_autotune_chooses_the_long_run_plan():
    """A batch in automatic mode with enough text per group takes the grouped
    plan; its autotune times one launch sequence per group against one
    work-queue launch for every group's long runs and keeps the faster.  The
    results stay the oracle's either way, also after a graph capture."""
    rx, motifs = gen.c2_regex_and_motifs(1)
    ref = MinRef(rx)
    xs = []
    for k in range(4):
        x, rej = gen.c2_texts(300 + k, n=(24 << 20) + 16 * k + 3, motifs=motifs)
        xs.append(x if k % 2 == 0 else rej)
    rec = ri.Recognizer(rx)
    texts = [dev(x) for x in xs]
    b = ri.Batch([(rec, t, ("rid", "dfa")[i % 2]) for i, t in enumerate(texts)], mode="auto")
    try:
        info = b.info()
        assert info["fused"] == 0 and info["queue"] == 0
        tun = b.autotune()
        assert tun["trials"] >= 8 and tun["best_ms"] > 0
        assert b.info()["queue"] in (0, 1)
        wants = [ref.serial(x) for x in xs]
        for run in (b.run, None):
            if run is None:
                b.capture()
                got = b.launch().cpu().numpy()
            else:
                got = run().cpu().numpy()
            for i, want in enumerate(wants):
                assert (bool(got[i, 0]), int(got[i, 1])) == want, (i, run is None)
    finally:
        b.close()
        rec.close()


@pytest.mark.parametrize("mode", MODES)
def test_batched_workload_sample(mode):
    """Four expressions of the batched workload, 48 texts of 1 KiB - 512 KiB,
    half derived from the expression and half changed at one byte."""
    spec = json.load(open(os.path.join(HERE, "golden", "c4_regexes.json")))
    seed = spec["seed"]
    chosen = spec["expressions"][::4]
    lengths = gen.c4_lengths(11, count=48, lo=1 << 10, hi=1 << 19)
    refs, recs, reqs = [], [], []
    for e in chosen:
        rx, tree, alphabet = gen.c4_candidate(seed, e["index"])
        assert rx.decode("latin-1") == e["regex"]
        refs.append(MinRef(rx))
        recs.append(ri.Recognizer(rx))
        reqs.append((tree, alphabet))
    items = []
    for i, n in enumerate(lengths):
        k = i % len(chosen)
        x, changed = gen.c4_text(11, i, reqs[k][0], reqs[k][1], int(n))
        items.append((k, x, changed))
    texts = [dev(x) for _, x, _ in items]
    try:
        for algo in ("rid", "dfa"):
            b = ri.Batch([(recs[k], t, algo) for (k, _, _), t in zip(items, texts)], mode=mode)
            try:
                got = b.run().cpu().numpy()
            finally:
                b.close()
            accepted = 0
            for i, (k, x, changed) in enumerate(items):
                want = refs[k].serial(x)
                assert (bool(got[i, 0]), int(got[i, 1])) == want, (algo, i, len(x))
                if not changed:
                    assert want[0], "a derived text is in the language"
                accepted += want[0]
            assert 0 < accepted < len(items)
    finally:
        for r in recs:
            r.close()


def test_batch_argument_errors():
    rec = ri.Recognizer(b"ab*")
    try:
        buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
        with pytest.raises(ri.RIError) as e:
            ri.Batch([(rec, buf[1:], "rid")])
        assert e.value.code == ri.binding.RI_ERR_ARG
        with pytest.raises(ri.RIError):
            ri.Batch([(rec, buf, "rid")], chunk_bytes=24)
        b = ri.Batch([(rec, buf, "rid")])
        try:
            with pytest.raises(TypeError):
                ri.ri_batch_run(b.handle, torch.zeros(1, dtype=torch.int32, device="cuda"))
            with pytest.raises(ri.RIError):
                ri.ri_batch_launch(b.handle)     # nothing captured yet
        finally:
            b.close()
        # an empty batch runs and launches nothing
        b = ri.Batch([])
        try:
            b.run()
            assert b.info()["texts"] == 0
        finally:
            b.close()
    finally:
        rec.close()


def test_fused_batch_of_large_automata():
    """Keyword unions with 20 and 300 keywords (interfaces below and beyond
    2048 states) and the never-merging counter beside a 300-keyword union,
    RID and DFA, in one fused batch (auto mode picks fused for them)."""
    kw20, k20 = gen.c5_automaton(7, 1, 20)
    kw300, k300 = gen.c5_automaton(7, 1, 300)
    count = b"((b*a){37})*b*|z" + kw300
    pats = [kw20, kw300, count]
    refs = {p: MinRef(p) for p in pats}
    recs = {p: ri.Recognizer(p) for p in pats}
    rng = gen.PCG(77)
    reqs = []
    for i, n in enumerate((0, 1, 300, 5000, 65536, 200003)):
        reqs.append((kw20, gen.c5_text(rng, k20, n, i % 2 == 0), ("rid", "dfa")[i % 2]))
        reqs.append((kw300, gen.c5_text(rng, k300, n, i % 2 == 1), ("rid", "dfa")[(i + 1) % 2]))
        reqs.append((count, gen.random_text(rng, b"ab", n), "rid"))
    try:
        texts = [dev(x) for _, x, _ in reqs]
        b = ri.Batch([(recs[p], t, a) for (p, _, a), t in zip(reqs, texts)], chunk_bytes=256)
        try:
            assert b.info()["fused"] == 1
            for rep in range(2):
                got = b.run().cpu().numpy()
                for i, (p, x, a) in enumerate(reqs):
                    assert (bool(got[i, 0]), int(got[i, 1])) == refs[p].serial(x), (rep, i, len(x), a)
        finally:
            b.close()
    finally:
        for r in recs.values():
            r.close()


def test_queue_with_tables_in_l2():
    """Work-queue batches mixing an automaton whose tables do not fit LDS
    (40 keywords under a star: B' of 1584 states over 38 classes, 241 KB,
    read from L2 by the queue) with small ones staged in LDS: every text
    gets the oracle's result, RID and DFA, run and graph."""
    rng = np.random.default_rng(5)
    letters = b"abcdefghijklmnopqrstuvwxyz0123456789"
    kws = [bytes(rng.choice(list(letters), size=int(rng.integers(4, 9)))) for _ in range(40)]
    big = b"(" + b"|".join(kws) + b")*"
    pats = [big, gen.c1_regex(), b"ab*"]
    refs = {p: MinRef(p) for p in pats}
    recs = {p: ri.Recognizer(p) for p in pats}
    assert recs[big].info()["table_bytes"][0] > 160 * 1024
    prng = gen.PCG(77)
    reqs = []
    for i, n_words in enumerate((0, 1, 7, 300, 4000, 20000)):
        x = np.frombuffer(b"".join(kws[int(j)] for j in rng.integers(0, len(kws), size=n_words)), np.uint8).copy()
        if i % 2 and len(x):
            x[int(rng.integers(0, len(x)))] = ord("#")   # rejected
        reqs.append((big, x, ("rid", "dfa")[i % 2]))
        reqs.append((big, x, ("dfa", "rid")[i % 2]))
    for p in pats[1:]:
        for n in (100, 70001):
            x = gen.random_text(prng, b"ab", n)
            reqs.append((p, x, "rid"))
            reqs.append((p, x, "dfa"))
    try:
        for launch in ("run", "graph"):
            info = check_batch(reqs, 0, refs, recs, launch=launch, mode="queue")
            assert info["texts"] == len(reqs)
    finally:
        for r in recs.values():
            r.close()
