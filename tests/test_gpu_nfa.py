"""GPU parity of the NFA device (RI_ALGO_NFA, Sect. 2 / Fig. 1): the
position NFA as chunk automaton, every NFA state speculated, runs as sets of
states, chunk relations composed.  Bit-exact (accept, final state) against
the oracle's serial recognizer, and the oracle's own NFA chunked simulator
agrees on acceptance (Lemma 1's NFA form is pinned in the oracle tests)."""

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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint8)).to("cuda")


def small_pattern(rng, alphabet, depth, maxpos=60):
    while True:
        p = gen.random_regex(rng, alphabet, depth)
        if oracle.position_nfa(p).n <= maxpos:
            return p


@pytest.mark.parametrize("seed", range(16))
def test_random_expressions(seed):
    rng = gen.PCG(4400 + seed)
    alphabet = b"abcd"[: 2 + seed % 3]
    pattern = small_pattern(rng, alphabet, int(rng.integers(1, 4)))
    b = oracle.build(pattern)
    table = oracle.dense_table(b.dfa.n, b.dfa.delta)
    rec = ri.Recognizer(pattern)
    try:
        assert rec.info()["starts"][3] == b.nfa.n
        for n in (1, 5, 16, 17, 63, 200, 4097, 70001):
            x = gen.random_text(rng, alphabet + (b"z" if seed % 4 == 0 else b""), n)
            want = oracle.serial(b.dfa, x, table)
            for chunks in (1, 3, n, 0):
                got = rec.recognize(dev(x), algo="nfa", chunks=chunks)
                assert (got["accept"], got["final_state"]) == want, (pattern, n, chunks)
            if n <= 200:
                res = oracle.nfa_csdpa(b.nfa, x, oracle.even_bounds(n, 3))
                assert res["accept"] == want[0]
    finally:
        rec.close()


@pytest.mark.parametrize("k", [3, 8, 12])
def test_regexp_family(k):
    rx = gen.regexp_family(k)
    b = oracle.build(rx)
    rec = ri.Recognizer(rx)
    try:
        assert rec.info()["starts"][3] == 2 * k + 4
        acc, rej = gen.c1_texts(500 + k, n=(1 << 20) + 3)
        for x in (acc, rej):
            want = oracle.serial(b.dfa, x)
            for chunks in (64, 4096, 0):
                got = rec.recognize(dev(x), algo="nfa", chunks=chunks)
                assert (got["accept"], got["final_state"]) == want, (k, chunks)
    finally:
        rec.close()


def test_motif_and_log_lines():
    """The motif union (105 NFA states: two words per set) and the log-lines
    expression (231 NFA states: four words per set) on 16 MiB texts and their
    rejected copies; queued calls too."""
    rx, motifs = gen.c2_regex_and_motifs(0)
    cases = [(rx, gen.c2_texts(0, n=1 << 24, motifs=motifs))]
    cases.append((gen.c3_regex(), gen.c3_texts(1, n=1 << 24)))
    for rx, texts in cases:
        b = oracle.build(rx)
        table = oracle.dense_table(b.dfa.n, b.dfa.delta)
        rec = ri.Recognizer(rx)
        try:
            res = torch.full((len(texts), 2), -7, dtype=torch.int32, device="cuda")
            wants = []
            for i, x in enumerate(texts):
                want = oracle.serial(b.dfa, x, table)
                wants.append(want)
                t = dev(x)
                for chunks in (0, 1000):
                    got = rec.recognize(t, algo="nfa", chunks=chunks)
                    assert (got["accept"], got["final_state"]) == want, (rx[:20], i, chunks)
                rec.recognize_async(t, res[i], algo="nfa")
                torch.cuda.synchronize()
            for g, w in zip(res.cpu().numpy(), wants):
                assert (bool(g[0]), int(g[1])) == w
        finally:
            rec.close()


def test_limits_and_errors():
    big = b"(" + b"|".join(b"k%03d" % i for i in range(80)) + b")*"     # > 256 NFA states
    rec = ri.Recognizer(big)
    try:
        with pytest.raises(ri.RIError) as e:
            rec.recognize(dev(np.frombuffer(b"k001k002", np.uint8)), algo="nfa")
        assert e.value.code == ri.binding.RI_ERR_LIMIT
    finally:
        rec.close()
    rec = ri.Recognizer(gen.c1_regex())
    try:
        x = dev(gen.c1_texts(0, n=4096)[0])
        with pytest.raises(ri.RIError) as e:
            rec.chunk_maps(x, algo="nfa", chunks=4)
        assert e.value.code == ri.binding.RI_ERR_ARG
        r = rec.recognize(torch.empty(0, dtype=torch.uint8, device="cuda"), algo="nfa")
        assert (r["accept"], r["final_state"]) == (False, 0)
        tun = rec.autotune(x, algo="nfa")
        assert tun["trials"] >= 1
        got = rec.recognize(x, algo="nfa")
        want = oracle.serial(oracle.build(gen.c1_regex()).dfa, gen.c1_texts(0, n=4096)[0])
        assert (got["accept"], got["final_state"]) == want
    finally:
        rec.close()
