"""GPU parity for large automata: keyword unions .*(k1|...|kn).* whose
interface exceeds the 2048 states of dense content bitsets (member lists,
hit-matrix join over them), and an expression whose runs never merge on top
of such an interface (join by propagation).  Expected values: the oracle's
minimal DFA and serial scan.
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint8)).to("cuda")


class MinRef:
    def __init__(self, pattern):
        self.dfa = oracle.min_dfa_of(oracle.trim(oracle.position_nfa(pattern)))
        self.table = oracle.dense_table(self.dfa.n, self.dfa.delta)

    def serial(self, x):
        return oracle.serial(self.dfa, x, self.table)


@pytest.fixture(scope="module", params=[20, 300])
def keywords(request):
    rx, kws = gen.c5_automaton(7, 1, request.param)
    rec = ri.Recognizer(rx)
    yield rx, kws, rec, MinRef(rx)
    rec.close()


def test_keyword_unions(keywords):
    rx, kws, rec, ref = keywords
    info = rec.info()
    if len(kws) == 300:
        assert info["interface_states"] > 2048      # beyond dense bitsets
    rng = gen.PCG(55)
    for n in (1, 100, 4097, 1 << 16, (1 << 20) + 3):
        for plant in (False, True):
            x = gen.c5_text(rng, kws, n, plant)
            want = ref.serial(x)
            for algo in ("rid", "dfa"):
                for chunks in (0, 7, 1000):
                    got = rec.recognize(dev(x), algo=algo, chunks=chunks)
                    assert (got["accept"], got["final_state"]) == want, (len(kws), n, plant, algo, chunks)


def test_keyword_union_chunk_maps(keywords):
    rx, kws, rec, ref = keywords
    rng = gen.PCG(56)
    x = gen.c5_text(rng, kws, 3000, True)
    res, maps = rec.chunk_maps(dev(x), algo="dfa", chunks=5)
    cs = res["chunk_size"]
    for i in range(res["chunks"]):
        lo, hi = i * cs, min(len(x), (i + 1) * cs)
        for s in range(0, ref.dfa.n, max(1, ref.dfa.n // 97)):
            want = -1 if (i == 0 and s != 0) else oracle.run(ref.table, s, x, lo, hi)[0]
            assert maps[i, s] == want, (i, s)


def test_runs_that_never_merge_on_a_large_interface():
    """Counting a's modulo 37 beside a 300-keyword union behind 'z': the
    interface exceeds 2048 states and every chunk keeps 37 runs, so the
    join falls back to propagation."""
    kw_rx, _ = gen.c5_automaton(7, 1, 300)
    rx = b"((b*a){37})*b*|z" + kw_rx
    ref = MinRef(rx)
    rec = ri.Recognizer(rx)
    try:
        assert rec.info()["interface_states"] > 2048
        rng = gen.PCG(37)
        for n in (37 * 5, 100003):
            x = gen.random_text(rng, b"ab", n)
            want = ref.serial(x)
            for chunks in (3, 64, 0):
                got = rec.recognize(dev(x), algo="rid", chunks=chunks)
                assert (got["accept"], got["final_state"]) == want, (n, chunks)
    finally:
        rec.close()


def test_warm_up_with_starts_read_from_global_memory():
    """520 keywords: 4447 interface starts (RID) and 6246 minimal-DFA states,
    more than the warm-up stages in LDS (4096), so the warm-up reads its start
    list from global memory; the results must still be the oracle's."""
    rx, kws = gen.c5_automaton(7, 1, 520)
    ref = MinRef(rx)
    rec = ri.Recognizer(rx)
    try:
        info = rec.info()
        assert info["starts"][0] > 4096 and info["starts"][1] > 4096
        rng = gen.PCG(91)
        for n in (4097, 1 << 16, (1 << 20) + 3):
            for plant in (False, True):
                x = gen.c5_text(rng, kws, n, plant)
                want = ref.serial(x)
                for algo in ("rid", "dfa"):
                    for chunks in (0, 64):
                        got = rec.recognize(dev(x), algo=algo, chunks=chunks)
                        assert (got["accept"], got["final_state"]) == want, (algo, n, chunks)
    finally:
        rec.close()
