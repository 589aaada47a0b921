"""GPU parity: the HIP path (through the C ABI) against the oracle.

Every comparison is bit-exact: ``accept`` and ``final_state`` (canonical
minimal-DFA id) against the oracle's serial recognizer, and the chunk maps
lambda_i against the oracle's own runs over the same chunk boundaries:
RI-DFA end states are compared by content (the set of N' states they stand
for), since state ids depend on construction order; DFA end states are
canonical ids and are compared directly.
"""

import numpy as np
import pytest

import oracle
from workloads import gen

torch = pytest.importorskip("torch")
ri = pytest.importorskip("paper_2412_14975_amd")

pytestmark = pytest.mark.gpu

ALGOS = ("rid", "dfa", "subset")

# reach pipelines: converging (warm-up + merge) with two warm-up lengths and
# the hit-matrix join, converging with the class join, and plain
MODES = {"conv64": dict(converge=1, warmup_bytes=64), "conv16": dict(converge=1, warmup_bytes=16),
         "cls64": dict(converge=1, warmup_bytes=64, join=1), "plain": dict(converge=0),
         # warm-ups longer than 64 bytes (four registers of byte codes), also
         # longer than many chunks of the small texts below
         "conv80": dict(converge=1, warmup_bytes=80), "conv128": dict(converge=1, warmup_bytes=128),
         "conv256": dict(converge=1, warmup_bytes=256),
         # every start stepping from the first byte (no transformation-automaton walk)
         "noprefix64": dict(converge=1, warmup_bytes=64, prefix=0)}


def make(pattern, mode="conv64", runs_per_lane=0):
    rec = ri.Recognizer(pattern)
    for k, v in MODES[mode].items():
        rec.set_option(k, v)
    rec.set_option("runs_per_lane", runs_per_lane)
    return rec


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ri.binding.lib()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint8)).to("cuda")


class Ref:
    """Oracle automata for one expression, with dense tables for the C scan."""

    def __init__(self, pattern):
        self.b = oracle.build(pattern)
        self.tdfa = oracle.dense_table(self.b.dfa.n, self.b.dfa.delta)
        self._tbq = None

    @property
    def tbq(self):
        if self._tbq is None:
            self._tbq = oracle.dense_table(self.b.Bq.n, self.b.Bq.delta)
        return self._tbq

    def serial(self, x):
        return oracle.serial(self.b.dfa, x, self.tdfa)


def check_maps(rec, ref, x, algo, chunks, sample=None, rng=None):
    """Compare the chunk maps of the HIP path with the oracle's runs."""
    res, maps = rec.chunk_maps(dev(x), algo=algo, chunks=chunks)
    n, cs, c = len(x), res["chunk_size"], res["chunks"]
    assert c == -(-n // cs)
    idx = range(c) if sample is None else sorted(set([0, c - 1] + list(rng.choice(c, size=sample))))
    for i in idx:
        lo, hi = i * cs, min(n, (i + 1) * cs)
        if algo == "rid":
            B = ref.b.Bq
            for q in range(ref.b.nfa_q.n):
                want = None
                if i == 0 and q != 0:
                    want = None
                else:
                    end, _ = oracle.run(ref.tbq, B.initial[q], x, lo, hi)
                    want = B.content[end] if end >= 0 else None
                got = maps[i, q]
                got_c = frozenset(rec.state_content("rid", int(got))) if got >= 0 else None
                assert got_c == want, (i, q)
        elif algo == "dfa":
            for s in range(ref.b.dfa.n):
                want = -1 if (i == 0 and s != 0) else oracle.run(ref.tdfa, s, x, lo, hi)[0]
                assert maps[i, s] == want, (i, s)
    return res


# ---------------------------------------------------------------------------
# tiny workload: (a|b)*a(a|b)^3, 1 MiB
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module", params=sorted(MODES))
def tiny(request):
    rx = gen.c1_regex()
    rec = make(rx, request.param)
    yield rec, Ref(rx)
    rec.close()


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("chunks", [64, 0, 1, 1000, 65536])
def test_tiny_accept_and_final(tiny, seed, algo, chunks):
    rec, ref = tiny
    acc, rej = gen.c1_texts(seed)
    for x, expect in ((acc, True), (rej, False)):
        want = ref.serial(x)
        assert want[0] is expect
        got = rec.recognize(dev(x), algo=algo, chunks=chunks)
        assert (got["accept"], got["final_state"]) == want
        assert got["n"] == len(x)


@pytest.mark.parametrize("c", [4096, 4097, 4098, 4161, 4162])
def test_join_level_boundaries(tiny, c):
    """16-byte chunks, c of them: c - 1 = 64 x 64 (+1, ...) hit matrices, so
    the last level of the product gets exactly 64 members or needs one more
    level; the functional join of the DFA sees the same group boundaries."""
    rec, ref = tiny
    acc, rej = gen.c1_texts(70 + c % 7, n=c * 16)
    for x in (acc, rej):
        want = ref.serial(x)
        for algo in ALGOS:
            got = rec.recognize(dev(x), algo=algo, chunks=c)
            assert got["chunks"] == c
            assert (got["accept"], got["final_state"]) == want, (algo, c)


@pytest.mark.parametrize("algo", ["rid", "dfa"])
def test_tiny_chunk_maps(tiny, algo):
    rec, ref = tiny
    acc, _ = gen.c1_texts(3, n=(1 << 14) + 5)      # ragged last chunk
    check_maps(rec, ref, acc, algo, 64)
    check_maps(rec, ref, acc, algo, 1000)


# ---------------------------------------------------------------------------
# random expressions, ragged sizes, every algorithm
# ---------------------------------------------------------------------------

def small_pattern(rng, alphabet, depth, maxpos=40):
    while True:
        p = gen.random_regex(rng, alphabet, depth)
        if oracle.position_nfa(p).n <= maxpos:
            return p


@pytest.mark.parametrize("seed", range(24))
@pytest.mark.parametrize("mode", sorted(MODES))
def test_random_expressions(seed, mode):
    rng = gen.PCG(777 + seed)
    alphabet = b"abcd"[: 2 + seed % 3]
    pattern = small_pattern(rng, alphabet, int(rng.integers(1, 4)))
    ref = Ref(pattern)
    rec = make(pattern, mode, runs_per_lane=(0, 1, 2, 4)[seed % 4])
    try:
        for n in (1, 5, 15, 16, 17, 63, 200, 4097, 70001):
            x = gen.random_text(rng, alphabet + b"z", n) if seed % 4 == 0 else gen.random_text(rng, alphabet, n)
            want = ref.serial(x)
            for algo in ALGOS:
                for chunks in (1, 3, n, 0):
                    got = rec.recognize(dev(x), algo=algo, chunks=chunks)
                    assert (got["accept"], got["final_state"]) == want, (pattern, n, algo, chunks)
        x = gen.random_text(rng, alphabet, 3001)
        check_maps(rec, ref, x, "rid", 37)
        check_maps(rec, ref, x, "dfa", 37)
    finally:
        rec.close()


def test_accepted_texts_of_random_expressions():
    """Texts built as members (random walks to acceptance on the oracle DFA),
    so that acceptance, not just rejection, is exercised on long inputs."""
    rng = gen.PCG(4242)
    for _ in range(8):
        pattern = small_pattern(rng, b"abc", 3)
        ref = Ref(pattern)
        d = ref.b.dfa
        if d.n == 0 or not d.final:
            continue
        # walk, then finish along a shortest path to a final state
        s, out = 0, []
        for _ in range(5000):
            moves = sorted(d.delta[s].items())
            if not moves:
                break
            b, s = moves[int(rng.integers(0, len(moves)))]
            out.append(b)
        dist = {f: [] for f in d.final}
        frontier = list(d.final)
        pred = [[] for _ in range(d.n)]
        for q in range(d.n):
            for b, t in d.delta[q].items():
                pred[t].append((q, b))
        while frontier:
            nxt = []
            for t in frontier:
                for q, b in pred[t]:
                    if q not in dist:
                        dist[q] = [b] + dist[t]
                        nxt.append(q)
            frontier = nxt
        if s not in dist:
            continue
        x = np.frombuffer(bytes(out + dist[s]), dtype=np.uint8)
        want = ref.serial(x)
        assert want[0] is True
        mode = ("conv64", "conv16", "plain")[_ % 3]
        rec = make(pattern, mode)
        try:
            for algo in ALGOS:
                for chunks in (1, 7, 100, 0):
                    got = rec.recognize(dev(x), algo=algo, chunks=chunks)
                    assert (got["accept"], got["final_state"]) == want, (pattern, mode, algo, chunks, got)
        finally:
            rec.close()


@pytest.mark.parametrize("mode", ["conv64", "conv16"])
def test_runs_that_never_converge(mode):
    """Counting a's modulo 37: the minimal DFA permutes its 37 states, so
    runs never die and never merge; each chunk keeps more distinct states
    than the merge step searches and falls back to one run per start."""
    rx = b"((b*a){37})*b*"
    ref = Ref(rx)
    rec = make(rx, mode)
    try:
        assert rec.info()["starts"][1] == 37
        rng = gen.PCG(37)
        for n in (37 * 5, 100003):
            x = gen.random_text(rng, b"ab", n)
            want = ref.serial(x)
            for algo in ALGOS:
                for chunks in (3, 64, 0):
                    got = rec.recognize(dev(x), algo=algo, chunks=chunks)
                    assert (got["accept"], got["final_state"]) == want, (algo, chunks)
        x = gen.random_text(rng, b"ab", 20000)
        check_maps(rec, ref, x, "dfa", 50)
        check_maps(rec, ref, x, "rid", 50)
    finally:
        rec.close()


@pytest.mark.parametrize("k", [2, 7, 8, 9, 16])
def test_runs_per_chunk_around_the_hit_row_cap(k):
    """Counting a's modulo k keeps k runs per chunk after merging: up to 8
    the hit-matrix join handles them, above it the call falls back to the
    class join.  Both must give the oracle's result."""
    rx = b"((b*a){%d})*b*" % k
    ref = Ref(rx)
    rec = make(rx, "conv16")
    try:
        rng = gen.PCG(100 + k)
        for n in (5000, 300001):
            for accept in (False, True):
                x = gen.random_text(rng, b"ab", n)
                if accept:   # flip b's to a's until the count of a's is a multiple of k
                    need = (-int((x == ord("a")).sum())) % k
                    x[np.flatnonzero(x == ord("b"))[:need]] = ord("a")
                want = ref.serial(x)
                assert not accept or want[0]
                for chunks in (1, 2, 64, 0):
                    got = rec.recognize(dev(x), algo="rid", chunks=chunks)
                    assert (got["accept"], got["final_state"]) == want, (k, n, chunks)
    finally:
        rec.close()


@pytest.mark.parametrize("k", [6, 10, 12])
def test_regexp_family_sweep(k):
    """(a|b)*a(a|b)^k: the minimal DFA has 2^(k+1) states (all speculated by
    the baseline), the interface k + 2.  Accepted and rejected texts, both
    algorithms, converging and plain reach."""
    rx = gen.regexp_family(k)
    ref = Ref(rx)
    acc, rej = gen.c1_texts(300 + k, n=(1 << 20) + 9)
    for mode in ("conv16", "plain"):
        rec = make(rx, mode)
        try:
            assert rec.info()["min_dfa_states"] == 2 ** (k + 1)
            assert rec.info()["interface_states"] == k + 2
            for x in (acc, rej):
                want = ref.serial(x)
                for algo in ("rid", "dfa"):
                    for chunks in (64, 0):
                        got = rec.recognize(dev(x), algo=algo, chunks=chunks)
                        assert (got["accept"], got["final_state"]) == want, (k, mode, algo, chunks)
            if k == 10:
                check_maps(rec, ref, acc[:40000], "rid", 16)
        finally:
            rec.close()


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", sorted(MODES))
def test_edge_cases(mode):
    rec = make(b"ab*", mode)
    ref = Ref(b"ab*")
    try:
        # empty text: decided on the host, no device work
        r = rec.recognize(torch.empty(0, dtype=torch.uint8, device="cuda"))
        assert (r["accept"], r["final_state"]) == (False, 0)
        # one byte, more chunks than bytes
        for x in (b"a", b"b", b"abbb", b"ab\x00b"):
            xx = np.frombuffer(x, dtype=np.uint8)
            for algo in ALGOS:
                for chunks in (1, 2, 100):
                    got = rec.recognize(dev(xx), algo=algo, chunks=chunks)
                    assert (got["accept"], got["final_state"]) == ref.serial(xx)
                    assert got["chunks"] >= 1
        # misaligned text is refused, not read
        buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
        with pytest.raises(ri.RIError) as e:
            rec.recognize(buf[1:])
        assert e.value.code == ri.binding.RI_ERR_ARG
        # no CPU path
        with pytest.raises(TypeError):
            rec.recognize(torch.zeros(16, dtype=torch.uint8))
    finally:
        rec.close()


def test_empty_language_and_empty_string_language():
    e = ri.Recognizer(b"a[^\\x00-\\xff]")
    try:
        x = dev(np.frombuffer(b"a" * 100, dtype=np.uint8))
        for algo in ALGOS:
            assert e.recognize(x, algo=algo) == dict(accept=False, final_state=-1, n=100, chunks=0,
                                                     chunk_size=0)
    finally:
        e.close()
    eps = ri.Recognizer(b"()")
    try:
        r = eps.recognize(torch.empty(0, dtype=torch.uint8, device="cuda"))
        assert (r["accept"], r["final_state"]) == (True, 0)
        r = eps.recognize(dev(np.frombuffer(b"x" * 33, dtype=np.uint8)), algo="dfa")
        assert (r["accept"], r["final_state"]) == (False, -1)
    finally:
        eps.close()


def test_autotune_keeps_results_exact():
    rx, motifs = gen.c2_regex_and_motifs(1)
    ref = Ref(rx)
    x, rej = gen.c2_texts(1, n=1 << 24, motifs=motifs)
    rec = ri.Recognizer(rx)
    try:
        t = dev(x)
        for algo in ("rid", "dfa"):
            tun = rec.autotune(t, algo=algo)
            assert tun["trials"] >= 6 and tun["best_ms"] > 0
            for text in (x, rej):
                got = rec.recognize(dev(text), algo=algo)
                assert (got["accept"], got["final_state"]) == ref.serial(text)
        rec.set_option("warmup_bytes", 32)     # explicit options drop the tuned setting
        got = rec.recognize(t, algo="rid")
        assert (got["accept"], got["final_state"]) == ref.serial(x)
    finally:
        rec.close()


def test_autotune_skips_settings_the_automaton_does_not_support():
    """An interface wider than the plain reach's join (more than 2048 starts)
    makes those trials RI_ERR_LIMIT: the autotuner skips them, keeps a
    converging setting and the tuned call stays exact."""
    rx, kws = gen.c5_automaton(11, 3, nkw=300)
    dmin = oracle.min_dfa_of(oracle.trim(oracle.position_nfa(rx)))
    rec = ri.Recognizer(rx)
    try:
        assert rec.info()["interface_states"] > 2048
        rng = gen.PCG(17)
        x = gen.c5_text(rng, kws, 3 << 20, plant=True)
        t = dev(x)
        tun = rec.autotune(t, algo="rid")
        assert tun["converge"] == 1 and tun["trials"] > 0
        got = rec.recognize(t, algo="rid")
        assert (got["accept"], got["final_state"]) == oracle.serial(dmin, x)
    finally:
        rec.close()


def test_side_stream_and_handle_reuse(tiny):
    rec, ref = tiny
    acc, rej = gen.c1_texts(9, n=1 << 18)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ta, tr = dev(acc), dev(rej)
        for _ in range(3):
            for x, t in ((acc, ta), (rej, tr)):
                got = rec.recognize(t, algo="rid", chunks=0, stream=s)
                assert (got["accept"], got["final_state"]) == ref.serial(x)


# ---------------------------------------------------------------------------
# motif union over {A,C,G,T}: 256 MiB
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_motif_union_full_size(seed):
    rx, motifs = gen.c2_regex_and_motifs(seed)
    ref = Ref(rx)
    x, rej = gen.c2_texts(seed, motifs=motifs)
    rec = make(rx, "conv64")
    plain = make(rx, "plain")
    try:
        for text in (x, rej):
            want = ref.serial(text)
            t = dev(text)
            for algo in ("rid", "dfa") + (("subset",) if seed == 0 else ()):
                for chunks in ((0, 1024, 262144) if algo != "subset" else (0,)):
                    got = rec.recognize(t, algo=algo, chunks=chunks)
                    assert (got["accept"], got["final_state"]) == want, (algo, chunks)
            if seed == 0:
                for algo in ("rid", "dfa"):
                    got = plain.recognize(t, algo=algo, chunks=16384)
                    assert (got["accept"], got["final_state"]) == want, ("plain", algo)
            del t
        res = check_maps(rec, ref, x, "rid", 0, sample=6, rng=gen.PCG(seed))
        assert res["chunks"] > 1000
        check_maps(plain, ref, x, "rid", 4096, sample=4, rng=gen.PCG(seed + 9))
    finally:
        rec.close()
        plain.close()
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# the walk of the transformation automaton over the first warm-up bytes
# ---------------------------------------------------------------------------

def _prefix_texts(grammar):
    if grammar == "log":
        x, r1, _ = gen.c3_texts(5, n=1 << 20)
        return gen.c3_regex(), x, r1, 24
    rx, motifs = gen.c2_regex_and_motifs(0)
    x, r1 = gen.c2_texts(5, n=1 << 20, motifs=motifs, mean_gap=512)
    return rx, x, r1, 8


@pytest.mark.parametrize("grammar", ["log", "motif"])
@pytest.mark.parametrize("size", [16, 32, 48, 8320])
def test_prefix_walk_chunk_lengths(grammar, size):
    """The log-lines grammar walks 24 bytes of every chunk in the
    transformation automaton of its 227 starts (then direct merging), the
    motif union 8 bytes of its 88 starts (then hashed merging).  Chunks
    shorter than the walk end it early (and may keep more than 64 runs, which
    takes every start instead); results and sampled chunk maps with the walk
    on and off against the oracle."""
    rx, x, r1, depth = _prefix_texts(grammar)
    ref = Ref(rx)
    for pf in (1, 0):
        rec = make(rx, "conv64")
        rec.set_option("prefix", pf)
        try:
            assert rec.info()["prefix_depth"][0] >= depth
            chunks = -(-len(x) // size)
            for text in (x, r1):
                want = ref.serial(text)
                got = rec.recognize(dev(text), algo="rid", chunks=chunks)
                assert (got["accept"], got["final_state"]) == want, (size, pf)
                assert got["chunk_size"] == size or size == 8320
            check_maps(rec, ref, x, "rid", chunks, sample=8, rng=gen.PCG(size + pf))
        finally:
            rec.close()


@pytest.mark.parametrize("mode,runs", [("conv64", 0), ("conv16", 0), ("conv64", 2), ("conv64", 4), ("plain", 0)])
def test_runs_that_enter_a_sink(mode, runs):
    """Expressions with a sink (a state that every byte maps back to itself,
    like the state after a match of .*(...).*): converging runs stop there,
    since their end state is known; results and chunk maps must be the
    oracle's, for texts that reach the sink early, late, in many chunks or
    never, RID and the all-states DFA."""
    rng = gen.PCG(4242)
    for rx, alphabet, never in ((b".*(ab|bca)a.*", b"abc", b"bc"), (b"[ab]*c.*", b"abc", b"ab"),
                                (b"(a|b)*b.*", b"ab", b"a")):
        ref = Ref(rx)
        rec = make(rx, mode, runs_per_lane=runs)
        try:
            texts = [gen.random_text(rng, alphabet, 200001), gen.random_text(rng, never, 70001)]
            late = gen.random_text(rng, never, 150001)
            late[-3:] = np.frombuffer(alphabet[-1:] * 3, np.uint8) if rx != b".*(ab|bca)a.*" else \
                np.frombuffer(b"aba", np.uint8)
            texts.append(late)
            for x in texts:
                want = ref.serial(x)
                for algo in ("rid", "dfa"):
                    for chunks in (1, 7, 1000, 0):
                        got = rec.recognize(dev(x), algo=algo, chunks=chunks)
                        assert (got["accept"], got["final_state"]) == want, (rx, mode, runs, algo, chunks)
            check_maps(rec, ref, texts[0], "rid", 1000, sample=10, rng=gen.PCG(7))
            check_maps(rec, ref, texts[0], "dfa", 1000, sample=10, rng=gen.PCG(8))
        finally:
            rec.close()


def _counter_text(seed, n_runs):
    """Runs of 1..100 a's, each closed by b (in the language (a{1,100}b)*),
    and a copy with one run of 101 a's (rejected)."""
    rng = gen.PCG(seed)
    lens = rng.integers(1, 101, size=n_runs)
    parts = [b"a" * int(k) + b"b" for k in lens]
    x = np.frombuffer(b"".join(parts), dtype=np.uint8)
    j = n_runs // 2
    bad = np.frombuffer(b"".join(parts[:j] + [b"a" * 101 + b"b"] + parts[j + 1:]), dtype=np.uint8)
    return x, bad


@pytest.mark.parametrize("mode", ["conv64", "conv80", "conv128", "conv256"])
@pytest.mark.parametrize("size", [160, 1024, 4096])
def test_prefix_walk_many_live_runs(mode, size):
    """(a{1,100}b)*: 101 starts, a walk of 64 bytes.  A chunk that begins
    inside a long run of a's keeps one live run per count that has not yet
    overflowed (more than 32 after the walk), a chunk that meets a b early
    keeps one or two: with warm-ups beyond the walk, chunks of both kinds sit
    side by side in the waves of the warm-up tail.  Results and sampled chunk
    maps against the oracle."""
    rx = b"(a{1,100}b)*"
    ref = Ref(rx)
    x, bad = _counter_text(11 + size, 6000)
    rec = make(rx, mode)
    try:
        info = rec.info()
        assert info["interface_states"] == 101 and info["prefix_depth"][0] >= 64
        chunks = -(-len(x) // size)
        for text in (x, bad):
            want = ref.serial(text)
            assert want[0] == (text is x)
            got = rec.recognize(dev(text), algo="rid", chunks=chunks)
            assert (got["accept"], got["final_state"]) == want, (mode, size)
            got = rec.recognize(dev(text), algo="dfa", chunks=chunks)
            assert (got["accept"], got["final_state"]) == want, (mode, size, "dfa")
        check_maps(rec, ref, x, "rid", chunks, sample=12, rng=gen.PCG(size))
    finally:
        rec.close()


# ---------------------------------------------------------------------------
# log lines: 1 GiB
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_log_lines_full_size(seed):
    """The 1 GiB log-lines text and its two rejected copies: synchronous
    calls (RID, all-states DFA; tuned and fixed chunk counts), the queued
    call (the path the benchmark times) and the plain reach, against the
    oracle's serial result; chunk maps sampled against the oracle's runs."""
    rx = gen.c3_regex()
    ref = Ref(rx)
    x, r1, r2 = gen.c3_texts(seed)
    assert len(x) > (1 << 30) - 4096
    rec = make(rx, "conv64")
    plain = make(rx, "plain")
    try:
        res = torch.full((6, 2), -7, dtype=torch.int32, device="cuda")
        wants = []
        for j, text in enumerate((x, r1, r2)):
            want = ref.serial(text)
            wants.append(want)
            t = dev(text)
            for algo in ("rid", "dfa"):
                for chunks in ((0, 262144) if j == 0 else (0,)):
                    got = rec.recognize(t, algo=algo, chunks=chunks)
                    assert (got["accept"], got["final_state"]) == want, (seed, j, algo, chunks)
                rec.recognize_async(t, res[2 * j + (algo == "dfa")], algo=algo)
            if j != 1:
                got = plain.recognize(t, algo="rid", chunks=65536)
                assert (got["accept"], got["final_state"]) == want, (seed, j, "plain")
            if seed == 0:
                rec.set_option("prefix", 0)
                got = rec.recognize(t, algo="rid")
                rec.set_option("prefix", 1)
                assert (got["accept"], got["final_state"]) == want, (seed, j, "no prefix walk")
            torch.cuda.synchronize()
            del t
        got = res.cpu().numpy()
        for j, want in enumerate(wants):
            for a in range(2):
                assert (bool(got[2 * j + a][0]), int(got[2 * j + a][1])) == want, (seed, j, a, "queued")
        if seed == 0:
            check_maps(rec, ref, x, "rid", 0, sample=4, rng=gen.PCG(1))
            check_maps(rec, ref, x, "dfa", 0, sample=4, rng=gen.PCG(2))
    finally:
        rec.close()
        plain.close()
    torch.cuda.empty_cache()


def test_text_beyond_4_gib():
    """17 copies of a 256 MiB log-lines text: 4.25 GiB, so chunk offsets run
    past 32 bits.  The whole text, the text with its last 9 bytes cut, and
    the text whose last copy is a rejected one; RID and the all-states DFA,
    synchronous and queued, automatic chunk counts.  The expected result is
    the serial run of the minimal DFA over the concatenation, carried copy by
    copy (the end state of one copy is the start of the next)."""
    rx = gen.c3_regex()
    ref = Ref(rx)
    base, bad, _ = gen.c3_texts(6, n=1 << 28)
    assert len(bad) == len(base)
    copies, nb = 17, len(base)
    n = copies * nb
    assert n > (1 << 32)

    def carry(s, x, end):
        return oracle.run(ref.tdfa, s, x, 0, end)[0] if s >= 0 else -1

    after = {}
    s = 0
    for _ in range(copies - 1):
        if s not in after:
            after[s] = carry(s, base, nb)
        s = after[s]
    ends = {"whole": carry(s, base, nb), "cut": carry(s, base, nb - 9), "bad": carry(s, bad, nb)}
    wants = {k: (e >= 0 and e in ref.b.dfa.final, e) for k, e in ends.items()}
    assert wants["whole"][0] and not wants["bad"][0]

    t = torch.empty(n, dtype=torch.uint8, device="cuda")
    bd = dev(base)
    for i in range(copies):
        t[i * nb:(i + 1) * nb].copy_(bd)
    del bd
    rec = make(rx, "conv64")
    res = torch.full((6, 2), -7, dtype=torch.int32, device="cuda")
    try:
        for j, case in enumerate(("whole", "cut", "bad")):
            if case == "bad":
                t[(copies - 1) * nb:].copy_(dev(bad))
            text = t[: n - 9] if case == "cut" else t
            for a, algo in enumerate(("rid", "dfa")):
                got = rec.recognize(text, algo=algo)
                assert (got["accept"], got["final_state"]) == wants[case], (case, algo)
                assert got["n"] == len(text)
                rec.recognize_async(text, res[2 * j + a], algo=algo)
            torch.cuda.synchronize()
        got = res.cpu().numpy()
        for j, case in enumerate(("whole", "cut", "bad")):
            for a in range(2):
                assert (bool(got[2 * j + a][0]), int(got[2 * j + a][1])) == wants[case], (case, a, "queued")
    finally:
        rec.close()
        del t
        torch.cuda.empty_cache()


def test_ri_recognize_entry_point_on_a_side_stream():
    """ri_recognize itself (RID, automatic chunk count), called through the
    C ABI on a non-default stream, on the tiny and log-lines expressions."""
    s = torch.cuda.Stream()
    for rx, texts in ((gen.c1_regex(), gen.c1_texts(4)), (gen.c3_regex(), gen.c3_texts(3, n=1 << 24)[:3])):
        ref = Ref(rx)
        h = ri.binding.ri_build(rx)
        try:
            with torch.cuda.stream(s):
                for x in texts:
                    t = dev(x)
                    got = ri.binding.ri_recognize(h, t, stream=s)
                    assert (got["accept"], got["final_state"]) == ref.serial(x)
                    assert got["n"] == len(x) and got["chunks"] >= 1
        finally:
            ri.binding.ri_free(h)
