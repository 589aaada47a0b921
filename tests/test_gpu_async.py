"""GPU parity of ri_recognize_async (include/ri.h): calls enqueued back to
back on one stream, each writing its [accept, final_state] to its own slot
of a device array, give exactly the oracle's serial results, across every
reach/join pipeline, the three chunk automata, texts that grow from call to
call (scratch reallocated between queued calls), the hit-matrix join's
fallback (more runs per chunk than a row holds), the empty text and the
empty language.
"""

import numpy as np
import pytest

import oracle
from workloads import gen

torch = pytest.importorskip("torch")
ri = pytest.importorskip("paper_2412_14975_amd")

pytestmark = pytest.mark.gpu

ALGOS = ("rid", "dfa", "subset")
MODES = {"conv64": dict(converge=1, warmup_bytes=64), "conv16": dict(converge=1, warmup_bytes=16),
         "cls64": dict(converge=1, warmup_bytes=64, join=1), "plain": dict(converge=0),
         "conv80": dict(converge=1, warmup_bytes=80), "conv128": dict(converge=1, warmup_bytes=128),
         "conv256": dict(converge=1, warmup_bytes=256),
         # every start stepping from the first byte (no transformation-automaton walk)
         "noprefix64": dict(converge=1, warmup_bytes=64, prefix=0)}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ri.binding.lib()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint8)).to("cuda")


def serial_ref(pattern):
    d = oracle.min_dfa_of(oracle.trim(oracle.position_nfa(pattern)))
    table = oracle.dense_table(d.n, d.delta)
    return lambda x: oracle.serial(d, x, table)


def run_queue(rec, items, stream=None):
    """items: (text tensor, algo, chunks); one async call each, then one wait."""
    res = torch.full((len(items), 2), -7, dtype=torch.int32, device="cuda")
    for i, (t, algo, chunks) in enumerate(items):
        rec.recognize_async(t, res[i], algo=algo, chunks=chunks, stream=stream)
    torch.cuda.synchronize()
    return [(bool(a), int(f)) for a, f in res.cpu().numpy()]


@pytest.mark.parametrize("mode", sorted(MODES))
def test_queued_calls_match_the_oracle(mode):
    pats = [gen.c1_regex(), b"((b*a){9})*b*", b"(ab|b)*a?"]
    rng = gen.PCG(808)
    for p in pats:
        ref = serial_ref(p)
        rec = ri.Recognizer(p)
        try:
            for k, v in MODES[mode].items():
                rec.set_option(k, v)
            xs = []
            for i, n in enumerate((1, 17, 4096, 70001, 300007, 1 << 20, 33)):   # growing, then small
                x = gen.random_text(rng, b"ab", n)
                if p == gen.c1_regex() and n >= 4 and i % 2 == 0:
                    x[-4:] = np.frombuffer(b"abab", np.uint8)
                xs.append(x)
            ts = [dev(x) for x in xs]
            items = [(t, ALGOS[i % 3], (0, 64, 5)[i % 3]) for i, t in enumerate(ts)]
            items += [(t, "rid", 0) for t in ts]
            got = run_queue(rec, items)
            want = [ref(x) for x in xs] * 2
            assert got == want, (p, mode)
        finally:
            rec.close()


@pytest.mark.parametrize("k", [8, 9, 16])
def test_hit_join_fallback_on_the_device(k):
    """Counting a's modulo k keeps k runs per chunk: above 8 the hit-matrix
    result is invalid and the queued call redoes the join on the device (the
    class join, one launch gated on the hit join's flag), with no host
    decision."""
    rx = b"((b*a){%d})*b*" % k
    ref = serial_ref(rx)
    rec = ri.Recognizer(rx)
    try:
        rec.set_option("warmup_bytes", 16)
        rng = gen.PCG(900 + k)
        xs = []
        for n in (5000, 300001):
            for accept in (False, True):
                x = gen.random_text(rng, b"ab", n)
                if accept:
                    need = (-int((x == ord("a")).sum())) % k
                    x[np.flatnonzero(x == ord("b"))[:need]] = ord("a")
                xs.append(x)
        ts = [dev(x) for x in xs]
        items = [(t, "rid", c) for t in ts for c in (1, 2, 64, 0)]
        got = run_queue(rec, items)
        want = [ref(x) for x in xs for _ in (1, 2, 64, 0)]
        assert got == want
        assert any(a for a, _ in want) and not all(a for a, _ in want)
    finally:
        rec.close()


def test_hit_join_fallback_with_a_three_level_class_join():
    """As above with k = 9 on 4 MiB: 8192 and about 16 384 chunks give the
    gated class join three levels -- level 0 inside the hit join's first
    launch, the others with the hit join's last level -- and it must still
    replace the invalid hit result; a call with k = 2 (valid hit result)
    queued in between must keep its own."""
    rx9, rx2 = b"((b*a){9})*b*", b"((b*a){2})*b*"
    ref9, ref2 = serial_ref(rx9), serial_ref(rx2)
    r9, r2 = ri.Recognizer(rx9), ri.Recognizer(rx2)
    try:
        rng = gen.PCG(931)
        xs = []
        for accept in (False, True):
            x = gen.random_text(rng, b"ab", (1 << 22) + 5)
            if accept:
                need = (-int((x == ord("a")).sum())) % 9
                x[np.flatnonzero(x == ord("b"))[:need]] = ord("a")
            xs.append(x)
        ts = [dev(x) for x in xs]
        stream = torch.cuda.Stream()
        res = torch.full((8, 2), -7, dtype=torch.int32, device="cuda")
        want = []
        i = 0
        for t, x in zip(ts, xs):
            for chunks in (8192, 0):
                r9.recognize_async(t, res[i], algo="rid", chunks=chunks, stream=stream)
                want.append(ref9(x))
                r2.recognize_async(t, res[i + 1], algo="rid", chunks=chunks, stream=stream)
                want.append(ref2(x))
                i += 2
        stream.synchronize()
        got = [(bool(a), int(f)) for a, f in res.cpu().numpy()]
        assert got == want
        assert want[4][0] and not want[0][0]
    finally:
        r9.close()
        r2.close()


def test_empty_text_and_empty_language_side_stream():
    s = torch.cuda.Stream()
    e = ri.Recognizer(b"a[^\\x00-\\xff]")
    eps = ri.Recognizer(b"()")
    star = ri.Recognizer(b"ab*")
    try:
        with torch.cuda.stream(s):
            x = dev(np.frombuffer(b"a" * 100, dtype=np.uint8))
            empty = torch.empty(0, dtype=torch.uint8, device="cuda")
            abb = dev(np.frombuffer(b"abbbbbbbbb" * 7, dtype=np.uint8)[:61])
            res = torch.full((5, 2), -7, dtype=torch.int32, device="cuda")
            e.recognize_async(x, res[0], stream=s)
            eps.recognize_async(empty, res[1], stream=s)
            eps.recognize_async(x, res[2], algo="dfa", stream=s)
            star.recognize_async(empty, res[3], stream=s)
            star.recognize_async(abb, res[4], algo="subset", stream=s)
        s.synchronize()
        got = [(bool(a), int(f)) for a, f in res.cpu().numpy()]
        assert got[:4] == [(False, -1), (True, 0), (False, -1), (False, 0)]
        assert got[4] == serial_ref(b"ab*")(np.frombuffer(b"abbbbbbbbb" * 7, dtype=np.uint8)[:61])
    finally:
        for r in (e, eps, star):
            r.close()


def test_async_argument_errors():
    rec = ri.Recognizer(b"ab*")
    try:
        t = dev(np.frombuffer(b"ab" * 40, dtype=np.uint8))
        with pytest.raises(TypeError):
            rec.recognize_async(t, torch.zeros(2, dtype=torch.int64, device="cuda"))
        with pytest.raises(TypeError):
            rec.recognize_async(t, torch.zeros(1, dtype=torch.int32, device="cuda"))
        raw = torch.zeros(8, dtype=torch.int32, device="cuda")
        lib = ri.binding.lib()
        rc = lib.ri_recognize_async(rec.handle, t.data_ptr(), t.numel(), None, 0, 0, raw.data_ptr() + 2)
        assert rc == ri.binding.RI_ERR_ARG
        rc = lib.ri_recognize_async(rec.handle, t.data_ptr(), t.numel(), None, 0, 0, None)
        assert rc == ri.binding.RI_ERR_ARG
        torch.cuda.synchronize()
        assert raw.abs().sum().item() == 0      # nothing was written by a refused call
    finally:
        rec.close()
