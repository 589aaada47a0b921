"""ri_recognize_noalloc (fixed scratch array, no allocation) against the
queued entry point it varies, ri_recognize_async, on the same inputs: two
calls in a row, the second with a smaller input, every algorithm; and
against the oracle's serial result."""

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


def serial_ref(pattern):
    d = oracle.min_dfa_of(oracle.trim(oracle.position_nfa(pattern)))
    table = oracle.dense_table(d.n, d.delta)
    return lambda x: oracle.serial(d, x, table)


def both(rec, t, algo, chunks=0):
    """(no-alloc result, async result) for one text, on the current stream."""
    a = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    b = torch.full((2,), -7, dtype=torch.int32, device="cuda")
    ri.binding.ri_recognize_noalloc(rec.handle, t, a, algo=algo, chunks=chunks)
    rec.recognize_async(t, b, algo=algo, chunks=chunks)
    torch.cuda.synchronize()
    ga, gb = a.cpu().numpy(), b.cpu().numpy()
    return (bool(ga[0]), int(ga[1])), (bool(gb[0]), int(gb[1]))


@pytest.mark.parametrize("pattern,alphabet", [(gen.c1_regex(), b"ab"), (b"((b*a){9})*b*", b"ab"),
                                              (b"(ab|b)*a?", b"ab")])
def test_two_calls_second_smaller(pattern, alphabet):
    ref = serial_ref(pattern)
    rec = ri.Recognizer(pattern)
    try:
        rng = gen.PCG(99)
        big = gen.random_text(rng, alphabet, 3 << 20)
        small = gen.random_text(rng, alphabet, 70001)
        rec.recognize(dev(small[:64]))            # puts the tables on the device
        for algo in ("rid", "dfa", "subset"):
            for x in (big, small):
                got, want = both(rec, dev(x), algo)
                assert got == want == ref(x), (pattern, algo, len(x))
            for x in (big, small):                # explicit chunk counts that fit
                got, want = both(rec, dev(x), algo, chunks=1000)
                assert got == want == ref(x), (pattern, algo, len(x), 1000)
    finally:
        rec.close()


def test_log_lines_fit_by_fewer_chunks():
    """16 MiB and then 1 MiB of log lines (interface of 227 starts): the
    automatic chunk count is lowered until the call fits the array."""
    rx = gen.c3_regex()
    ref = serial_ref(rx)
    rec = ri.Recognizer(rx)
    try:
        x, r1, r2 = gen.c3_texts(5, n=16 << 20)
        rec.recognize(dev(x[:4096]))
        for text in (x, r2, x[: 1 << 20]):
            for algo in ("rid", "dfa"):
                got, want = both(rec, dev(text), algo)
                assert got == want == ref(text), (algo, len(text))
    finally:
        rec.close()


def test_errors():
    rx = gen.c3_regex()
    x = gen.c3_texts(2, n=16 << 20)[0]
    rec = ri.Recognizer(rx)
    try:
        t = dev(x)
        res = torch.zeros(2, dtype=torch.int32, device="cuda")
        with pytest.raises(ri.RIError) as e:       # tables not on the device yet
            ri.binding.ri_recognize_noalloc(rec.handle, t, res)
        assert e.value.code == ri.binding.RI_ERR_ARG
        rec.recognize(t[:4096])
        with pytest.raises(ri.RIError) as e:       # 2^20 chunks x 227 starts: beyond the array
            ri.binding.ri_recognize_noalloc(rec.handle, t, res, chunks=1 << 20)
        assert e.value.code == ri.binding.RI_ERR_LIMIT
        assert "fixed scratch" in str(e.value)
        ri.binding.ri_recognize_noalloc(rec.handle, t, res)   # still usable afterwards
        torch.cuda.synchronize()
        assert (bool(res[0]), int(res[1])) == serial_ref(rx)(x)
    finally:
        rec.close()
