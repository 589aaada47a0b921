"""Host-side checks of the C ABI (no GPU needed).

* libri.so loads and exports every function include/ri.h declares;
* ri_build's error handling (parse errors with offsets, state caps, bad args);
* the host constructor agrees with the oracle: automaton sizes, and the
  RI-DFA B' = RI-DFA(N') as a set of contents (sets of N' states), which are
  unique for the expression (state ids are construction-order dependent).
"""

import ctypes
import os
import re

import pytest

import oracle
from workloads import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ri.h")

ri = pytest.importorskip("paper_2412_14975_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ri_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(ri.binding.LIB_PATH)
    names = declared_functions()
    assert "ri_build" in names and "ri_recognize" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ri.binding.SYMBOLS)


@pytest.mark.parametrize("bad,offset", [(b"(ab", 3), (b"ab)", 2), (b"*a", 0), (b"a{3,1}", 1),
                                        (b"[ab", 0), (b"a\\x4", 1)])
def test_parse_errors_report_offset(bad, offset):
    with pytest.raises(ri.RIError) as e:
        ri.ri_build(bad)
    assert e.value.code == ri.binding.RI_ERR_PARSE
    assert f"offset {offset}" in str(e.value)


def test_state_cap_gives_limit_error():
    with pytest.raises(ri.RIError) as e:
        ri.ri_build(gen.regexp_family(10), max_states=100)
    assert e.value.code == ri.binding.RI_ERR_LIMIT


def test_null_and_bad_arguments():
    lib = ri.binding.lib()
    h = ctypes.c_void_p()
    assert lib.ri_build(None, 0, None, ctypes.byref(h)) == ri.binding.RI_ERR_ARG
    opts = ri.binding.ri_build_opts(0, 7)
    assert lib.ri_build(b"a", 1, ctypes.byref(opts), ctypes.byref(h)) == ri.binding.RI_ERR_ARG
    assert lib.ri_info(None, None) == ri.binding.RI_ERR_ARG
    r = ri.binding.ri_result()
    hh = ri.ri_build(b"a")
    try:
        assert lib.ri_recognize_ex(hh, None, 16, None, 0, 0, ctypes.byref(r)) == ri.binding.RI_ERR_ARG
        assert lib.ri_recognize_ex(hh, None, 0, None, 7, 0, ctypes.byref(r)) == ri.binding.RI_ERR_ARG
        # n = 0 is decided on the host: "a" does not contain the empty text
        assert lib.ri_recognize_ex(hh, None, 0, None, 0, 0, ctypes.byref(r)) == 0
        assert (r.accept, r.final_state) == (0, 0)
    finally:
        ri.ri_free(hh)
    ri.ri_free(None)


def test_batch_argument_checks_before_any_device_call():
    """ri_batch_create validates every request on the host and returns
    RI_ERR_ARG before touching a device."""
    lib = ri.binding.lib()
    Req = ri.binding.ri_request
    out = ctypes.c_void_p()
    hh = ri.ri_build(b"ab*")
    try:
        def create(reqs, chunk_bytes=0):
            arr = (Req * max(1, len(reqs)))(*reqs)
            return lib.ri_batch_create(arr, len(reqs), chunk_bytes, ctypes.byref(out))
        assert create([Req(None, 0x1000, 16, 0, 0)]) == ri.binding.RI_ERR_ARG       # NULL handle
        assert create([Req(hh, 0x1000, 16, 9, 0)]) == ri.binding.RI_ERR_ARG         # bad algo
        assert create([Req(hh, 0x1000, 16, 0, 1)]) == ri.binding.RI_ERR_ARG         # reserved
        assert create([Req(hh, None, 16, 0, 0)]) == ri.binding.RI_ERR_ARG           # NULL text, n > 0
        assert create([Req(hh, 0x1001, 16, 0, 0)]) == ri.binding.RI_ERR_ARG         # misaligned
        assert create([Req(hh, 0x1000, 16, 0, 0)], chunk_bytes=24) == ri.binding.RI_ERR_ARG
        assert "16-byte" in ri.ri_last_error() or "multiple of 16" in ri.ri_last_error()
        assert lib.ri_batch_create(None, 1, 0, ctypes.byref(out)) == ri.binding.RI_ERR_ARG
        assert lib.ri_batch_run(None, None, None) == ri.binding.RI_ERR_ARG
        assert lib.ri_batch_launch(None, None) == ri.binding.RI_ERR_ARG
        assert lib.ri_batch_get_info(None, None) == ri.binding.RI_ERR_ARG
        lib.ri_batch_free(None)
    finally:
        ri.ri_free(hh)


def test_request_footprint_is_host_only_and_grows_with_the_text():
    hh = ri.ri_build(gen.c5_automaton(3, 0, 20)[0])
    try:
        f = [ri.ri_request_footprint(hh, algo, n) for algo in ("rid", "dfa") for n in (0, 100, 1 << 16, 1 << 24)]
        assert all(v > 0 for v in f)
        assert f[0] < f[1] < f[2] < f[3] and f[4] < f[5] < f[6] < f[7]
        assert f[3] >= 1 << 24
        lib = ri.binding.lib()
        v = ctypes.c_uint64()
        assert lib.ri_request_footprint(None, 0, 10, 0, ctypes.byref(v)) == ri.binding.RI_ERR_ARG
        assert lib.ri_request_footprint(hh, 9, 10, 0, ctypes.byref(v)) == ri.binding.RI_ERR_ARG
        assert lib.ri_request_footprint(hh, 0, 10, 24, ctypes.byref(v)) == ri.binding.RI_ERR_ARG
        assert lib.ri_batch_update(None, None, 0) == ri.binding.RI_ERR_ARG
    finally:
        ri.ri_free(hh)


def _compare_with_oracle(pattern):
    ref = oracle.build(pattern)
    h = ri.ri_build(pattern)
    try:
        info = ri.ri_info(h)
        assert info["nfa_states"] == ref.nfa.n
        if ref.nfa.n == 0:
            return
        assert info["interface_states"] == ref.nfa_q.n == len(ref.red.kept)
        assert info["ridfa_full_states"] == ref.B.n
        assert info["ridfa_states"] == ref.Bq.n
        assert info["min_dfa_states"] == ref.dfa.n
        assert info["subset_dfa_states"] == oracle.subset_dfa(ref.nfa)[0].n
        assert info["accepts_empty"] == (0 in ref.dfa.final)
        assert info["starts"] == [ref.nfa_q.n, ref.dfa.n, info["subset_dfa_states"], ref.nfa.n]
        got = {frozenset(ri.ri_state_content(h, "rid", p)) for p in range(info["ridfa_states"])}
        assert got == set(ref.Bq.content)
    finally:
        ri.ri_free(h)


@pytest.mark.parametrize("pattern", [
    gen.c1_regex(), gen.regexp_family(6), gen.c3_regex(), gen.c2_regex_and_motifs(0)[0],
    gen.c2_regex_and_motifs(2)[0], b"b*a(ab*a|b+a)*", b"()", b"a[^\\x00-\\xff]", b"(ab|a)*b{1,}",
])
def test_constructor_matches_oracle(pattern):
    _compare_with_oracle(pattern)


@pytest.mark.parametrize("seed", range(40))
def test_constructor_matches_oracle_random(seed):
    rng = gen.PCG(31000 + seed)
    while True:
        p = gen.random_regex(rng, b"abc"[: 2 + seed % 2], int(rng.integers(1, 4)))
        if oracle.position_nfa(p).n <= 40:
            break
    _compare_with_oracle(p)
