"""Seeded generators for the regular expressions and texts of the workloads.

Every generator takes an integer seed and draws from
``numpy.random.Generator(PCG64(seed))``, so that a (workload, seed) pair
names one exact byte string on every machine with the same numpy.

Workloads (sizes are the full ones; callers may pass smaller sizes):

* regexp family ``(a|b)*a(a|b)^k``: the paper's synthetic *regexp*
  benchmark, whose minimal DFA grows as 2^(k+1) states (Sect. 4.1, Tab. 1).
* tiny (k = 3): 1 MiB of i.i.d. uniform {a,b} whose last four symbols are
  forced to ``abab`` (accepted), plus a copy whose fourth-from-last byte is
  ``b`` (rejected).  Stands in for the paper's *regexp* texts.
* motif union over {A,C,G,T}: 256 MiB of uniform bases with motif instances
  planted at exponential gaps of mean 4 KiB.  Stands in for *fasta*.
* log lines: about 1 GiB of syslog-like lines sampled from the expression.
  Stands in for *traffic*.

None of the paper's datasets is reproduced; the texts only share the shape
(alphabet, automaton size, text length) of those workloads.
"""

from __future__ import annotations

import numpy as np

ACGT = b"ACGT"


def PCG(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# ---------------------------------------------------------------------------
# regexp family and the tiny workload
# ---------------------------------------------------------------------------

def regexp_family(k: int) -> bytes:
    """``(a|b)*a(a|b)^k`` written out with k explicit copies."""
    return b"(a|b)*a" + b"(a|b)" * int(k)


def c1_regex() -> bytes:
    return regexp_family(3)


def c1_texts(seed: int, n: int = 1 << 20):
    """Return (accepted, rejected) uint8 texts of length n (n >= 4)."""
    if n < 4:
        raise ValueError("n must be >= 4")
    rng = PCG(seed)
    t = np.frombuffer(b"ab", dtype=np.uint8)[rng.integers(0, 2, size=n)]
    t = np.ascontiguousarray(t)
    t[n - 4:] = np.frombuffer(b"abab", dtype=np.uint8)
    r = t.copy()
    r[n - 4] = ord("b")
    return t, r


# ---------------------------------------------------------------------------
# motif union over {A,C,G,T}
# ---------------------------------------------------------------------------

def _motif(rng: np.random.Generator):
    """One motif: a list of positions, each ('base', b) | ('class', bytes) | ('rep',)."""
    npos = int(rng.integers(6, 13))
    out = []
    for _ in range(npos):
        u = rng.random()
        if u < 0.6:
            out.append(("base", ACGT[int(rng.integers(0, 4))]))
        elif u < 0.9:
            k = int(rng.integers(2, 4))
            idx = np.sort(rng.choice(4, size=k, replace=False))
            out.append(("class", bytes(ACGT[i] for i in idx)))
        else:
            out.append(("rep",))
    return out


def _motif_regex(m) -> bytes:
    parts = []
    for p in m:
        if p[0] == "base":
            parts.append(bytes([p[1]]))
        elif p[0] == "class":
            parts.append(b"[" + p[1] + b"]")
        else:
            parts.append(b"[ACGT]{1,3}")
    return b"".join(parts)


def c2_regex_and_motifs(seed: int, nmotifs: int = 8):
    """Return (regex, motifs) for ``([ACGT]*(m1|...|m8))*[ACGT]*``."""
    rng = PCG(seed)
    motifs = [_motif(rng) for _ in range(nmotifs)]
    body = b"|".join(_motif_regex(m) for m in motifs)
    return b"([ACGT]*(" + body + b"))*[ACGT]*", motifs


def _motif_instance(rng: np.random.Generator, m) -> bytes:
    out = bytearray()
    for p in m:
        if p[0] == "base":
            out.append(p[1])
        elif p[0] == "class":
            out.append(p[1][int(rng.integers(0, len(p[1])))])
        else:
            for _ in range(int(rng.integers(1, 4))):
                out.append(ACGT[int(rng.integers(0, 4))])
    return bytes(out)


def c2_texts(seed: int, n: int = 1 << 28, motifs=None, mean_gap: int = 4096):
    """Return (text, rejected): uniform bases with planted motif instances;
    the second copy has one byte replaced by ``N`` (outside the alphabet)."""
    if motifs is None:
        motifs = c2_regex_and_motifs(seed)[1]
    rng = PCG(seed + 1_000_003)
    t = np.frombuffer(ACGT, dtype=np.uint8)[rng.integers(0, 4, size=n, dtype=np.int8)]
    t = np.ascontiguousarray(t)
    pos = 0
    while True:
        pos += int(rng.exponential(mean_gap)) + 1
        if pos >= n:
            break
        inst = _motif_instance(rng, motifs[int(rng.integers(0, len(motifs)))])
        end = min(n, pos + len(inst))
        t[pos:end] = np.frombuffer(inst[: end - pos], dtype=np.uint8)
        pos = end
    r = t.copy()
    r[int(rng.integers(0, n))] = ord("N")
    return t, r


# ---------------------------------------------------------------------------
# log lines over the byte alphabet
# ---------------------------------------------------------------------------

def c3_regex() -> bytes:
    d = b"[0-9]"
    ts = d + b"{4}-" + d + b"{2}-" + d + b"{2} " + d + b"{2}:" + d + b"{2}:" + d + b"{2}"
    octet = d + b"{1,3}"
    ip = octet + b"\\." + octet + b"\\." + octet + b"\\." + octet
    level = b"(INFO|WARN|ERROR|DEBUG)"
    field = b"[a-z]{1,12}=[0-9A-Za-z]{1,16}"
    line = ts + b" " + ip + b" " + level + b" (" + field + b"){1,6}"
    return b"(" + line + b"\\n)*"


_DIG = np.frombuffer(b"0123456789", dtype=np.uint8)
_LOW = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz", dtype=np.uint8)
_ALNUM = np.frombuffer(b"0123456789ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz",
                       dtype=np.uint8)
_LEVELS = [b"INFO", b"WARN", b"ERROR", b"DEBUG"]

# segment kinds
_K_DIG, _K_LOW, _K_ALNUM, _K_LIT = 0, 1, 2, 3


def _c3_batch(rng: np.random.Generator, nlines: int) -> np.ndarray:
    """Generate ``nlines`` whole log lines as one uint8 array."""
    B = nlines
    ipl = rng.integers(1, 4, size=(B, 4))
    lvl = rng.integers(0, 4, size=B)
    nf = rng.integers(1, 7, size=B)
    kl = rng.integers(1, 13, size=(B, 6))
    vl = rng.integers(1, 17, size=(B, 6))
    fmask = np.arange(6)[None, :] < nf[:, None]
    kl = np.where(fmask, kl, 0)
    vl = np.where(fmask, vl, 0)
    eq = fmask.astype(np.int64)

    # segments per line: (kind, length, literal byte or -1)
    segs_len = []
    segs_kind = []
    segs_lit = []

    def add(kind, length, lit=0):
        segs_kind.append(np.full(B, kind, dtype=np.int64) if np.isscalar(kind) else kind)
        segs_len.append(np.broadcast_to(np.asarray(length, dtype=np.int64), (B,)).copy())
        segs_lit.append(np.broadcast_to(np.asarray(lit, dtype=np.int64), (B,)).copy())

    for i, L in enumerate((4, 2, 2, 2, 2, 2)):
        add(_K_DIG, L)
        if i < 5:
            add(_K_LIT, 1, ord(b"-- ::"[i:i + 1]))
    add(_K_LIT, 1, ord(" "))
    for o in range(4):
        add(_K_DIG, ipl[:, o])
        if o < 3:
            add(_K_LIT, 1, ord("."))
    add(_K_LIT, 1, ord(" "))
    # level: up to 5 literal bytes
    lvl_tab = np.zeros((4, 5), dtype=np.int64)
    lvl_len = np.zeros(4, dtype=np.int64)
    for j, s in enumerate(_LEVELS):
        lvl_tab[j, : len(s)] = np.frombuffer(s, dtype=np.uint8)
        lvl_len[j] = len(s)
    for c in range(5):
        add(_K_LIT, (lvl_len[lvl] > c).astype(np.int64), lvl_tab[lvl, c])
    add(_K_LIT, 1, ord(" "))
    for f in range(6):
        add(_K_LOW, kl[:, f])
        add(_K_LIT, eq[:, f], ord("="))
        add(_K_ALNUM, vl[:, f])
    add(_K_LIT, 1, ord("\n"))

    kind = np.stack(segs_kind, axis=1).ravel().astype(np.uint8)
    length = np.stack(segs_len, axis=1).ravel()
    lit = np.stack(segs_lit, axis=1).ravel().astype(np.uint8)
    bkind = np.repeat(kind, length)
    out = np.repeat(lit, length)          # literal bytes in place
    for k, alpha in ((_K_DIG, _DIG), (_K_LOW, _LOW), (_K_ALNUM, _ALNUM)):
        idx = np.flatnonzero(bkind == k)
        out[idx] = alpha[rng.integers(0, len(alpha), size=len(idx), dtype=np.uint8)]
    return out


def c3_texts(seed: int, n: int = 1 << 30, batch_lines: int = 1 << 17, workers: int = 0):
    """Return (text, rejected_random, rejected_guaranteed).

    ``text`` is whole lines only, at most ``n`` bytes.  ``rejected_random``
    has one byte replaced by a different random byte (it may still be in the
    language); ``rejected_guaranteed`` has the same byte replaced by 0x01.

    Batch i of ``batch_lines`` lines draws from the i-th child of
    ``SeedSequence(seed)``, so the bytes do not depend on ``workers`` (the
    number of threads generating batches concurrently; 0 = all cores, at
    most 16).
    """
    import os
    from concurrent.futures import ThreadPoolExecutor

    if workers <= 0:
        workers = max(1, min(16, os.cpu_count() or 1))
    children = np.random.SeedSequence(int(seed)).spawn(1 << 14)
    pieces = []
    have = 0
    nxt = 0
    with ThreadPoolExecutor(max_workers=workers) as pool:
        while have < n:
            if nxt + workers > len(children):
                raise ValueError("text too long for the batch schedule")
            rngs = [np.random.Generator(np.random.PCG64(children[nxt + i])) for i in range(workers)]
            nxt += workers
            for b in pool.map(lambda r: _c3_batch(r, batch_lines), rngs):
                if have >= n:
                    break
                room = n - have
                if len(b) > room:
                    nl = np.flatnonzero(b[:room] == ord("\n"))
                    b = b[: int(nl[-1]) + 1] if len(nl) else b[:0]
                    pieces.append(b)
                    have = n
                    break
                pieces.append(b)
                have += len(b)
    t = np.concatenate(pieces) if pieces else np.zeros(0, dtype=np.uint8)
    r1 = t.copy()
    r2 = t.copy()
    if len(t):
        rng2 = PCG(seed + 7_777)
        p = int(rng2.integers(0, len(t)))
        v = int(rng2.integers(0, 255))
        r1[p] = v if v < t[p] else v + 1
        r2[p] = 1
    return t, r1, r2


# ---------------------------------------------------------------------------
# small random expressions and texts (property tests)
# ---------------------------------------------------------------------------

def random_regex(rng: np.random.Generator, alphabet: bytes, depth: int) -> bytes:
    """A random expression in the syntax subset shared with Python's ``re``:
    literals, bracket classes, groups, ``|``, ``*``, ``+``, ``?`` and
    ``{m}``, ``{m,}``, ``{m,n}``."""
    def atom(d):
        u = rng.random()
        if d <= 0 or u < 0.35:
            if rng.random() < 0.75 or len(alphabet) == 1:
                return bytes([alphabet[int(rng.integers(0, len(alphabet)))]])
            k = int(rng.integers(1, len(alphabet) + 1))
            idx = np.sort(rng.choice(len(alphabet), size=k, replace=False))
            neg = rng.random() < 0.15
            body = bytes(alphabet[i] for i in idx)
            return b"[" + (b"^" if neg else b"") + body + b"]"
        if u < 0.65:
            nparts = int(rng.integers(2, 4))
            return b"(" + b"".join(expr(d - 1) for _ in range(nparts)) + b")"
        nalt = int(rng.integers(2, 4))
        alts = [expr(d - 1) if rng.random() < 0.9 else b"" for _ in range(nalt)]
        return b"(" + b"|".join(alts) + b")"

    def post(d):
        a = atom(d)
        u = rng.random()
        if u < 0.15:
            return a + b"*"
        if u < 0.25:
            return a + b"+"
        if u < 0.35:
            return a + b"?"
        if u < 0.42:
            m = int(rng.integers(0, 3))
            hi = m + int(rng.integers(0, 3))
            form = int(rng.integers(0, 3))
            if form == 0:
                return a + b"{%d}" % m
            if form == 1:
                return a + b"{%d,}" % m
            return a + b"{%d,%d}" % (m, hi)
        return a

    def expr(d):
        n = int(rng.integers(1, 4))
        return b"".join(post(d) for _ in range(n))

    return expr(depth)


def random_text(rng: np.random.Generator, alphabet: bytes, n: int) -> np.ndarray:
    a = np.frombuffer(alphabet, dtype=np.uint8)
    return np.ascontiguousarray(a[rng.integers(0, len(a), size=n)])
