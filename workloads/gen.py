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


# ---------------------------------------------------------------------------
# batched workload: random expressions of a small grammar, texts sampled
# from their syntax trees
# ---------------------------------------------------------------------------
#
# Trees: ('lit', b) | ('cls', bytes, neg) | ('cat', [t...]) | ('alt', [t...])
# | ('rep', t, m, hi) with hi None for an unbounded repeat.  Every subtree
# denotes a non-empty language (the grammar has no empty set), so a text can
# always be derived.  Derivations pick uniformly among alternatives and
# class members; repeats draw their counts; one unbounded repeat takes the
# length budget by concatenating independently derived copies of its body.

def _lit_bytes(b: int) -> bytes:
    c = bytes([b])
    return c if c.isalnum() else b"\\x%02x" % b


def c4_tree(rng: np.random.Generator, alphabet: bytes, depth: int):
    def atom(d):
        u = rng.random()
        if d <= 0 or u < 0.4:
            if rng.random() < 0.7:
                return ("lit", alphabet[int(rng.integers(0, len(alphabet)))])
            k = int(rng.integers(2, max(3, min(len(alphabet), 8) + 1)))
            idx = np.sort(rng.choice(len(alphabet), size=min(k, len(alphabet)), replace=False))
            return ("cls", bytes(alphabet[i] for i in idx), bool(rng.random() < 0.1))
        if u < 0.7:
            return ("cat", [post(d - 1) for _ in range(int(rng.integers(2, 4)))])
        return ("alt", [post(d - 1) for _ in range(int(rng.integers(2, 4)))])

    def post(d):
        a = atom(d)
        u = rng.random()
        if u < 0.2:
            return ("rep", a, 0, None)
        if u < 0.28:
            return ("rep", a, 1, None)
        if u < 0.36:
            return ("rep", a, 0, 1)
        if u < 0.46:
            m = int(rng.integers(1, 4))
            return ("rep", a, m, m + int(rng.integers(0, 4)))
        return a

    return ("cat", [post(depth) for _ in range(int(rng.integers(2, 4)))])


def render(t) -> bytes:
    kind = t[0]
    if kind == "lit":
        return _lit_bytes(t[1])
    if kind == "cls":
        return b"[" + (b"^" if t[2] else b"") + b"".join(_lit_bytes(b) for b in t[1]) + b"]"
    if kind == "cat":
        return b"(" + b"".join(render(c) for c in t[1]) + b")"
    if kind == "alt":
        return b"(" + b"|".join(render(c) for c in t[1]) + b")"
    body = render(t[1])
    m, hi = t[2], t[3]
    if hi is None:
        return body + (b"*" if m == 0 else b"+" if m == 1 else b"{%d,}" % m)
    if (m, hi) == (0, 1):
        return body + b"?"
    return body + (b"{%d}" % m if m == hi else b"{%d,%d}" % (m, hi))


def _nonempty(t) -> bool:
    """Whether t derives some non-empty text."""
    kind = t[0]
    if kind in ("lit", "cls"):
        return True
    if kind in ("cat", "alt"):
        return any(_nonempty(c) for c in t[1])
    return (t[3] is None or t[3] > 0) and _nonempty(t[1])


def unbounded(t) -> bool:
    """Whether t derives texts of every length beyond some bound, i.e. has an
    unbounded repeat of a body that derives a non-empty text."""
    kind = t[0]
    if kind in ("lit", "cls"):
        return False
    if kind in ("cat", "alt"):
        return any(unbounded(c) for c in t[1])
    return (t[3] is None and _nonempty(t[1])) or ((t[3] is None or t[3] > 0) and unbounded(t[1]))


def _class_pick(rng, members: bytes, neg: bool, alphabet: bytes) -> int:
    if not neg:
        return members[int(rng.integers(0, len(members)))]
    pool = [b for b in alphabet if b not in members] or [b for b in range(256) if b not in members]
    return pool[int(rng.integers(0, len(pool)))]


def derive(rng: np.random.Generator, t, alphabet: bytes, budget: int = 0) -> np.ndarray:
    """A text of L(t).  With budget > 0 the first unbounded repeat met takes
    the budget: copies of its body are derived (a pool of 64) and
    concatenated in random order until the budget is used."""
    out = []
    state = {"budget": int(budget)}

    def go(t):
        kind = t[0]
        if kind == "lit":
            out.append(np.array([t[1]], np.uint8))
        elif kind == "cls":
            out.append(np.array([_class_pick(rng, t[1], t[2], alphabet)], np.uint8))
        elif kind == "cat":
            for c in t[1]:
                go(c)
        elif kind == "alt":
            kids = t[1]
            if state["budget"] > 0:
                long = [c for c in kids if unbounded(c)]
                if long:
                    go(long[int(rng.integers(0, len(long)))])
                    return
            go(kids[int(rng.integers(0, len(kids)))])
        else:
            body, m, hi = t[1], t[2], t[3]
            if hi is None and state["budget"] > 0 and _nonempty(body):
                b = state["budget"]
                state["budget"] = 0
                pool = []
                for _ in range(64):
                    sub = derive(rng, body, alphabet)
                    if len(sub):
                        pool.append(sub)
                lens = np.array([len(p) for p in pool], np.int64)
                flat = np.concatenate(pool)
                starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
                cnt = max(m, int(b // max(1.0, lens.mean())) + 1)
                pick = rng.integers(0, len(pool), size=cnt)
                plen = lens[pick]
                total = int(plen.sum())
                first = np.repeat(starts[pick] - np.concatenate([[0], np.cumsum(plen)[:-1]]), plen)
                out.append(flat[first + np.arange(total)])
                return
            if state["budget"] > 0 and unbounded(body):
                reps = max(m, 1)
            else:
                top = hi if hi is not None else m + int(rng.geometric(0.5))
                reps = int(rng.integers(m, top + 1))
            for _ in range(reps):
                go(body)

    go(t)
    return np.concatenate(out) if out else np.zeros(0, np.uint8)


def c4_alphabet(k: int) -> bytes:
    """The first k printable bytes."""
    return bytes(range(0x20, 0x20 + int(k)))


def c4_candidate(seed: int, index: int):
    """Candidate expression `index` of the batched workload: (regex, tree,
    alphabet).  Candidates are filtered by automaton size elsewhere."""
    rng = PCG((int(seed) << 20) + int(index))
    alphabet = c4_alphabet(int(rng.integers(4, 65)))
    t = c4_tree(rng, alphabet, int(rng.integers(4, 8)))
    return render(t), t, alphabet


def c4_lengths(seed: int, count: int = 4096, lo: int = 1 << 10, hi: int = 1 << 22) -> np.ndarray:
    """Text lengths, log-uniform in [lo, hi]."""
    rng = PCG(seed)
    return np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def c4_text(seed: int, i: int, tree, alphabet: bytes, n: int):
    """Text i: derived from the tree to about n bytes (even i), or derived
    and then changed at one uniform position to a different byte of the
    alphabet (odd i).  Returns (text, changed)."""
    rng = PCG((int(seed) << 24) + 7919 * int(i) + 1)
    x = derive(rng, tree, alphabet, budget=n)
    if len(x) > n:
        # keep the derivation whole: a cut could leave L; only the budget is approximate
        pass
    changed = bool(i % 2 == 1 and len(x) > 0)
    if changed:
        x = x.copy()
        p = int(rng.integers(0, len(x)))
        others = [b for b in alphabet if b != x[p]]
        x[p] = others[int(rng.integers(0, len(others)))]
    return np.ascontiguousarray(x, dtype=np.uint8), changed


# ---------------------------------------------------------------------------
# serving workload: keyword unions .*(k1|...|kn).*
# ---------------------------------------------------------------------------
#
# A keyword is a list of positions, each a set of printable bytes with a
# repeat range: a literal (p = 0.9), a class of 2-5 bytes (p = 0.08) or a
# class repeated 1-3 times (p = 0.02).  Keywords are dropped from the end
# until the keyword positions (a repeat counted at its upper bound) are at
# most `max_positions`: that is the size of the expression's position NFA
# and about the size of its keyword trie.

PRINTABLE = bytes(range(0x20, 0x7F))


def _c5_keyword(rng: np.random.Generator):
    n = int(rng.integers(4, 17))
    out = []
    for _ in range(n):
        u = rng.random()
        if u < 0.9:
            out.append((bytes([PRINTABLE[int(rng.integers(0, len(PRINTABLE)))]]), 1, 1))
        else:
            k = int(rng.integers(2, 6))
            idx = np.sort(rng.choice(len(PRINTABLE), size=k, replace=False))
            members = bytes(PRINTABLE[i] for i in idx)
            out.append((members, 1, 1) if u < 0.98 else (members, 1, 3))
    return out


def _keyword_positions(kw) -> int:
    return sum(hi for _, _, hi in kw)


def _render_keyword(kw) -> bytes:
    out = b""
    for members, lo, hi in kw:
        body = _lit_bytes(members[0]) if len(members) == 1 else b"[" + b"".join(_lit_bytes(b) for b in members) + b"]"
        out += body if (lo, hi) == (1, 1) else body + b"{%d,%d}" % (lo, hi)
    return out


def c5_automaton(seed: int, index: int, nkw: int = 0, max_positions: int = 20000):
    """Expression `index` of the serving pool: (regex, keywords).  nkw = 0
    draws the keyword count from U{200..2000}."""
    rng = PCG((int(seed) << 16) + 977 * int(index) + 5)
    n = int(nkw) if nkw else int(rng.integers(200, 2001))
    kws = [_c5_keyword(rng) for _ in range(n)]
    while len(kws) > 1 and sum(_keyword_positions(k) for k in kws) > max_positions:
        kws.pop()
    rx = b".*(" + b"|".join(_render_keyword(k) for k in kws) + b").*"
    return rx, kws


def keyword_instance(rng: np.random.Generator, kw) -> bytes:
    out = b""
    for members, lo, hi in kw:
        for _ in range(int(rng.integers(lo, hi + 1))):
            out += bytes([members[int(rng.integers(0, len(members)))]])
    return out


def c5_text(rng: np.random.Generator, kws, n: int, plant: bool) -> np.ndarray:
    """n uniform printable bytes; with plant, one instance of a random keyword
    at a uniform position."""
    x = random_text(rng, PRINTABLE, n)
    if plant and kws and n > 0:
        k = keyword_instance(rng, kws[int(rng.integers(0, len(kws)))])
        if len(k) <= n:
            p = int(rng.integers(0, n - len(k) + 1))
            x[p:p + len(k)] = np.frombuffer(k, np.uint8)
    return x


def c5_length(rng: np.random.Generator, median: int = 1 << 16, sigma: float = 1.0, cap: int = 1 << 26) -> int:
    return int(min(cap, max(1, round(float(rng.lognormal(np.log(median), sigma))))))


SERVE_SEED = 11


def c5_requests(count: int, kws_of, seed: int = SERVE_SEED, keep=None):
    """The request stream of the serving workload: request i picks automaton
    k uniform in [0, len(kws_of)), a log-normal length and printable bytes,
    with a keyword of automaton k planted when i is even.  Yields (i, k, x)
    for every request whose automaton is in `keep` (all when None); the draws
    of the skipped requests are still made, so request i is the same byte
    string whatever `keep` is."""
    rng = PCG(seed + 1)
    for i in range(count):
        k = int(rng.integers(0, len(kws_of)))
        n = c5_length(rng)
        if keep is None or k in keep:
            yield i, k, c5_text(rng, kws_of[k], n, plant=i % 2 == 0)
        else:
            c5_text(rng, kws_of[k], n, plant=i % 2 == 0)
