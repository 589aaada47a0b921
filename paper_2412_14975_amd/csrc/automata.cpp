// Host-side automaton construction for the recognizer (see automata.hpp).
//
// Expression syntax (bytes): alternation |, concatenation, grouping ( ),
// postfix * + ? {m} {m,} {m,n} (0 <= m <= n <= 1000), . (any byte),
// bracket classes [...] with ranges and a leading ^ for the complement,
// escapes \n \t \r \f \v \0 \xHH \d, and a backslash before any other byte
// makes it literal.  Every other byte stands for itself.
//
// Bounded repeats are expanded before positions are numbered:
//   e{m} = e...e,  e{m,} = e...e e*,  e{m,n} = e...e (e (e (...)?)?)?
// and positions are numbered left to right in the expanded expression, so
// the position automaton is fixed by the expression.
#include "automata.hpp"

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>

#include "ri.h"

namespace ri {
namespace {

// ---------------------------------------------------------------------------
// parser
// ---------------------------------------------------------------------------

enum Kind : uint8_t { K_SYM, K_EPS, K_CAT, K_ALT, K_STAR, K_PLUS, K_OPT, K_REP };

struct Node {
    Kind kind;
    ByteSet sym;
    std::vector<int> kids;
    int lo = 0;
    int hi = 0;   // -1: unbounded
};

constexpr int kMaxRepeat = 1000;

class Parser {
  public:
    explicit Parser(const std::string &s) : s_(s) {}

    int parse() {
        int r = alternation();
        if (i_ != s_.size()) fail("unbalanced ')'", i_);
        return r;
    }

    std::vector<Node> nodes;

  private:
    const std::string &s_;
    size_t i_ = 0;

    [[noreturn]] void fail(const char *m, size_t at) {
        throw BuildError(RI_ERR_PARSE, std::string(m) + " at offset " + std::to_string(at));
    }
    int peek() const { return i_ < s_.size() ? (unsigned char)s_[i_] : -1; }
    int take() {
        if (i_ >= s_.size()) fail("unexpected end of pattern", i_);
        return (unsigned char)s_[i_++];
    }
    int make(Kind k) {
        nodes.push_back(Node{k, ByteSet(), {}, 0, 0});
        return (int)nodes.size() - 1;
    }
    int make_sym(const ByteSet &b) {
        int n = make(K_SYM);
        nodes[n].sym = b;
        return n;
    }
    int make_unary(Kind k, int kid) {
        int n = make(k);
        nodes[n].kids.push_back(kid);
        return n;
    }

    int alternation() {
        std::vector<int> br{sequence()};
        while (peek() == '|') {
            ++i_;
            br.push_back(sequence());
        }
        if (br.size() == 1) return br[0];
        int n = make(K_ALT);
        nodes[n].kids = std::move(br);
        return n;
    }

    int sequence() {
        std::vector<int> items;
        while (peek() != -1 && peek() != '|' && peek() != ')') items.push_back(postfix());
        if (items.empty()) return make(K_EPS);
        if (items.size() == 1) return items[0];
        int n = make(K_CAT);
        nodes[n].kids = std::move(items);
        return n;
    }

    int postfix() {
        int a = atom();
        for (;;) {
            int c = peek();
            if (c == '*') { ++i_; a = make_unary(K_STAR, a); }
            else if (c == '+') { ++i_; a = make_unary(K_PLUS, a); }
            else if (c == '?') { ++i_; a = make_unary(K_OPT, a); }
            else if (c == '{') a = braces(a);
            else return a;
        }
    }

    int number() {
        size_t j = i_;
        long v = 0;
        while (peek() >= '0' && peek() <= '9') {
            v = v * 10 + (take() - '0');
            if (v > kMaxRepeat) fail("repeat count too large", j);
        }
        if (j == i_) fail("expected a number", i_);
        return (int)v;
    }

    int braces(int a) {
        size_t at = i_;
        ++i_;
        int lo = number(), hi = lo;
        if (peek() == ',') {
            ++i_;
            hi = (peek() == '}') ? -1 : number();
        }
        if (peek() != '}') fail("expected '}'", i_);
        ++i_;
        if (hi >= 0 && hi < lo) fail("bad repeat bounds", at);
        int n = make_unary(K_REP, a);
        nodes[n].lo = lo;
        nodes[n].hi = hi;
        return n;
    }

    int atom() {
        size_t at = i_;
        int c = take();
        switch (c) {
        case '(': {
            int n = alternation();
            if (peek() != ')') fail("missing ')'", i_);
            ++i_;
            return n;
        }
        case ')': fail("unbalanced ')'", at);
        case '*': case '+': case '?': case '{': fail("nothing to repeat", at);
        case '.': { ByteSet b; b.set(); return make_sym(b); }
        case '[': return make_sym(bracket());
        case '\\': return make_sym(escape());
        default: { ByteSet b; b.set(c); return make_sym(b); }
        }
    }

    ByteSet escape() {
        size_t at = i_ - 1;
        int c = take();
        ByteSet b;
        switch (c) {
        case 'n': b.set(10); break;
        case 't': b.set(9); break;
        case 'r': b.set(13); break;
        case 'f': b.set(12); break;
        case 'v': b.set(11); break;
        case '0': b.set(0); break;
        case 'd': for (int d = '0'; d <= '9'; ++d) b.set(d); break;
        case 'x': {
            auto hex = [&](int ch) -> int {
                if (ch >= '0' && ch <= '9') return ch - '0';
                if (ch >= 'a' && ch <= 'f') return ch - 'a' + 10;
                if (ch >= 'A' && ch <= 'F') return ch - 'A' + 10;
                return -1;
            };
            int h1 = i_ < s_.size() ? hex((unsigned char)s_[i_]) : -1;
            int h2 = i_ + 1 < s_.size() ? hex((unsigned char)s_[i_ + 1]) : -1;
            if (h1 < 0 || h2 < 0) fail("bad \\x escape", at);
            i_ += 2;
            b.set(h1 * 16 + h2);
            break;
        }
        default: b.set(c);
        }
        return b;
    }

    ByteSet class_item() {
        int c = take();
        if (c == '\\') return escape();
        ByteSet b;
        b.set(c);
        return b;
    }

    ByteSet bracket() {
        size_t at = i_ - 1;
        bool neg = false;
        if (peek() == '^') { neg = true; ++i_; }
        ByteSet out;
        bool first = true;
        for (;;) {
            int c = peek();
            if (c < 0) fail("missing ']'", at);
            if (c == ']' && !first) { ++i_; break; }
            first = false;
            ByteSet lo = class_item();
            if (peek() == '-' && i_ + 1 < s_.size() && s_[i_ + 1] != ']') {
                ++i_;
                ByteSet hi = class_item();
                if (lo.count() != 1 || hi.count() != 1) fail("bad range", i_);
                int a = 0, z = 0;
                while (!lo.test(a)) ++a;
                while (!hi.test(z)) ++z;
                if (z < a) fail("bad range", i_);
                for (int x = a; x <= z; ++x) out.set(x);
            } else {
                out |= lo;
            }
        }
        if (neg) out.flip();
        return out;
    }
};

// ---------------------------------------------------------------------------
// position automaton
// ---------------------------------------------------------------------------

class Glushkov {
  public:
    Glushkov(const std::vector<Node> &nodes, uint32_t max_pos) : nodes_(nodes), max_pos_(max_pos) {
        sym.emplace_back();
        follow.emplace_back();
    }

    struct Res {
        bool nullable = true;
        std::vector<uint32_t> first, last;
    };

    std::vector<ByteSet> sym;
    std::vector<std::vector<uint32_t>> follow;

    Res walk(int id) {
        const Node &nd = nodes_[id];
        switch (nd.kind) {
        case K_SYM: return leaf(nd.sym);
        case K_EPS: return Res{};
        case K_CAT: {
            Res acc;
            for (int k : nd.kids) acc = cat(std::move(acc), walk(k));
            return acc;
        }
        case K_ALT: {
            Res acc;
            acc.nullable = false;
            for (int k : nd.kids) {
                Res r = walk(k);
                acc.nullable = acc.nullable || r.nullable;
                acc.first.insert(acc.first.end(), r.first.begin(), r.first.end());
                acc.last.insert(acc.last.end(), r.last.begin(), r.last.end());
            }
            return acc;
        }
        case K_STAR: { Res r = walk(nd.kids[0]); loop(r); r.nullable = true; return r; }
        case K_PLUS: { Res r = walk(nd.kids[0]); loop(r); return r; }
        case K_OPT: { Res r = walk(nd.kids[0]); r.nullable = true; return r; }
        case K_REP: {
            Res acc;
            for (int c = 0; c < nd.lo; ++c) acc = cat(std::move(acc), walk(nd.kids[0]));
            if (nd.hi < 0) {
                Res r = walk(nd.kids[0]);
                loop(r);
                r.nullable = true;
                acc = cat(std::move(acc), std::move(r));
            } else if (nd.hi > nd.lo) {
                acc = cat(std::move(acc), nested(nd.kids[0], nd.hi - nd.lo));
            }
            return acc;
        }
        }
        return Res{};
    }

  private:
    const std::vector<Node> &nodes_;
    uint32_t max_pos_;

    Res leaf(const ByteSet &b) {
        if (sym.size() > max_pos_)
            throw BuildError(RI_ERR_LIMIT, "position automaton exceeds max_states");
        uint32_t p = (uint32_t)sym.size();
        sym.push_back(b);
        follow.emplace_back();
        Res r;
        r.nullable = false;
        r.first.push_back(p);
        r.last.push_back(p);
        return r;
    }

    // (e (e (...)?)?)? with `levels` copies of e, leftmost copy numbered first
    Res nested(int kid, int levels) {
        Res head = walk(kid);
        if (levels > 1) head = cat(std::move(head), nested(kid, levels - 1));
        head.nullable = true;
        return head;
    }

    void loop(const Res &r) {
        for (uint32_t x : r.last) follow[x].insert(follow[x].end(), r.first.begin(), r.first.end());
    }

    Res cat(Res a, Res b) {
        for (uint32_t x : a.last) follow[x].insert(follow[x].end(), b.first.begin(), b.first.end());
        Res r;
        r.nullable = a.nullable && b.nullable;
        r.first = std::move(a.first);
        if (a.nullable) r.first.insert(r.first.end(), b.first.begin(), b.first.end());
        r.last = std::move(b.last);
        if (b.nullable) r.last.insert(r.last.end(), a.last.begin(), a.last.end());
        return r;
    }
};

void sort_unique(std::vector<uint32_t> &v) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
}

PositionNfa position_automaton(const std::string &re, uint32_t max_states) {
    Parser ps(re);
    int root = ps.parse();
    Glushkov g(ps.nodes, max_states);
    Glushkov::Res r = g.walk(root);
    PositionNfa N;
    N.n = (uint32_t)g.sym.size();
    N.sym = std::move(g.sym);
    N.next.resize(N.n);
    N.next[0] = r.first;
    for (uint32_t p = 1; p < N.n; ++p) N.next[p] = std::move(g.follow[p]);
    for (auto &v : N.next) sort_unique(v);
    N.final.assign(N.n, 0);
    for (uint32_t p : r.last) N.final[p] = 1;
    if (r.nullable) N.final[0] = 1;
    return N;
}

// Keep states reachable from 0 that can reach a final state, renumbered in
// increasing order (0 stays 0).  n = 0 when the language is empty.
PositionNfa trim(const PositionNfa &N) {
    std::vector<uint8_t> fwd(N.n, 0), bwd(N.n, 0);
    std::vector<uint32_t> stack{0};
    fwd[0] = 1;
    while (!stack.empty()) {
        uint32_t q = stack.back();
        stack.pop_back();
        for (uint32_t p : N.next[q])
            if (N.sym[p].any() && !fwd[p]) { fwd[p] = 1; stack.push_back(p); }
    }
    std::vector<std::vector<uint32_t>> pred(N.n);
    for (uint32_t q = 0; q < N.n; ++q)
        for (uint32_t p : N.next[q])
            if (N.sym[p].any()) pred[p].push_back(q);
    for (uint32_t q = 0; q < N.n; ++q)
        if (N.final[q]) { bwd[q] = 1; stack.push_back(q); }
    while (!stack.empty()) {
        uint32_t p = stack.back();
        stack.pop_back();
        for (uint32_t q : pred[p])
            if (!bwd[q]) { bwd[q] = 1; stack.push_back(q); }
    }
    PositionNfa T;
    if (!(fwd[0] && bwd[0])) return T;
    std::vector<int64_t> id(N.n, -1);
    for (uint32_t q = 0; q < N.n; ++q)
        if (fwd[q] && bwd[q]) id[q] = T.n++;
    T.sym.resize(T.n);
    T.next.resize(T.n);
    T.final.resize(T.n);
    for (uint32_t q = 0; q < N.n; ++q) {
        if (id[q] < 0) continue;
        uint32_t nq = (uint32_t)id[q];
        T.sym[nq] = N.sym[q];
        T.final[nq] = N.final[q];
        for (uint32_t p : N.next[q])
            if (id[p] >= 0 && N.sym[p].any()) T.next[nq].push_back((uint32_t)id[p]);
    }
    return T;
}

// ---------------------------------------------------------------------------
// byte classes and class-labelled NFAs
// ---------------------------------------------------------------------------

// Partition of the 256 bytes into classes of bytes that no symbol set tells
// apart; classes are numbered in increasing order of their smallest byte.
uint32_t byte_classes(const PositionNfa &N, uint8_t cls[256]) {
    std::vector<uint32_t> c(256, 0);
    uint32_t K = 1;
    std::vector<uint8_t> seen;
    for (uint32_t p = 1; p < N.n; ++p) {
        std::vector<int32_t> remap(2 * K, -1);
        uint32_t nk = 0;
        for (int b = 0; b < 256; ++b) {
            uint32_t key = 2 * c[b] + (N.sym[p].test(b) ? 1 : 0);
            if (remap[key] < 0) remap[key] = (int32_t)nk++;
            c[b] = (uint32_t)remap[key];
        }
        K = nk;
    }
    // renumber by smallest byte (the loop above already does: ids are given
    // on first appearance while scanning bytes in ascending order)
    for (int b = 0; b < 256; ++b) cls[b] = (uint8_t)c[b];
    return K;
}

struct MaskPool {
    uint32_t words;
    std::vector<uint64_t> data;
    std::map<std::vector<uint64_t>, uint32_t> ids;
    uint32_t intern(const std::vector<uint64_t> &m) {
        auto it = ids.find(m);
        if (it != ids.end()) return it->second;
        uint32_t id = (uint32_t)ids.size();
        ids.emplace(m, id);
        data.insert(data.end(), m.begin(), m.end());
        return id;
    }
};

ClassNfa class_nfa(const PositionNfa &N, uint32_t K, const uint8_t cls[256]) {
    ClassNfa C;
    C.n = N.n;
    C.K = K;
    C.mask_words = (K + 63) / 64;
    MaskPool pool{C.mask_words, {}, {}};
    std::vector<uint32_t> pmask(N.n, 0);
    for (uint32_t p = 1; p < N.n; ++p) {
        std::vector<uint64_t> m(C.mask_words, 0);
        for (int b = 0; b < 256; ++b)
            if (N.sym[p].test(b)) m[cls[b] / 64] |= 1ull << (cls[b] % 64);
        pmask[p] = pool.intern(m);
    }
    C.edges.resize(N.n);
    for (uint32_t q = 0; q < N.n; ++q)
        for (uint32_t p : N.next[q]) C.edges[q].push_back({p, pmask[p]});
    C.masks = std::move(pool.data);
    C.final = N.final;
    return C;
}

ClassNfa quotient(const ClassNfa &N, const std::vector<uint32_t> &cid, uint32_t nq) {
    ClassNfa Q;
    Q.n = nq;
    Q.K = N.K;
    Q.mask_words = N.mask_words;
    MaskPool pool{Q.mask_words, {}, {}};
    std::vector<std::map<uint32_t, std::vector<uint64_t>>> acc(nq);
    Q.final.assign(nq, 0);
    for (uint32_t q = 0; q < N.n; ++q) {
        if (N.final[q]) Q.final[cid[q]] = 1;
        for (auto [t, mid] : N.edges[q]) {
            auto &m = acc[cid[q]][cid[t]];
            if (m.empty()) m.assign(Q.mask_words, 0);
            for (uint32_t w = 0; w < Q.mask_words; ++w) m[w] |= N.masks[(size_t)mid * Q.mask_words + w];
        }
    }
    Q.edges.resize(nq);
    for (uint32_t c = 0; c < nq; ++c)
        for (auto &[t, m] : acc[c]) Q.edges[c].push_back({t, pool.intern(m)});
    Q.masks = std::move(pool.data);
    return Q;
}

// ---------------------------------------------------------------------------
// powerset constructions
// ---------------------------------------------------------------------------

struct VecHash {
    size_t operator()(const std::vector<uint32_t> &v) const {
        uint64_t h = 1469598103934665603ull;
        for (uint32_t x : v) { h ^= x; h *= 1099511628211ull; }
        return (size_t)h;
    }
};
using SubsetIndex = std::unordered_map<std::vector<uint32_t>, uint32_t, VecHash>;

// Deterministic transition graph over the subsets of NFA states reachable
// from the singletons of `starts`, processed in order; each pass only adds
// states not yet present (the incremental construction of Sect. 3.1 when
// `starts` lists every NFA state, the textbook powerset DFA when it is {0}).
DetAutomaton powerset(const ClassNfa &N, const std::vector<uint32_t> &starts, uint32_t max_states,
                      SubsetIndex *index_out) {
    DetAutomaton A;
    A.K = N.K;
    SubsetIndex index;
    std::vector<std::vector<uint32_t>> buckets(N.K);
    auto add = [&](std::vector<uint32_t> &&S) -> uint32_t {
        if (A.n >= max_states) throw BuildError(RI_ERR_LIMIT, "automaton exceeds max_states");
        uint32_t id = A.n++;
        index.emplace(S, id);
        A.content.push_back(std::move(S));
        A.delta.resize((size_t)A.n * A.K, -1);
        return id;
    };
    std::deque<uint32_t> work;
    for (uint32_t q : starts) {
        std::vector<uint32_t> S{q};
        if (index.count(S)) continue;
        work.push_back(add(std::move(S)));
        while (!work.empty()) {
            uint32_t p = work.front();
            work.pop_front();
            for (auto &b : buckets) b.clear();
            for (uint32_t s : A.content[p])
                for (auto [t, mid] : N.edges[s]) {
                    const uint64_t *m = &N.masks[(size_t)mid * N.mask_words];
                    for (uint32_t w = 0; w < N.mask_words; ++w)
                        for (uint64_t bits = m[w]; bits; bits &= bits - 1)
                            buckets[w * 64 + __builtin_ctzll(bits)].push_back(t);
                }
            for (uint32_t k = 0; k < N.K; ++k) {
                if (buckets[k].empty()) continue;
                sort_unique(buckets[k]);
                auto it = index.find(buckets[k]);
                uint32_t t = (it != index.end()) ? it->second : 0;
                if (it == index.end()) {
                    t = add(std::vector<uint32_t>(buckets[k]));
                    work.push_back(t);
                }
                A.delta[(size_t)p * A.K + k] = (int32_t)t;
            }
        }
    }
    A.final.assign(A.n, 0);
    for (uint32_t p = 0; p < A.n; ++p)
        for (uint32_t q : A.content[p])
            if (N.final[q]) { A.final[p] = 1; break; }
    A.initial.assign(N.n, UINT32_MAX);
    for (uint32_t q = 0; q < N.n; ++q) {
        auto it = index.find(std::vector<uint32_t>{q});
        if (it != index.end()) A.initial[q] = it->second;
    }
    if (index_out) *index_out = std::move(index);
    return A;
}

// Nerode classes of a deterministic graph completed by a dead state
// (index n): Moore refinement from {final, non-final} until stable.
std::vector<uint32_t> nerode(const DetAutomaton &A) {
    const uint32_t n = A.n, K = A.K;
    std::vector<uint32_t> cls(n + 1, 0), next(n + 1);
    for (uint32_t s = 0; s < n; ++s) cls[s] = A.final[s] ? 1 : 0;
    uint32_t count = 0;
    {
        bool has[2] = {false, false};
        for (uint32_t c : cls) has[c] = true;
        count = (uint32_t)has[0] + (uint32_t)has[1];
    }
    std::vector<uint32_t> sig(K + 1);
    for (;;) {
        std::unordered_map<std::vector<uint32_t>, uint32_t, VecHash> ids;
        ids.reserve(2 * (n + 1));
        for (uint32_t s = 0; s <= n; ++s) {
            sig[0] = cls[s];
            for (uint32_t k = 0; k < K; ++k) {
                int32_t t = (s < n) ? A.delta[(size_t)s * K + k] : -1;
                sig[k + 1] = (t < 0) ? cls[n] : cls[t];
            }
            next[s] = ids.emplace(sig, (uint32_t)ids.size()).first->second;
        }
        cls.swap(next);
        if (ids.size() == count) return cls;
        count = (uint32_t)ids.size();
    }
}

}  // namespace

void build_automata(const std::string &re, uint32_t max_states, Automata &out) {
    PositionNfa raw = position_automaton(re, max_states);
    PositionNfa N = trim(raw);
    out = Automata();
    out.nfa_states = N.n;
    if (N.n == 0) {
        out.empty_language = true;
        out.K = 1;
        std::memset(out.cls, 0, sizeof(out.cls));
        return;
    }
    out.K = byte_classes(N, out.cls);
    ClassNfa CN = class_nfa(N, out.K, out.cls);
    if (N.n <= kNfaMaxStates) {
        const uint32_t W = N.n <= 64 ? 1 : N.n <= 128 ? 2 : 4;
        out.nfa_words = W;
        out.nfa_follow.assign((size_t)N.n * W, 0);
        for (uint32_t q = 0; q < N.n; ++q)
            for (uint32_t p : N.next[q]) out.nfa_follow[(size_t)q * W + p / 64] |= 1ull << (p % 64);
        out.nfa_mask.assign((size_t)out.K * W, 0);
        for (uint32_t p = 1; p < N.n; ++p)
            for (int b = 0; b < 256; ++b)
                if (N.sym[p].test(b)) out.nfa_mask[(size_t)out.cls[b] * W + p / 64] |= 1ull << (p % 64);
    }

    // B = RI-DFA(N) and its Nerode classes (Sect. 3.1, 3.4)
    std::vector<uint32_t> all(N.n);
    for (uint32_t q = 0; q < N.n; ++q) all[q] = q;
    DetAutomaton B = powerset(CN, all, max_states, nullptr);
    out.ridfa_full_states = B.n;
    std::vector<uint32_t> clsB = nerode(B);

    // delegation: the lowest NFA state of each class of initial singletons
    // keeps the initial role; N' merges each class into one state
    std::vector<uint32_t> rep(N.n);
    std::unordered_map<uint32_t, uint32_t> first_of_class;
    for (uint32_t q = 0; q < N.n; ++q) {
        auto it = first_of_class.emplace(clsB[B.initial[q]], q).first;
        rep[q] = it->second;
    }
    out.cid.assign(N.n, 0);
    uint32_t nq = 0;
    {
        std::vector<int64_t> id_of_rep(N.n, -1);
        for (uint32_t q = 0; q < N.n; ++q) {
            if (id_of_rep[rep[q]] < 0) id_of_rep[rep[q]] = nq++;
            out.cid[q] = (uint32_t)id_of_rep[rep[q]];
        }
    }
    out.nq = quotient(CN, out.cid, nq);

    // B' = RI-DFA(N')
    std::vector<uint32_t> allq(nq);
    for (uint32_t q = 0; q < nq; ++q) allq[q] = q;
    SubsetIndex indexBq;
    out.Bq = powerset(out.nq, allq, max_states, &indexBq);
    const DetAutomaton &Bq = out.Bq;
    const uint32_t K = out.K;

    // minimal DFA from the Nerode classes of B' restricted to the states
    // reachable from {0}; canonical breadth-first numbering over classes in
    // increasing order of their smallest byte
    std::vector<uint32_t> clsBq = nerode(Bq);
    std::vector<uint8_t> reach(Bq.n, 0);
    std::vector<uint32_t> order{Bq.initial[0]};
    reach[Bq.initial[0]] = 1;
    for (size_t i = 0; i < order.size(); ++i)
        for (uint32_t k = 0; k < K; ++k) {
            int32_t t = Bq.delta[(size_t)order[i] * K + k];
            if (t >= 0 && !reach[t]) { reach[t] = 1; order.push_back((uint32_t)t); }
        }
    std::unordered_map<uint32_t, uint32_t> rep_state;   // class -> a reachable member
    for (uint32_t p : order) rep_state.emplace(clsBq[p], p);
    std::unordered_map<uint32_t, int32_t> canon;        // class -> canonical id
    std::vector<uint32_t> cq{clsBq[Bq.initial[0]]};
    canon[cq[0]] = 0;
    for (size_t i = 0; i < cq.size(); ++i) {
        uint32_t r = rep_state.at(cq[i]);
        for (uint32_t k = 0; k < K; ++k) {
            int32_t t = Bq.delta[(size_t)r * K + k];
            if (t < 0) continue;
            if (canon.emplace(clsBq[t], (int32_t)cq.size()).second) cq.push_back(clsBq[t]);
        }
    }
    out.dmin_n = (uint32_t)cq.size();
    if (out.dmin_n > max_states) throw BuildError(RI_ERR_LIMIT, "minimal DFA exceeds max_states");
    out.dmin_delta.assign((size_t)out.dmin_n * K, -1);
    out.dmin_final.assign(out.dmin_n, 0);
    for (uint32_t i = 0; i < out.dmin_n; ++i) {
        uint32_t r = rep_state.at(cq[i]);
        out.dmin_final[i] = Bq.final[r];
        for (uint32_t k = 0; k < K; ++k) {
            int32_t t = Bq.delta[(size_t)r * K + k];
            if (t >= 0) out.dmin_delta[(size_t)i * K + k] = canon.at(clsBq[t]);
        }
    }
    out.final_id.assign(Bq.n, -1);
    for (uint32_t p : order) out.final_id[p] = canon.at(clsBq[p]);
    out.accepts_empty = out.dmin_final[0] != 0;

    // powerset DFA of N (the unminimized baseline).  Both it and the minimal
    // DFA are trimmed DFAs of L, so walking them in lockstep from their
    // initial states pairs every powerset state with its minimal-DFA state.
    DetAutomaton D = powerset(CN, std::vector<uint32_t>{0}, max_states, nullptr);
    out.dsub_n = D.n;
    out.dsub_final_id.assign(D.n, -1);
    out.dsub_accept.assign(D.n, 0);
    std::vector<uint32_t> work{0};
    out.dsub_final_id[0] = 0;
    for (size_t i = 0; i < work.size(); ++i) {
        const uint32_t s = work[i];
        const int32_t m = out.dsub_final_id[s];
        for (uint32_t k = 0; k < K; ++k) {
            const int32_t t = D.delta[(size_t)s * K + k];
            const int32_t u = out.dmin_delta[(size_t)m * K + k];
            if ((t < 0) != (u < 0))
                throw BuildError(RI_ERR_LIMIT, "internal: powerset and minimal DFA disagree");
            if (t < 0) continue;
            if (out.dsub_final_id[t] < 0) {
                out.dsub_final_id[t] = u;
                work.push_back((uint32_t)t);
            } else if (out.dsub_final_id[t] != u) {
                throw BuildError(RI_ERR_LIMIT, "internal: powerset and minimal DFA disagree");
            }
        }
    }
    for (uint32_t s = 0; s < D.n; ++s) out.dsub_accept[s] = D.final[s];
    out.dsub_delta = std::move(D.delta);
    out.dsub_content = std::move(D.content);
    out.pos = std::move(N);
}

}  // namespace ri
