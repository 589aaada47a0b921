// C ABI of the recognizer (include/ri.h): handle, device tables, per-stream
// workspaces and the launch sequence reach -> join tree -> finalize.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "automata.hpp"
#include "kernels.hpp"
#include "ri.h"

namespace {

thread_local std::string g_error;

int fail(int code, const std::string &msg) {
    g_error = msg;
    return code;
}

constexpr uint32_t kJoinGroup = 64;          // members per join group
constexpr uint64_t kMinAutoChunk = 256;      // smallest automatic chunk size (bytes)
constexpr uint64_t kMaxLamBytes = 1ull << 31;
constexpr uint64_t kMaxAutoPairs = 1ull << 27;   // (start, chunk) pairs of an automatic chunking
constexpr int kMaxDevices = 64;

uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

// FNV-1a over the members of a set in ascending order; the finalize kernels
// use the same function.
uint32_t hash_members(const std::vector<uint32_t> &m) {
    uint32_t h = 2166136261u;
    for (uint32_t x : m) { h ^= x; h *= 16777619u; }
    return h;
}

constexpr uint32_t kMaxDenseWords = 64;   // dense content bitsets up to 2048 interface states

// The transformation automaton of the starts over their first bytes (built
// for the grouped warm-up, at most 256 starts; see ri::PrefixArgs).
struct PrefixHost {
    uint32_t depth = 0;                        // every word of up to `depth` bytes is expanded; 0 = none
    uint32_t n = 0;                            // states
    std::vector<uint16_t> next;                // [n][K], 0xFFFF where not expanded
    std::vector<uint8_t> count;                // [n] distinct live states, kPrefixWide above 64
    std::vector<uint16_t> tgt;                 // [n][64] their ids
    std::vector<uint8_t> map;                  // [n][L] start -> index into tgt, 0xFF = dead
};

struct AlgoHost {
    bool relational = false;
    uint32_t nstates = 0, K = 0, L = 0, W = 0;
    uint32_t entry_bytes = 0, lam_bytes = 2;
    uint32_t dead = 0;                         // byte offset of the dead row
    uint32_t sink[2] = {0xFFFFFFFFu, 0xFFFFFFFFu};   // offsets of up to two sink rows, ~0 = none
    uint16_t code[256] = {};                   // byte -> class * entry_bytes
    std::vector<uint8_t> table;                // padded to 16 bytes
    std::vector<uint32_t> starts;              // entry offsets of the start states
    std::vector<uint32_t> content;             // relations, W <= kMaxDenseWords: [nstates][W] bitsets
    std::vector<uint32_t> csr_off, csr_idx;    // relations: content as sorted member lists
    std::vector<uint32_t> fmask;               // relations: [W] final states of N'
    std::vector<uint32_t> hash;                // relations: [cap][2] = (state, final id), state ~0 = empty
    uint32_t hash_cap = 0;
    std::vector<int32_t> final_of_state;       // functions
    std::vector<uint8_t> accept_of_state;      // functions
    // RI_ALGO_NFA: sets of N's states (nfa_words 64-bit words); fmask, hash
    // and csr_* then describe the powerset DFA's states as sets of N's states
    bool nfa = false;
    uint32_t nfa_words = 0;                    // 0: N is too large for the device NFA
    std::vector<uint64_t> follow, mask;        // [L][nfa_words], [K][nfa_words]
    PrefixHost prefix;
};

struct AlgoDevice {
    void *table = nullptr;
    uint32_t *starts = nullptr, *content = nullptr, *fmask = nullptr, *hash = nullptr;
    uint32_t *csr_off = nullptr, *csr_idx = nullptr;
    uint16_t *code = nullptr;
    int32_t *final_of_state = nullptr;
    uint8_t *accept_of_state = nullptr;
    uint64_t *follow = nullptr, *mask = nullptr;
    uint16_t *pfx_next = nullptr, *pfx_tgt = nullptr;
    uint8_t *pfx_count = nullptr, *pfx_map = nullptr;
};

struct DeviceCopy {
    bool ready = false;
    uint8_t *cls = nullptr;
    AlgoDevice algo[RI_NUM_ALGOS];
    int cus = 0;
    size_t max_lds = 0;
};

// A device buffer that only grows.  A buffer it replaces may still be read
// by work enqueued without a host wait, so it is kept in `retired` and freed
// with its owner (no device-wide synchronization on the way).
struct Buf { void *p = nullptr; size_t cap = 0; };

struct Workspace {
    std::mutex mu;
    int device = -1;
    hipStream_t stream = nullptr;
    uint32_t *counters = nullptr;   // [4], zero between calls
    int32_t *dres = nullptr;
    int32_t *hres = nullptr;        // pinned
    Buf lam, alias, run_base, run_count, run_chunk, run_state, run_final, dbg, join[2], ncls[2], hprod[2],
        hrows[2], block_count;
    std::vector<void *> retired;
    hipEvent_t ev[6] = {};
};

struct Options {
    int converge = 1;
    int join = 0;              // 0: hit-matrix products (class join when a chunk has too many runs); 1: class join
    uint32_t warm = 64;
    uint32_t runs_per_lane = 0;
    uint32_t chunk_target = 131072;
    int prefix = 1;            // transformation-automaton walk of the first warm-up bytes
};

}  // namespace

struct ri_handle {
    ri::Automata A;
    AlgoHost algo[RI_NUM_ALGOS];
    std::mutex mu;
    DeviceCopy dev[kMaxDevices];
    std::vector<std::unique_ptr<Workspace>> ws;
    bool profiling = false;
    float last_ms[5] = {0, 0, 0, 0, 0};
    Options opt;
    bool tuned_valid[RI_NUM_ALGOS] = {false, false, false};
    Options tuned[RI_NUM_ALGOS];
};

namespace {

// Entries and byte codes are byte offsets: entry = next_state * K * eb, code[b]
// = class(b) * eb, so a step is one add and one load.  eb (1, 2 or 4 bytes)
// is the narrowest width that holds the dead row's offset n * K * eb.
void pack_table(AlgoHost &h, uint32_t n, uint32_t K, const std::vector<int32_t> &delta,
                const uint8_t cls[256]) {
    h.nstates = n;
    h.K = K;
    const uint64_t rows = (uint64_t)n * K;
    h.entry_bytes = rows <= 0xFF ? 1 : rows * 2 <= 0xFFFF ? 2 : 4;
    const uint32_t eb = h.entry_bytes;
    h.dead = (uint32_t)(rows * eb);
    const uint64_t entries = (uint64_t)(n + 1) * K;
    h.table.assign(round_up(entries * eb, 16), 0);
    auto put = [&](uint64_t i, uint32_t v) {
        if (eb == 1) h.table[i] = (uint8_t)v;
        else if (eb == 2) reinterpret_cast<uint16_t *>(h.table.data())[i] = (uint16_t)v;
        else reinterpret_cast<uint32_t *>(h.table.data())[i] = v;
    };
    for (uint32_t s = 0; s <= n; ++s)
        for (uint32_t k = 0; k < K; ++k) {
            int32_t t = s < n ? delta[(size_t)s * K + k] : -1;
            put((uint64_t)s * K + k, t < 0 ? h.dead : (uint32_t)t * K * eb);
        }
    for (int b = 0; b < 256; ++b) h.code[b] = (uint16_t)(cls[b] * eb);
    h.lam_bytes = n < 0xFFFF ? 2 : 4;
    // sinks: every class leads back to the state (e.g. the state after a
    // match of .*(...).*); the first two found are passed to the kernels
    h.sink[0] = h.sink[1] = 0xFFFFFFFFu;
    uint32_t ns = 0;
    for (uint32_t s = 0; s < n && ns < 2; ++s) {
        bool sink = K > 0;
        for (uint32_t k = 0; k < K && sink; ++k) sink = delta[(size_t)s * K + k] == (int32_t)s;
        if (sink) h.sink[ns++] = s * K * eb;
    }
}

// Breadth-first expansion of the transformation automaton: its root is the
// vector of the start states, and class c maps a vector v to (delta(v[s], c))_s.
// Level d holds the vectors of the words of exactly d bytes.  Levels are
// added while the states stay within the cap (and the work n K L, and the
// level visits, within a budget); a level that would cross the cap is dropped
// whole, so every word of up to `depth` bytes ends in a state whose
// transitions below that depth exist.
constexpr uint32_t kPrefixCap = 65535;   // ids are u16, 0xFFFF marks a transition not expanded
constexpr uint64_t kPrefixWork = 1ull << 27;
constexpr uint32_t kPrefixMaxDepth = 64;

void build_prefix(AlgoHost &H) {
    PrefixHost &P = H.prefix;
    P = PrefixHost{};
    if (H.nfa || H.L == 0 || H.L > 256 || H.nstates >= 0xFFFF) return;
    const uint32_t K = H.K, L = H.L, eb = H.entry_bytes, rb = K * eb;
    const uint32_t dead = H.dead / rb;
    const uint64_t cap64 = std::min<uint64_t>(kPrefixCap, kPrefixWork / ((uint64_t)K * L));
    if (cap64 < 2) return;
    const uint32_t cap = (uint32_t)cap64;
    // transitions by state id (the dead row included)
    std::vector<uint16_t> tr((size_t)(H.nstates + 1) * K);
    for (uint32_t q = 0; q <= H.nstates; ++q)
        for (uint32_t c = 0; c < K; ++c) {
            const size_t off = (size_t)q * rb + (size_t)c * eb;
            uint32_t e = 0;
            for (uint32_t i = 0; i < eb; ++i) e |= (uint32_t)H.table[off + i] << (8 * i);
            tr[(size_t)q * K + c] = (uint16_t)(e / rb);
        }
    std::vector<uint16_t> vec;                 // [n][L]
    uint32_t hcap = 1;
    while (hcap < 2 * cap) hcap *= 2;
    std::vector<uint32_t> slot(hcap, 0xFFFFFFFFu);
    auto hash = [&](const uint16_t *v) {
        uint64_t x = 1469598103934665603ull;
        for (uint32_t s = 0; s < L; ++s) x = (x ^ v[s]) * 1099511628211ull;
        return (uint32_t)(x ^ (x >> 29));
    };
    uint32_t n = 0;
    // id of v, added when new; 0xFFFFFFFF when the cap is reached
    auto find_or_add = [&](const uint16_t *v) -> uint32_t {
        uint32_t i = hash(v) & (hcap - 1);
        while (slot[i] != 0xFFFFFFFFu) {
            if (std::memcmp(&vec[(size_t)slot[i] * L], v, (size_t)L * 2) == 0) return slot[i];
            i = (i + 1) & (hcap - 1);
        }
        if (n >= cap) return 0xFFFFFFFFu;
        slot[i] = n;
        vec.insert(vec.end(), v, v + L);
        return n++;
    };
    std::vector<uint16_t> v(L);
    for (uint32_t s = 0; s < L; ++s) v[s] = (uint16_t)(H.starts[s] / rb);
    find_or_add(v.data());
    std::vector<uint16_t> next;                // grows with n
    std::vector<uint8_t> expanded;
    std::vector<uint32_t> level{0}, nlevel, stamp;
    uint32_t depth = 0;
    uint64_t lwork = 0;                        // level x class visits, bounded like the expansion
    for (uint32_t d = 0; d < kPrefixMaxDepth; ++d) {
        const uint32_t n0 = n;
        const size_t vec0 = vec.size();
        std::vector<uint32_t> fresh;           // states expanded in this level
        bool over = false;
        nlevel.clear();
        stamp.resize(cap, 0);
        for (uint32_t f : level) {
            if (f < expanded.size() && expanded[f]) continue;
            if (next.size() < (size_t)(f + 1) * K) next.resize((size_t)(f + 1) * K, 0xFFFF);
            if (expanded.size() < (size_t)f + 1) expanded.resize((size_t)f + 1, 0);
            for (uint32_t c = 0; c < K && !over; ++c) {
                for (uint32_t s = 0; s < L; ++s) v[s] = tr[(size_t)vec[(size_t)f * L + s] * K + c];
                const uint32_t g = find_or_add(v.data());
                if (g == 0xFFFFFFFFu) over = true;
                else next[(size_t)f * K + c] = (uint16_t)g;
            }
            expanded[f] = 1;
            fresh.push_back(f);
            if (over) break;
        }
        if (over) {
            // undo the level: its new states and transitions are never reached
            for (uint32_t f : fresh) {
                expanded[f] = 0;
                for (uint32_t c = 0; c < K; ++c) next[(size_t)f * K + c] = 0xFFFF;
            }
            n = n0;
            vec.resize(vec0);
            break;
        }
        for (uint32_t f : level)
            for (uint32_t c = 0; c < K; ++c) {
                const uint32_t g = next[(size_t)f * K + c];
                if (stamp[g] != d + 1) { stamp[g] = d + 1; nlevel.push_back(g); }
            }
        level.swap(nlevel);
        depth = d + 1;
        lwork += (uint64_t)level.size() * K;
        if (lwork > kPrefixWork) break;
    }
    if (depth == 0) return;
    P.depth = depth;
    P.n = n;
    next.resize((size_t)n * K, 0xFFFF);
    P.next = std::move(next);
    P.count.assign(n, 0);
    P.tgt.assign((size_t)n * 64, 0);
    P.map.assign((size_t)n * L, 0xFF);
    std::vector<int32_t> where(H.nstates + 1, -1);
    for (uint32_t f = 0; f < n; ++f) {
        const uint16_t *x = &vec[(size_t)f * L];
        uint32_t cnt = 0;
        bool wide = false;
        for (uint32_t s = 0; s < L && !wide; ++s) {
            const uint32_t q = x[s];
            if (q == dead) continue;
            if (where[q] < 0) {
                if (cnt == 64) { wide = true; break; }
                where[q] = (int32_t)cnt;
                P.tgt[(size_t)f * 64 + cnt++] = (uint16_t)q;
            }
            P.map[(size_t)f * L + s] = (uint8_t)where[q];
        }
        for (uint32_t i = 0; i < cnt; ++i) where[P.tgt[(size_t)f * 64 + i]] = -1;
        P.count[f] = wide ? ri::kPrefixWide : (uint8_t)cnt;
    }
}

void pack_all(ri_handle *h) {
    const ri::Automata &A = h->A;
    if (A.empty_language) return;
    const uint32_t K = A.K;

    // RI_ALGO_RID: B' with the singletons of N' as starts; relational join
    AlgoHost &r = h->algo[RI_ALGO_RID];
    pack_table(r, A.Bq.n, K, A.Bq.delta, A.cls);
    r.relational = true;
    r.L = A.nq.n;
    uint32_t W = 1;
    while (W * 32 < r.L) W *= 2;
    r.W = W;
    r.starts.resize(r.L);
    for (uint32_t q = 0; q < r.L; ++q) r.starts[q] = A.Bq.initial[q] * K * r.entry_bytes;
    if (W <= kMaxDenseWords) {
        r.content.assign((size_t)A.Bq.n * W, 0);
        for (uint32_t p = 0; p < A.Bq.n; ++p)
            for (uint32_t q : A.Bq.content[p]) r.content[(size_t)p * W + q / 32] |= 1u << (q % 32);
    }
    r.csr_off.assign(A.Bq.n + 1, 0);
    for (uint32_t p = 0; p < A.Bq.n; ++p) {
        r.csr_off[p + 1] = r.csr_off[p] + (uint32_t)A.Bq.content[p].size();
        r.csr_idx.insert(r.csr_idx.end(), A.Bq.content[p].begin(), A.Bq.content[p].end());   // ascending
    }
    r.fmask.assign(W, 0);
    for (uint32_t q = 0; q < A.nq.n; ++q)
        if (A.nq.final[q]) r.fmask[q / 32] |= 1u << (q % 32);
    uint32_t nkeys = 0;
    for (uint32_t p = 0; p < A.Bq.n; ++p) nkeys += A.final_id[p] >= 0;
    uint32_t cap = 1;
    while (cap < 2 * nkeys + 2) cap *= 2;
    r.hash_cap = cap;
    r.hash.assign((size_t)cap * 2, 0xFFFFFFFFu);
    for (uint32_t p = 0; p < A.Bq.n; ++p) {
        if (A.final_id[p] < 0) continue;
        uint32_t slot = hash_members(A.Bq.content[p]) & (cap - 1);
        while (r.hash[(size_t)slot * 2] != 0xFFFFFFFFu) slot = (slot + 1) & (cap - 1);
        r.hash[(size_t)slot * 2] = p;
        r.hash[(size_t)slot * 2 + 1] = (uint32_t)A.final_id[p];
    }

    // RI_ALGO_DFA: minimal DFA, all states as starts; functional join
    AlgoHost &d = h->algo[RI_ALGO_DFA];
    pack_table(d, A.dmin_n, K, A.dmin_delta, A.cls);
    d.L = A.dmin_n;
    d.starts.resize(d.L);
    for (uint32_t s = 0; s < d.L; ++s) d.starts[s] = s * K * d.entry_bytes;
    d.final_of_state.resize(d.L);
    d.accept_of_state.resize(d.L);
    for (uint32_t s = 0; s < d.L; ++s) {
        d.final_of_state[s] = (int32_t)s;
        d.accept_of_state[s] = A.dmin_final[s];
    }

    // RI_ALGO_SUBSET: powerset DFA of N, all states as starts
    AlgoHost &u = h->algo[RI_ALGO_SUBSET];
    pack_table(u, A.dsub_n, K, A.dsub_delta, A.cls);
    u.L = A.dsub_n;
    u.starts.resize(u.L);
    for (uint32_t s = 0; s < u.L; ++s) u.starts[s] = s * K * u.entry_bytes;
    u.final_of_state = A.dsub_final_id;
    u.accept_of_state = A.dsub_accept;

    // RI_ALGO_NFA: N itself over sets of states, every state a start; the
    // set reached from q0 is a state of the powerset DFA, found by the hash
    // of its members
    AlgoHost &v = h->algo[RI_ALGO_NFA];
    v.nfa = true;
    v.L = A.nfa_states;
    v.K = K;
    v.nfa_words = A.nfa_words;
    if (v.nfa_words) {
        v.W = 2 * v.nfa_words;
        v.follow = A.nfa_follow;
        v.mask = A.nfa_mask;
        v.fmask.assign(v.W, 0);
        for (uint32_t q = 0; q < A.pos.n; ++q)
            if (A.pos.final[q]) v.fmask[q / 32] |= 1u << (q % 32);
        v.csr_off.assign(A.dsub_n + 1, 0);
        for (uint32_t t = 0; t < A.dsub_n; ++t) {
            v.csr_off[t + 1] = v.csr_off[t] + (uint32_t)A.dsub_content[t].size();
            v.csr_idx.insert(v.csr_idx.end(), A.dsub_content[t].begin(), A.dsub_content[t].end());
        }
        uint32_t cap = 1;
        while (cap < 2 * A.dsub_n + 2) cap *= 2;
        v.hash_cap = cap;
        v.hash.assign((size_t)cap * 2, 0xFFFFFFFFu);
        for (uint32_t t = 0; t < A.dsub_n; ++t) {
            uint32_t slot = hash_members(A.dsub_content[t]) & (cap - 1);
            while (v.hash[(size_t)slot * 2] != 0xFFFFFFFFu) slot = (slot + 1) & (cap - 1);
            v.hash[(size_t)slot * 2] = t;
            v.hash[(size_t)slot * 2 + 1] = (uint32_t)A.dsub_final_id[t];
        }
    }
    for (int a : {RI_ALGO_RID, RI_ALGO_DFA, RI_ALGO_SUBSET}) build_prefix(h->algo[a]);
}

// Zero device memory and wait for it: the memset runs on the null stream,
// which does not order it before kernels on non-blocking streams.
hipError_t zero_now(void *p, size_t bytes) {
    hipError_t e = hipMemset(p, 0, bytes);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    return e;
}

template <typename T>
hipError_t upload(T **dst, const void *src, size_t bytes) {
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), bytes ? bytes : 16);
    if (e != hipSuccess) return e;
    if (bytes == 0 || !src) return zero_now(*dst, bytes ? bytes : 16);
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e__ = (expr);                                                           \
        if (e__ != hipSuccess)                                                             \
            return fail(e__ == hipErrorOutOfMemory ? RI_ERR_NOMEM : RI_ERR_DEVICE,         \
                        std::string(#expr) + ": " + hipGetErrorString(e__));               \
    } while (0)

int ensure_device(ri_handle *h, int device) {
    DeviceCopy &dc = h->dev[device];
    if (dc.ready) return RI_OK;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    dc.cus = prop.multiProcessorCount;
    dc.max_lds = prop.sharedMemPerBlock;
    HIP_TRY(upload(&dc.cls, h->A.cls, 256));
    for (int a = 0; a < RI_NUM_ALGOS; ++a) {
        const AlgoHost &H = h->algo[a];
        AlgoDevice &D = dc.algo[a];
        HIP_TRY(upload(&D.table, H.table.data(), H.table.size()));
        HIP_TRY(upload(&D.code, H.code, sizeof(H.code)));
        HIP_TRY(upload(&D.starts, H.starts.data(), H.starts.size() * 4));
        if (H.prefix.depth) {
            const PrefixHost &P = H.prefix;
            HIP_TRY(upload(&D.pfx_next, P.next.data(), P.next.size() * 2));
            HIP_TRY(upload(&D.pfx_count, P.count.data(), P.count.size()));
            HIP_TRY(upload(&D.pfx_tgt, P.tgt.data(), P.tgt.size() * 2));
            HIP_TRY(upload(&D.pfx_map, P.map.data(), P.map.size()));
        }
        if (H.nfa) {
            HIP_TRY(upload(&D.follow, H.follow.data(), H.follow.size() * 8));
            HIP_TRY(upload(&D.mask, H.mask.data(), H.mask.size() * 8));
            HIP_TRY(upload(&D.csr_off, H.csr_off.data(), H.csr_off.size() * 4));
            HIP_TRY(upload(&D.csr_idx, H.csr_idx.data(), H.csr_idx.size() * 4));
            HIP_TRY(upload(&D.fmask, H.fmask.data(), H.fmask.size() * 4));
            HIP_TRY(upload(&D.hash, H.hash.data(), H.hash.size() * 4));
        } else if (H.relational) {
            HIP_TRY(upload(&D.content, H.content.data(), H.content.size() * 4));
            HIP_TRY(upload(&D.csr_off, H.csr_off.data(), H.csr_off.size() * 4));
            HIP_TRY(upload(&D.csr_idx, H.csr_idx.data(), H.csr_idx.size() * 4));
            HIP_TRY(upload(&D.fmask, H.fmask.data(), H.fmask.size() * 4));
            HIP_TRY(upload(&D.hash, H.hash.data(), H.hash.size() * 4));
        } else {
            HIP_TRY(upload(&D.final_of_state, H.final_of_state.data(), H.final_of_state.size() * 4));
            HIP_TRY(upload(&D.accept_of_state, H.accept_of_state.data(), H.accept_of_state.size()));
        }
    }
    dc.ready = true;
    return RI_OK;
}

int get_workspace(ri_handle *h, int device, hipStream_t stream, Workspace **out) {
    for (auto &w : h->ws)
        if (w->device == device && w->stream == stream) { *out = w.get(); return RI_OK; }
    auto w = std::make_unique<Workspace>();
    w->device = device;
    w->stream = stream;
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(&w->counters), 64));
    HIP_TRY(zero_now(w->counters, 64));
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(&w->dres), 16));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&w->hres), 16, hipHostMallocDefault));
    for (auto &e : w->ev) HIP_TRY(hipEventCreate(&e));
    *out = w.get();
    h->ws.push_back(std::move(w));
    return RI_OK;
}

// Grows b to at least `need` bytes (geometrically, so the retired buffers
// of one owner add up to less than its live ones).  The old buffer goes to
// `retired`, or is freed at once when retired is null (the caller knows
// that nothing in flight uses it).
int grow(Buf &b, size_t need, std::vector<void *> *retired) {
    if (need <= b.cap) return RI_OK;
    need = round_up(std::max<size_t>(need, b.cap + b.cap / 2), 1 << 20);
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, need));
    if (b.p) {
        if (retired) retired->push_back(b.p);
        else (void)hipFree(b.p);
    }
    b.p = p;
    b.cap = need;
    return RI_OK;
}

struct Plan {
    uint64_t cs = 0;
    uint32_t nchunks = 0;
};

// Automatic chunk sizes of 2 KiB and more are odd multiples of 128 bytes.
// The runs of a wave read their chunks in lockstep, and chunk starts a large
// power of two apart fall into the same L2 sets and channels: with 8 KiB
// chunks of the 1 GiB log text the long-run kernel fetched 1.46 times the
// text from HBM, with 8320-byte chunks 1.02 times.
uint64_t spread_chunk(uint64_t cs) {
    if (cs < 2048) return cs;
    cs = round_up(cs, 128);
    return (cs / 128) % 2 == 0 ? cs + 128 : cs;
}

int plan_chunks(const AlgoHost &H, uint64_t n, uint32_t chunks, uint32_t target, Plan *p) {
    uint64_t cs;
    if (chunks == 0) {
        cs = std::max<uint64_t>(round_up((n + target - 1) / target, 16), kMinAutoChunk);
        while ((uint64_t)H.L * ((n + cs - 1) / cs) > kMaxAutoPairs) cs *= 2;
        cs = spread_chunk(cs);
    } else {
        cs = round_up((n + chunks - 1) / chunks, 16);
        if ((uint64_t)H.L * ((n + cs - 1) / cs) * H.lam_bytes > kMaxLamBytes)
            return fail(RI_ERR_LIMIT, "chunk maps for this chunk count exceed the device budget");
    }
    if (cs < 16) cs = 16;
    uint64_t nc = (n + cs - 1) / cs;
    if (nc > 0x7fffffffull) return fail(RI_ERR_LIMIT, "too many chunks");
    p->cs = cs;
    p->nchunks = (uint32_t)nc;
    return RI_OK;
}

ri::KernelShape base_shape(const AlgoHost &H, const DeviceCopy &dc) {
    ri::KernelShape shape;
    shape.entry_bytes = (int)H.entry_bytes;
    shape.tile_bytes = (int)H.lam_bytes;
    shape.alias_bytes = H.L <= 254 ? 1 : 2;
    shape.runs_per_lane = 1;
    shape.block_threads = 1024;
    shape.table_in_lds = H.table.size() + ri::kCodeLdsBytes <= dc.max_lds;
    return shape;
}

// Launch configuration of the converging reach over `nchunks` chunks.
struct ConvCfg {
    ri::KernelShape warm_shape, long_shape;
    size_t lds_w = 0, lds_l = 0;
    int grid_w = 1, grid_l = 1;
    uint64_t run_cap = 0;   // run slots of all warm-up blocks' regions
    uint32_t cpi = ri::kWarmChunksPerBlock;   // chunks per warm-up block iteration
};

int conv_config(const AlgoHost &H, const DeviceCopy &dc, const Options &opt, uint32_t nchunks, ConvCfg *c) {
    if (H.L > 65534) return fail(RI_ERR_LIMIT, "too many starts for the converging reach");
    const ri::KernelShape shape = base_shape(H, dc);
    const size_t lds_tables = H.table.size() + ri::kCodeLdsBytes;
    // warm-up: starts held 64 per lane register, up to 4 registers per lane
    c->warm_shape = shape;
    c->warm_shape.runs_per_lane = H.L <= 64 ? 1 : H.L <= 128 ? 2 : 4;
    c->warm_shape.code_regs = opt.warm <= 64 ? 1 : 4;   // registers of 64 warm-up byte codes
    // merging by hashing when the starts fit one block of 64 R starts; a
    // wave then takes several chunks at a time
    c->warm_shape.hashed = H.L <= 64u * (uint32_t)c->warm_shape.runs_per_lane;
    // and through a table indexed by state when a byte per state fits
    c->warm_shape.direct = c->warm_shape.hashed && ri::warm_direct_fits(H.nstates);
    c->cpi = ri::kWarmChunksPerBlock *
             ri::warm_chunks_per_wave(c->warm_shape.hashed, c->warm_shape.direct, c->warm_shape.runs_per_lane,
                                       c->warm_shape.code_regs);
    c->lds_w = ri::warm_lds_bytes(c->warm_shape, (uint32_t)H.table.size(), H.L);
    if (c->lds_w > dc.max_lds) {   // table and starts do not fit together: table from global memory
        c->warm_shape.table_in_lds = false;
        c->lds_w = ri::warm_lds_bytes(c->warm_shape, (uint32_t)H.table.size(), H.L);
    }
    const uint32_t iters = (nchunks + c->cpi - 1) / c->cpi;
    const int per_cu_w = std::max(1, ri::blocks_per_cu(1, c->warm_shape, c->lds_w));
    c->grid_w = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)dc.cus * per_cu_w, iters));
    c->run_cap = (uint64_t)iters * c->cpi * H.L;   // every block's region
    // long runs: one run per lane unless set; LDS also holds the prefix of
    // the warm-up blocks' run counts
    c->long_shape = shape;
    c->long_shape.runs_per_lane = (int)(opt.runs_per_lane ? opt.runs_per_lane : 1);
    const size_t pre = round_up(((size_t)c->grid_w + 1) * 4, 16);
    c->lds_l = (shape.table_in_lds ? lds_tables : ri::kCodeLdsBytes) + pre;
    if (c->lds_l > dc.max_lds) {
        c->long_shape.table_in_lds = false;
        c->lds_l = ri::kCodeLdsBytes + pre;
    }
    const uint64_t pairs = (uint64_t)H.L * nchunks;
    const int per_cu_l = std::max(1, ri::blocks_per_cu(2, c->long_shape, c->lds_l));
    const uint64_t max_jobs = (pairs + 64ull * c->long_shape.runs_per_lane - 1) / (64ull * c->long_shape.runs_per_lane);
    c->grid_l = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)dc.cus * per_cu_l, (max_jobs + 15) / 16));
    return RI_OK;
}

struct ReachBufs {
    void *alias;
    uint32_t *run_base, *run_chunk, *run_state, *run_final, *counters;
    uint32_t *run_count;
    uint32_t *block_count;   // [warm-up grid]
    ri::PrefixArgs pfx{};     // k = 0: no transformation-automaton walk
};

// The walk of the first warm-up bytes: every word of up to `depth` bytes is
// expanded; k is rounded down to a multiple of 8 (the rest of the warm-up then
// steps 8 bytes per broadcast of codes) and is at most the warm-up.  Starts
// that fit one register (64) step byte by byte: there a walk of dependent
// loads from L2 saves no lookups, it only adds their latency.
ri::PrefixArgs prefix_args(const AlgoHost &H, const AlgoDevice &D, const Options &opt) {
    ri::PrefixArgs p{};
    const uint32_t depth = H.prefix.depth;
    if (!opt.prefix || !opt.converge || depth == 0 || !D.pfx_next || H.L <= 64) return p;
    p.k = std::min<uint32_t>(depth >= 8 ? depth & ~7u : depth, opt.warm);
    p.next = D.pfx_next;
    p.count = D.pfx_count;
    p.tgt = D.pfx_tgt;
    p.map = D.pfx_map;
    p.K = H.K;
    p.shift = H.entry_bytes == 1 ? 0 : H.entry_bytes == 2 ? 1 : 2;
    return p;
}

ri::WarmArgs warm_args(const ConvCfg &c, const ri::ScanArgs &sa, const Options &opt, const ReachBufs &rb) {
    ri::WarmArgs wa{};
    wa.s = sa;
    wa.pfx = rb.pfx;
    wa.warm = opt.warm;
    wa.alias = rb.alias;
    wa.run_base = rb.run_base;
    wa.run_count = rb.run_count;
    wa.run_chunk = rb.run_chunk;
    wa.run_state = rb.run_state;
    wa.counters = rb.counters;
    wa.block_count = rb.block_count;
    wa.cpi = c.cpi;
    return wa;
}

// Warm-up and merging, then the merged runs to the chunk ends; `mid`
// (optional) is recorded between the two kernels.
int launch_conv(const ConvCfg &c, const ri::ScanArgs &sa, const Options &opt, const ReachBufs &rb,
                hipStream_t stream, hipEvent_t mid) {
    HIP_TRY(ri::launch_warm(warm_args(c, sa, opt, rb), c.warm_shape, c.grid_w, c.lds_w, stream));
    if (mid) HIP_TRY(hipEventRecord(mid, stream));
    ri::LongArgs la{};
    la.s = sa;
    la.warm = opt.warm;
    la.run_chunk = rb.run_chunk;
    la.run_state = rb.run_state;
    la.run_final = rb.run_final;
    la.block_count = rb.block_count;
    la.warm_blocks = (uint32_t)c.grid_w;
    la.cpi = c.cpi;
    HIP_TRY(ri::launch_long(la, c.long_shape, c.grid_l, c.lds_l, stream));
    return RI_OK;
}

// Members per group of the class-partitioned join: the widest power of two
// <= 64 whose LDS stays within 64 KiB; 0 if none does.
uint32_t cls_group(const AlgoHost &H, int alias_bytes) {
    ri::ClsJoinArgs ca{};
    ca.L = H.L;
    for (uint32_t gc = 64; gc >= 2; gc /= 2) {
        ca.G = gc;
        if (ri::cls_join_lds(ca, (int)H.W, alias_bytes) <= 65536) return gc;
    }
    return 0;
}

// Members per group of the staged level-0 join (functions or relations): the
// widest power of two <= 64 whose tile of chunk maps (L x G x 4 bytes) stays
// within 64 KiB; 0 = unstaged join.
uint32_t tile_group(const AlgoHost &H) {
    uint32_t g0 = 64;
    while (g0 > 0 && (size_t)H.L * g0 * 4 > 65536) g0 /= 2;
    return g0;
}

// Device scratch of one recognition call, taken from the stream's cached
// workspace or carved from a fixed arena (ri_recognize_noalloc).
struct Scratch {
    void *lam = nullptr, *alias = nullptr, *dbg = nullptr;
    uint32_t *run_base = nullptr, *run_count = nullptr, *run_chunk = nullptr, *run_state = nullptr;
    uint32_t *run_final = nullptr, *block_count = nullptr;
    void *join[2] = {nullptr, nullptr};
    uint32_t *ncls[2] = {nullptr, nullptr}, *hrows[2] = {nullptr, nullptr};
    uint64_t *hprod[2] = {nullptr, nullptr};
    uint32_t *counters = nullptr;   // [16], zero on entry
    int32_t *dres = nullptr;        // [4]
};

// Launch plan and scratch sizes of one call for a given chunking.
struct CallPlan {
    Plan plan;
    bool conv = false;
    ConvCfg cc;
    ri::KernelShape shape;
    uint32_t g0 = 0, ng0 = 0, gc = 0;
    bool hit = false, dense_join = false;
    size_t row_words = 1, pairs = 0, nh = 0, nrel_max = 0;
};

int plan_call(const AlgoHost &H, const DeviceCopy &dc, const Options &opt, const Plan &plan, CallPlan *cp) {
    cp->plan = plan;
    cp->conv = opt.converge != 0;
    if (!cp->conv && H.relational && H.W > kMaxDenseWords)
        return fail(RI_ERR_LIMIT, "the plain reach joins interfaces of at most 2048 states; use RI_OPT_CONVERGE = 1");
    cp->g0 = tile_group(H);
    cp->ng0 = (plan.nchunks + (cp->g0 ? cp->g0 : kJoinGroup) - 1) / (cp->g0 ? cp->g0 : kJoinGroup);
    cp->row_words = H.relational ? H.W : 1;
    cp->pairs = (size_t)H.L * plan.nchunks;
    cp->shape = base_shape(H, dc);
    if (cp->conv) {
        int rc = conv_config(H, dc, opt, plan.nchunks, &cp->cc);
        if (rc) return rc;
    }
    cp->nh = std::max<size_t>(1, (plan.nchunks + 62) / 64);   // level-0 hit products
    // join buffers of the dense joins (class join, relations, functions): at
    // most ceil(nchunks / 2) relations of L rows (or classes); the hit-matrix
    // join and the join by propagation do not use them
    const bool rel_conv = cp->conv && H.relational;
    cp->gc = rel_conv && H.W <= kMaxDenseWords ? cls_group(H, cp->shape.alias_bytes) : 0;
    cp->hit = rel_conv && (opt.join == 0 || cp->gc == 0);
    cp->dense_join = !rel_conv || cp->gc != 0;
    cp->nrel_max = std::max<size_t>(cp->ng0, (plan.nchunks + 1) / 2);
    return RI_OK;
}

// The buffers of a call in a fixed order: (pointer slot, bytes).
template <class F>
void for_each_buffer(const AlgoHost &H, const CallPlan &cp, bool maps, Scratch &sc, F &&f) {
    if (cp.conv) {
        f(reinterpret_cast<void **>(&sc.alias), cp.pairs * cp.shape.alias_bytes);
        f(reinterpret_cast<void **>(&sc.run_base), (size_t)cp.plan.nchunks * 4);
        f(reinterpret_cast<void **>(&sc.run_chunk), cp.cc.run_cap * 4);
        f(reinterpret_cast<void **>(&sc.run_state), cp.cc.run_cap * 4);
        f(reinterpret_cast<void **>(&sc.run_final), cp.cc.run_cap * 4);
        f(reinterpret_cast<void **>(&sc.run_count), (size_t)cp.plan.nchunks * 4);
        f(reinterpret_cast<void **>(&sc.block_count), (size_t)cp.cc.grid_w * 4);
        for (int i = 0; i < 2; ++i) {
            f(reinterpret_cast<void **>(&sc.hprod[i]), cp.nh * ri::kRowCap * 8);
            f(reinterpret_cast<void **>(&sc.hrows[i]), cp.nh * 4);
        }
    } else {
        f(reinterpret_cast<void **>(&sc.lam), cp.pairs * H.lam_bytes);
    }
    if (cp.dense_join) {
        for (int i = 0; i < 2; ++i) {
            f(reinterpret_cast<void **>(&sc.join[i]), cp.nrel_max * H.L * cp.row_words * 4);
            f(reinterpret_cast<void **>(&sc.ncls[i]), cp.nrel_max * 4);
        }
    }
    if (maps) f(reinterpret_cast<void **>(&sc.dbg), cp.pairs * 4);
}

constexpr size_t kArenaAlign = 256;

// Bytes of the arena a call needs: counters and result, then every buffer.
size_t arena_bytes(const AlgoHost &H, const CallPlan &cp) {
    size_t total = 2 * kArenaAlign;
    Scratch tmp;
    for_each_buffer(H, cp, false, tmp, [&](void **, size_t bytes) { total += round_up(bytes ? bytes : 1, kArenaAlign); });
    return total;
}

}  // namespace

namespace ri {
// A fixed device region that a call carves its scratch from; the caller of
// recognize() provides it and guarantees that no other call uses it meanwhile.
struct Arena {
    uint8_t *base;
    size_t bytes;
};
}  // namespace ri

namespace {

// ---------------------------------------------------------------------------
// RI_ALGO_NFA: the position NFA as chunk automaton over sets of states
// ---------------------------------------------------------------------------

constexpr uint64_t kNfaMapBytes = 1ull << 29;   // chunk maps of one call

int nfa_plan(const AlgoHost &H, uint64_t n, uint32_t chunks, uint32_t target, Plan *p) {
    const uint64_t row = (uint64_t)H.L * H.nfa_words * 8;   // one chunk's map
    uint64_t cs;
    if (chunks == 0) {
        cs = std::max<uint64_t>(round_up((n + target - 1) / target, 16), kMinAutoChunk);
        while (((n + cs - 1) / cs) * row > kNfaMapBytes) cs *= 2;
        cs = spread_chunk(cs);
    } else {
        cs = round_up((n + chunks - 1) / chunks, 16);
        if (((n + cs - 1) / cs) * row > kNfaMapBytes)
            return fail(RI_ERR_LIMIT, "NFA chunk maps for this chunk count exceed the device budget");
    }
    const uint64_t nc = (n + cs - 1) / cs;
    if (nc * H.L > 0x7fffffffull) return fail(RI_ERR_LIMIT, "too many chunks");
    p->cs = cs;
    p->nchunks = (uint32_t)nc;
    return RI_OK;
}

// Scratch of an NFA call: maps [c][L][W] and two join buffers of
// ceil(c / 64) relations.
void nfa_buffer_sizes(const AlgoHost &H, const Plan &plan, size_t *maps, size_t *join) {
    const size_t row = (size_t)H.L * H.nfa_words * 8;
    *maps = (size_t)plan.nchunks * row;
    *join = (size_t)((plan.nchunks + 63) / 64) * row;
}

size_t nfa_arena_bytes(const AlgoHost &H, const Plan &plan) {
    size_t m, j;
    nfa_buffer_sizes(H, plan, &m, &j);
    return 2 * kArenaAlign + round_up(m, kArenaAlign) + 2 * round_up(j, kArenaAlign);
}

int recognize_nfa(ri_handle *h, const AlgoHost &H, const DeviceCopy &dc, const AlgoDevice &D, const uint8_t *text,
                  size_t n, hipStream_t stream, const Plan &plan, Workspace *ws, const ri::Arena *arena,
                  int32_t *result_dev, ri_result *out) {
    size_t mbytes, jbytes;
    nfa_buffer_sizes(H, plan, &mbytes, &jbytes);
    uint64_t *maps, *join[2];
    uint32_t *counters;
    int32_t *dres;
    if (arena) {
        uint8_t *p = arena->base;
        counters = reinterpret_cast<uint32_t *>(p);
        dres = reinterpret_cast<int32_t *>(p + kArenaAlign);
        p += 2 * kArenaAlign;
        maps = reinterpret_cast<uint64_t *>(p);
        p += round_up(mbytes, kArenaAlign);
        join[0] = reinterpret_cast<uint64_t *>(p);
        p += round_up(jbytes, kArenaAlign);
        join[1] = reinterpret_cast<uint64_t *>(p);
        HIP_TRY(ri::launch_zero_words(counters, 16, stream));
    } else {
        int rc = grow(ws->lam, mbytes, &ws->retired);
        if (!rc) rc = grow(ws->join[0], jbytes, &ws->retired);
        if (!rc) rc = grow(ws->join[1], jbytes, &ws->retired);
        if (rc) return rc;
        maps = static_cast<uint64_t *>(ws->lam.p);
        join[0] = static_cast<uint64_t *>(ws->join[0].p);
        join[1] = static_cast<uint64_t *>(ws->join[1].p);
        counters = ws->counters;
        dres = ws->dres;
    }
    const bool prof = h->profiling && !result_dev;
    if (prof) HIP_TRY(hipEventRecord(ws->ev[0], stream));
    ri::NfaArgs na{};
    na.text = text;
    na.n = n;
    na.cs = plan.cs;
    na.nchunks = plan.nchunks;
    na.follow = D.follow;
    na.mask = D.mask;
    na.cls = dc.cls;
    na.L = H.L;
    na.K = H.K;
    na.W = H.nfa_words;
    na.maps = maps;
    na.job_counter = counters + 3;
    na.chunk_groups = (plan.nchunks + 63) / 64;
    na.njobs = H.L * na.chunk_groups;
    // 256-thread blocks, 8 per CU, persistent over the jobs
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)dc.cus * 8, (na.njobs + 3) / 4));
    HIP_TRY(ri::launch_nfa_reach(na, grid, stream));
    if (prof) {
        HIP_TRY(hipEventRecord(ws->ev[4], stream));
        HIP_TRY(hipEventRecord(ws->ev[1], stream));
    }
    const uint64_t *total = maps;
    uint32_t nin = plan.nchunks;
    int cur = 0;
    while (nin > 1) {
        ri::NfaJoinArgs ja{total, nin, join[cur], H.L, H.nfa_words, kJoinGroup};
        HIP_TRY(ri::launch_nfa_join(ja, stream));
        total = join[cur];
        cur ^= 1;
        nin = (nin + kJoinGroup - 1) / kJoinGroup;
    }
    ri::FinalArgs fa{};
    fa.fmask = D.fmask;
    fa.hash = D.hash;
    fa.hash_cap = H.hash_cap;
    fa.csr_off = D.csr_off;
    fa.csr_idx = D.csr_idx;
    fa.result = result_dev ? result_dev : dres;
    fa.counters = counters;
    HIP_TRY(ri::launch_nfa_final(fa, total, H.nfa_words, nullptr, stream));
    out->chunks = plan.nchunks;
    out->chunk_size = (uint32_t)plan.cs;
    if (result_dev) {
        out->accept = -1;
        out->final_state = -1;
        return RI_OK;
    }
    if (prof) HIP_TRY(hipEventRecord(ws->ev[2], stream));
    HIP_TRY(hipMemcpyAsync(ws->hres, ws->dres, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    if (prof) HIP_TRY(hipEventRecord(ws->ev[3], stream));
    HIP_TRY(hipStreamSynchronize(stream));
    out->accept = ws->hres[0];
    out->final_state = ws->hres[1];
    if (out->final_state == -3) return fail(RI_ERR_DEVICE, "internal: final subset not found");
    if (prof) {
        float ms[5] = {0, 0, 0, 0, 0};
        HIP_TRY(hipEventElapsedTime(&ms[0], ws->ev[0], ws->ev[1]));
        HIP_TRY(hipEventElapsedTime(&ms[1], ws->ev[1], ws->ev[2]));
        HIP_TRY(hipEventElapsedTime(&ms[2], ws->ev[0], ws->ev[3]));
        HIP_TRY(hipEventElapsedTime(&ms[3], ws->ev[0], ws->ev[4]));
        std::lock_guard<std::mutex> lk(h->mu);
        std::memcpy(h->last_ms, ms, sizeof(ms));
    }
    return RI_OK;
}

// result_dev != nullptr: everything is enqueued on the stream and the
// result is left in result_dev[0..1]; no host wait, no profiling, no maps.
// arena != nullptr (with result_dev): scratch is carved from the arena, the
// chunk count is lowered until it fits, and nothing is allocated.
int recognize(const ri_handle *hc, const uint8_t *text, size_t n, void *stream_v, int algo,
              uint32_t chunks, ri_result *out, int32_t *maps, size_t maps_cap, int32_t *result_dev = nullptr,
              const ri::Arena *arena = nullptr) {
    ri_handle *h = const_cast<ri_handle *>(hc);
    if (!h || !out) return fail(RI_ERR_ARG, "NULL handle or result pointer");
    if (result_dev && (reinterpret_cast<uintptr_t>(result_dev) & 3))
        return fail(RI_ERR_ARG, "result must be 4-byte aligned");
    if (arena && (!result_dev || maps)) return fail(RI_ERR_ARG, "internal: arena calls are queued calls");
    if (algo < 0 || algo >= RI_NUM_ALGOS) return fail(RI_ERR_ARG, "unknown algorithm");
    if (n > 0 && !text) return fail(RI_ERR_ARG, "NULL text pointer");
    if (n > 0 && (reinterpret_cast<uintptr_t>(text) & 15)) return fail(RI_ERR_ARG, "text must be 16-byte aligned");
    std::memset(out, 0, sizeof(*out));
    out->n = n;
    const ri::Automata &A = h->A;
    if (n == 0 || A.empty_language) {
        out->accept = (n == 0 && !A.empty_language && A.accepts_empty) ? 1 : 0;
        out->final_state = (n == 0 && !A.empty_language) ? 0 : -1;
        if (maps && maps_cap > 0) std::memset(maps, 0xff, sizeof(int32_t) * maps_cap);
        if (result_dev) {
            hipError_t e = ri::launch_store_result(result_dev, out->accept, out->final_state,
                                                   reinterpret_cast<hipStream_t>(stream_v));
            if (e != hipSuccess) return fail(RI_ERR_DEVICE, std::string("store result: ") + hipGetErrorString(e));
        }
        return RI_OK;
    }
    const AlgoHost &H = h->algo[algo];
    if (H.nfa && maps) return fail(RI_ERR_ARG, "RI_ALGO_NFA: chunk maps are sets of NFA states, not state ids");
    if (H.nfa && !H.nfa_words) return fail(RI_ERR_LIMIT, "RI_ALGO_NFA: the NFA has more than 256 states");
    if (H.relational && H.W > ri::kPropMaxWords)
        return fail(RI_ERR_LIMIT, "interface larger than 32768 states is not supported by the device join");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    if (device < 0 || device >= kMaxDevices) return fail(RI_ERR_DEVICE, "device index out of range");

    Options opt;
    uint32_t target = h->opt.chunk_target;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        if (chunks == 0 && h->tuned_valid[algo]) target = h->tuned[algo].chunk_target;
        opt = (chunks == 0 && h->tuned_valid[algo]) ? h->tuned[algo] : h->opt;
    }
    Plan plan;
    int rc = H.nfa ? nfa_plan(H, n, chunks, target, &plan) : plan_chunks(H, n, chunks, target, &plan);
    if (rc) return rc;
    if (maps && maps_cap < (size_t)plan.nchunks * H.L)
        return fail(RI_ERR_ARG, "maps buffer too small");

    Workspace *ws = nullptr;
    std::unique_lock<std::mutex> wlk;
    if (arena) {
        std::lock_guard<std::mutex> lk(h->mu);
        if (!h->dev[device].ready)
            return fail(RI_ERR_ARG, "the handle's tables are not on the current device yet: make one "
                                    "ri_recognize* call on this device first");
    } else {
        std::lock_guard<std::mutex> lk(h->mu);
        rc = ensure_device(h, device);
        if (rc) return rc;
        rc = get_workspace(h, device, stream, &ws);
        if (rc) return rc;
    }
    if (ws) wlk = std::unique_lock<std::mutex>(ws->mu);
    DeviceCopy &dc = h->dev[device];
    const AlgoDevice &D = dc.algo[algo];
    const bool prof = h->profiling && !result_dev;

    if (H.nfa) {
        if (arena) {
            while (nfa_arena_bytes(H, plan) > arena->bytes) {
                if (chunks != 0 || plan.nchunks <= 1)
                    return fail(RI_ERR_LIMIT, "the text does not fit the fixed scratch memory with this chunk count "
                                              "(" + std::to_string(nfa_arena_bytes(H, plan)) + " bytes needed, " +
                                              std::to_string(arena->bytes) + " available)");
                rc = nfa_plan(H, n, 0, std::max<uint32_t>(1, plan.nchunks / 2), &plan);
                if (rc) return rc;
            }
        }
        return recognize_nfa(h, H, dc, D, text, n, stream, plan, ws, arena, result_dev, out);
    }
    CallPlan cp;
    rc = plan_call(H, dc, opt, plan, &cp);
    if (rc) return rc;
    Scratch sc;
    if (arena) {
        // fewer, longer chunks until the call fits the arena
        while (arena_bytes(H, cp) > arena->bytes) {
            if (chunks != 0 || plan.nchunks <= 1)
                return fail(RI_ERR_LIMIT, "the text does not fit the fixed scratch memory with this chunk count "
                                          "(" + std::to_string(arena_bytes(H, cp)) + " bytes needed, " +
                                          std::to_string(arena->bytes) + " available)");
            target = std::max<uint32_t>(1, plan.nchunks / 2);
            rc = plan_chunks(H, n, 0, target, &plan);
            if (!rc) rc = plan_call(H, dc, opt, plan, &cp);
            if (rc) return rc;
        }
        uint8_t *p = arena->base;
        sc.counters = reinterpret_cast<uint32_t *>(p);
        sc.dres = reinterpret_cast<int32_t *>(p + kArenaAlign);
        p += 2 * kArenaAlign;
        for_each_buffer(H, cp, false, sc, [&](void **slot, size_t bytes) {
            *slot = p;
            p += round_up(bytes ? bytes : 1, kArenaAlign);
        });
        // the counters start at zero (a fill kernel: capturable, unlike a memset)
        HIP_TRY(ri::launch_zero_words(sc.counters, 16, stream));
    } else {
        // the workspace buffer that backs each scratch pointer
        const std::pair<void *, Buf *> backing[] = {
            {&sc.lam, &ws->lam}, {&sc.alias, &ws->alias}, {&sc.dbg, &ws->dbg}, {&sc.run_base, &ws->run_base},
            {&sc.run_count, &ws->run_count}, {&sc.run_chunk, &ws->run_chunk}, {&sc.run_state, &ws->run_state},
            {&sc.run_final, &ws->run_final}, {&sc.block_count, &ws->block_count}, {&sc.join[0], &ws->join[0]},
            {&sc.join[1], &ws->join[1]}, {&sc.ncls[0], &ws->ncls[0]}, {&sc.ncls[1], &ws->ncls[1]},
            {&sc.hrows[0], &ws->hrows[0]}, {&sc.hrows[1], &ws->hrows[1]}, {&sc.hprod[0], &ws->hprod[0]},
            {&sc.hprod[1], &ws->hprod[1]}};
        for_each_buffer(H, cp, maps != nullptr, sc, [&](void **slot, size_t bytes) {
            Buf *b = nullptr;
            for (const auto &e : backing)
                if (e.first == static_cast<void *>(slot)) b = e.second;
            if (!b) { rc = fail(RI_ERR_DEVICE, "internal: scratch slot without a buffer"); return; }
            if (!rc) rc = grow(*b, bytes, &ws->retired);
            *slot = b->p;
        });
        if (rc) return rc;
        sc.counters = ws->counters;
        sc.dres = ws->dres;
    }
    const bool conv = cp.conv;
    const ConvCfg &cc = cp.cc;
    ri::KernelShape shape = cp.shape;
    const uint32_t g0 = cp.g0, ng0 = cp.ng0, gc = cp.gc;
    const bool hit = cp.hit;
    const size_t pairs = cp.pairs;
    uint32_t R = opt.runs_per_lane ? opt.runs_per_lane : 4;
    const size_t lds_tables = H.table.size() + ri::kCodeLdsBytes;

    ri::ScanArgs sa{};
    sa.text = text;
    sa.n = n;
    sa.cs = plan.cs;
    sa.nchunks = plan.nchunks;
    sa.table = D.table;
    sa.table_bytes = (uint32_t)H.table.size();
    sa.code = D.code;
    sa.starts = D.starts;
    sa.L = H.L;
    sa.row_bytes = H.K * H.entry_bytes;
    sa.dead = H.dead;
    sa.sink0 = H.sink[0];
    sa.sink1 = H.sink[1];
    const uint32_t chunk_groups = (plan.nchunks + 63) / 64;

    if (prof) HIP_TRY(hipEventRecord(ws->ev[0], stream));
    if (!conv) {
        while (R > 1 && R / 2 >= H.L) R /= 2;
        shape.runs_per_lane = (int)R;
        const size_t lds = shape.table_in_lds ? lds_tables : ri::kCodeLdsBytes;
        ri::PlainArgs pa{};
        pa.s = sa;
        pa.lam = sc.lam;
        pa.job_counter = sc.counters + 3;
        pa.chunk_groups = chunk_groups;
        pa.njobs = ((H.L + R - 1) / R) * chunk_groups;
        const int per_cu = std::max(1, ri::blocks_per_cu(0, shape, lds));
        const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)dc.cus * per_cu, (pa.njobs + 15) / 16));
        HIP_TRY(ri::launch_plain(pa, shape, grid, lds, stream));
        if (prof) HIP_TRY(hipEventRecord(ws->ev[4], stream));
    } else {
        ReachBufs rb{sc.alias, sc.run_base, sc.run_chunk, sc.run_state, sc.run_final, sc.counters, sc.run_count,
                     sc.block_count, prefix_args(H, D, opt)};
        rc = launch_conv(cc, sa, opt, rb, stream, prof ? ws->ev[5] : nullptr);
        if (rc) return rc;
        if (prof) HIP_TRY(hipEventRecord(ws->ev[4], stream));
    }
    if (prof) HIP_TRY(hipEventRecord(ws->ev[1], stream));

    // join tree
    ri::JoinArgs ja{};
    ja.converged = conv;
    ja.lam = sc.lam;
    ja.alias = sc.alias;
    ja.run_base = sc.run_base;
    ja.run_final = sc.run_final;
    ja.tile_bytes = (int)H.lam_bytes;
    ja.alias_bytes = shape.alias_bytes;
    ja.nchunks = plan.nchunks;
    ja.content = D.content;
    ja.L = H.L;
    ja.G = kJoinGroup;
    ja.in = nullptr;
    ja.nin = 0;
    ja.out = sc.join[0];
    ri::FinalArgs fa{};
    fa.fmask = D.fmask;
    fa.hash = D.hash;
    fa.hash_cap = H.hash_cap;
    fa.csr_off = D.csr_off;
    fa.csr_idx = D.csr_idx;
    fa.content = H.relational && H.W <= kMaxDenseWords ? D.content : nullptr;
    fa.final_of_state = D.final_of_state;
    fa.accept_of_state = D.accept_of_state;
    fa.result = result_dev && !hit ? result_dev : sc.dres;   // the hit join needs result[2]
    fa.counters = sc.counters;

    // class-partitioned join for merged runs of a relational chunk automaton:
    // the group size is the widest power of two <= 64 whose LDS stays in 64 KiB
    ri::ClsJoinArgs ca{};
    ca.alias = sc.alias;
    ca.nchunks = plan.nchunks;
    ca.L = H.L;
    ca.run_base = ja.run_base;
    ca.run_final = ja.run_final;
    ca.content = D.content;
    auto cls_join = [&]() -> int {
        ca.G = gc;
        ca.nmembers = plan.nchunks;
        ca.span = 1;
        ca.ncls_in = nullptr;
        ca.cont_in = nullptr;
        ca.ncls_out = sc.ncls[0];
        ca.cont_out = static_cast<uint32_t *>(sc.join[0]);
        HIP_TRY(ri::launch_join_cls(ca, (int)H.W, shape.alias_bytes, true, stream));
        int cur = 0;
        uint32_t nm = (plan.nchunks + gc - 1) / gc;
        uint64_t span = gc;
        while (nm > 1) {
            ca.nmembers = nm;
            ca.span = span;
            ca.ncls_in = sc.ncls[cur];
            ca.cont_in = static_cast<const uint32_t *>(sc.join[cur]);
            ca.ncls_out = sc.ncls[cur ^ 1];
            ca.cont_out = static_cast<uint32_t *>(sc.join[cur ^ 1]);
            HIP_TRY(ri::launch_join_cls(ca, (int)H.W, shape.alias_bytes, false, stream));
            cur ^= 1;
            span *= gc;
            nm = (nm + gc - 1) / gc;
        }
        ca.cont_in = static_cast<const uint32_t *>(sc.join[cur]);
        HIP_TRY(ri::launch_finalize_cls(fa, ca, (int)H.W, shape.alias_bytes, stream));
        return RI_OK;
    };
    ri::HitArgs ha{};
    // queued calls: a result that a chunk with too many runs made invalid is
    // redone by the class join, whose kernels are enqueued behind the hit join
    // and return at once unless the flag is set (interfaces of at most 2048
    // states), or else by propagation inside the final kernel.  Its levels:
    // level 0, then level 1 in one launch whose last block takes the higher
    // levels (few groups) and the final step (a single launch when level 0 is
    // the only level); one launch per level when there are too many levels.
    const bool gated_cls = hit && result_dev && gc != 0;
    ri::ClsJoinAll all{};
    uint32_t gated_levels = 0;
    bool gated_tree = false;    // every level fits the launches above
    if (gated_cls) {
        ca.gate = sc.counters + 2;
        ca.G = gc;
        ca.nmembers = plan.nchunks;
        ca.span = 1;
        ca.ncls_in = nullptr;
        ca.cont_in = nullptr;
        ca.ncls_out = sc.ncls[0];
        ca.cont_out = static_cast<uint32_t *>(sc.join[0]);
        all.lv[gated_levels++] = ca;
        int cur = 0;
        uint32_t nm = (plan.nchunks + gc - 1) / gc;
        uint64_t span = gc;
        while (nm > 1 && gated_levels < ri::kMaxClsLevels) {
            ri::ClsJoinArgs l = ca;
            l.nmembers = nm;
            l.span = span;
            l.ncls_in = sc.ncls[cur];
            l.cont_in = static_cast<const uint32_t *>(sc.join[cur]);
            l.ncls_out = sc.ncls[cur ^ 1];
            l.cont_out = static_cast<uint32_t *>(sc.join[cur ^ 1]);
            all.lv[gated_levels++] = l;
            cur ^= 1;
            span *= gc;
            nm = (nm + gc - 1) / gc;
        }
        gated_tree = nm == 1;
        if (gated_tree) {
            all.final_rel = static_cast<const uint32_t *>(sc.join[cur]);
            all.done = sc.counters + 8;
        }
    }
    // the gated level 0 rides in the hit join's first launch (extra blocks)
    // and the upper levels in its last one, when the hit join has a level 0
    // and the class join more than one level
    const bool fuse_cls0 = gated_cls && gated_tree && gated_levels > 1 && plan.nchunks > 1 && H.W > 0 &&
                           H.W <= kMaxDenseWords;
    if (hit) {
        // products of hit matrices: level 0 over the K - 1 matrices, then
        // groups of 64 products until at most 64 are left; the last level and
        // the final step run in one wave
        ha.alias = sc.alias;
        ha.L = H.L;
        ha.nchunks = plan.nchunks;
        ha.run_base = ja.run_base;
        ha.run_count = sc.run_count;
        ha.run_final = ja.run_final;
        ha.csr_off = D.csr_off;
        ha.csr_idx = D.csr_idx;
        ha.content = H.W <= kMaxDenseWords ? D.content : nullptr;
        ha.prod_in = nullptr;
        ha.nmembers = 0;
        if (plan.nchunks > 1) {
            int cur = 0;
            ha.nmembers = plan.nchunks - 1;
            ha.prod_out = sc.hprod[0];
            ha.rows_out = sc.hrows[0];
            if (fuse_cls0)
                HIP_TRY(ri::launch_hit_prod_cls(ha, all.lv[0], (int)H.W, shape.alias_bytes, stream));
            else
                HIP_TRY(ri::launch_hit_prod(ha, H.W <= kMaxDenseWords ? (int)H.W : 0, shape.alias_bytes, true, stream));
            uint32_t nm = (ha.nmembers + 63) / 64;
            while (nm > ri::kHitTailMax) {
                ha.nmembers = nm;
                ha.prod_in = sc.hprod[cur];
                ha.rows_in = sc.hrows[cur];
                ha.prod_out = sc.hprod[cur ^ 1];
                ha.rows_out = sc.hrows[cur ^ 1];
                HIP_TRY(ri::launch_hit_prod(ha, 0, shape.alias_bytes, false, stream));
                cur ^= 1;
                nm = (nm + 63) / 64;
            }
            ha.prod_in = sc.hprod[cur];
            ha.nmembers = nm;
        }
        if (maps) HIP_TRY(ri::launch_materialize(ja, static_cast<int32_t *>(sc.dbg), stream));
        if (fuse_cls0) {
            // the class join's level 0 ran in the first launch: the last hit
            // level, the final step and the gated upper levels in one launch
            ri::FinalArgs fr = fa;
            fr.result = result_dev;
            all.f = fr;
            for (uint32_t l = 1; l < gated_levels; ++l) all.lv[l - 1] = all.lv[l];
            all.nlevels = gated_levels - 1;
            HIP_TRY(ri::launch_hit_tail_cls(fa, ha, result_dev, all, (int)H.W, shape.alias_bytes, stream));
        } else {
            HIP_TRY(ri::launch_finalize_hit(fa, ha, H.W <= kMaxDenseWords ? (int)H.W : 0, shape.alias_bytes, stream,
                                            result_dev, result_dev && !gated_cls ? H.W : 0, gated_cls));
            if (gated_cls) {
                fa.result = result_dev;
                if (gated_tree) {
                    all.f = fa;
                    if (gated_levels == 1) {
                        all.nlevels = 1;
                        HIP_TRY(ri::launch_cls_join_all(all, (int)H.W, shape.alias_bytes, true, stream));
                    } else {
                        HIP_TRY(ri::launch_join_cls(all.lv[0], (int)H.W, shape.alias_bytes, true, stream));
                        for (uint32_t l = 1; l < gated_levels; ++l) all.lv[l - 1] = all.lv[l];
                        all.nlevels = gated_levels - 1;
                        HIP_TRY(ri::launch_cls_join_all(all, (int)H.W, shape.alias_bytes, false, stream));
                    }
                } else {
                    rc = cls_join();
                    if (rc) return rc;
                }
            }
        }
    } else if (gc) {
        if (maps) HIP_TRY(ri::launch_materialize(ja, static_cast<int32_t *>(sc.dbg), stream));
        rc = cls_join();
        if (rc) return rc;
    } else {
        if (g0 > 0) {
            ja.G = g0;
            HIP_TRY(ri::launch_join0_tile(ja, H.relational ? (int)H.W : 0, stream));
            ja.G = kJoinGroup;
        } else if (H.relational) {
            HIP_TRY(ri::launch_join0_rel(ja, (int)H.W, stream));
        } else {
            HIP_TRY(ri::launch_join0_fun(ja, stream));
        }
        int cur = 0;
        uint32_t nin = ng0;
        while (nin > 1) {
            ja.in = sc.join[cur];
            ja.nin = nin;
            ja.out = sc.join[cur ^ 1];
            if (H.relational) HIP_TRY(ri::launch_joinN_rel(ja, (int)H.W, stream));
            else HIP_TRY(ri::launch_joinN_fun(ja, stream));
            cur ^= 1;
            nin = (nin + kJoinGroup - 1) / kJoinGroup;
        }
        if (maps) HIP_TRY(ri::launch_materialize(ja, static_cast<int32_t *>(sc.dbg), stream));
        fa.total = sc.join[cur];
        if (H.relational) HIP_TRY(ri::launch_finalize_rel(fa, (int)H.W, stream));
        else HIP_TRY(ri::launch_finalize_fun(fa, stream));
    }
    if (result_dev) {
        // the result stays on the device (written by the final kernel)
        out->chunks = plan.nchunks;
        out->chunk_size = (uint32_t)plan.cs;
        out->accept = -1;
        out->final_state = -1;
        return RI_OK;
    }
    if (prof) HIP_TRY(hipEventRecord(ws->ev[2], stream));
    HIP_TRY(hipMemcpyAsync(ws->hres, ws->dres, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    std::vector<int32_t> lam_host;
    if (maps) {
        lam_host.resize(pairs);
        HIP_TRY(hipMemcpyAsync(lam_host.data(), sc.dbg, pairs * 4, hipMemcpyDeviceToHost, stream));
    }
    if (prof) HIP_TRY(hipEventRecord(ws->ev[3], stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (hit && ws->hres[2] != 0) {
        // some chunk kept more runs than a hit-matrix row can index: join
        // again (the reach results are still in place) with the class join,
        // or by propagation when the interface is too large for it
        if (gc) {
            rc = cls_join();
            if (rc) return rc;
        } else {
            HIP_TRY(ri::launch_propagate(fa, ha, H.W, shape.alias_bytes, stream));
        }
        HIP_TRY(hipMemcpyAsync(ws->hres, ws->dres, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
    }

    out->accept = ws->hres[0];
    out->final_state = ws->hres[1];
    out->chunks = plan.nchunks;
    out->chunk_size = (uint32_t)plan.cs;
    if (out->final_state == -3) return fail(RI_ERR_DEVICE, "internal: final subset not found");
    if (prof) {
        float ms[5] = {0, 0, 0, 0, 0};
        HIP_TRY(hipEventElapsedTime(&ms[0], ws->ev[0], ws->ev[1]));
        HIP_TRY(hipEventElapsedTime(&ms[1], ws->ev[1], ws->ev[2]));
        HIP_TRY(hipEventElapsedTime(&ms[2], ws->ev[0], ws->ev[3]));
        if (conv) {
            HIP_TRY(hipEventElapsedTime(&ms[4], ws->ev[0], ws->ev[5]));
            HIP_TRY(hipEventElapsedTime(&ms[3], ws->ev[5], ws->ev[4]));
        } else {
            HIP_TRY(hipEventElapsedTime(&ms[3], ws->ev[0], ws->ev[4]));
        }
        std::lock_guard<std::mutex> lk(h->mu);
        std::memcpy(h->last_ms, ms, sizeof(ms));
    }
    if (maps) {
        for (uint32_t s2 = 0; s2 < H.L; ++s2)
            for (uint32_t c = 0; c < plan.nchunks; ++c)
                maps[(size_t)c * H.L + s2] = lam_host[(size_t)s2 * plan.nchunks + c];
    }
    return RI_OK;
}

// ---------------------------------------------------------------------------
// batches: texts grouped by (automaton, algorithm); every group is one
// converging reach over all of its texts' chunks (chunk descriptors), a join
// tree whose groups never mix two texts, and one result per text
// ---------------------------------------------------------------------------

constexpr uint64_t kBatchAutoChunkTarget = 131072;   // chunks aimed at per group when unset
constexpr uint64_t kBatchMinChunk = 256;
constexpr uint64_t kBatchMaxChunk = 1ull << 20;
constexpr int kBatchSide = 4;                         // concurrent branches of a captured batch
constexpr uint64_t kGroupedMinBytes = 4ull << 20;     // text per group for the automatic grouped mode

struct BatchLevel {
    uint32_t ngroups = 0;
    size_t first = 0, count = 0, gchunk = 0;   // byte offsets in the descriptor block
};

struct BatchGroup {
    ri_handle *h = nullptr;
    int algo = 0;
    std::vector<uint32_t> req;                // request indices
    uint64_t cs = 0;                          // chunk bytes
    Options opt;
    bool empty = false;                       // the automaton accepts nothing
    uint32_t slots = 0;
    uint64_t bytes = 0;
    uint32_t gjoin = 0;                       // level-0 group size
    uint32_t gupper = 0;                      // group size above level 0
    ConvCfg cc;
    std::vector<BatchLevel> levels;
    size_t off_addr = 0, off_len = 0, off_slot = 0, off_out = 0;
    Buf desc, alias, run_base, run_chunk, run_state, run_final, join[2], ncls[2], block_count;
    uint32_t *counters = nullptr;
    float tuned_ms = 0;
};

}  // namespace

namespace {

constexpr uint64_t kFusedTextPairs = 1ull << 22;   // (start, chunk) pairs of one text in a fused batch
constexpr size_t kMaxQueueGroups = 4096;             // automata of one queued batch

// Plan of a fused batch: all texts, all automata, one launch sequence.
struct FusedPlan {
    uint32_t cs = 0, warm = 64;
    uint32_t nslots = 0, ntexts = 0, max_words = 1;
    uint64_t alias_entries = 0;
    size_t off_addr = 0, off_len = 0, off_sauto = 0, off_stext = 0, off_arow = 0;
    size_t off_tslot = 0, off_tn = 0, off_tauto = 0, off_tout = 0, off_tprod = 0;
    struct Level {
        uint32_t ngroups = 0, prod_out = 0;
        size_t first = 0, count = 0;
    };
    std::vector<Level> levels;
    uint32_t nprod = 0;
    Buf blob, autos, alias, run_base, run_count, run_chunk, run_state, run_final, prod, prod_rows,
        text_flag, counters;
    int grid_w = 1, grid_l = 1;
    float tuned_ms = 0;
};

}  // namespace

struct ri_batch {
    int device = 0;
    std::vector<ri_request> reqs;
    std::vector<BatchGroup> groups;
    uint64_t bytes = 0;
    uint32_t fixed_chunk = 0;
    bool fused = false;
    FusedPlan fz;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t *graph_results = nullptr;
    hipStream_t side[kBatchSide] = {};
    hipEvent_t fork = nullptr, joins[kBatchSide] = {};
    // grouped batches: the long runs of every group in one work-queue launch
    bool queue = false;
    bool auto_mode = false;         // created with RI_BATCH_AUTO: the autotuner may switch `queue`
    Buf qdesc;                      // ri::QueueGroup per non-empty group
    uint32_t *qcounters = nullptr;  // items taken per group
    uint32_t qgroups = 0;
    int qgrid = 0;
    size_t qlds = 0;
    hipEvent_t fork2 = nullptr, joins2[kBatchSide] = {};
    std::vector<void *> retired;    // buffers replaced by a re-plan, freed with the batch
};

namespace {

template <typename T>
size_t put_array(std::vector<uint8_t> &blob, const std::vector<T> &v) {
    const size_t off = round_up(blob.size(), 16);
    blob.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

void release(Buf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// Chunk descriptors, join levels and buffers of one group for its chunk size.
int plan_group(ri_batch *b, BatchGroup &g) {
    ri_handle *h = g.h;
    const AlgoHost &H = h->algo[g.algo];
    DeviceCopy &dc = h->dev[b->device];
    std::vector<uint8_t> blob;
    std::vector<uint32_t> text_slot, text_out;
    for (uint32_t r : g.req) text_out.push_back(r);
    g.levels.clear();
    g.slots = 0;
    g.bytes = 0;
    if (g.empty) {
        text_slot.assign(g.req.size(), 0);
        g.off_slot = put_array(blob, text_slot);
        g.off_out = put_array(blob, text_out);
    } else {
        if (H.relational && H.W > 64)
            return fail(RI_ERR_LIMIT, "interface larger than 2048 states is not supported by the device join");
        const uint64_t cs = g.cs;
        std::vector<uint64_t> addr;
        std::vector<uint32_t> len;
        std::vector<uint32_t> mfirst, mcount;   // member range of each text at the current level
        for (uint32_t r : g.req) {
            const ri_request &q = b->reqs[r];
            const uint64_t nc = q.n == 0 ? 1 : (q.n + cs - 1) / cs;
            if (addr.size() + nc > 0x7fffffffull) return fail(RI_ERR_LIMIT, "too many chunks in one batch group");
            text_slot.push_back((uint32_t)addr.size());
            mfirst.push_back((uint32_t)addr.size());
            mcount.push_back((uint32_t)nc);
            for (uint64_t j = 0; j < nc; ++j) {
                const uint64_t o = j * cs;
                addr.push_back(reinterpret_cast<uint64_t>(q.text_dev) + (q.n ? o : 0));
                const uint64_t l = q.n ? std::min<uint64_t>(cs, q.n - o) : 0;
                len.push_back((uint32_t)l | (j == 0 ? 0x80000000u : 0u));
            }
            g.bytes += q.n;
        }
        g.slots = (uint32_t)addr.size();
        if ((uint64_t)H.L * g.slots > 0x7fffffffull) return fail(RI_ERR_LIMIT, "chunk maps of one batch group exceed the device budget");
        g.off_addr = put_array(blob, addr);
        g.off_len = put_array(blob, len);
        g.off_slot = put_array(blob, text_slot);
        g.off_out = put_array(blob, text_out);
        // join levels: groups of consecutive members of one text, until every
        // text has a single group (group i of the last level is text i)
        const int alias_bytes = H.L <= 254 ? 1 : 2;
        if (H.relational) {
            g.gjoin = g.gupper = cls_group(H, alias_bytes);
            if (!g.gjoin) return fail(RI_ERR_LIMIT, "interface too large for the batched join");
        } else {
            g.gjoin = tile_group(H);
            if (!g.gjoin) g.gjoin = kJoinGroup;
            g.gupper = kJoinGroup;
        }
        std::vector<uint32_t> mchunk;   // first chunk of each member (level >= 1)
        uint32_t G = g.gjoin;
        size_t max_groups = 0;
        for (int level = 0;; ++level) {
            std::vector<uint32_t> first, count, gchunk;
            bool done = true;
            for (size_t t = 0; t < mfirst.size(); ++t) {
                const uint32_t f0 = (uint32_t)first.size();
                uint32_t k = 0;
                for (uint32_t j = 0; j < mcount[t]; j += G, ++k) {
                    const uint32_t m = mfirst[t] + j;
                    first.push_back(m);
                    count.push_back(std::min(G, mcount[t] - j));
                    gchunk.push_back(level == 0 ? m : mchunk[m]);
                }
                mfirst[t] = f0;
                mcount[t] = k;
                done &= k == 1;
            }
            BatchLevel lv;
            lv.ngroups = (uint32_t)first.size();
            lv.first = put_array(blob, first);
            lv.count = put_array(blob, count);
            lv.gchunk = put_array(blob, gchunk);
            g.levels.push_back(lv);
            max_groups = std::max<size_t>(max_groups, first.size());
            mchunk.swap(gchunk);
            G = g.gupper;
            if (done) break;
        }
        const size_t pairs = (size_t)H.L * g.slots;
        const size_t row_words = H.relational ? H.W : 1;
        int rc = conv_config(H, dc, g.opt, g.slots, &g.cc);
        if (!rc) rc = grow(g.alias, pairs * alias_bytes, &b->retired);
        if (!rc) rc = grow(g.run_base, (size_t)g.slots * 4, &b->retired);
        if (!rc) rc = grow(g.run_chunk, g.cc.run_cap * 4, &b->retired);
        if (!rc) rc = grow(g.run_state, g.cc.run_cap * 4, &b->retired);
        if (!rc) rc = grow(g.run_final, g.cc.run_cap * 4, &b->retired);
        if (!rc) rc = grow(g.block_count, (size_t)g.cc.grid_w * 4, &b->retired);
        for (int i = 0; i < 2 && !rc; ++i) {
            rc = grow(g.join[i], max_groups * H.L * row_words * 4, &b->retired);
            if (!rc) rc = grow(g.ncls[i], max_groups * 4, &b->retired);
        }
        if (rc) return rc;
        if (!g.counters) {
            HIP_TRY(hipMalloc(reinterpret_cast<void **>(&g.counters), 64));
            HIP_TRY(zero_now(g.counters, 64));
        }
    }
    int rc = grow(g.desc, blob.size(), &b->retired);
    if (rc) return rc;
    HIP_TRY(hipMemcpy(g.desc.p, blob.data(), blob.size(), hipMemcpyHostToDevice));
    return RI_OK;
}

template <typename T>
const T *at_off(const BatchGroup &g, size_t off) {
    return reinterpret_cast<const T *>(static_cast<const uint8_t *>(g.desc.p) + off);
}

// Reach arguments of one group (chunk descriptors, tables, starts).
ri::ScanArgs group_scan_args(const ri_batch *b, const BatchGroup &g) {
    const AlgoHost &H = g.h->algo[g.algo];
    const AlgoDevice &D = g.h->dev[b->device].algo[g.algo];
    ri::ScanArgs sa{};
    sa.text = nullptr;
    sa.n = 0;
    sa.cs = g.cs;
    sa.nchunks = g.slots;
    sa.chunk_addr = at_off<uint64_t>(g, g.off_addr);
    sa.chunk_len = at_off<uint32_t>(g, g.off_len);
    sa.table = D.table;
    sa.table_bytes = (uint32_t)H.table.size();
    sa.code = D.code;
    sa.starts = D.starts;
    sa.L = H.L;
    sa.row_bytes = H.K * H.entry_bytes;
    sa.dead = H.dead;
    sa.sink0 = H.sink[0];
    sa.sink1 = H.sink[1];
    return sa;
}

// Long-run arguments of one group (as launch_conv sets them).
ri::LongArgs group_long_args(const ri_batch *b, const BatchGroup &g) {
    ri::LongArgs la{};
    la.s = group_scan_args(b, g);
    la.warm = g.opt.warm;
    la.run_chunk = static_cast<const uint32_t *>(g.run_chunk.p);
    la.run_state = static_cast<const uint32_t *>(g.run_state.p);
    la.run_final = static_cast<uint32_t *>(g.run_final.p);
    la.block_count = static_cast<const uint32_t *>(g.block_count.p);
    la.warm_blocks = (uint32_t)g.cc.grid_w;
    la.cpi = g.cc.cpi;
    return la;
}

// Phases of a group's launch sequence: everything, or (queued batches) the
// warm-up alone and the joins alone, with the long runs of every group in
// between in one work-queue launch.
enum GroupPhase { kAllPhases, kWarmPhase, kJoinPhase };

// Enqueue one group's kernels; results[2 * request] = (accept, final state).
int run_group(ri_batch *b, const BatchGroup &g, hipStream_t stream, int32_t *results, GroupPhase phase = kAllPhases) {
    ri::BatchFinalArgs bf{};
    bf.ntexts = (uint32_t)g.req.size();
    bf.text_slot = at_off<uint32_t>(g, g.off_slot);
    bf.text_out = at_off<uint32_t>(g, g.off_out);
    bf.results = results;
    if (g.empty) {
        if (phase != kWarmPhase) HIP_TRY(ri::launch_batch_fill(bf, stream));
        return RI_OK;
    }
    const AlgoHost &H = g.h->algo[g.algo];
    const AlgoDevice &D = g.h->dev[b->device].algo[g.algo];
    const ri::ScanArgs sa = group_scan_args(b, g);
    ReachBufs rb{g.alias.p, static_cast<uint32_t *>(g.run_base.p), static_cast<uint32_t *>(g.run_chunk.p),
                 static_cast<uint32_t *>(g.run_state.p), static_cast<uint32_t *>(g.run_final.p), g.counters, nullptr,
                 static_cast<uint32_t *>(g.block_count.p), prefix_args(H, D, g.opt)};
    if (phase == kAllPhases) {
        const int rc = launch_conv(g.cc, sa, g.opt, rb, stream, nullptr);
        if (rc) return rc;
    } else if (phase == kWarmPhase) {
        HIP_TRY(ri::launch_warm(warm_args(g.cc, sa, g.opt, rb), g.cc.warm_shape, g.cc.grid_w, g.cc.lds_w, stream));
        return RI_OK;
    }

    const int alias_bytes = g.cc.long_shape.alias_bytes;
    ri::FinalArgs fa{};
    fa.fmask = D.fmask;
    fa.hash = D.hash;
    fa.hash_cap = H.hash_cap;
    fa.csr_off = D.csr_off;
    fa.csr_idx = D.csr_idx;
    fa.content = H.relational && H.W <= kMaxDenseWords ? D.content : nullptr;
    fa.final_of_state = D.final_of_state;
    fa.accept_of_state = D.accept_of_state;
    fa.counters = g.counters;
    int cur = 0;
    if (H.relational) {
        ri::ClsJoinArgs ca{};
        ca.alias = g.alias.p;
        ca.nchunks = g.slots;
        ca.L = H.L;
        ca.run_base = rb.run_base;
        ca.run_final = rb.run_final;
        ca.content = D.content;
        ca.span = 1;
        for (size_t l = 0; l < g.levels.size(); ++l) {
            const BatchLevel &lv = g.levels[l];
            ca.G = l == 0 ? g.gjoin : g.gupper;
            ca.grp_first = at_off<uint32_t>(g, lv.first);
            ca.grp_count = at_off<uint32_t>(g, lv.count);
            ca.ngroups = lv.ngroups;
            ca.member_chunk = l == 0 ? nullptr : at_off<uint32_t>(g, g.levels[l - 1].gchunk);
            ca.nmembers = l == 0 ? g.slots : g.levels[l - 1].ngroups;
            ca.ncls_in = l == 0 ? nullptr : static_cast<const uint32_t *>(g.ncls[cur].p);
            ca.cont_in = l == 0 ? nullptr : static_cast<const uint32_t *>(g.join[cur].p);
            const int o = l == 0 ? 0 : cur ^ 1;
            ca.ncls_out = static_cast<uint32_t *>(g.ncls[o].p);
            ca.cont_out = static_cast<uint32_t *>(g.join[o].p);
            HIP_TRY(ri::launch_join_cls(ca, (int)H.W, alias_bytes, l == 0, stream));
            cur = o;
        }
        ca.cont_in = static_cast<const uint32_t *>(g.join[cur].p);
        HIP_TRY(ri::launch_batch_final_cls(bf, fa, ca, (int)H.W, alias_bytes, stream));
    } else {
        ri::JoinArgs ja{};
        ja.converged = true;
        ja.alias = g.alias.p;
        ja.run_base = rb.run_base;
        ja.run_final = rb.run_final;
        ja.tile_bytes = (int)H.lam_bytes;
        ja.alias_bytes = alias_bytes;
        ja.nchunks = g.slots;
        ja.L = H.L;
        for (size_t l = 0; l < g.levels.size(); ++l) {
            const BatchLevel &lv = g.levels[l];
            ja.G = l == 0 ? g.gjoin : g.gupper;
            ja.grp_first = at_off<uint32_t>(g, lv.first);
            ja.grp_count = at_off<uint32_t>(g, lv.count);
            ja.ngroups = lv.ngroups;
            const int o = l == 0 ? 0 : cur ^ 1;
            ja.out = g.join[o].p;
            if (l == 0) {
                if (tile_group(H)) HIP_TRY(ri::launch_join0_tile(ja, 0, stream));
                else HIP_TRY(ri::launch_join0_fun(ja, stream));
            } else {
                ja.in = g.join[cur].p;
                ja.nin = g.levels[l - 1].ngroups;
                HIP_TRY(ri::launch_joinN_fun(ja, stream));
            }
            cur = o;
        }
        fa.total = g.join[cur].p;
        HIP_TRY(ri::launch_batch_final_fun(bf, fa, H.L, stream));
    }
    return RI_OK;
}

// Descriptors of the queued long runs (after every group is planned).  The
// launch's LDS holds the largest group table that fits a workgroup's LDS
// (with the byte codes and the group's dense run prefix); groups with larger
// tables read them from L2.
int plan_queue(ri_batch *b) {
    std::vector<ri::QueueGroup> qg;
    size_t lds = ri::kCodeLdsBytes;
    int budget = 0;
    HIP_TRY(hipDeviceGetAttribute(&budget, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device));

    for (const auto &g : b->groups) {
        if (g.empty || g.slots == 0) continue;
        const AlgoHost &H = g.h->algo[g.algo];
        ri::QueueGroup d{};
        d.la = group_long_args(b, g);
        d.entry_bytes = H.entry_bytes;
        const size_t need = H.table.size() + ri::kCodeLdsBytes;
        const size_t pre = round_up(((size_t)g.cc.grid_w + 1) * 4, 16);   // dense run prefix
        d.lds = need + pre <= (size_t)budget ? 1u : 0u;
        lds = std::max(lds, (d.lds ? need : ri::kCodeLdsBytes) + pre);
        qg.push_back(d);
    }
    b->qgroups = (uint32_t)qg.size();
    b->qlds = lds;
    if (qg.empty()) return RI_OK;
    int rc = grow(b->qdesc, qg.size() * sizeof(ri::QueueGroup), &b->retired);
    if (rc) return rc;
    HIP_TRY(hipMemcpy(b->qdesc.p, qg.data(), qg.size() * sizeof(ri::QueueGroup), hipMemcpyHostToDevice));
    if (!b->qcounters) HIP_TRY(hipMalloc(reinterpret_cast<void **>(&b->qcounters), kMaxQueueGroups * 4));
    if (qg.size() > kMaxQueueGroups) return fail(RI_ERR_LIMIT, "too many automata in one queued batch");
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    const int per_cu = std::max(1, ri::queue_long_blocks_per_cu(lds));
    b->qgrid = cus * per_cu;
    return RI_OK;
}

// The long runs of every group: counters cleared by a kernel (capturable),
// then the work-queue launch.
int run_queue(ri_batch *b, hipStream_t stream) {
    if (b->qgroups == 0) return RI_OK;
    HIP_TRY(ri::launch_zero_words(b->qcounters, b->qgroups, stream));
    ri::QueueArgs qa{};
    qa.groups = static_cast<const ri::QueueGroup *>(b->qdesc.p);
    qa.ngroups = b->qgroups;
    qa.counters = b->qcounters;
    HIP_TRY(ri::launch_queue_long(qa, b->qgrid, b->qlds, stream));
    return RI_OK;
}

// Every group of a grouped batch on one stream.
int run_groups(ri_batch *b, hipStream_t stream, int32_t *results) {
    int rc = RI_OK;
    if (!b->queue) {
        for (const auto &g : b->groups)
            if ((rc = run_group(b, g, stream, results)) != RI_OK) return rc;
        return RI_OK;
    }
    for (const auto &g : b->groups)
        if ((rc = run_group(b, g, stream, results, kWarmPhase)) != RI_OK) return rc;
    if ((rc = run_queue(b, stream)) != RI_OK) return rc;
    for (const auto &g : b->groups)
        if ((rc = run_group(b, g, stream, results, kJoinPhase)) != RI_OK) return rc;
    return RI_OK;
}

void drop_graph(ri_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_results = nullptr;
}

int check_device(const ri_batch *b) {
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    if (device != b->device) return fail(RI_ERR_ARG, "the batch was created on another device");
    return RI_OK;
}

// Chunking of one text in a fused batch: (chunk bytes, chunks).
void fused_chunking(uint64_t n, uint32_t L, uint64_t cs, uint64_t *cs_out, uint64_t *nc_out) {
    const uint64_t maxc = std::max<uint64_t>(1, kFusedTextPairs / std::max<uint32_t>(L, 1));
    if (n && (n + cs - 1) / cs > maxc) cs = round_up((n + maxc - 1) / maxc, 16);
    *cs_out = cs;
    *nc_out = n ? (n + cs - 1) / cs : 1;
}

int check_requests(const ri_request *reqs, uint32_t count) {
    for (uint32_t i = 0; i < count; ++i) {
        const ri_request &q = reqs[i];
        if (!q.h) return fail(RI_ERR_ARG, "request " + std::to_string(i) + ": NULL handle");
        if (q.algo < 0 || q.algo >= RI_NUM_ALGOS) return fail(RI_ERR_ARG, "request " + std::to_string(i) + ": unknown algorithm");
        if (q.algo == RI_ALGO_NFA)
            return fail(RI_ERR_ARG, "request " + std::to_string(i) + ": RI_ALGO_NFA is not available in batches");
        if (q.reserved != 0) return fail(RI_ERR_ARG, "request " + std::to_string(i) + ": reserved must be 0");
        if (q.n > 0 && !q.text_dev) return fail(RI_ERR_ARG, "request " + std::to_string(i) + ": NULL text pointer");
        if (q.n > 0 && (reinterpret_cast<uintptr_t>(q.text_dev) & 15))
            return fail(RI_ERR_ARG, "request " + std::to_string(i) + ": text must be 16-byte aligned");
    }
    return RI_OK;
}

// Automaton descriptor of a group for the fused kernels.
ri::AutoDesc auto_desc(const BatchGroup &g, int device) {
    ri::AutoDesc d{};
    if (g.empty) return d;
    const AlgoHost &H = g.h->algo[g.algo];
    const AlgoDevice &D = g.h->dev[device].algo[g.algo];
    d.table = D.table;
    d.code = D.code;
    d.starts = D.starts;
    d.L = H.L;
    d.row_bytes = H.K * H.entry_bytes;
    d.dead = H.dead;
    d.sink0 = H.sink[0];
    d.sink1 = H.sink[1];
    d.entry_bytes = H.entry_bytes;
    d.functional = H.relational ? 0u : 1u;
    d.W = H.relational ? H.W : (H.L + 31) / 32;
    d.csr_off = D.csr_off;
    d.csr_idx = D.csr_idx;
    d.fmask = D.fmask;
    d.hash = D.hash;
    d.hash_cap = H.hash_cap;
    d.final_of_state = D.final_of_state;
    d.accept_of_state = D.accept_of_state;
    return d;
}

int plan_fused(ri_batch *b) {
    FusedPlan &z = b->fz;
    std::vector<ri::AutoDesc> descs;
    z.max_words = 1;
    for (const auto &g : b->groups) {
        descs.push_back(auto_desc(g, b->device));
        if (descs.back().W > ri::kPropMaxWords) return fail(RI_ERR_LIMIT, "automaton too large for the fused batch join");
        z.max_words = std::max(z.max_words, descs.back().W);
    }
    std::vector<uint64_t> addr, arow;
    std::vector<uint32_t> len, sauto, stext, tslot, tn, tauto, tout, tprod;
    uint64_t alias_entries = 0;
    for (uint32_t gi = 0; gi < b->groups.size(); ++gi) {
        const uint32_t L = descs[gi].L;
        for (uint32_t r : b->groups[gi].req) {
            const ri_request &q = b->reqs[r];
            uint64_t cs, nc;
            fused_chunking(q.n, L, z.cs, &cs, &nc);
            if (addr.size() + nc > 0x7fffffffull) return fail(RI_ERR_LIMIT, "too many chunks in one batch");
            const uint32_t t = (uint32_t)tslot.size();
            tslot.push_back((uint32_t)addr.size());
            tn.push_back((uint32_t)nc);
            tauto.push_back(gi);
            tout.push_back(r);
            for (uint64_t j = 0; j < nc; ++j) {
                const uint64_t o = j * cs;
                addr.push_back(reinterpret_cast<uint64_t>(q.text_dev) + (q.n ? o : 0));
                const uint64_t l = q.n ? std::min<uint64_t>(cs, q.n - o) : 0;
                len.push_back((uint32_t)l | (j == 0 ? 0x80000000u : 0u));
                sauto.push_back(gi);
                stext.push_back(t);
                arow.push_back(alias_entries);
                alias_entries += L;
            }
        }
    }
    z.nslots = (uint32_t)addr.size();
    z.ntexts = (uint32_t)tslot.size();
    z.alias_entries = alias_entries;
    // join levels: level 0 groups the matrices (slot k -> k + 1) of one text,
    // higher levels group the products of one text, until each text has one
    std::vector<uint8_t> blob;
    tprod.assign(z.ntexts, 0xFFFFFFFFu);
    std::vector<uint32_t> pfirst(z.ntexts, 0), pn(z.ntexts, 0);
    z.levels.clear();
    z.nprod = 0;
    std::vector<std::vector<uint32_t>> firsts, counts;
    for (int level = 0;; ++level) {
        std::vector<uint32_t> first, count;
        const uint32_t out0 = z.nprod;
        for (uint32_t t = 0; t < z.ntexts; ++t) {
            uint32_t m0, mn;
            if (level == 0) {
                if (tn[t] < 2) continue;
                m0 = tslot[t];
                mn = tn[t] - 1;
            } else {
                if (pn[t] < 2) continue;
                m0 = pfirst[t];
                mn = pn[t];
            }
            const uint32_t f0 = z.nprod;
            uint32_t k = 0;
            for (uint32_t j = 0; j < mn; j += 64, ++k) {
                first.push_back(m0 + j);
                count.push_back(std::min<uint32_t>(64, mn - j));
                ++z.nprod;
            }
            pfirst[t] = f0;
            pn[t] = k;
            if (k == 1) tprod[t] = f0;
        }
        if (first.empty()) break;
        FusedPlan::Level lv;
        lv.ngroups = (uint32_t)first.size();
        lv.prod_out = out0;
        firsts.push_back(first);
        counts.push_back(count);
        z.levels.push_back(lv);
    }
    z.off_addr = put_array(blob, addr);
    z.off_arow = put_array(blob, arow);
    z.off_len = put_array(blob, len);
    z.off_sauto = put_array(blob, sauto);
    z.off_stext = put_array(blob, stext);
    z.off_tslot = put_array(blob, tslot);
    z.off_tn = put_array(blob, tn);
    z.off_tauto = put_array(blob, tauto);
    z.off_tout = put_array(blob, tout);
    z.off_tprod = put_array(blob, tprod);
    for (size_t l = 0; l < z.levels.size(); ++l) {
        z.levels[l].first = put_array(blob, firsts[l]);
        z.levels[l].count = put_array(blob, counts[l]);
    }
    int rc = grow(z.blob, std::max<size_t>(blob.size(), 16), &b->retired);
    if (!rc) rc = grow(z.autos, std::max<size_t>(descs.size(), 1) * sizeof(ri::AutoDesc), &b->retired);
    if (!rc) rc = grow(z.alias, std::max<uint64_t>(alias_entries, 1) * 2, &b->retired);
    if (!rc) rc = grow(z.run_base, std::max<size_t>(z.nslots, 1) * 4, &b->retired);
    if (!rc) rc = grow(z.run_count, std::max<size_t>(z.nslots, 1) * 4, &b->retired);
    if (!rc) rc = grow(z.run_chunk, std::max<uint64_t>(alias_entries, 1) * 4, &b->retired);
    if (!rc) rc = grow(z.run_state, std::max<uint64_t>(alias_entries, 1) * 4, &b->retired);
    if (!rc) rc = grow(z.run_final, std::max<uint64_t>(alias_entries, 1) * 4, &b->retired);
    if (!rc) rc = grow(z.prod, std::max<size_t>(z.nprod, 1) * ri::kRowCap * 8, &b->retired);
    if (!rc) rc = grow(z.prod_rows, std::max<size_t>(z.nprod, 1) * 4, &b->retired);
    if (!rc) rc = grow(z.text_flag, std::max<size_t>(z.ntexts, 1) * 4, &b->retired);
    if (!rc) rc = grow(z.counters, 64, &b->retired);
    if (rc) return rc;
    if (!blob.empty()) HIP_TRY(hipMemcpy(z.blob.p, blob.data(), blob.size(), hipMemcpyHostToDevice));
    if (!descs.empty())
        HIP_TRY(hipMemcpy(z.autos.p, descs.data(), descs.size() * sizeof(ri::AutoDesc), hipMemcpyHostToDevice));
    HIP_TRY(zero_now(z.text_flag.p, z.text_flag.cap));
    HIP_TRY(zero_now(z.counters.p, 64));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    const uint32_t iters = (z.nslots + ri::kWarmChunksPerBlock - 1) / ri::kWarmChunksPerBlock;
    z.grid_w = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)cus * std::max(1, ri::multi_blocks_per_cu(1)), iters));
    z.grid_l = std::max(1, cus * std::max(1, ri::multi_blocks_per_cu(2)));
    return RI_OK;
}

int run_fused(ri_batch *b, hipStream_t stream, int32_t *results) {
    const FusedPlan &z = b->fz;
    if (z.ntexts == 0) return RI_OK;
    auto at8 = [&](size_t off) { return static_cast<const uint8_t *>(z.blob.p) + off; };
    ri::MultiArgs a{};
    a.autos = static_cast<const ri::AutoDesc *>(z.autos.p);
    a.nslots = z.nslots;
    a.ntexts = z.ntexts;
    a.chunk_addr = reinterpret_cast<const uint64_t *>(at8(z.off_addr));
    a.chunk_len = reinterpret_cast<const uint32_t *>(at8(z.off_len));
    a.slot_auto = reinterpret_cast<const uint32_t *>(at8(z.off_sauto));
    a.slot_text = reinterpret_cast<const uint32_t *>(at8(z.off_stext));
    a.alias_row = reinterpret_cast<const uint64_t *>(at8(z.off_arow));
    a.alias = static_cast<uint16_t *>(z.alias.p);
    a.warm = z.warm;
    a.run_base = static_cast<uint32_t *>(z.run_base.p);
    a.run_count = static_cast<uint32_t *>(z.run_count.p);
    a.run_chunk = static_cast<uint32_t *>(z.run_chunk.p);
    a.run_state = static_cast<uint32_t *>(z.run_state.p);
    a.run_final = static_cast<uint32_t *>(z.run_final.p);
    a.counters = static_cast<uint32_t *>(z.counters.p);
    a.text_flag = static_cast<uint32_t *>(z.text_flag.p);
    a.text_slot = reinterpret_cast<const uint32_t *>(at8(z.off_tslot));
    a.text_nslots = reinterpret_cast<const uint32_t *>(at8(z.off_tn));
    a.text_auto = reinterpret_cast<const uint32_t *>(at8(z.off_tauto));
    a.text_out = reinterpret_cast<const uint32_t *>(at8(z.off_tout));
    a.text_prod = reinterpret_cast<const uint32_t *>(at8(z.off_tprod));
    a.results = results;
    a.prod = static_cast<uint64_t *>(z.prod.p);
    a.prod_rows = static_cast<uint32_t *>(z.prod_rows.p);
    HIP_TRY(ri::launch_mwarm(a, z.grid_w, stream));
    HIP_TRY(ri::launch_mlong(a, z.grid_l, stream));
    for (size_t l = 0; l < z.levels.size(); ++l) {
        a.grp_first = reinterpret_cast<const uint32_t *>(at8(z.levels[l].first));
        a.grp_count = reinterpret_cast<const uint32_t *>(at8(z.levels[l].count));
        a.ngroups = z.levels[l].ngroups;
        a.prod_out = z.levels[l].prod_out;
        HIP_TRY(ri::launch_mhit(a, l == 0, stream));
    }
    HIP_TRY(ri::launch_mfinal(a, stream));
    HIP_TRY(ri::launch_mprop(a, z.max_words, stream));
    return RI_OK;
}

void release_fused(FusedPlan &z) {
    for (Buf *x : {&z.blob, &z.autos, &z.alias, &z.run_base, &z.run_count, &z.run_chunk, &z.run_state,
                              &z.run_final, &z.prod, &z.prod_rows, &z.text_flag, &z.counters})
        release(*x);
}

// Whole-batch grid search of (chunk size, warm-up) for a fused batch.
int autotune_fused(ri_batch *b, hipStream_t stream, const uint32_t *chunks, size_t nchunks, const uint32_t *warms,
                   size_t nwarms, ri_batch_tuning *out) {
    FusedPlan &z = b->fz;
    const size_t nr = b->reqs.size();
    int32_t *dres = nullptr;
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(&dres), std::max<size_t>(nr, 1) * 8));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = RI_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventCreate");
    std::vector<int32_t> ref, got(nr * 2);
    float best = 1e30f;
    uint32_t best_cs = z.cs, best_warm = z.warm, trials = 0;
    for (size_t ci = 0; ci < nchunks && !rc; ++ci) {
        if (b->fixed_chunk && ci > 0) break;
        for (size_t wi = 0; wi < nwarms && !rc; ++wi) {
            z.cs = b->fixed_chunk ? b->fixed_chunk : chunks[ci];
            z.warm = warms[wi];
            rc = plan_fused(b);
            float ms = 0;
            for (int it = 0; it < 3 && !rc; ++it) {   // first pass is a warm-up
                if (hipEventRecord(e0, stream) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventRecord");
                if (!rc) rc = run_fused(b, stream, dres);
                if (!rc && hipEventRecord(e1, stream) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventRecord");
                if (!rc && hipStreamSynchronize(stream) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipStreamSynchronize");
                float t = 0;
                if (!rc && it > 0 && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventElapsedTime");
                ms += it > 0 ? t / 2 : 0.f;
            }
            if (!rc && nr && hipMemcpy(got.data(), dres, nr * 8, hipMemcpyDeviceToHost) != hipSuccess)
                rc = fail(RI_ERR_DEVICE, "hipMemcpy");
            if (rc) break;
            if (ref.empty()) ref = got;
            else if (got != ref) rc = fail(RI_ERR_DEVICE, "internal: results differ between tuning trials");
            ++trials;
            if (!rc && ms < best) {
                best = ms;
                best_cs = z.cs;
                best_warm = z.warm;
            }
        }
    }
    (void)hipFree(dres);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    z.cs = best_cs;
    z.warm = best_warm;
    z.tuned_ms = best;
    rc = plan_fused(b);
    if (rc) return rc;
    if (out) {
        out->trials = trials;
        out->best_ms = best;
    }
    return RI_OK;
}

int batch_setup(ri_batch *b, const ri_request *reqs, uint32_t count, const ri_batch_opts &o) {
    HIP_TRY(hipGetDevice(&b->device));
    if (b->device < 0 || b->device >= kMaxDevices) return fail(RI_ERR_DEVICE, "device index out of range");
    b->reqs.assign(reqs, reqs + count);
    b->fixed_chunk = o.chunk_bytes;
    for (uint32_t i = 0; i < count; ++i) {
        ri_handle *h = const_cast<ri_handle *>(reqs[i].h);
        BatchGroup *g = nullptr;
        for (auto &x : b->groups)
            if (x.h == h && x.algo == reqs[i].algo) g = &x;
        if (!g) {
            b->groups.emplace_back();
            g = &b->groups.back();
            g->h = h;
            g->algo = reqs[i].algo;
            g->empty = h->A.empty_language;
        }
        g->req.push_back(i);
        b->bytes += reqs[i].n;
    }
    for (auto &s : b->side) HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&b->fork2, hipEventDisableTiming));
    for (auto &e : b->joins) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto &e : b->joins2) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    bool wide = false;   // an interface beyond the grouped path's dense join
    for (auto &g : b->groups) {
        std::lock_guard<std::mutex> lk(g.h->mu);
        g.opt = g.h->tuned_valid[g.algo] ? g.h->tuned[g.algo] : g.h->opt;
        if (o.warmup_bytes) g.opt.warm = o.warmup_bytes;
        if (!g.empty) {
            const int rc = ensure_device(g.h, b->device);
            if (rc) return rc;
            wide |= g.h->algo[g.algo].relational && g.h->algo[g.algo].W > kMaxDenseWords;
        }
    }
    // automatic mode: the grouped path (tables in LDS, one launch sequence per
    // group) when every group has enough text to fill the GPU; else fused
    const bool small_groups = b->groups.size() > 0 && b->bytes / b->groups.size() < kGroupedMinBytes;
    b->fused = o.mode == RI_BATCH_FUSED || (o.mode == RI_BATCH_AUTO && (wide || small_groups));
    if (b->fused) {
        b->fz.cs = o.chunk_bytes ? o.chunk_bytes : 4096;
        b->fz.warm = o.warmup_bytes ? o.warmup_bytes : 64;
        return plan_fused(b);
    }
    b->queue = o.mode == RI_BATCH_QUEUE;
    b->auto_mode = o.mode == RI_BATCH_AUTO;
    for (auto &g : b->groups) {
        uint64_t bytes = 0;
        for (uint32_t r : g.req) bytes += b->reqs[r].n;
        g.cs = o.chunk_bytes ? o.chunk_bytes
                             : spread_chunk(std::min(kBatchMaxChunk,
                                                     std::max(kBatchMinChunk,
                                                              round_up((bytes + kBatchAutoChunkTarget - 1) /
                                                                           kBatchAutoChunkTarget, 16))));
        const int rc = plan_group(b, g);
        if (rc) return rc;
    }
    return b->queue ? plan_queue(b) : RI_OK;
}

}  // namespace

namespace ri {
// Entry points in other translation units of the library (not part of ri.h).
int set_error(int code, const char *msg) { return fail(code, msg); }
int recognize_in_arena(const ri_handle *h, const uint8_t *text, size_t n, void *stream, int algo,
                       uint32_t chunks, int32_t *result_dev, void *arena, size_t arena_bytes) {
    if (!result_dev) return fail(RI_ERR_ARG, "NULL result pointer");
    ri_result r;
    const Arena a{static_cast<uint8_t *>(arena), arena_bytes};
    return recognize(h, text, n, stream, algo, chunks, &r, nullptr, 0, result_dev, &a);
}
}  // namespace ri

extern "C" {

int ri_build(const char *re, size_t re_len, const ri_build_opts *opts, ri_handle **out) {
    if (!re || !out) return fail(RI_ERR_ARG, "NULL expression or output pointer");
    *out = nullptr;
    if (opts && opts->flags != 0) return fail(RI_ERR_ARG, "flags must be 0");
    uint32_t max_states = (opts && opts->max_states) ? opts->max_states : (1u << 20);
    try {
        std::unique_ptr<ri_handle> h(new ri_handle());
        ri::build_automata(std::string(re, re_len), max_states, h->A);
        pack_all(h.get());
        *out = h.release();
        return RI_OK;
    } catch (const ri::BuildError &e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(RI_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(RI_ERR_ARG, e.what());
    }
}

void ri_free(ri_handle *h) {
    if (!h) return;
    for (int d = 0; d < kMaxDevices; ++d) {
        DeviceCopy &dc = h->dev[d];
        if (!dc.ready) continue;
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(d);
        (void)hipFree(dc.cls);
        for (auto &D : dc.algo) {
            (void)hipFree(D.table);
            (void)hipFree(D.code);
            (void)hipFree(D.starts);
            (void)hipFree(D.content);
            (void)hipFree(D.csr_off);
            (void)hipFree(D.csr_idx);
            (void)hipFree(D.fmask);
            (void)hipFree(D.hash);
            (void)hipFree(D.final_of_state);
            (void)hipFree(D.accept_of_state);
            (void)hipFree(D.pfx_next);
            (void)hipFree(D.pfx_count);
            (void)hipFree(D.pfx_tgt);
            (void)hipFree(D.pfx_map);
            (void)hipFree(D.follow);
            (void)hipFree(D.mask);
        }
        (void)hipSetDevice(prev);
    }
    for (auto &w : h->ws) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(w->device);
        (void)hipFree(w->counters);
        (void)hipFree(w->dres);
        (void)hipHostFree(w->hres);
        for (Buf *b : {&w->lam, &w->alias, &w->run_base, &w->run_count, &w->hprod[0], &w->hprod[1], &w->block_count,
                                  &w->hrows[0], &w->hrows[1], &w->run_chunk, &w->run_state,
                                  &w->run_final, &w->dbg, &w->join[0], &w->join[1], &w->ncls[0],
                                  &w->ncls[1]})
            (void)hipFree(b->p);
        for (void *p : w->retired) (void)hipFree(p);
        for (auto e : w->ev) (void)hipEventDestroy(e);
        (void)hipSetDevice(prev);
    }
    delete h;
}

int ri_info(const ri_handle *h, ri_info_t *out) {
    if (!h || !out) return fail(RI_ERR_ARG, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    const ri::Automata &A = h->A;
    out->nfa_states = A.nfa_states;
    out->interface_states = A.nq.n;
    out->ridfa_states = A.Bq.n;
    out->ridfa_full_states = A.ridfa_full_states;
    out->min_dfa_states = A.dmin_n;
    out->subset_dfa_states = A.dsub_n;
    out->classes = A.K;
    out->accepts_empty = A.accepts_empty ? 1 : 0;
    for (int a = 0; a < RI_NUM_ALGOS; ++a) {
        out->starts[a] = h->algo[a].L;
        out->entry_bytes[a] = h->algo[a].nfa ? 8 * h->algo[a].nfa_words : h->algo[a].entry_bytes;
        out->table_bytes[a] = h->algo[a].nfa ? 8 * (h->algo[a].follow.size() + h->algo[a].mask.size())
                                             : h->algo[a].table.size();
        out->prefix_depth[a] = h->algo[a].prefix.depth;
        out->prefix_states[a] = h->algo[a].prefix.n;
    }
    return RI_OK;
}

int ri_recognize(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream, ri_result *out) {
    return recognize(h, text_dev, n, stream, RI_ALGO_RID, 0, out, nullptr, 0);
}

int ri_recognize_ex(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream, int algo,
                    uint32_t chunks, ri_result *out) {
    return recognize(h, text_dev, n, stream, algo, chunks, out, nullptr, 0);
}

int ri_recognize_async(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream, int algo,
                       uint32_t chunks, int32_t *result_dev) {
    if (!result_dev) return fail(RI_ERR_ARG, "NULL result pointer");
    ri_result r;
    return recognize(h, text_dev, n, stream, algo, chunks, &r, nullptr, 0, result_dev);
}

int ri_chunk_maps(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream, int algo,
                  uint32_t chunks, int32_t *maps, size_t cap, ri_result *out) {
    if (!maps) return fail(RI_ERR_ARG, "NULL maps pointer");
    return recognize(h, text_dev, n, stream, algo, chunks, out, maps, cap);
}

int ri_state_content(const ri_handle *h, int algo, uint32_t state, uint32_t *members, uint32_t cap,
                     uint32_t *count) {
    if (!h || !count || (cap > 0 && !members)) return fail(RI_ERR_ARG, "NULL argument");
    if (algo < 0 || algo >= RI_NUM_ALGOS) return fail(RI_ERR_ARG, "unknown algorithm");
    const ri::Automata &A = h->A;
    std::vector<uint32_t> v;
    if (algo == RI_ALGO_RID) {
        if (state >= A.Bq.n) return fail(RI_ERR_ARG, "state out of range");
        v = A.Bq.content[state];
    } else if (algo == RI_ALGO_DFA) {
        if (state >= A.dmin_n) return fail(RI_ERR_ARG, "state out of range");
        v.push_back(state);
    } else if (algo == RI_ALGO_SUBSET) {
        if (state >= A.dsub_n) return fail(RI_ERR_ARG, "state out of range");
        if (A.dsub_final_id[state] >= 0) v.push_back((uint32_t)A.dsub_final_id[state]);
    } else {
        return fail(RI_ERR_ARG, "RI_ALGO_NFA has no state ids (its runs are sets of NFA states)");
    }
    *count = (uint32_t)v.size();
    if (v.size() > cap) return fail(RI_ERR_ARG, "members buffer too small");
    std::copy(v.begin(), v.end(), members);
    return RI_OK;
}

int ri_set_profiling(ri_handle *h, int enable) {
    if (!h) return fail(RI_ERR_ARG, "NULL handle");
    std::lock_guard<std::mutex> lk(h->mu);
    h->profiling = enable != 0;
    return RI_OK;
}

int ri_last_timings(const ri_handle *h, float ms[5]) {
    if (!h || !ms) return fail(RI_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(const_cast<ri_handle *>(h)->mu);
    std::memcpy(ms, h->last_ms, sizeof(h->last_ms));
    return RI_OK;
}

int ri_set_option(ri_handle *h, int option, int64_t value) {
    if (!h) return fail(RI_ERR_ARG, "NULL handle");
    std::lock_guard<std::mutex> lk(h->mu);
    for (bool &v : h->tuned_valid) v = false;
    switch (option) {
    case RI_OPT_CONVERGE:
        if (value != 0 && value != 1) return fail(RI_ERR_ARG, "RI_OPT_CONVERGE must be 0 or 1");
        h->opt.converge = (int)value;
        return RI_OK;
    case RI_OPT_WARMUP_BYTES:
        if (value < 16 || value > 256 || value % 16) return fail(RI_ERR_ARG, "bad warm-up length");
        h->opt.warm = (uint32_t)value;
        return RI_OK;
    case RI_OPT_RUNS_PER_LANE:
        if (value != 0 && value != 1 && value != 2 && value != 4) return fail(RI_ERR_ARG, "runs per lane: 0, 1, 2 or 4");
        h->opt.runs_per_lane = (uint32_t)value;
        return RI_OK;
    case RI_OPT_JOIN:
        if (value != 0 && value != 1) return fail(RI_ERR_ARG, "RI_OPT_JOIN must be 0 or 1");
        h->opt.join = (int)value;
        return RI_OK;
    case RI_OPT_CHUNK_TARGET:
        if (value < 1 || value > (1ll << 30)) return fail(RI_ERR_ARG, "bad chunk target");
        h->opt.chunk_target = (uint32_t)value;
        return RI_OK;
    case RI_OPT_PREFIX:
        if (value != 0 && value != 1) return fail(RI_ERR_ARG, "RI_OPT_PREFIX must be 0 or 1");
        h->opt.prefix = (int)value;
        return RI_OK;
    }
    return fail(RI_ERR_ARG, "unknown option");
}

int ri_get_option(const ri_handle *h, int option, int64_t *value) {
    if (!h || !value) return fail(RI_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(const_cast<ri_handle *>(h)->mu);
    switch (option) {
    case RI_OPT_CONVERGE: *value = h->opt.converge; return RI_OK;
    case RI_OPT_WARMUP_BYTES: *value = h->opt.warm; return RI_OK;
    case RI_OPT_RUNS_PER_LANE: *value = h->opt.runs_per_lane; return RI_OK;
    case RI_OPT_CHUNK_TARGET: *value = h->opt.chunk_target; return RI_OK;
    case RI_OPT_JOIN: *value = h->opt.join; return RI_OK;
    case RI_OPT_PREFIX: *value = h->opt.prefix; return RI_OK;
    }
    return fail(RI_ERR_ARG, "unknown option");
}

int ri_autotune(ri_handle *h, const uint8_t *text, size_t n, void *stream, int algo, ri_tuning *out) {
    if (!h) return fail(RI_ERR_ARG, "NULL handle");
    if (algo < 0 || algo >= RI_NUM_ALGOS) return fail(RI_ERR_ARG, "unknown algorithm");
    Options saved;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        saved = h->opt;
        h->tuned_valid[algo] = false;
    }
    static const uint32_t kTargets[] = {32768, 65536, 98304, 131072, 196608, 262144, 524288};
    static const uint32_t kWarm[] = {16, 32, 48, 64, 96, 128};
    static const uint32_t kRuns[] = {1, 2};
    // the grid: converging reach over targets x warm-up x runs per lane, then
    // the plain reach over targets x runs per lane
    std::vector<Options> grid;
    if (algo == RI_ALGO_NFA) {   // chunk count only: the NFA runs neither merge nor share lanes
        for (uint32_t tgt : {4096u, 16384u, 65536u, 131072u, 262144u}) {
            Options o = saved;
            o.chunk_target = tgt;
            grid.push_back(o);
        }
    }
    for (int conv = 1; conv >= 0 && algo != RI_ALGO_NFA; --conv)
        for (uint32_t tgt : kTargets)
            for (uint32_t w : (conv ? std::vector<uint32_t>(std::begin(kWarm), std::end(kWarm)) : std::vector<uint32_t>{saved.warm}))
                for (uint32_t R : kRuns) {
                    Options o = saved;
                    o.converge = conv;
                    o.chunk_target = tgt;
                    o.warm = w;
                    o.runs_per_lane = R;
                    grid.push_back(o);
                }
    ri_result first{}, r{};
    int rc = recognize(h, text, n, stream, algo, 0, &first, nullptr, 0);
    if (rc) return rc;
    Options best = saved;
    double best_ms = 1e30;
    uint32_t trials = 0;
    auto timed = [&](double *ms) -> int {
        auto t0 = std::chrono::steady_clock::now();
        const int e = recognize(h, text, n, stream, algo, 0, &r, nullptr, 0);
        *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return e;
    };
    for (const Options &o : grid) {
        {
            std::lock_guard<std::mutex> lk(h->mu);
            h->opt = o;
        }
        double t[3];
        rc = timed(&t[0]);   // warm-up call; a setting far slower than the best is not timed further
        if (rc == RI_ERR_LIMIT) {   // a setting this automaton does not support (e.g. the plain
            rc = RI_OK;             // reach of an interface too wide for its join): skipped
            continue;
        }
        if (rc) break;
        if (t[0] > 4 * best_ms) continue;
        for (double &ti : t) {
            rc = timed(&ti);
            if (rc) break;
        }
        if (rc) break;
        if (r.accept != first.accept || r.final_state != first.final_state) {
            std::lock_guard<std::mutex> lk(h->mu);
            h->opt = saved;
            return fail(RI_ERR_DEVICE, "internal: results differ between tuning trials");
        }
        std::sort(t, t + 3);
        ++trials;
        if (t[1] < best_ms) {
            best_ms = t[1];
            best = o;
        }
    }
    std::lock_guard<std::mutex> lk(h->mu);
    h->opt = saved;
    if (rc) return rc;
    h->tuned[algo] = best;
    h->tuned_valid[algo] = true;
    if (out) {
        out->chunk_target = best.chunk_target;
        out->warmup_bytes = best.warm;
        out->runs_per_lane = best.runs_per_lane;
        out->trials = trials;
        out->best_ms = (float)best_ms;
        out->converge = (uint32_t)best.converge;
    }
    return RI_OK;
}

int ri_batch_create_ex(const ri_request *reqs, uint32_t count, const ri_batch_opts *opts, ri_batch **out) {
    if (!out || (count > 0 && !reqs)) return fail(RI_ERR_ARG, "NULL argument");
    *out = nullptr;
    ri_batch_opts o{};
    if (opts) o = *opts;
    if (o.chunk_bytes % 16) return fail(RI_ERR_ARG, "chunk_bytes must be a multiple of 16");
    if (o.chunk_bytes > (1u << 30)) return fail(RI_ERR_ARG, "chunk_bytes too large");
    if (o.mode > RI_BATCH_QUEUE) return fail(RI_ERR_ARG, "unknown batch mode");
    if (o.warmup_bytes && (o.warmup_bytes < 16 || o.warmup_bytes > 256 || o.warmup_bytes % 16))
        return fail(RI_ERR_ARG, "bad warm-up length");
    if (o.reserved) return fail(RI_ERR_ARG, "reserved must be 0");
    int rc0 = check_requests(reqs, count);
    if (rc0) return rc0;
    ri_batch *b = new ri_batch();
    const int rc = batch_setup(b, reqs, count, o);
    if (rc) {
        ri_batch_free(b);
        return rc;
    }
    *out = b;
    return RI_OK;
}

int ri_batch_create(const ri_request *reqs, uint32_t count, uint32_t chunk_bytes, ri_batch **out) {
    ri_batch_opts o{};
    o.chunk_bytes = chunk_bytes;
    return ri_batch_create_ex(reqs, count, &o, out);
}

int ri_batch_update(ri_batch *b, const ri_request *reqs, uint32_t count) {
    if (!b || (count > 0 && !reqs)) return fail(RI_ERR_ARG, "NULL argument");
    if (!b->fused) return fail(RI_ERR_ARG, "only fused batches can be updated");
    int rc = check_device(b);
    if (!rc) rc = check_requests(reqs, count);
    if (rc) return rc;
    drop_graph(b);
    b->reqs.assign(reqs, reqs + count);
    b->groups.clear();
    b->bytes = 0;
    for (uint32_t i = 0; i < count; ++i) {
        ri_handle *h = const_cast<ri_handle *>(reqs[i].h);
        BatchGroup *g = nullptr;
        for (auto &x : b->groups)
            if (x.h == h && x.algo == reqs[i].algo) g = &x;
        if (!g) {
            b->groups.emplace_back();
            g = &b->groups.back();
            g->h = h;
            g->algo = reqs[i].algo;
            g->empty = h->A.empty_language;
            if (!g->empty) {
                std::lock_guard<std::mutex> lk(h->mu);
                rc = ensure_device(h, b->device);
                if (rc) return rc;
            }
        }
        g->req.push_back(i);
        b->bytes += reqs[i].n;
    }
    return plan_fused(b);
}

int ri_request_footprint(const ri_handle *h, int algo, uint64_t n, uint32_t chunk_bytes, uint64_t *bytes) {
    if (!h || !bytes) return fail(RI_ERR_ARG, "NULL argument");
    if (algo < 0 || algo >= RI_NUM_ALGOS) return fail(RI_ERR_ARG, "unknown algorithm");
    if (chunk_bytes % 16) return fail(RI_ERR_ARG, "chunk_bytes must be a multiple of 16");
    const uint32_t L = h->A.empty_language ? 0 : h->algo[algo].L;
    uint64_t cs, nc;
    fused_chunking(n, L, chunk_bytes ? chunk_bytes : 4096, &cs, &nc);
    // text, alias rows (2 B), run records (chunk, state, final: 12 B) per
    // (start, chunk) pair, per-chunk descriptors and run counts, products
    *bytes = round_up(n, 16) + nc * (uint64_t)L * 14 + nc * 40 + (nc / 64 + 2) * (ri::kRowCap * 8 + 4) + 64;
    return RI_OK;
}

void ri_batch_free(ri_batch *b) {
    if (!b) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    drop_graph(b);
    for (auto &g : b->groups) {
        for (Buf *x : {&g.desc, &g.alias, &g.run_base, &g.run_chunk, &g.run_state, &g.run_final,
                                  &g.join[0], &g.join[1], &g.ncls[0], &g.ncls[1], &g.block_count})
            release(*x);
        if (g.counters) (void)hipFree(g.counters);
    }
    release_fused(b->fz);
    release(b->qdesc);
    if (b->qcounters) (void)hipFree(b->qcounters);
    for (void *p : b->retired) (void)hipFree(p);
    for (auto s : b->side)
        if (s) (void)hipStreamDestroy(s);
    for (hipEvent_t e : {b->fork, b->fork2})
        if (e) (void)hipEventDestroy(e);
    for (auto e : b->joins)
        if (e) (void)hipEventDestroy(e);
    for (auto e : b->joins2)
        if (e) (void)hipEventDestroy(e);
    (void)hipSetDevice(prev);
    delete b;
}

int ri_batch_run(ri_batch *b, void *stream_v, int32_t *results_dev) {
    if (!b || (!results_dev && !b->reqs.empty())) return fail(RI_ERR_ARG, "NULL argument");
    int rc = check_device(b);
    if (rc) return rc;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
    if (b->fused) return run_fused(b, stream, results_dev);
    return run_groups(b, stream, results_dev);
}

int ri_batch_capture(ri_batch *b, int32_t *results_dev) {
    if (!b || (!results_dev && !b->reqs.empty())) return fail(RI_ERR_ARG, "NULL argument");
    int rc = check_device(b);
    if (rc) return rc;
    drop_graph(b);
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return fail(RI_ERR_DEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    // groups are independent: spread them over concurrent branches
    e = hipEventRecord(b->fork, cap);
    for (int k = 0; k < kBatchSide && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->side[k], b->fork, 0);
    if (b->fused && e == hipSuccess) rc = run_fused(b, b->side[0], results_dev);
    const GroupPhase first = b->queue ? kWarmPhase : kAllPhases;
    for (size_t i = 0; !b->fused && i < b->groups.size() && e == hipSuccess && rc == RI_OK; ++i)
        rc = run_group(b, b->groups[i], b->side[i % kBatchSide], results_dev, first);
    for (int k = 0; k < kBatchSide && e == hipSuccess; ++k) {
        e = hipEventRecord(b->joins[k], b->side[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cap, b->joins[k], 0);
    }
    if (!b->fused && b->queue && e == hipSuccess && rc == RI_OK) {
        // every group's warm-up is done: the long runs of all groups in one
        // launch, then the joins spread over the branches again
        rc = run_queue(b, cap);
        if (rc == RI_OK) e = hipEventRecord(b->fork2, cap);
        for (int k = 0; k < kBatchSide && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->side[k], b->fork2, 0);
        for (size_t i = 0; i < b->groups.size() && e == hipSuccess && rc == RI_OK; ++i)
            rc = run_group(b, b->groups[i], b->side[i % kBatchSide], results_dev, kJoinPhase);
        for (int k = 0; k < kBatchSide && e == hipSuccess; ++k) {
            e = hipEventRecord(b->joins2[k], b->side[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(cap, b->joins2[k], 0);
        }
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cap, &graph);
    (void)hipStreamDestroy(cap);
    if (rc || e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (rc) return rc;
        return fail(RI_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = graph;
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return fail(RI_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    b->graph_results = results_dev;
    return RI_OK;
}

int ri_batch_launch(ri_batch *b, void *stream) {
    if (!b) return fail(RI_ERR_ARG, "NULL batch");
    if (!b->exec) return fail(RI_ERR_ARG, "the batch has no captured graph (ri_batch_capture)");
    int rc = check_device(b);
    if (rc) return rc;
    HIP_TRY(hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)));
    return RI_OK;
}

int ri_batch_get_info(const ri_batch *b, ri_batch_info *out) {
    if (!b || !out) return fail(RI_ERR_ARG, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->texts = (uint32_t)b->reqs.size();
    out->groups = (uint32_t)b->groups.size();
    out->bytes = b->bytes;
    out->queue = !b->fused && b->queue ? 1u : 0u;
    if (b->fused) {
        const FusedPlan &z = b->fz;
        out->slots = z.nslots;
        out->kernels = z.ntexts ? 4 + (uint32_t)z.levels.size() : 0;
        for (const Buf *x : {&z.blob, &z.autos, &z.alias, &z.run_base, &z.run_count, &z.run_chunk,
                                        &z.run_state, &z.run_final, &z.prod, &z.prod_rows, &z.text_flag, &z.counters})
            out->device_bytes += x->cap;
    }
    for (const auto &g : b->groups) {
        if (b->fused) break;
        out->slots += g.slots;
        out->kernels += g.empty ? 1 : (b->queue ? 1 : 2) + (uint32_t)g.levels.size() + 1;
        for (const Buf *x : {&g.desc, &g.alias, &g.run_base, &g.run_chunk, &g.run_state, &g.run_final,
                                        &g.join[0], &g.join[1], &g.ncls[0], &g.ncls[1]})
            out->device_bytes += x->cap;
    }
    if (!b->fused && b->queue && b->qgroups) {
        out->kernels += 2;   // counter clear and the work-queue launch
        out->device_bytes += b->qdesc.cap + kMaxQueueGroups * 4;
    }
    out->captured = b->exec != nullptr;
    out->fused = b->fused ? 1u : 0u;
    return RI_OK;
}

int ri_batch_get_group(const ri_batch *b, uint32_t index, ri_batch_group *out) {
    if (!b || !out) return fail(RI_ERR_ARG, "NULL argument");
    if (index >= b->groups.size()) return fail(RI_ERR_ARG, "group index out of range");
    const BatchGroup &g = b->groups[index];
    std::memset(out, 0, sizeof(*out));
    out->h = g.h;
    out->algo = g.algo;
    out->texts = (uint32_t)g.req.size();
    if (b->fused) {
        const FusedPlan &z = b->fz;
        for (uint32_t r : g.req) out->bytes += b->reqs[r].n;
        out->chunk_bytes = z.cs;
        out->warmup_bytes = z.warm;
        out->join_levels = (uint32_t)z.levels.size();
        out->tuned_ms = z.tuned_ms;
        return RI_OK;
    }
    out->slots = g.slots;
    out->bytes = g.bytes;
    out->chunk_bytes = (uint32_t)g.cs;
    out->warmup_bytes = g.opt.warm;
    out->runs_per_lane = g.opt.runs_per_lane;
    out->join_levels = (uint32_t)g.levels.size();
    out->tuned_ms = g.tuned_ms;
    return RI_OK;
}

int ri_batch_autotune(ri_batch *b, void *stream_v, ri_batch_tuning *out) {
    if (!b) return fail(RI_ERR_ARG, "NULL batch");
    int rc = check_device(b);
    if (rc) return rc;
    drop_graph(b);
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
    static const uint32_t kChunk[] = {1024, 2048, 4096, 8192, 16384, 65536};
    static const uint32_t kWarm[] = {32, 64, 128};
    if (b->fused) return autotune_fused(b, stream, kChunk, sizeof(kChunk) / 4, kWarm, sizeof(kWarm) / 4, out);
    const size_t ng = b->groups.size();
    const size_t nr = b->reqs.size();
    int32_t *dres = nullptr;
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(&dres), std::max<size_t>(nr, 1) * 8));
    std::vector<int32_t> ref(nr * 2), got(nr * 2);
    std::vector<hipEvent_t> ev(ng + 1);
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    std::vector<float> best(ng, 1e30f);
    std::vector<uint64_t> best_cs(ng);
    std::vector<uint32_t> best_warm(ng);
    uint32_t trials = 0;
    bool have_ref = false;
    auto cleanup = [&]() {
        (void)hipFree(dres);
        for (auto e : ev) (void)hipEventDestroy(e);
    };
    for (uint32_t cs : kChunk) {
        if (b->fixed_chunk && cs != kChunk[0]) break;
        for (uint32_t w : kWarm) {
            for (auto &g : b->groups) {
                g.cs = b->fixed_chunk ? b->fixed_chunk : spread_chunk(cs);
                g.opt.warm = w;
                rc = g.empty ? RI_OK : plan_group(b, g);
                if (rc) { cleanup(); return rc; }
            }
            std::vector<float> ms(ng, 0.f);
            for (int it = 0; it < 3 && !rc; ++it) {   // first pass is a warm-up
                for (size_t i = 0; i < ng && !rc; ++i) {
                    if (hipEventRecord(ev[i], stream) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventRecord");
                    if (!rc) rc = run_group(b, b->groups[i], stream, dres);
                }
                if (!rc && hipEventRecord(ev[ng], stream) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventRecord");
                if (!rc && hipStreamSynchronize(stream) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipStreamSynchronize");
                for (size_t i = 0; i < ng && !rc && it > 0; ++i) {
                    float t = 0;
                    if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventElapsedTime");
                    ms[i] += t / 2;
                }
            }
            if (!rc && nr && hipMemcpy(got.data(), dres, nr * 8, hipMemcpyDeviceToHost) != hipSuccess)
                rc = fail(RI_ERR_DEVICE, "hipMemcpy");
            if (rc) { cleanup(); return rc; }
            if (!have_ref) {
                ref = got;
                have_ref = true;
            } else if (got != ref) {
                cleanup();
                return fail(RI_ERR_DEVICE, "internal: results differ between tuning trials");
            }
            ++trials;
            for (size_t i = 0; i < ng; ++i)
                if (ms[i] < best[i]) {
                    best[i] = ms[i];
                    best_cs[i] = b->groups[i].cs;
                    best_warm[i] = w;
                }
        }
    }
    float total = 0;
    for (size_t i = 0; i < ng; ++i) {
        BatchGroup &g = b->groups[i];
        g.cs = best_cs[i];
        g.opt.warm = best_warm[i];
        g.tuned_ms = best[i];
        total += best[i];
        rc = g.empty ? RI_OK : plan_group(b, g);
        if (rc) { cleanup(); return rc; }
    }
    // an automatic-mode batch also chooses where its long runs go: one
    // launch sequence per group (groups overlapping on the side streams) or
    // every group's long runs in one work-queue launch.  Both are timed as
    // ri_batch_run runs them and must give the per-group trials' results.
    if (b->auto_mode && nr && ng) {
        float tm[2] = {0.f, 0.f};
        for (int q = 0; q < 2 && !rc; ++q) {
            b->queue = q == 1;
            if (b->queue) rc = plan_queue(b);
            for (int it = 0; it < 3 && !rc; ++it) {   // first pass is a warm-up
                if (hipEventRecord(ev[0], stream) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventRecord");
                if (!rc) rc = run_groups(b, stream, dres);
                if (!rc && hipEventRecord(ev[1], stream) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventRecord");
                if (!rc && hipStreamSynchronize(stream) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipStreamSynchronize");
                float t = 0;
                if (!rc && hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess) rc = fail(RI_ERR_DEVICE, "hipEventElapsedTime");
                if (!rc && it > 0) tm[q] += t / 2;
            }
            if (!rc && hipMemcpy(got.data(), dres, nr * 8, hipMemcpyDeviceToHost) != hipSuccess)
                rc = fail(RI_ERR_DEVICE, "hipMemcpy");
            if (!rc && got != ref) rc = fail(RI_ERR_DEVICE, "internal: results differ between batch plans");
            ++trials;
        }
        if (rc) { cleanup(); return rc; }
        b->queue = tm[1] < tm[0];   // the work-queue plan is still in place when chosen
        total = b->queue ? tm[1] : tm[0];
    } else if (b->queue && (rc = plan_queue(b)) != RI_OK) {
        cleanup();
        return rc;
    }
    cleanup();
    if (out) {
        out->trials = trials;
        out->best_ms = total;
    }
    return RI_OK;
}

const char *ri_last_error(void) { return g_error.c_str(); }

}  // extern "C"
