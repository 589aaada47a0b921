// C ABI of the recognizer (include/ri.h): handle, device tables, per-stream
// workspaces and the launch sequence reach -> join tree -> finalize.
#include <hip/hip_runtime.h>

#include <algorithm>
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
constexpr uint32_t kAutoChunks = 131072;     // chunk count aimed at by chunks = 0
constexpr uint64_t kMinAutoChunk = 256;      // smallest automatic chunk size (bytes)
constexpr uint64_t kMaxLamBytes = 1ull << 31;
constexpr int kMaxDevices = 64;

uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

// FNV-1a over words; the finalize kernel uses the same function.
uint32_t hash_words(const uint32_t *x, uint32_t W) {
    uint32_t h = 2166136261u;
    for (uint32_t w = 0; w < W; ++w) { h ^= x[w]; h *= 16777619u; }
    return h;
}

struct AlgoHost {
    bool relational = false;
    uint32_t nstates = 0, K = 0, L = 0, W = 0;
    uint32_t entry_bytes = 0, lam_bytes = 2;
    uint32_t dead = 0;                         // entry offset of the dead row
    std::vector<uint8_t> table;                // padded to 16 bytes
    std::vector<uint32_t> starts;              // entry offsets of the start states
    std::vector<uint32_t> content;             // relations: [nstates][W]
    std::vector<uint32_t> fmask;               // relations: [W]
    std::vector<uint32_t> hash;                // relations: [cap][W + 1]
    uint32_t hash_cap = 0;
    std::vector<int32_t> final_of_state;       // functions
    std::vector<uint8_t> accept_of_state;      // functions
};

struct AlgoDevice {
    void *table = nullptr;
    uint32_t *starts = nullptr, *content = nullptr, *fmask = nullptr, *hash = nullptr;
    int32_t *final_of_state = nullptr;
    uint8_t *accept_of_state = nullptr;
};

struct DeviceCopy {
    bool ready = false;
    uint8_t *cls = nullptr;
    AlgoDevice algo[RI_NUM_ALGOS];
    int cus = 0;
    size_t max_lds = 0;
};

struct Workspace {
    std::mutex mu;
    int device = -1;
    hipStream_t stream = nullptr;
    uint32_t *counter = nullptr;
    int32_t *dres = nullptr;
    int32_t *hres = nullptr;        // pinned
    void *lam = nullptr;
    size_t lam_cap = 0;
    void *buf[2] = {nullptr, nullptr};
    size_t buf_cap[2] = {0, 0};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

}  // namespace

struct ri_handle {
    ri::Automata A;
    AlgoHost algo[RI_NUM_ALGOS];
    std::mutex mu;
    DeviceCopy dev[kMaxDevices];
    std::vector<std::unique_ptr<Workspace>> ws;
    bool profiling = false;
    float last_ms[3] = {0, 0, 0};
    uint32_t runs_per_lane[RI_NUM_ALGOS] = {0, 0, 0};
};

namespace {

void pack_table(AlgoHost &h, uint32_t n, uint32_t K, const std::vector<int32_t> &delta) {
    h.nstates = n;
    h.K = K;
    const uint64_t maxv = (uint64_t)n * K;     // offset of the dead row
    h.entry_bytes = maxv <= 0xFF ? 1 : maxv <= 0xFFFF ? 2 : 4;
    h.dead = (uint32_t)maxv;
    const uint64_t entries = (uint64_t)(n + 1) * K;
    h.table.assign(round_up(entries * h.entry_bytes, 16), 0);
    auto put = [&](uint64_t i, uint32_t v) {
        if (h.entry_bytes == 1) h.table[i] = (uint8_t)v;
        else if (h.entry_bytes == 2) reinterpret_cast<uint16_t *>(h.table.data())[i] = (uint16_t)v;
        else reinterpret_cast<uint32_t *>(h.table.data())[i] = v;
    };
    for (uint32_t s = 0; s <= n; ++s)
        for (uint32_t k = 0; k < K; ++k) {
            int32_t t = s < n ? delta[(size_t)s * K + k] : -1;
            put((uint64_t)s * K + k, t < 0 ? h.dead : (uint32_t)t * K);
        }
    h.lam_bytes = n < 0xFFFF ? 2 : 4;
}

void pack_all(ri_handle *h) {
    const ri::Automata &A = h->A;
    if (A.empty_language) return;
    const uint32_t K = A.K;

    // RI_ALGO_RID: B' with the singletons of N' as starts; relational join
    AlgoHost &r = h->algo[RI_ALGO_RID];
    pack_table(r, A.Bq.n, K, A.Bq.delta);
    r.relational = true;
    r.L = A.nq.n;
    uint32_t W = 1;
    while (W * 32 < r.L) W *= 2;
    r.W = W;
    r.starts.resize(r.L);
    for (uint32_t q = 0; q < r.L; ++q) r.starts[q] = A.Bq.initial[q] * K;
    r.content.assign((size_t)A.Bq.n * W, 0);
    for (uint32_t p = 0; p < A.Bq.n; ++p)
        for (uint32_t q : A.Bq.content[p]) r.content[(size_t)p * W + q / 32] |= 1u << (q % 32);
    r.fmask.assign(W, 0);
    for (uint32_t q = 0; q < A.nq.n; ++q)
        if (A.nq.final[q]) r.fmask[q / 32] |= 1u << (q % 32);
    uint32_t nkeys = 0;
    for (uint32_t p = 0; p < A.Bq.n; ++p) nkeys += A.final_id[p] >= 0;
    uint32_t cap = 1;
    while (cap < 2 * nkeys + 2) cap *= 2;
    r.hash_cap = cap;
    r.hash.assign((size_t)cap * (W + 1), 0);
    for (uint32_t s = 0; s < cap; ++s) r.hash[(size_t)s * (W + 1) + W] = (uint32_t)-2;
    for (uint32_t p = 0; p < A.Bq.n; ++p) {
        if (A.final_id[p] < 0) continue;
        const uint32_t *key = &r.content[(size_t)p * W];
        uint32_t slot = hash_words(key, W) & (cap - 1);
        while (r.hash[(size_t)slot * (W + 1) + W] != (uint32_t)-2) slot = (slot + 1) & (cap - 1);
        std::memcpy(&r.hash[(size_t)slot * (W + 1)], key, W * sizeof(uint32_t));
        r.hash[(size_t)slot * (W + 1) + W] = (uint32_t)A.final_id[p];
    }

    // RI_ALGO_DFA: minimal DFA, all states as starts; functional join
    AlgoHost &d = h->algo[RI_ALGO_DFA];
    pack_table(d, A.dmin_n, K, A.dmin_delta);
    d.L = A.dmin_n;
    d.starts.resize(d.L);
    for (uint32_t s = 0; s < d.L; ++s) d.starts[s] = s * K;
    d.final_of_state.resize(d.L);
    d.accept_of_state.resize(d.L);
    for (uint32_t s = 0; s < d.L; ++s) {
        d.final_of_state[s] = (int32_t)s;
        d.accept_of_state[s] = A.dmin_final[s];
    }

    // RI_ALGO_SUBSET: powerset DFA of N, all states as starts
    AlgoHost &u = h->algo[RI_ALGO_SUBSET];
    pack_table(u, A.dsub_n, K, A.dsub_delta);
    u.L = A.dsub_n;
    u.starts.resize(u.L);
    for (uint32_t s = 0; s < u.L; ++s) u.starts[s] = s * K;
    u.final_of_state = A.dsub_final_id;
    u.accept_of_state = A.dsub_accept;
}

template <typename T>
hipError_t upload(T **dst, const void *src, size_t bytes) {
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), bytes ? bytes : 16);
    if (e != hipSuccess) return e;
    if (bytes == 0 || !src) return hipMemset(*dst, 0, bytes ? bytes : 16);
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
        HIP_TRY(upload(&D.starts, H.starts.data(), H.starts.size() * 4));
        if (H.relational) {
            HIP_TRY(upload(&D.content, H.content.data(), H.content.size() * 4));
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
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(&w->counter), 16));
    HIP_TRY(hipMemset(w->counter, 0, 16));
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(&w->dres), 16));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&w->hres), 16, hipHostMallocDefault));
    for (auto &e : w->ev) HIP_TRY(hipEventCreate(&e));
    *out = w.get();
    h->ws.push_back(std::move(w));
    return RI_OK;
}

int grow(void **p, size_t *cap, size_t need) {
    if (need <= *cap) return RI_OK;
    if (*p) HIP_TRY(hipFree(*p));
    *p = nullptr;
    *cap = 0;
    need = round_up(need, 1 << 20);
    HIP_TRY(hipMalloc(p, need));
    *cap = need;
    return RI_OK;
}

struct Plan {
    uint64_t cs = 0;
    uint32_t nchunks = 0;
};

int plan_chunks(const AlgoHost &H, uint64_t n, uint32_t chunks, Plan *p) {
    uint64_t cs;
    if (chunks == 0) {
        cs = std::max<uint64_t>(round_up((n + kAutoChunks - 1) / kAutoChunks, 16), kMinAutoChunk);
        while ((uint64_t)H.L * ((n + cs - 1) / cs) * H.lam_bytes > kMaxLamBytes) cs *= 2;
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

int recognize(const ri_handle *hc, const uint8_t *text, size_t n, void *stream_v, int algo,
              uint32_t chunks, ri_result *out, int32_t *maps, size_t maps_cap) {
    ri_handle *h = const_cast<ri_handle *>(hc);
    if (!h || !out) return fail(RI_ERR_ARG, "NULL handle or result pointer");
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
        return RI_OK;
    }
    const AlgoHost &H = h->algo[algo];
    if (H.relational && H.W > 64)
        return fail(RI_ERR_LIMIT, "interface larger than 2048 states is not supported by the device join");
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    if (device < 0 || device >= kMaxDevices) return fail(RI_ERR_DEVICE, "device index out of range");

    Plan plan;
    int rc = plan_chunks(H, n, chunks, &plan);
    if (rc) return rc;
    if (maps && maps_cap < (size_t)plan.nchunks * H.L)
        return fail(RI_ERR_ARG, "maps buffer too small");

    Workspace *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        rc = ensure_device(h, device);
        if (rc) return rc;
        rc = get_workspace(h, device, stream, &ws);
        if (rc) return rc;
    }
    std::lock_guard<std::mutex> wlk(ws->mu);
    DeviceCopy &dc = h->dev[device];
    const AlgoDevice &D = dc.algo[algo];

    // buffers
    const uint32_t ng0 = (plan.nchunks + kJoinGroup - 1) / kJoinGroup;
    const size_t row_words = H.relational ? H.W : 1;
    rc = grow(&ws->lam, &ws->lam_cap, (size_t)H.L * plan.nchunks * H.lam_bytes);
    if (rc) return rc;
    const size_t bufneed = (size_t)ng0 * H.L * row_words * 4;
    for (int b = 0; b < 2; ++b) {
        rc = grow(&ws->buf[b], &ws->buf_cap[b], bufneed);
        if (rc) return rc;
    }

    // reach configuration
    ri::ReachConfig cfg;
    cfg.entry_bytes = (int)H.entry_bytes;
    cfg.lam_bytes = (int)H.lam_bytes;
    uint32_t R = h->runs_per_lane[algo];
    if (R == 0) R = 4;
    while (R > 1 && R / 2 >= H.L) R /= 2;
    cfg.runs_per_lane = (int)R;
    cfg.block_threads = 1024;
    const size_t lds_table = H.table.size() + 256;
    cfg.table_in_lds = lds_table <= dc.max_lds;
    const size_t lds = cfg.table_in_lds ? lds_table : 256;

    ri::ReachArgs ra;
    ra.text = text;
    ra.n = n;
    ra.cs = plan.cs;
    ra.nchunks = plan.nchunks;
    ra.table = D.table;
    ra.table_bytes = (uint32_t)H.table.size();
    ra.cls = dc.cls;
    ra.starts = D.starts;
    ra.L = H.L;
    ra.K = H.K;
    ra.dead = H.dead;
    ra.lam = ws->lam;
    ra.job_counter = ws->counter;
    ra.chunk_groups = (plan.nchunks + 63) / 64;
    const uint32_t groups = (H.L + R - 1) / R;
    ra.njobs = groups * ra.chunk_groups;
    const int per_cu = std::max(1, ri::reach_blocks_per_cu(cfg, lds));
    const uint32_t waves_per_block = cfg.block_threads / 64;
    int grid = (int)std::min<uint64_t>((uint64_t)dc.cus * per_cu,
                                       (ra.njobs + waves_per_block - 1) / waves_per_block);
    grid = std::max(grid, 1);

    if (h->profiling) HIP_TRY(hipEventRecord(ws->ev[0], stream));
    HIP_TRY(ri::launch_reach(ra, cfg, grid, lds, stream));
    if (h->profiling) HIP_TRY(hipEventRecord(ws->ev[1], stream));

    // join tree
    ri::JoinArgs ja;
    ja.lam = ws->lam;
    ja.lam_bytes = (int)H.lam_bytes;
    ja.nchunks = plan.nchunks;
    ja.content = D.content;
    ja.L = H.L;
    ja.G = kJoinGroup;
    ja.in = nullptr;
    ja.nin = 0;
    ja.out = ws->buf[0];
    if (H.relational) HIP_TRY(ri::launch_join0_rel(ja, (int)H.W, stream));
    else HIP_TRY(ri::launch_join0_fun(ja, stream));
    int cur = 0;
    uint32_t nin = ng0;
    while (nin > 1) {
        ja.in = ws->buf[cur];
        ja.nin = nin;
        ja.out = ws->buf[cur ^ 1];
        if (H.relational) HIP_TRY(ri::launch_joinN_rel(ja, (int)H.W, stream));
        else HIP_TRY(ri::launch_joinN_fun(ja, stream));
        cur ^= 1;
        nin = (nin + kJoinGroup - 1) / kJoinGroup;
    }
    ri::FinalArgs fa;
    fa.total = ws->buf[cur];
    fa.fmask = D.fmask;
    fa.hash = D.hash;
    fa.hash_cap = H.hash_cap;
    fa.final_of_state = D.final_of_state;
    fa.accept_of_state = D.accept_of_state;
    fa.result = ws->dres;
    fa.job_counter = ws->counter;
    if (H.relational) HIP_TRY(ri::launch_finalize_rel(fa, (int)H.W, stream));
    else HIP_TRY(ri::launch_finalize_fun(fa, stream));
    if (h->profiling) HIP_TRY(hipEventRecord(ws->ev[2], stream));
    HIP_TRY(hipMemcpyAsync(ws->hres, ws->dres, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    std::vector<uint8_t> lam_host;
    if (maps) {
        lam_host.resize((size_t)H.L * plan.nchunks * H.lam_bytes);
        HIP_TRY(hipMemcpyAsync(lam_host.data(), ws->lam, lam_host.size(), hipMemcpyDeviceToHost, stream));
    }
    if (h->profiling) HIP_TRY(hipEventRecord(ws->ev[3], stream));
    HIP_TRY(hipStreamSynchronize(stream));

    out->accept = ws->hres[0];
    out->final_state = ws->hres[1];
    out->chunks = plan.nchunks;
    out->chunk_size = (uint32_t)plan.cs;
    if (out->final_state == -3) return fail(RI_ERR_DEVICE, "internal: final subset not found");
    if (h->profiling) {
        float ms[3];
        HIP_TRY(hipEventElapsedTime(&ms[0], ws->ev[0], ws->ev[1]));
        HIP_TRY(hipEventElapsedTime(&ms[1], ws->ev[1], ws->ev[2]));
        HIP_TRY(hipEventElapsedTime(&ms[2], ws->ev[0], ws->ev[3]));
        std::lock_guard<std::mutex> lk(h->mu);
        std::memcpy(h->last_ms, ms, sizeof(ms));
    }
    if (maps) {
        for (uint32_t s = 0; s < H.L; ++s)
            for (uint32_t c = 0; c < plan.nchunks; ++c) {
                const size_t i = (size_t)s * plan.nchunks + c;
                int32_t v;
                if (H.lam_bytes == 2) {
                    uint16_t x = reinterpret_cast<const uint16_t *>(lam_host.data())[i];
                    v = x == 0xFFFF ? -1 : x;
                } else {
                    uint32_t x = reinterpret_cast<const uint32_t *>(lam_host.data())[i];
                    v = x == 0xFFFFFFFFu ? -1 : (int32_t)x;
                }
                maps[(size_t)c * H.L + s] = v;
            }
    }
    return RI_OK;
}

}  // namespace

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
            (void)hipFree(D.starts);
            (void)hipFree(D.content);
            (void)hipFree(D.fmask);
            (void)hipFree(D.hash);
            (void)hipFree(D.final_of_state);
            (void)hipFree(D.accept_of_state);
        }
        (void)hipSetDevice(prev);
    }
    for (auto &w : h->ws) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(w->device);
        (void)hipFree(w->counter);
        (void)hipFree(w->dres);
        (void)hipHostFree(w->hres);
        (void)hipFree(w->lam);
        (void)hipFree(w->buf[0]);
        (void)hipFree(w->buf[1]);
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
        out->entry_bytes[a] = h->algo[a].entry_bytes;
        out->table_bytes[a] = h->algo[a].table.size();
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
    } else {
        if (state >= A.dsub_n) return fail(RI_ERR_ARG, "state out of range");
        if (A.dsub_final_id[state] >= 0) v.push_back((uint32_t)A.dsub_final_id[state]);
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

int ri_last_timings(const ri_handle *h, float ms[3]) {
    if (!h || !ms) return fail(RI_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(const_cast<ri_handle *>(h)->mu);
    std::memcpy(ms, h->last_ms, sizeof(h->last_ms));
    return RI_OK;
}

const char *ri_last_error(void) { return g_error.c_str(); }

}  // extern "C"
