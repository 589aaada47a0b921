// HIP kernels of the recognizer for gfx950 (CDNA4, wave64).
//
// Reach phase (Sect. 2): for every chunk and every start state of the chunk
// automaton, one deterministic run over the chunk; its end state (or "no
// run") is the chunk map lambda_i.  Integer table lookups only; no MFMA work
// exists on this path.
//
//   plain_kernel  every (chunk, start) run to the chunk end or its death, as
//                 the paper's reach phase is stated.
//   warm_kernel + long_kernel
//                 the same chunk maps with state convergence, an optimization
//                 the paper names as compatible with the RI-DFA (Sect. 5):
//                 every run is scanned for a short warm-up; the runs of one
//                 chunk that are then in the same state have the same future
//                 (the chunk automaton is deterministic), so they are merged
//                 into one run that alone is scanned to the chunk end.
//
// Join phase: an associative composition of chunk maps over a tree of
// groups of G consecutive members.
//   Relations (RI-DFA, Sect. 3.2): row s of a chunk is the content of
//   lambda_i({s}), a set of interface states.  Composing two chunks unions
//   the rows of the second over the set bits of the first, which is
//   PLAS_i = lambda_i(if(PLAS_{i-1}) & PIS_i) taken for every PLAS_{i-1}.
//   Functions (DFA, Sect. 2): lambda_i is a partial map Q -> Q; composition
//   is a gather.
// finalize: row 0 (the initial state) of the composition of all chunks,
// the acceptance test and the minimal-DFA state of the result.
#include "kernels.hpp"

#include <mutex>
#include <type_traits>
#include <unordered_map>

namespace ri {
namespace {

constexpr int kWave = 64;

template <typename T> __device__ __forceinline__ constexpr T all_ones() { return (T)~(T)0; }

// Copy the transition table (optionally) and the byte-code map into LDS.
// Layout: [table_bytes if LDS][256 x u16 byte codes][caller's area].
// Table and codes hold byte offsets, so one step is next = *(TE *)(tab + st + code).
template <typename TE, bool LDS>
__device__ __forceinline__ void stage_tables(const ScanArgs &s, uint8_t *smem, const TE *&tab,
                                             const uint16_t *&cls) {
    uint32_t off = 0;
    if constexpr (LDS) {
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        const uint4 *src = reinterpret_cast<const uint4 *>(s.table);
        for (uint32_t i = threadIdx.x; i < s.table_bytes / 16; i += blockDim.x) dst[i] = src[i];
        tab = reinterpret_cast<const TE *>(smem);
        off = s.table_bytes;
    } else {
        tab = reinterpret_cast<const TE *>(s.table);
    }
    uint16_t *c = reinterpret_cast<uint16_t *>(smem + off);
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) c[i] = s.code[i];
    cls = c;
}

template <typename TE, bool LDS>
__host__ __device__ constexpr uint32_t tables_lds(uint32_t table_bytes) {
    return (LDS ? table_bytes : 0u) + 512u;
}

// One transition: st and c are byte offsets into the table.
template <typename TE>
__device__ __forceinline__ uint32_t next_state(const TE *tab, uint32_t st, uint32_t c) {
    return *reinterpret_cast<const TE *>(reinterpret_cast<const uint8_t *>(tab) + st + c);
}

// 16 steps of R runs over the same 16 bytes (runs of one chunk).
template <typename TE, int R>
__device__ __forceinline__ void step16_shared(uint32_t (&st)[R], const uint4 v, const TE *tab,
                                              const uint16_t *cls) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t c = cls[(w[i >> 2] >> ((i & 3) * 8)) & 0xffu];
#pragma unroll
        for (int r = 0; r < R; ++r) st[r] = next_state<TE>(tab, st[r], c);
    }
}

// 16 steps of R runs over R different 16-byte blocks (runs of R chunks).
template <typename TE, int R>
__device__ __forceinline__ void step16_each(uint32_t (&st)[R], const uint4 (&v)[R], const TE *tab,
                                            const uint16_t *cls) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t w = i < 4 ? v[r].x : i < 8 ? v[r].y : i < 12 ? v[r].z : v[r].w;
            const uint32_t c = cls[(w >> ((i & 3) * 8)) & 0xffu];
            st[r] = next_state<TE>(tab, st[r], c);
        }
    }
}

// Text bytes are read through global (address space 1) pointers: the loads
// are then global loads, tracked by the vector-memory counter only, so a wait
// for an LDS table lookup does not also wait for text loads still in flight
// (generic pointers give flat loads, which count against both counters).
typedef const __attribute__((address_space(1))) uint8_t gbyte;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4 gu32x4;

__device__ __forceinline__ uint4 load16(gbyte *p) {
    const u32x4 v = *(gu32x4 *)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void load64(uint4 (&b)[4], gbyte *p) {
    b[0] = load16(p); b[1] = load16(p + 16); b[2] = load16(p + 32); b[3] = load16(p + 48);
}

// Chunk `chunk` as absolute addresses [b, e), and whether it begins its text
// (such a chunk is scanned from the initial state only).
__device__ __forceinline__ void chunk_bounds(const ScanArgs &s, uint32_t chunk, uint64_t &b, uint64_t &e,
                                             bool &first) {
    if (s.chunk_addr) {
        const uint32_t l = s.chunk_len[chunk];
        b = s.chunk_addr[chunk];
        e = b + (l & 0x7fffffffu);
        first = (l >> 31) != 0;
    } else {
        const uint64_t o = (uint64_t)chunk * s.cs;
        const uint64_t t = reinterpret_cast<uint64_t>(s.text);
        b = t + o;
        e = t + (o + s.cs < s.n ? o + s.cs : s.n);
        first = chunk == 0;
    }
}

__device__ __forceinline__ gbyte *at(uint64_t p) { return (gbyte *)p; }

// Values that are equal on every lane of the wave, marked as such so that the
// compiler keeps them in scalar registers and branches on them with scalar
// branches instead of exec masks.
__device__ __forceinline__ uint32_t wave_uniform(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t wave_uniform(uint64_t x) {
    return (uint64_t)wave_uniform((uint32_t)x) | (uint64_t)wave_uniform((uint32_t)(x >> 32)) << 32;
}

template <int R>
__device__ __forceinline__ bool any_alive(const uint32_t (&st)[R], uint32_t dead) {
    bool a = false;
#pragma unroll
    for (int r = 0; r < R; ++r) a |= st[r] != dead;
    return a;
}

// Scan text[p, end) with R runs of one chunk.  64-byte blocks are scanned
// while the next one is already being loaded (one block of read-ahead hides
// the HBM latency behind 64 dependent lookups); then 16-byte blocks and the
// ragged tail.  The wave leaves the block loop when no lane has a live run
// with work left.
template <typename TE, int R>
__device__ __forceinline__ void scan_shared(uint32_t (&st)[R], uint64_t p, uint64_t end, const TE *tab,
                                            const uint16_t *cls, uint32_t dead) {
    const uint64_t vend = p + ((end - p) & ~(uint64_t)15);
    const uint64_t bend = p + ((end - p) & ~(uint64_t)63);
    uint4 cur[4];
    if (p < bend) load64(cur, at(p));
    for (;;) {
        const bool work = p < bend && any_alive<R>(st, dead);
        if (__ballot(work) == 0) break;
        if (work) {
            uint4 nxt[4];
            load64(nxt, at(p + 64 < bend ? p + 64 : p));
#pragma unroll
            for (int q = 0; q < 4; ++q) step16_shared<TE, R>(st, cur[q], tab, cls);
#pragma unroll
            for (int q = 0; q < 4; ++q) cur[q] = nxt[q];
            p += 64;
        }
    }
    for (; p < vend && any_alive<R>(st, dead); p += 16)
        step16_shared<TE, R>(st, load16(at(p)), tab, cls);
    for (p = p < vend ? vend : p; p < end && any_alive<R>(st, dead); ++p) {
        const uint32_t c = cls[*at(p)];
#pragma unroll
        for (int r = 0; r < R; ++r) st[r] = next_state<TE>(tab, st[r], c);
    }
}

// One run over text[p, end) without wave votes (p .. vend in 16-byte blocks).
template <typename TE>
__device__ __forceinline__ uint32_t scan_lane(uint32_t st, uint64_t p, uint64_t vend, uint64_t end,
                                              const TE *tab, const uint16_t *cls, uint32_t dead) {
    uint32_t s1[1] = {st};
    for (; p < vend && s1[0] != dead; p += 16)
        step16_shared<TE, 1>(s1, load16(at(p)), tab, cls);
    for (p = p < vend ? vend : p; p < end && s1[0] != dead; ++p) s1[0] = next_state<TE>(tab, s1[0], cls[*at(p)]);
    return s1[0];
}

__device__ __forceinline__ uint32_t wave_ticket(uint32_t *counter) {
    uint32_t t = 0;
    if (threadIdx.x % kWave == 0) t = atomicAdd(counter, 1u);
    return __shfl(t, 0);
}

// ---------------------------------------------------------------------------
// plain reach
// ---------------------------------------------------------------------------
//
// A job is 64 consecutive chunks x R consecutive starts: lane l scans chunk
// (64*cg + l) from the R starts at once, so the R runs share each byte and
// class lookup and give the lane R independent lookup chains.  Jobs are
// numbered start-group-major and handed out by a global counter to
// persistent blocks.
template <typename TE, typename TL, int R, bool LDS>
__global__ void __launch_bounds__(1024) plain_kernel(PlainArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const TE *tab;
    const uint16_t *cls;
    stage_tables<TE, LDS>(a.s, smem, tab, cls);
    __syncthreads();
    const uint32_t lane = threadIdx.x % kWave;
    TL *lam = reinterpret_cast<TL *>(a.lam);
    for (;;) {
        const uint32_t job = wave_ticket(a.job_counter);
        if (job >= a.njobs) break;
        const uint32_t g = job / a.chunk_groups;
        const uint32_t chunk = (job - g * a.chunk_groups) * kWave + lane;
        const bool ok = chunk < a.s.nchunks;
        uint64_t begin = 0, end = 0;
        bool first = false;
        if (ok) chunk_bounds(a.s, chunk, begin, end, first);
        uint32_t st[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t s = g * R + r;
            // the first chunk of a text is scanned from the initial state only (I_1 = {q0})
            st[r] = (ok && s < a.s.L && (!first || s == 0)) ? a.s.starts[s] : a.s.dead;
        }
        scan_shared<TE, R>(st, begin, end, tab, cls, a.s.dead);
        if (ok) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t s = g * R + r;
                if (s < a.s.L)
                    lam[(uint64_t)s * a.s.nchunks + chunk] =
                        st[r] == a.s.dead ? all_ones<TL>() : (TL)(st[r] / a.s.row_bytes);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// converging reach, step 1: warm-up and merging
// ---------------------------------------------------------------------------
//
// One wavefront per chunk; a block of 16 waves takes 16 consecutive chunks
// at a time (static grid-stride schedule).  The lanes hold the starts, R per
// lane (start s = base + r * 64 + lane), in blocks of 64 R starts.  The
// chunk's first `warm` bytes are loaded once, 64 per register, as byte codes;
// step j broadcasts code j to the wave with readlane, so every lookup of the
// warm-up is a table access.  After the warm-up the runs of the chunk that
// are in the same state form one class (one merged run): a leader loop finds
// the distinct states (one ballot each), lane i keeps the state of class i.
// A chunk with more than 64 distinct states keeps every live start as its own
// run (numbered in start order).  The run slots of the block's 16 chunks come
// from one atomic; the alias row of a chunk ([nchunks][L], class of every
// start) is written contiguously.
// Starts staged in LDS by the warm-up kernel when they fit.
constexpr uint32_t kStageStarts = 4096;

// The start list, read from LDS when staged and from global memory otherwise,
// through pointers of the matching address space (never a flat load, whose
// wait would also wait for the text read ahead for the next chunk).
struct StartList {
    const __attribute__((address_space(3))) uint32_t *lds;
    const __attribute__((address_space(1))) uint32_t *glb;
    bool staged;
    __device__ __forceinline__ uint32_t operator[](uint32_t s) const { return staged ? lds[s] : glb[s]; }
};

template <typename T> __host__ __device__ constexpr uint32_t tile_stride(uint32_t cols) {
    return cols + (sizeof(T) == 1 ? 4u : sizeof(T) == 2 ? 2u : 1u);
}

constexpr uint32_t kWarmWaves = kWarmChunksPerBlock;

// Warm-up of the start block at `base` over codes[0..wlen) (codes of bytes
// 64 q + lane in register q).
template <typename TE, int R, int NQ>
__device__ __forceinline__ void warm_block(uint32_t (&st)[R], const uint32_t (&code)[NQ], uint32_t wlen,
                                           const TE *tab, uint32_t dead) {
#pragma unroll
    for (uint32_t q = 0; q < (uint32_t)NQ; ++q) {
        const uint32_t j0 = q * kWave;
        if (j0 >= wlen) break;
        const uint32_t jn = wlen - j0 < kWave ? wlen - j0 : kWave;
        for (uint32_t j = 0; j < jn; j += 16) {
            if (__ballot(any_alive<R>(st, dead)) == 0) return;
            if (j + 16 <= jn) {
#pragma unroll
                for (uint32_t k = 0; k < 16; ++k) {
                    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)code[q], (int)(j + k));
#pragma unroll
                    for (int r = 0; r < R; ++r) st[r] = next_state<TE>(tab, st[r], c);
                }
            } else {
                for (uint32_t k = j; k < jn; ++k) {
                    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)code[q], (int)k);
#pragma unroll
                    for (int r = 0; r < R; ++r) st[r] = next_state<TE>(tab, st[r], c);
                }
            }
        }
    }
}

// Warm-up and classes of one chunk (all lanes of the wave).  al[r]: class of
// start base + r * 64 + lane of the last start block; with several start
// blocks the alias row is written as classes are found.  Once more than 64
// distinct states are seen the chunk spills: D counts its live starts.
template <typename TE, typename TA, int R, int NQ>
__device__ __forceinline__ void warm_classes(const TE *tab, const StartList &starts, uint32_t L, uint32_t dead,
                                             bool ok, bool first, const uint32_t (&code)[NQ], uint32_t wlen,
                                             TA *arow, uint32_t lane, uint32_t (&al)[R], uint32_t &D,
                                             uint32_t &cs, bool &spill) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    const uint32_t per_block = (uint32_t)kWave * R;
    const uint32_t nblk = (L + per_block - 1) / per_block;
    cs = dead;
    D = 0;
    spill = false;
    uint32_t st[R];
    for (uint32_t blk = 0; blk < nblk; ++blk) {
        const uint32_t base = blk * per_block;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t s = base + r * kWave + lane;
            st[r] = (ok && s < L && (!first || s == 0)) ? starts[s] : dead;
        }
        warm_block<TE, R, NQ>(st, code, wlen, tab, dead);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            al[r] = kNone;
            const bool live = st[r] != dead;
            if (spill) {
                D += (uint32_t)__builtin_popcountll(__ballot(live));
                continue;
            }
            uint64_t open = __ballot(live);
            while (open) {
                const int leader = __builtin_ctzll(open);
                const uint32_t lv = (uint32_t)__builtin_amdgcn_readlane((int)st[r], leader);
                const uint64_t hit = __ballot(lane < D && cs == lv);
                uint32_t ci;
                if (hit) {
                    ci = (uint32_t)__builtin_ctzll(hit);
                } else {
                    if (D == kWave) { spill = true; break; }
                    ci = D;
                    if (lane == D) cs = lv;
                    ++D;
                }
                const uint64_t same = __ballot(live && st[r] == lv);
                if (live && st[r] == lv) al[r] = ci;
                open &= ~same;
            }
            if (spill) {
                // count the live starts of every start seen so far
                D = 0;
                for (uint32_t b2 = 0; b2 <= blk; ++b2) {
                    uint32_t s2[R];
#pragma unroll
                    for (int r2 = 0; r2 < R; ++r2) {
                        const uint32_t s = b2 * per_block + r2 * kWave + lane;
                        s2[r2] = (ok && s < L && (!first || s == 0)) ? starts[s] : dead;
                    }
                    warm_block<TE, R, NQ>(s2, code, wlen, tab, dead);
#pragma unroll
                    for (int r2 = 0; r2 < R; ++r2)
                        if (b2 < blk || r2 <= r) D += (uint32_t)__builtin_popcountll(__ballot(s2[r2] != dead));
                }
                continue;
            }
            if (nblk > 1 && ok) {
                const uint32_t s = base + r * kWave + lane;
                if (s < L) arow[s] = al[r] == kNone ? all_ones<TA>() : (TA)al[r];
            }
        }
    }
}

// Run records of one chunk from slot `firstrun` on, and its alias row (when
// not written yet).  A spilled chunk's runs are recomputed: every live start
// is its own run, in start order.
template <typename TE, typename TA, int R, int NQ>
__device__ __forceinline__ void warm_records(const TE *tab, const StartList &starts, uint32_t L, uint32_t dead,
                                             uint32_t row_bytes, bool first, const uint32_t (&code)[NQ],
                                             uint32_t wlen, TA *arow, uint32_t lane, uint64_t lane_lt,
                                             const uint32_t (&al)[R], uint32_t D, uint32_t cs, bool spill,
                                             uint32_t firstrun, uint32_t chunk, uint32_t *run_chunk,
                                             uint32_t *run_state) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    const uint32_t per_block = (uint32_t)kWave * R;
    const uint32_t nblk = (L + per_block - 1) / per_block;
    if (!spill) {
        if (lane < D) {
            run_chunk[firstrun + lane] = chunk;
            run_state[firstrun + lane] = cs / row_bytes;
        }
        if (nblk == 1) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t s = r * kWave + lane;
                if (s < L) arow[s] = al[r] == kNone ? all_ones<TA>() : (TA)al[r];
            }
        }
        return;
    }
    uint32_t idx = 0;
    uint32_t st[R];
    for (uint32_t blk = 0; blk < nblk; ++blk) {
        const uint32_t base = blk * per_block;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t s = base + r * kWave + lane;
            st[r] = (s < L && (!first || s == 0)) ? starts[s] : dead;
        }
        warm_block<TE, R, NQ>(st, code, wlen, tab, dead);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t s = base + r * kWave + lane;
            const bool live = st[r] != dead;
            const uint64_t m = __ballot(live);
            const uint32_t my = idx + (uint32_t)__builtin_popcountll(m & lane_lt);
            if (live) {
                run_chunk[firstrun + my] = chunk;
                run_state[firstrun + my] = st[r] / row_bytes;
            }
            if (s < L) arow[s] = live ? (TA)my : all_ones<TA>();
            idx += (uint32_t)__builtin_popcountll(m);
        }
    }
}

// Run slots of the block's chunks (one per wave): one atomic.  Returns the
// first slot of this wave's chunk.
// s_cnt [kWarmWaves + 1] is used on alternate iterations from two buffers, so
// no barrier is needed after the last read: the next writes go to the other
// buffer, and the one after that follows this iteration's first barrier.
__device__ __forceinline__ uint32_t warm_slots(uint32_t *s_cnt, uint32_t lane, uint32_t wave, uint32_t D,
                                               uint32_t *counter) {
    if (lane == 0) s_cnt[wave] = D;
    __syncthreads();
    if (wave == 0) {
        const uint32_t d = lane < kWarmWaves ? s_cnt[lane] : 0u;
        uint32_t incl = d;
#pragma unroll
        for (int k = 1; k < (int)kWarmWaves; k <<= 1) {
            const uint32_t o = __shfl_up(incl, k);
            if ((int)lane >= k) incl += o;
        }
        if (lane == kWarmWaves - 1) s_cnt[kWarmWaves] = atomicAdd(counter, incl);
        if (lane < kWarmWaves) s_cnt[lane] = incl - d;
    }
    __syncthreads();
    return s_cnt[kWarmWaves] + s_cnt[wave];
}


// Occupancy: a block is 16 waves (4 per SIMD), so two blocks per CU need 8
// waves per SIMD; without the attribute the kernel's SGPR use allows 7 and
// only one block fits (the SGPRs over the limit live in VGPR lanes).
template <typename TE, typename TA, int R, bool LDS, int NQ>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) warm_kernel(WarmArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_count;   // runs placed in this block's region
    const TE *tab;
    const uint16_t *cls;
    stage_tables<TE, LDS>(a.s, smem, tab, cls);
    const uint32_t L = a.s.L;
    uint32_t *ss = reinterpret_cast<uint32_t *>(smem + tables_lds<TE, LDS>(a.s.table_bytes));
    StartList starts;
    starts.lds = (const __attribute__((address_space(3))) uint32_t *)ss;
    starts.glb = (const __attribute__((address_space(1))) uint32_t *)a.s.starts;
    starts.staged = L <= kStageStarts;
    if (starts.staged)
        for (uint32_t i = threadIdx.x; i < L; i += blockDim.x) ss[i] = a.s.starts[i];
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();   // tables and starts staged
    const uint32_t dead = a.s.dead;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t wave = wave_uniform(threadIdx.x / kWave);
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    TA *alias = reinterpret_cast<TA *>(a.alias);
    const uint32_t iters = (a.s.nchunks + kWarmWaves - 1) / kWarmWaves;

    // the warm-up bytes of this wave's chunk in iteration `it` (raw, 64 per
    // register); loaded one iteration ahead
    auto fetch = [&](uint32_t it, uint32_t (&raw)[NQ], uint64_t &b, uint32_t &wlen, bool &first) {
        const uint32_t chunk = it * kWarmWaves + wave;
        uint64_t e = 0;
        b = 0;
        first = false;
        wlen = 0;
        if (it < iters && chunk < a.s.nchunks) {
            chunk_bounds(a.s, chunk, b, e, first);
            wlen = (uint32_t)(e - b < a.warm ? e - b : a.warm);
        }
        b = wave_uniform(b);
        wlen = wave_uniform(wlen);
        first = wave_uniform((uint32_t)first) != 0;
#pragma unroll
        for (uint32_t q = 0; q < (uint32_t)NQ; ++q) {
            const uint32_t j = q * kWave + lane;
            raw[q] = j < wlen ? (uint32_t)*at(b + j) : 0u;
        }
    };
    uint32_t raw[NQ];
    uint64_t b;
    uint32_t wlen;
    bool first;
    fetch(blockIdx.x, raw, b, wlen, first);
    const uint64_t region = warm_region(blockIdx.x, gridDim.x, iters, L);
    for (uint32_t it = blockIdx.x; it < iters; it += gridDim.x) {
        const uint32_t chunk = it * kWarmWaves + wave;
        const bool ok = chunk < a.s.nchunks;
        uint32_t code[NQ];
#pragma unroll
        for (uint32_t q = 0; q < (uint32_t)NQ; ++q) code[q] = q * kWave + lane < wlen ? cls[raw[q]] : 0u;
        const uint32_t cur_wlen = wlen;
        const bool cur_first = first;
        fetch(it + gridDim.x, raw, b, wlen, first);   // next iteration's bytes, in flight meanwhile
        TA *arow = alias + (uint64_t)(ok ? chunk : 0) * L;
        uint32_t al[R], D, cs;
        bool spill;
        warm_classes<TE, TA, R, NQ>(tab, starts, L, dead, ok, cur_first, code, cur_wlen, arow, lane, al, D, cs, spill);
        // slots from the block's region: an LDS counter, no barrier
        uint32_t base = 0;
        if (lane == 0 && ok) base = atomicAdd(&s_count, D);
        const uint32_t firstrun = (uint32_t)(region + (uint32_t)__shfl((int)base, 0));
        if (ok) {
            if (lane == 0) {
                a.run_base[chunk] = firstrun;
                if (a.run_count) a.run_count[chunk] = D;
                if (D > kRowCap) atomicOr(&a.counters[2], 1u);
            }
            warm_records<TE, TA, R, NQ>(tab, starts, L, dead, a.s.row_bytes, cur_first, code, cur_wlen, arow, lane,
                                    lane_lt, al, D, cs, spill, firstrun, chunk, a.run_chunk, a.run_state);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) a.block_count[blockIdx.x] = s_count;
}

// ---------------------------------------------------------------------------
// converging reach, step 2: merged runs to the chunk end
// ---------------------------------------------------------------------------
//
// A job is 64 x R runs; lane l takes runs (job*64R + r*64 + l).  The R runs
// of a lane belong to different chunks: each loads its own 16-byte blocks,
// and the 16 x R lookups of one block step are interleaved so the lane has
// R independent chains in flight.  Runs of equal length (all but the last
// chunk's) advance in lockstep; a lane whose runs differ finishes them one
// by one.
// Exclusive prefix of the warm-up blocks' run counts in LDS: run i of the
// dense numbering is in the region of block b with pre[b] <= i < pre[b + 1].
// Ends with a barrier.
__device__ __forceinline__ void run_prefix(uint32_t *pre, const uint32_t *block_count, uint32_t G) {
    for (uint32_t i = threadIdx.x; i < G; i += blockDim.x) pre[i + 1] = block_count[i];
    __syncthreads();
    const uint32_t lane = threadIdx.x % kWave;
    if (threadIdx.x < kWave) {
        uint32_t carry = 0;
        for (uint32_t b0 = 0; b0 < G; b0 += kWave) {
            const uint32_t v = b0 + lane < G ? pre[b0 + lane + 1] : 0u;
            uint32_t incl = v;
#pragma unroll
            for (int k = 1; k < kWave; k <<= 1) {
                const uint32_t o = __shfl_up(incl, k);
                if ((int)lane >= k) incl += o;
            }
            if (b0 + lane < G) pre[b0 + lane + 1] = carry + incl;
            carry += (uint32_t)__shfl((int)incl, kWave - 1);
        }
        if (lane == 0) pre[0] = 0;
    }
    __syncthreads();
}

// Slot of dense run i (binary search of the prefix).
__device__ __forceinline__ uint32_t run_slot(const uint32_t *pre, uint32_t G, uint32_t iters, uint32_t L,
                                             uint32_t i) {
    uint32_t lo = 0, hi = G;   // pre[lo] <= i < pre[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (pre[mid] <= i) lo = mid;
        else hi = mid;
    }
    return (uint32_t)(warm_region(lo, G, iters, L) + (i - pre[lo]));
}

template <typename TE, int R, bool LDS>
__global__ void __launch_bounds__(1024) long_kernel(LongArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const TE *tab;
    const uint16_t *cls;
    stage_tables<TE, LDS>(a.s, smem, tab, cls);
    const uint32_t G = a.warm_blocks;
    uint32_t *pre = reinterpret_cast<uint32_t *>(smem + tables_lds<TE, LDS>(a.s.table_bytes));
    run_prefix(pre, a.block_count, G);
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t iters = (a.s.nchunks + kWarmChunksPerBlock - 1) / kWarmChunksPerBlock;
    auto phys = [&](uint32_t i) -> uint32_t { return run_slot(pre, G, iters, a.s.L, i); };
    const uint32_t nruns = pre[G];
    const uint32_t per_job = kWave * R;
    const uint32_t njobs = (nruns + per_job - 1) / per_job;
    const uint32_t dead = a.s.dead;
    // jobs cost about the same (runs of one chunk length): static schedule
    const uint32_t nwaves_grid = gridDim.x * (blockDim.x / kWave);
    for (uint32_t job = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; job < njobs;
         job += nwaves_grid) {
        uint64_t p[R], vend[R], end[R];
        uint32_t st[R];
        bool ok[R];
        uint32_t ri[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t i = job * per_job + r * kWave + lane;
            ok[r] = i < nruns;
            p[r] = vend[r] = end[r] = 0;
            st[r] = dead;
            ri[r] = 0;
            if (ok[r]) {
                ri[r] = phys(i);
                uint64_t b, e;
                bool first;
                chunk_bounds(a.s, a.run_chunk[ri[r]], b, e, first);
                p[r] = b + a.warm < e ? b + a.warm : e;
                vend[r] = p[r] + ((e - p[r]) & ~(uint64_t)15);
                end[r] = e;
                st[r] = a.run_state[ri[r]] * a.s.row_bytes;
            }
        }
        // lockstep 64-byte block loop with one block of read-ahead per run.
        // A run that has no whole block left is parked on the dead row (so
        // that stepping it changes nothing) until the lane's other runs are
        // done; its state is restored for the ragged remainder.
        uint64_t bend[R];
        uint32_t parked[R];
        bool pk[R];
        uint4 cur[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bend[r] = p[r] + ((end[r] - p[r]) & ~(uint64_t)63);
            pk[r] = false;
            parked[r] = dead;
            if (ok[r] && p[r] < bend[r]) load64(cur[r], at(p[r]));
            else cur[r][0] = cur[r][1] = cur[r][2] = cur[r][3] = make_uint4(0, 0, 0, 0);
        }
        for (;;) {
            bool work = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (ok[r] && !pk[r] && p[r] >= bend[r]) {
                    parked[r] = st[r];
                    st[r] = dead;
                    pk[r] = true;
                }
                work |= ok[r] && !pk[r] && st[r] != dead;
            }
            if (__ballot(work) == 0) break;
            if (work) {
                uint4 nxt[R][4];
                bool act[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    act[r] = ok[r] && !pk[r] && st[r] != dead;
                    const uint64_t q = act[r] && p[r] + 64 < bend[r] ? p[r] + 64 : p[r];
                    if (act[r]) load64(nxt[r], at(q));
                    else nxt[r][0] = nxt[r][1] = nxt[r][2] = nxt[r][3] = make_uint4(0, 0, 0, 0);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint4 v[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) v[r] = cur[r][q];
                    step16_each<TE, R>(st, v, tab, cls);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) cur[r][q] = nxt[r][q];
                    p[r] += act[r] ? 64 : 0;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (pk[r]) st[r] = parked[r];
        // remaining blocks and ragged tails, run by run
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (ok[r]) {
                const uint32_t f = scan_lane<TE>(st[r], p[r], vend[r], end[r], tab, cls, dead);
                a.run_final[ri[r]] = f == dead ? kNoState : f / a.s.row_bytes;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// views of the chunk maps for the join
// ---------------------------------------------------------------------------

template <typename TL>
struct PlainView {
    const TL *lam;
    uint32_t nchunks;
    __device__ __forceinline__ uint32_t get(uint32_t s, uint32_t c) const {
        const TL v = lam[(uint64_t)s * nchunks + c];
        return v == all_ones<TL>() ? kNoState : (uint32_t)v;
    }
};

template <typename TA>
struct ConvView {
    const TA *alias;           // [nchunks][L]
    const uint32_t *base;
    const uint32_t *fin;
    uint32_t L;
    __device__ __forceinline__ uint32_t get(uint32_t s, uint32_t c) const {
        const TA v = alias[(uint64_t)c * L + s];
        return v == all_ones<TA>() ? kNoState : fin[base[c] + v];
    }
};

template <class F>
hipError_t with_view(const JoinArgs &a, F &&f) {
    if (!a.converged) {
        if (a.tile_bytes == 2) return f(PlainView<uint16_t>{(const uint16_t *)a.lam, a.nchunks});
        return f(PlainView<uint32_t>{(const uint32_t *)a.lam, a.nchunks});
    }
    if (a.alias_bytes == 1)
        return f(ConvView<uint8_t>{(const uint8_t *)a.alias, a.run_base, a.run_final, a.L});
    return f(ConvView<uint16_t>{(const uint16_t *)a.alias, a.run_base, a.run_final, a.L});
}

// ---------------------------------------------------------------------------
// join: relations over interface states (RI-DFA)
// ---------------------------------------------------------------------------

template <int W>
__device__ __forceinline__ void or_row(uint32_t (&y)[W], const uint32_t *row) {
    if constexpr (W % 4 == 0) {
#pragma unroll
        for (int w = 0; w < W; w += 4) {
            const uint4 v = *reinterpret_cast<const uint4 *>(row + w);
            y[w] |= v.x; y[w + 1] |= v.y; y[w + 2] |= v.z; y[w + 3] |= v.w;
        }
    } else {
#pragma unroll
        for (int w = 0; w < W; ++w) y[w] |= row[w];
    }
}

template <int W>
__device__ __forceinline__ bool empty_row(const uint32_t (&x)[W]) {
    uint32_t o = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) o |= x[w];
    return o == 0;
}

// Level 0: thread per (group of G chunks, start s).  X starts as the content
// of lambda_first(s); each later chunk of the group replaces X by the union
// of content(lambda_c(t)) over t in X.
template <int W, class View>
__global__ void __launch_bounds__(256) join0_rel_kernel(JoinArgs a, View view) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ngroups = (a.nchunks + a.G - 1) / a.G;
    if (tid >= (uint64_t)ngroups * a.L) return;
    const uint32_t grp = (uint32_t)(tid / a.L), s = (uint32_t)(tid % a.L);
    const uint32_t c0 = grp * a.G;
    const uint32_t c1 = c0 + a.G < a.nchunks ? c0 + a.G : a.nchunks;
    uint32_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = 0;
    {
        const uint32_t v = view.get(s, c0);
        if (v != kNoState) or_row<W>(x, a.content + (uint64_t)v * W);
    }
    for (uint32_t c = c0 + 1; c < c1 && !empty_row<W>(x); ++c) {
        uint32_t y[W];
#pragma unroll
        for (int w = 0; w < W; ++w) y[w] = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            for (uint32_t bits = x[w]; bits; bits &= bits - 1) {
                const uint32_t v = view.get(w * 32 + __builtin_ctz(bits), c);
                if (v != kNoState) or_row<W>(y, a.content + (uint64_t)v * W);
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = y[w];
    }
    uint32_t *out = reinterpret_cast<uint32_t *>(a.out) + tid * W;
#pragma unroll
    for (int w = 0; w < W; ++w) out[w] = x[w];
}

// Level 0, staged: one block per group of G consecutive chunks.  The group's
// chunk maps are first gathered into LDS as state ids ([L][G], one coalesced
// sweep), so the chains of dependent lookups below run at LDS latency.
// W = 0: partial functions (DFA); W > 0: relations (RI-DFA).
template <int W, class View>
__global__ void __launch_bounds__(256) join0_tile_kernel(JoinArgs a, View view) {
    extern __shared__ __align__(16) uint32_t lt[];
    const uint32_t G = a.G;
    const uint32_t grp = blockIdx.x;
    const uint32_t c0 = a.grp_first ? a.grp_first[grp] : grp * G;
    const uint32_t gn = a.grp_first ? a.grp_count[grp] : c0 + G < a.nchunks ? G : a.nchunks - c0;
    for (uint32_t i = threadIdx.x; i < a.L * G; i += blockDim.x) {
        const uint32_t s = i / G, c = i - s * G;
        lt[i] = c < gn ? view.get(s, c0 + c) : kNoState;
    }
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < a.L; s += blockDim.x) {
        if constexpr (W == 0) {
            uint32_t v = lt[s * G];
            for (uint32_t c = 1; c < gn && v != kNoState; ++c) v = lt[v * G + c];
            reinterpret_cast<int32_t *>(a.out)[(uint64_t)grp * a.L + s] = v == kNoState ? -1 : (int32_t)v;
        } else {
            uint32_t x[W];
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] = 0;
            {
                const uint32_t v = lt[s * G];
                if (v != kNoState) or_row<W>(x, a.content + (uint64_t)v * W);
            }
            for (uint32_t c = 1; c < gn && !empty_row<W>(x); ++c) {
                uint32_t y[W];
#pragma unroll
                for (int w = 0; w < W; ++w) y[w] = 0;
                uint32_t last = kNoState;   // runs of one chunk are often shared: skip repeats
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    for (uint32_t bits = x[w]; bits; bits &= bits - 1) {
                        const uint32_t v = lt[(w * 32 + __builtin_ctz(bits)) * G + c];
                        if (v != kNoState && v != last) {
                            or_row<W>(y, a.content + (uint64_t)v * W);
                            last = v;
                        }
                    }
                }
#pragma unroll
                for (int w = 0; w < W; ++w) x[w] = y[w];
            }
            uint32_t *out = reinterpret_cast<uint32_t *>(a.out) + ((uint64_t)grp * a.L + s) * W;
#pragma unroll
            for (int w = 0; w < W; ++w) out[w] = x[w];
        }
    }
}

// ---------------------------------------------------------------------------
// join over merged runs: class-partitioned relations (RI-DFA)
// ---------------------------------------------------------------------------
//
// After merging, the starts of a chunk fall into a few classes (one per
// run); starts of one class have the same row.  A relation over a span of
// chunks is kept as the classes of its FIRST chunk (the alias column of that
// chunk) plus one propagated content bitset per class.  Composing relations
// propagates each class content X through the next member: the member's
// classes hit by X are {alias[t][first chunk] : t in X}, and the new X is the
// union of their contents.  Only the first member's classes are propagated,
// so a group costs (#classes) chains instead of L.
//
// One block per group of G members.  LDS holds the members' first-chunk
// alias columns [L][G] and the contents of each member's first kClsStage
// classes; larger classes are read from global memory.
constexpr uint32_t kClsStage = 8;

template <int W, typename TA, bool LEVEL0>
__global__ void __launch_bounds__(256) join_cls_kernel(ClsJoinArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *scont = reinterpret_cast<uint32_t *>(smem);                    // [G][kClsStage][W]
    uint32_t *sncls = scont + (size_t)a.G * kClsStage * W;                    // [G]
    TA *salias = reinterpret_cast<TA *>(sncls + a.G);                         // [L][GS]
    const uint32_t G = a.G, L = a.L;
    const uint32_t GS = tile_stride<TA>(G);
    const uint32_t grp = blockIdx.x;
    const uint32_t m0 = a.grp_first ? a.grp_first[grp] : grp * G;
    const uint32_t gn = a.grp_first ? a.grp_count[grp] : m0 + G < a.nmembers ? G : a.nmembers - m0;
    const TA *alias = reinterpret_cast<const TA *>(a.alias);

    // member k of the group: first chunk (m0 + k) * span, or as listed
    for (uint32_t i = threadIdx.x; i < G; i += blockDim.x) sncls[i] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < L * G; i += blockDim.x) {
        const uint32_t t = i / G, k = i - t * G;
        TA v = all_ones<TA>();
        if (k < gn) {
            const uint64_t c = a.member_chunk ? a.member_chunk[m0 + k] : (uint64_t)(m0 + k) * a.span;
            v = alias[c * L + t];
            if (LEVEL0 && v != all_ones<TA>()) atomicMax(&sncls[k], (uint32_t)v + 1);
        }
        salias[t * GS + k] = v;
    }
    if (!LEVEL0)
        for (uint32_t k = threadIdx.x; k < gn; k += blockDim.x) sncls[k] = a.ncls_in[m0 + k];
    __syncthreads();

    // contents of member k's class b (global)
    auto content_ptr = [&](uint32_t k, uint32_t b) -> const uint32_t * {
        if (LEVEL0) {
            const uint32_t c = m0 + k;
            const uint32_t f = a.run_final[a.run_base[c] + b];
            return f == kNoState ? nullptr : a.content + (uint64_t)f * W;
        }
        return a.cont_in + ((uint64_t)(m0 + k) * L + b) * W;
    };
    for (uint32_t i = threadIdx.x; i < gn * kClsStage; i += blockDim.x) {
        const uint32_t k = i / kClsStage, b = i - k * kClsStage;
        uint32_t *dst = scont + (size_t)i * W;
        const uint32_t *src = b < sncls[k] ? content_ptr(k, b) : nullptr;
#pragma unroll
        for (int w = 0; w < W; ++w) dst[w] = src ? src[w] : 0u;
    }
    __syncthreads();

    // one wave per class of member 0; lane w < W holds word w of the content
    const uint32_t lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const uint32_t nw = blockDim.x / kWave;
    const uint32_t ncls0 = sncls[0];
    for (uint32_t cls = wave; cls < ncls0; cls += nw) {
        uint32_t xw = 0;
        if (lane < (uint32_t)W) {
            const uint32_t *src = cls < kClsStage ? scont + (size_t)cls * W : content_ptr(0, cls);
            xw = src ? src[lane] : 0u;
        }
        for (uint32_t k = 1; k < gn; ++k) {
            if (__ballot(xw != 0) == 0) break;
            uint32_t hit = 0;          // staged classes (< kClsStage) hit, this lane's share
            uint32_t yw = 0;
            for (uint32_t t0 = 0; t0 < L; t0 += kWave) {
                const uint32_t t = t0 + lane;
                const uint32_t word = __shfl(xw, (int)((t0 + lane) / 32 < (uint32_t)W ? (t0 + lane) / 32 : 0));
                const bool in = t < L && ((word >> (t & 31)) & 1u);
                const TA b = in ? salias[t * GS + k] : all_ones<TA>();
                if (b != all_ones<TA>() && (uint32_t)b < kClsStage) hit |= 1u << b;
                // classes beyond the staged ones: OR their contents lane by lane
                uint64_t big = __ballot(b != all_ones<TA>() && (uint32_t)b >= kClsStage);
                while (big) {
                    const int src_lane = __builtin_ctzll(big);
                    big &= big - 1;
                    const uint32_t bb = (uint32_t)__shfl((int)b, src_lane);
                    const uint32_t *src = content_ptr(k, bb);
                    if (src && lane < (uint32_t)W) yw |= src[lane];
                }
            }
            // OR of the hit masks over the wave
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) hit |= (uint32_t)__shfl_xor((int)hit, d);
            if (lane < (uint32_t)W)
                for (; hit; hit &= hit - 1) yw |= scont[((size_t)k * kClsStage + __builtin_ctz(hit)) * W + lane];
            xw = yw;
        }
        if (lane < (uint32_t)W) a.cont_out[((uint64_t)grp * L + cls) * W + lane] = xw;
    }
    if (threadIdx.x == 0) a.ncls_out[grp] = ncls0;
}

// ---------------------------------------------------------------------------
// join over merged runs: products of hit matrices (RI-DFA)
// ---------------------------------------------------------------------------

// A hit matrix keeps kRowCap = 8 rows and 8 columns (a chunk with more
// classes flags the result as invalid, so wider columns are never needed):
// row r is byte r of one 64-bit word, bit c of that byte is column c.
constexpr uint64_t kByteLsb = 0x0101010101010101ull;

// Boolean product a * b: row r of the result is the union of the rows j of b
// for which a[r][j] is set.  For each j, bit j of every row of a is widened
// to a byte mask and selects a copy of row j of b; no data-dependent loop.
__device__ __forceinline__ uint64_t mat8_times(uint64_t a, uint64_t b) {
    uint64_t c = 0;
#pragma unroll
    for (uint32_t j = 0; j < kRowCap; ++j) {
        const uint64_t col = (a >> j) & kByteLsb;     // a[r][j] as 0 / 1 in byte r
        const uint64_t sel = (col << 8) - col;        // 0xFF in the selected rows
        c |= sel & (((b >> (8 * j)) & 0xFFull) * kByteLsb);
    }
    return c;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return (uint64_t)hi << 32 | lo;
}

// Tree product of the wave's gn members (lane l holds member l): after it
// lane 0 holds the product of all of them, in order.
__device__ __forceinline__ void wave_tree_product(uint64_t &m, uint32_t lane, uint32_t gn) {
#pragma unroll
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        const uint64_t b = shfl64(m, (int)((lane + d) % kWave));
        if ((lane & (2 * d - 1)) == 0 && lane + d < gn) m = mat8_times(m, b);
    }
}

// Level 0, fused with the hit rows: wave per group of 64 matrices; lane l
// builds M_k (k = 64 g + l) from the end states of chunk k's runs and the
// alias column of chunk k + 1.
template <int W, typename TA, bool STAGE>
__global__ void __launch_bounds__(256) hit_prod0_kernel(HitArgs a) {
    extern __shared__ __align__(16) uint8_t hsm[];
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t g = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const uint32_t ngroups = (a.nmembers + kWave - 1) / kWave;
    if (g >= ngroups) return;
    const uint32_t gn = g * kWave + kWave <= a.nmembers ? kWave : a.nmembers - g * kWave;
    const uint32_t k = g * kWave + lane;
    const TA *alias = reinterpret_cast<const TA *>(a.alias);
    // STAGE: the wave's next-chunk rows (chunks 64 g + 1 .. 64 g + gn, one
    // contiguous span) are copied to LDS first, lanes over elements
    TA *srow = reinterpret_cast<TA *>(hsm) + (size_t)(threadIdx.x / kWave) * kWave * a.L;
    if constexpr (STAGE) {
        const TA *src = alias + (uint64_t)(g * kWave + 1) * a.L;
        for (uint32_t i = lane; i < gn * a.L; i += kWave) srow[i] = src[i];
        __builtin_amdgcn_wave_barrier();   // the rows are read by other lanes of this wave
    }
    uint64_t M = 0;
    uint32_t R = 0;
    if (lane < gn) {
        R = a.run_count[k];
        R = R < kRowCap ? R : kRowCap;
    }
#pragma unroll
    for (uint32_t r = 0; r < kRowCap; ++r) {
        uint64_t m = 0;
        if (r < R) {
            const uint32_t f = a.run_final[a.run_base[k] + r];
            if (f != kNoState) {
                const TA *row = STAGE ? srow + (size_t)lane * a.L : alias + (uint64_t)(k + 1) * a.L;
                if constexpr (W > 0) {
                    const uint32_t *cw = a.content + (uint64_t)f * W;
                    for (uint32_t w = 0; w < (uint32_t)W; ++w)
                        for (uint32_t bits = cw[w]; bits; bits &= bits - 1) {
                            const TA j = row[w * 32 + __builtin_ctz(bits)];
                            if (j != all_ones<TA>() && (uint32_t)j < kRowCap) m |= 1ull << j;
                        }
                } else {
                    for (uint32_t i = a.csr_off[f], ie = a.csr_off[f + 1]; i < ie; ++i) {
                        const TA j = row[a.csr_idx[i]];
                        if (j != all_ones<TA>() && (uint32_t)j < kRowCap) m |= 1ull << j;
                    }
                }
            }
        }
        M |= m << (8 * r);
    }
    wave_tree_product(M, lane, gn);
    if (lane == 0) {
        a.prod_out[g] = M;
        a.rows_out[g] = R;
    }
}

// Level >= 1: wave per group of 64 products of the level below.
__global__ void __launch_bounds__(256) hit_prodN_kernel(HitArgs a) {
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t g = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const uint32_t ngroups = (a.nmembers + kWave - 1) / kWave;
    if (g >= ngroups) return;
    const uint32_t gn = g * kWave + kWave <= a.nmembers ? kWave : a.nmembers - g * kWave;
    const uint32_t m = g * kWave + lane;
    uint64_t M = lane < gn ? a.prod_in[m] : 0ull;
    const uint32_t R = lane < gn ? a.rows_in[m] : 0u;
    wave_tree_product(M, lane, gn);
    if (lane == 0) {
        a.prod_out[g] = M;
        a.rows_out[g] = R;
    }
}

// Level >= 1: thread per (group of G relations, row s).
template <int W>
__global__ void __launch_bounds__(256) joinN_rel_kernel(JoinArgs a) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ngroups = (a.nin + a.G - 1) / a.G;
    if (tid >= (uint64_t)ngroups * a.L) return;
    const uint32_t grp = (uint32_t)(tid / a.L), s = (uint32_t)(tid % a.L);
    const uint32_t *in = reinterpret_cast<const uint32_t *>(a.in);
    const uint32_t k0 = grp * a.G;
    const uint32_t k1 = k0 + a.G < a.nin ? k0 + a.G : a.nin;
    uint32_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = 0;
    or_row<W>(x, in + ((uint64_t)k0 * a.L + s) * W);
    for (uint32_t k = k0 + 1; k < k1 && !empty_row<W>(x); ++k) {
        uint32_t y[W];
#pragma unroll
        for (int w = 0; w < W; ++w) y[w] = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            for (uint32_t bits = x[w]; bits; bits &= bits - 1) {
                const uint32_t t = w * 32 + __builtin_ctz(bits);
                or_row<W>(y, in + ((uint64_t)k * a.L + t) * W);
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = y[w];
    }
    uint32_t *out = reinterpret_cast<uint32_t *>(a.out) + tid * W;
#pragma unroll
    for (int w = 0; w < W; ++w) out[w] = x[w];
}

// ---------------------------------------------------------------------------
// join: partial functions over DFA states
// ---------------------------------------------------------------------------

template <class View>
__global__ void __launch_bounds__(256) join0_fun_kernel(JoinArgs a, View view) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ngroups = a.grp_first ? a.ngroups : (a.nchunks + a.G - 1) / a.G;
    if (tid >= (uint64_t)ngroups * a.L) return;
    const uint32_t grp = (uint32_t)(tid / a.L), s = (uint32_t)(tid % a.L);
    const uint32_t c0 = a.grp_first ? a.grp_first[grp] : grp * a.G;
    const uint32_t c1 = a.grp_first ? c0 + a.grp_count[grp] : c0 + a.G < a.nchunks ? c0 + a.G : a.nchunks;
    uint32_t v = view.get(s, c0);
    for (uint32_t c = c0 + 1; c < c1 && v != kNoState; ++c) v = view.get(v, c);
    reinterpret_cast<int32_t *>(a.out)[tid] = v == kNoState ? -1 : (int32_t)v;
}

__global__ void __launch_bounds__(256) joinN_fun_kernel(JoinArgs a) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ngroups = a.grp_first ? a.ngroups : (a.nin + a.G - 1) / a.G;
    if (tid >= (uint64_t)ngroups * a.L) return;
    const uint32_t grp = (uint32_t)(tid / a.L), s = (uint32_t)(tid % a.L);
    const int32_t *in = reinterpret_cast<const int32_t *>(a.in);
    const uint32_t k0 = a.grp_first ? a.grp_first[grp] : grp * a.G;
    const uint32_t k1 = a.grp_first ? k0 + a.grp_count[grp] : k0 + a.G < a.nin ? k0 + a.G : a.nin;
    int32_t v = in[(uint64_t)k0 * a.L + s];
    for (uint32_t k = k0 + 1; k < k1 && v >= 0; ++k) v = in[(uint64_t)k * a.L + v];
    reinterpret_cast<int32_t *>(a.out)[tid] = v;
}

template <class View>
__global__ void __launch_bounds__(256) materialize_kernel(JoinArgs a, View view, int32_t *out) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (uint64_t)a.L * a.nchunks) return;
    const uint32_t s = (uint32_t)(tid / a.nchunks), c = (uint32_t)(tid % a.nchunks);
    const uint32_t v = view.get(s, c);
    out[tid] = v == kNoState ? -1 : (int32_t)v;
}

// ---------------------------------------------------------------------------
// finalize
// ---------------------------------------------------------------------------

__device__ __forceinline__ void reset_counters(uint32_t *c) {
    c[0] = 0; c[1] = 0; c[2] = 0; c[3] = 0;
}

// Acceptance and final state of a set X of N' states (the union content of
// the relation row of the initial state): accept iff X meets the final
// states of N'; final state = the canonical minimal-DFA id stored for the
// RI-DFA state whose content is X (found by the hash of X's members, then a
// comparison of member lists); -1 when X is empty.
__device__ __forceinline__ uint32_t fnv_step(uint32_t h, uint32_t m) { return (h ^ m) * 16777619u; }

// Probe for the state whose members equal X: `same(p)` compares.
template <class Same>
__device__ int32_t lookup_set(uint32_t h, Same same, const FinalArgs &f) {
    uint32_t slot = h & (f.hash_cap - 1);
    for (uint32_t probe = 0; probe < f.hash_cap; ++probe) {
        const uint32_t p = f.hash[(uint64_t)slot * 2];
        if (p == 0xFFFFFFFFu) break;   // empty slot
        if (same(p)) return (int32_t)f.hash[(uint64_t)slot * 2 + 1];
        slot = (slot + 1) & (f.hash_cap - 1);
    }
    return -3;   // not found: cannot happen for a reachable subset
}

// member list of p has exactly cnt members, all in X
template <class Has>
__device__ __forceinline__ bool same_list(uint32_t p, uint32_t cnt, Has has, const FinalArgs &f) {
    const uint32_t b = f.csr_off[p], e = f.csr_off[p + 1];
    if (e - b != cnt) return false;
    bool eq = true;
    for (uint32_t i = b; i < e && eq; ++i) eq = has(f.csr_idx[i]);
    return eq;
}

// X as a bitset of nw words (any memory)
__device__ void decide_bits(const uint32_t *x, uint32_t nw, const FinalArgs &f, int32_t *res) {
    uint32_t acc = 0, cnt = 0, h = 2166136261u;
    for (uint32_t w = 0; w < nw; ++w) {
        acc |= x[w] & f.fmask[w];
        cnt += __builtin_popcount(x[w]);
        for (uint32_t bits = x[w]; bits; bits &= bits - 1) h = fnv_step(h, w * 32 + __builtin_ctz(bits));
    }
    int32_t fin = -1;
    if (cnt)
        fin = lookup_set(h, [&](uint32_t p) {
            return same_list(p, cnt, [&](uint32_t m) { return ((x[m >> 5] >> (m & 31)) & 1u) != 0; }, f);
        }, f);
    res[0] = acc != 0;
    res[1] = fin;
}

// X as W <= 64 words in registers; candidates compared with their dense rows
template <int W>
__device__ __forceinline__ void decide(const uint32_t (&x)[W], const FinalArgs &f, int32_t *res) {
    uint32_t acc = 0, any = 0, h = 2166136261u;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        acc |= x[w] & f.fmask[w];
        any |= x[w];
        for (uint32_t bits = x[w]; bits; bits &= bits - 1) h = fnv_step(h, w * 32 + __builtin_ctz(bits));
    }
    int32_t fin = -1;
    if (any)
        fin = lookup_set(h, [&](uint32_t p) {
            const uint32_t *row = f.content + (uint64_t)p * W;
            bool eq = true;
#pragma unroll
            for (int w = 0; w < W; ++w) eq &= row[w] == x[w];
            return eq;
        }, f);
    res[0] = acc != 0;
    res[1] = fin;
}

// X as the union of up to kRowCap sorted member lists
struct ListUnion {
    const uint32_t *b[kRowCap];
    const uint32_t *e[kRowCap];
    uint32_t k;
    __device__ bool has(uint32_t m) const {
        for (uint32_t i = 0; i < k; ++i) {
            const uint32_t *lo = b[i], *hi = e[i];
            while (lo < hi) {
                const uint32_t *mid = lo + (hi - lo) / 2;
                if (*mid < m) lo = mid + 1;
                else hi = mid;
            }
            if (lo < e[i] && *lo == m) return true;
        }
        return false;
    }
};

__device__ void decide_lists(const ListUnion &u, const FinalArgs &f, int32_t *res) {
    const uint32_t *pos[kRowCap];
    for (uint32_t i = 0; i < u.k; ++i) pos[i] = u.b[i];
    uint32_t acc = 0, cnt = 0, h = 2166136261u;
    for (;;) {   // ascending merge without repeats
        uint32_t m = 0xFFFFFFFFu;
        for (uint32_t i = 0; i < u.k; ++i)
            if (pos[i] < u.e[i] && *pos[i] < m) m = *pos[i];
        if (m == 0xFFFFFFFFu) break;
        for (uint32_t i = 0; i < u.k; ++i)
            if (pos[i] < u.e[i] && *pos[i] == m) ++pos[i];
        acc |= (f.fmask[m >> 5] >> (m & 31)) & 1u;
        ++cnt;
        h = fnv_step(h, m);
    }
    int32_t fin = -1;
    if (cnt) fin = lookup_set(h, [&](uint32_t p) { return same_list(p, cnt, [&](uint32_t m) { return u.has(m); }, f); }, f);
    res[0] = acc != 0;
    res[1] = fin;
}

template <int W>
__device__ __forceinline__ void load_row(uint32_t (&x)[W], const uint32_t *row) {
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = row ? row[w] : 0u;
}

template <int W>
__global__ void finalize_rel_kernel(FinalArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t x[W];
    load_row<W>(x, reinterpret_cast<const uint32_t *>(a.total));   // row 0
    decide<W>(x, a, a.result);
    reset_counters(a.counters);
}

// Row of start 0 of the single remaining class-partitioned relation: the
// class alias[0][chunk 0].
template <int W, typename TA>
__global__ void finalize_cls_kernel(FinalArgs f, ClsJoinArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const TA c0 = reinterpret_cast<const TA *>(a.alias)[0];
    uint32_t x[W];
    load_row<W>(x, c0 != all_ones<TA>() ? a.cont_in + (uint64_t)c0 * W : nullptr);
    decide<W>(x, f, f.result);
    reset_counters(f.counters);
}

// Classes of the last chunk reached from start 0 (row a0 of the product, a0
// = class of start 0 in chunk 0), union of their end-state contents, then
// acceptance and final state.
// The join by propagation (defined below) run by the calling block; sm holds
// 3 W words.
template <typename TA>
__device__ void propagate_block(const FinalArgs &f, const HitArgs &a, uint32_t W, uint32_t *sm);

// prod: the whole product M_0 ... M_{K-2} when `have` (not for a single
// chunk).  One thread.
template <int W, typename TA>
__device__ uint32_t finalize_hit_one(const FinalArgs &f, const HitArgs &a, bool have, uint64_t prod) {
    const TA a0 = reinterpret_cast<const TA *>(a.alias)[0];
    uint64_t v = 0;
    if (a0 != all_ones<TA>() && (uint32_t)a0 < kRowCap) v = have ? (prod >> (8 * (uint32_t)a0)) & 0xFFull : 1ull << a0;
    const uint32_t last = a.nchunks - 1;
    const uint32_t R = a.run_count[last];
    if constexpr (W > 0) {
        uint32_t x[W];
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = 0;
        for (; v; v &= v - 1) {
            const uint32_t c = __builtin_ctzll(v);
            if (c >= R) continue;
            const uint32_t fs = a.run_final[a.run_base[last] + c];
            if (fs == kNoState) continue;
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] |= a.content[(uint64_t)fs * W + w];
        }
        decide<W>(x, f, f.result);
    } else {
        ListUnion u;
        u.k = 0;
        for (; v && u.k < kRowCap; v &= v - 1) {
            const uint32_t c = __builtin_ctzll(v);
            if (c >= R) continue;
            const uint32_t fs = a.run_final[a.run_base[last] + c];
            if (fs == kNoState) continue;
            u.b[u.k] = a.csr_idx + a.csr_off[fs];
            u.e[u.k] = a.csr_idx + a.csr_off[fs + 1];
            ++u.k;
        }
        decide_lists(u, f, f.result);
    }
    const uint32_t flag = f.counters[2];
    f.result[2] = (int32_t)flag;
    reset_counters(f.counters);
    return flag;
}

// The last level of the hit-matrix product (at most 64 products, a.nmembers
// of them in a.prod_in; 0 for a single chunk) and the final step, in one wave.
// With out != nullptr the result is also copied to out; when a chunk kept
// more runs than a hit row holds, the wave first joins again by propagation
// (prop_words words per set of N' states, 12 bytes per word of dynamic LDS).
template <int W, typename TA>
__global__ void __launch_bounds__(64) hit_tail_kernel(FinalArgs f, HitArgs a, uint32_t prop_words, int32_t *out) {
    const uint32_t lane = threadIdx.x;
    const uint32_t nm = a.nmembers;
    uint64_t M = lane < nm ? a.prod_in[lane] : 0ull;
    if (nm > 1) wave_tree_product(M, lane, nm);
    uint32_t redo = 0;
    if (lane == 0) redo = finalize_hit_one<W, TA>(f, a, nm > 0, M);
    if (!out) return;
    redo = (uint32_t)__shfl((int)redo, 0);
    if (redo) {
        extern __shared__ __align__(16) uint32_t tsm[];
        propagate_block<TA>(f, a, prop_words, tsm);   // ends with the result in f.result
    }
    if (lane == 0) {
        out[0] = f.result[0];
        out[1] = f.result[1];
    }
}

// One block: the set X of N' states (a bitset in LDS) is carried from chunk
// to chunk: the classes of chunk k hit by X are {alias[k][t] : t in X}, and
// the new X is the union of the contents of their end states.  Exact for any
// number of runs per chunk.
template <typename TA>
__device__ void propagate_block(const FinalArgs &f, const HitArgs &a, uint32_t W, uint32_t *sm) {
    uint32_t *X = sm;               // [W]
    uint32_t *Y = sm + W;           // [W]
    uint32_t *H = sm + 2 * W;       // [W] classes hit (a chunk has at most L runs)
    const TA *alias = reinterpret_cast<const TA *>(a.alias);
    for (uint32_t w = threadIdx.x; w < W; w += blockDim.x) X[w] = 0;
    __syncthreads();
    // chunk 0: start 0 only
    {
        const TA c0 = alias[0];
        if (c0 != all_ones<TA>()) {
            const uint32_t fs = a.run_final[a.run_base[0] + c0];
            if (fs != kNoState)
                for (uint32_t i = a.csr_off[fs] + threadIdx.x; i < a.csr_off[fs + 1]; i += blockDim.x) {
                    const uint32_t m = a.csr_idx[i];
                    atomicOr(&X[m >> 5], 1u << (m & 31));
                }
        }
    }
    __syncthreads();
    for (uint32_t k = 1; k < a.nchunks; ++k) {
        for (uint32_t w = threadIdx.x; w < W; w += blockDim.x) { H[w] = 0; Y[w] = 0; }
        __syncthreads();
        const TA *row = alias + (uint64_t)k * a.L;
        for (uint32_t w = threadIdx.x; w < W; w += blockDim.x)
            for (uint32_t bits = X[w]; bits; bits &= bits - 1) {
                const TA c = row[w * 32 + __builtin_ctz(bits)];
                if (c != all_ones<TA>()) atomicOr(&H[(uint32_t)c >> 5], 1u << ((uint32_t)c & 31));
            }
        __syncthreads();
        const uint32_t base = a.run_base[k];
        for (uint32_t w = threadIdx.x; w < W; w += blockDim.x)
            for (uint32_t bits = H[w]; bits; bits &= bits - 1) {
                const uint32_t fs = a.run_final[base + w * 32 + __builtin_ctz(bits)];
                if (fs == kNoState) continue;
                for (uint32_t i = a.csr_off[fs]; i < a.csr_off[fs + 1]; ++i) {
                    const uint32_t m = a.csr_idx[i];
                    atomicOr(&Y[m >> 5], 1u << (m & 31));
                }
            }
        __syncthreads();
        for (uint32_t w = threadIdx.x; w < W; w += blockDim.x) X[w] = Y[w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        decide_bits(X, W, f, f.result);
        f.result[2] = 0;
        reset_counters(f.counters);
    }
}

template <typename TA>
__global__ void __launch_bounds__(1024) propagate_kernel(FinalArgs f, HitArgs a, uint32_t W) {
    extern __shared__ __align__(16) uint32_t sm[];
    propagate_block<TA>(f, a, W, sm);
}

__global__ void store_result_kernel(int32_t *out, int32_t accept, int32_t final_state) {
    if (threadIdx.x == 0) {
        out[0] = accept;
        out[1] = final_state;
    }
}

// Batch: thread per text; group t of the last level holds text t's relation.
template <int W, typename TA>
__global__ void batch_final_cls_kernel(BatchFinalArgs b, FinalArgs f, ClsJoinArgs a) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) reset_counters(f.counters);
    if (t >= b.ntexts) return;
    const TA c0 = reinterpret_cast<const TA *>(a.alias)[(uint64_t)b.text_slot[t] * a.L];   // start 0's class
    uint32_t x[W];
    load_row<W>(x, c0 != all_ones<TA>() ? a.cont_in + ((uint64_t)t * a.L + c0) * W : nullptr);
    decide<W>(x, f, b.results + (uint64_t)b.text_out[t] * 2);
}

__global__ void batch_final_fun_kernel(BatchFinalArgs b, FinalArgs f, uint32_t L) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) reset_counters(f.counters);
    if (t >= b.ntexts) return;
    const int32_t v = reinterpret_cast<const int32_t *>(f.total)[(uint64_t)t * L];
    int32_t *res = b.results + (uint64_t)b.text_out[t] * 2;
    res[0] = v >= 0 ? (int32_t)f.accept_of_state[v] : 0;
    res[1] = v >= 0 ? f.final_of_state[v] : -1;
}

__global__ void batch_fill_kernel(BatchFinalArgs b) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.ntexts) return;
    int32_t *res = b.results + (uint64_t)b.text_out[t] * 2;
    res[0] = 0;
    res[1] = -1;
}

__global__ void finalize_fun_kernel(FinalArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int32_t t = reinterpret_cast<const int32_t *>(a.total)[0];
    a.result[0] = t >= 0 ? (int32_t)a.accept_of_state[t] : 0;
    a.result[1] = t >= 0 ? a.final_of_state[t] : -1;
    reset_counters(a.counters);
}

uint32_t blocks_for(uint64_t threads, uint32_t per) { return (uint32_t)((threads + per - 1) / per); }

// ---------------------------------------------------------------------------
// fused batches: every slot and text names its automaton
// ---------------------------------------------------------------------------

template <class F>
__device__ __forceinline__ void with_entry(uint32_t eb, F &&f) {
    if (eb == 1) f((uint8_t)0);
    else if (eb == 2) f((uint16_t)0);
    else f((uint32_t)0);
}

__device__ __forceinline__ void slot_bounds(const MultiArgs &a, uint32_t slot, uint64_t &b, uint64_t &e, bool &first) {
    const uint32_t l = a.chunk_len[slot];
    b = a.chunk_addr[slot];
    e = b + (l & 0x7fffffffu);
    first = (l >> 31) != 0;
}

// warm-up and merging: one wavefront per slot, 16 slots per block iteration
// (8 waves per SIMD: two 16-wave blocks per CU, as for warm_kernel)
__global__ void __launch_bounds__(1024, 8) mwarm_kernel(MultiArgs a) {
    __shared__ uint32_t s_cnt[2][kWarmWaves + 1];
    uint32_t buf = 0;
    constexpr int R = 4;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t wave = wave_uniform(threadIdx.x / kWave);
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const uint32_t iters = (a.nslots + kWarmWaves - 1) / kWarmWaves;
    for (uint32_t it = blockIdx.x; it < iters; it += gridDim.x, buf ^= 1) {
        const uint32_t slot = it * kWarmWaves + wave;
        const bool ok = slot < a.nslots;
        const AutoDesc &d = a.autos[ok ? a.slot_auto[slot] : 0];
        const bool okl = ok && d.L > 0;
        uint64_t b = 0, e = 0;
        bool first = false;
        if (ok) slot_bounds(a, slot, b, e, first);
        b = wave_uniform(b);
        first = wave_uniform((uint32_t)first) != 0;
        const uint32_t wlen = wave_uniform(okl ? (uint32_t)(e - b < a.warm ? e - b : a.warm) : 0u);
        StartList starts;
        starts.lds = nullptr;
        starts.glb = (const __attribute__((address_space(1))) uint32_t *)d.starts;
        starts.staged = false;
        uint32_t code[4] = {0, 0, 0, 0};
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t j = q * kWave + lane;
            if (j < wlen) code[q] = d.code[*at(b + j)];
        }
        uint16_t *arow = a.alias + (ok ? a.alias_row[slot] : 0);
        uint32_t al[R], D = 0, cs = 0;
        bool spill = false;
        if (okl)
            with_entry(d.entry_bytes, [&](auto te) {
                using TE = decltype(te);
                warm_classes<TE, uint16_t, R, 4>(reinterpret_cast<const TE *>(d.table), starts, d.L, d.dead, true,
                                              first, code, wlen, arow, lane, al, D, cs, spill);
            });
        const uint32_t firstrun = warm_slots(s_cnt[buf], lane, wave, ok ? D : 0u, &a.counters[1]);
        if (ok) {
            if (lane == 0) {
                a.run_base[slot] = firstrun;
                a.run_count[slot] = D;
                if (D > kRowCap) a.text_flag[a.slot_text[slot]] = 1u;
            }
            if (okl)
                with_entry(d.entry_bytes, [&](auto te) {
                    using TE = decltype(te);
                    warm_records<TE, uint16_t, R, 4>(reinterpret_cast<const TE *>(d.table), starts, d.L, d.dead,
                                                  d.row_bytes, first, code, wlen, arow, lane, lane_lt, al, D, cs,
                                                  spill, firstrun, slot, a.run_chunk, a.run_state);
                });
        }
    }
}

// merged runs to the end of their chunks: one run per lane, grid-stride
__global__ void __launch_bounds__(256) mlong_kernel(MultiArgs a) {
    const uint32_t nruns = *reinterpret_cast<volatile uint32_t *>(&a.counters[1]);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nruns; i += gridDim.x * blockDim.x) {
        const uint32_t slot = a.run_chunk[i];
        const AutoDesc &d = a.autos[a.slot_auto[slot]];
        uint64_t b, e;
        bool first;
        slot_bounds(a, slot, b, e, first);
        const uint64_t p = b + a.warm < e ? b + a.warm : e;
        const uint64_t vend = p + ((e - p) & ~(uint64_t)15);
        uint32_t f = 0;
        with_entry(d.entry_bytes, [&](auto te) {
            using TE = decltype(te);
            f = scan_lane<TE>(a.run_state[i] * d.row_bytes, p, vend, e, reinterpret_cast<const TE *>(d.table), d.code,
                              d.dead);
        });
        a.run_final[i] = f == d.dead ? kNoState : f / d.row_bytes;
    }
}

// Members of the set a state stands for: its content (RI-DFA) or itself.
template <class F>
__device__ __forceinline__ void for_members(const AutoDesc &d, uint32_t st, F &&f) {
    if (d.functional) {
        f(st);
        return;
    }
    for (uint32_t i = d.csr_off[st], ie = d.csr_off[st + 1]; i < ie; ++i) f(d.csr_idx[i]);
}

// Hit products.  Level 0: wave per group of matrices M_k (slots k and k + 1
// of one text); level >= 1: wave per group of products of the level below.
template <bool LEVEL0>
__global__ void __launch_bounds__(256) mhit_kernel(MultiArgs a) {
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t g = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (g >= a.ngroups) return;
    const uint32_t m0 = a.grp_first[g], gn = a.grp_count[g];
    uint64_t M = 0;
    uint32_t R = 0;
    if (lane < gn) {
        const uint32_t m = m0 + lane;
        if (LEVEL0) {
            const AutoDesc &d = a.autos[a.slot_auto[m]];
            R = a.run_count[m];
            R = R < kRowCap ? R : kRowCap;
            const uint16_t *row = a.alias + a.alias_row[m + 1];
            for (uint32_t r = 0; r < R; ++r) {
                const uint32_t fs = a.run_final[a.run_base[m] + r];
                uint64_t bits = 0;
                if (fs != kNoState)
                    for_members(d, fs, [&](uint32_t t) {
                        const uint16_t j = row[t];
                        if (j != 0xFFFFu && j < kRowCap) bits |= 1ull << j;
                    });
                M |= bits << (8 * r);
            }
        } else {
            M = a.prod[m];
            R = a.prod_rows[m];
        }
    }
    wave_tree_product(M, lane, gn);
    if (lane == 0) {
        const uint64_t o = (uint64_t)(a.prod_out + g);
        a.prod[o] = M;
        a.prod_rows[o] = R;
    }
}

__device__ __forceinline__ FinalArgs final_args(const AutoDesc &d) {
    FinalArgs f{};
    f.fmask = d.fmask;
    f.hash = d.hash;
    f.hash_cap = d.hash_cap;
    f.csr_off = d.csr_off;
    f.csr_idx = d.csr_idx;
    return f;
}

// thread per text: classes of the last slot reached from start 0 of the first
__global__ void __launch_bounds__(256) mfinal_kernel(MultiArgs a) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) reset_counters(a.counters);   // every reader of the counters has run
    if (t >= a.ntexts) return;
    const AutoDesc &d = a.autos[a.text_auto[t]];
    int32_t *res = a.results + (uint64_t)a.text_out[t] * 2;
    res[0] = 0;
    res[1] = -1;
    if (d.L == 0) return;
    const uint32_t s0 = a.text_slot[t], c = a.text_nslots[t], last = s0 + c - 1;
    const uint16_t a0 = a.alias[a.alias_row[s0]];
    uint64_t v = 0;
    if (a0 != 0xFFFFu && a0 < kRowCap) v = c == 1 ? 1ull << a0 : (a.prod[a.text_prod[t]] >> (8 * a0)) & 0xFFull;
    const uint32_t R = a.run_count[last];
    if (d.functional) {
        for (; v; v &= v - 1) {
            const uint32_t ci = __builtin_ctzll(v);
            if (ci >= R) continue;
            const uint32_t fs = a.run_final[a.run_base[last] + ci];
            if (fs == kNoState) continue;
            res[0] = d.accept_of_state[fs];
            res[1] = d.final_of_state[fs];
            break;
        }
        return;
    }
    ListUnion u;
    u.k = 0;
    for (; v && u.k < kRowCap; v &= v - 1) {
        const uint32_t ci = __builtin_ctzll(v);
        if (ci >= R) continue;
        const uint32_t fs = a.run_final[a.run_base[last] + ci];
        if (fs == kNoState) continue;
        u.b[u.k] = d.csr_idx + d.csr_off[fs];
        u.e[u.k] = d.csr_idx + d.csr_off[fs + 1];
        ++u.k;
    }
    decide_lists(u, final_args(d), res);
}

// block per text whose chunks kept more than kRowCap runs: the set of starts
// (members) is carried slot by slot, as in propagate_kernel
__global__ void __launch_bounds__(1024) mprop_kernel(MultiArgs a) {
    extern __shared__ __align__(16) uint32_t sm[];
    const uint32_t t = blockIdx.x;
    if (a.text_flag[t] == 0) return;
    const AutoDesc &d = a.autos[a.text_auto[t]];
    const uint32_t W = d.functional ? (d.L + 31) / 32 : d.W;
    uint32_t *X = sm, *Y = sm + W, *H = sm + 2 * W;
    const uint32_t s0 = a.text_slot[t], c = a.text_nslots[t];
    for (uint32_t w = threadIdx.x; w < W; w += blockDim.x) X[w] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint16_t c0 = a.alias[a.alias_row[s0]];
        if (c0 != 0xFFFFu) {
            const uint32_t fs = a.run_final[a.run_base[s0] + c0];
            if (fs != kNoState) for_members(d, fs, [&](uint32_t m) { X[m >> 5] |= 1u << (m & 31); });
        }
    }
    __syncthreads();
    for (uint32_t k = s0 + 1; k < s0 + c; ++k) {
        for (uint32_t w = threadIdx.x; w < W; w += blockDim.x) { H[w] = 0; Y[w] = 0; }
        __syncthreads();
        const uint16_t *row = a.alias + a.alias_row[k];
        for (uint32_t w = threadIdx.x; w < W; w += blockDim.x)
            for (uint32_t bits = X[w]; bits; bits &= bits - 1) {
                const uint16_t ci = row[w * 32 + __builtin_ctz(bits)];
                if (ci != 0xFFFFu) atomicOr(&H[ci >> 5], 1u << (ci & 31));
            }
        __syncthreads();
        const uint32_t base = a.run_base[k];
        for (uint32_t w = threadIdx.x; w < W; w += blockDim.x)
            for (uint32_t bits = H[w]; bits; bits &= bits - 1) {
                const uint32_t fs = a.run_final[base + w * 32 + __builtin_ctz(bits)];
                if (fs != kNoState) for_members(d, fs, [&](uint32_t m) { atomicOr(&Y[m >> 5], 1u << (m & 31)); });
            }
        __syncthreads();
        for (uint32_t w = threadIdx.x; w < W; w += blockDim.x) X[w] = Y[w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int32_t *res = a.results + (uint64_t)a.text_out[t] * 2;
        if (d.functional) {
            res[0] = 0;
            res[1] = -1;
            for (uint32_t w = 0; w < W; ++w)
                if (X[w]) {
                    const uint32_t st = w * 32 + __builtin_ctz(X[w]);
                    res[0] = d.accept_of_state[st];
                    res[1] = d.final_of_state[st];
                    break;
                }
        } else {
            decide_bits(X, W, final_args(d), res);
        }
        a.text_flag[t] = 0;
    }
}



// ---- template dispatch ----------------------------------------------------

template <class F>
hipError_t dispatch_te(int eb, F &&f) {
    switch (eb) {
    case 1: return f((uint8_t)0);
    case 2: return f((uint16_t)0);
    case 4: return f((uint32_t)0);
    }
    return hipErrorInvalidValue;
}

template <int N> struct IntC { static constexpr int value = N; };

template <class F>
hipError_t dispatch_r(int r, F &&f) {
    switch (r) {
    case 1: return f(IntC<1>{});
    case 2: return f(IntC<2>{});
    case 4: return f(IntC<4>{});
    }
    return hipErrorInvalidValue;
}

template <class F>
hipError_t dispatch_b(bool b, F &&f) {
    return b ? f(std::true_type{}) : f(std::false_type{});
}

template <class F>
hipError_t dispatch_tl(int tb, F &&f) {
    if (tb == 2) return f((uint16_t)0);
    if (tb == 4) return f((uint32_t)0);
    return hipErrorInvalidValue;
}

template <class F>
hipError_t dispatch_ta(int ab, F &&f) {
    if (ab == 1) return f((uint8_t)0);
    if (ab == 2) return f((uint16_t)0);
    return hipErrorInvalidValue;
}

const void *g_fn = nullptr;   // set by the dispatch below when only the function is wanted

}  // namespace

hipError_t launch_plain(const PlainArgs &a, const KernelShape &k, int grid, size_t lds, hipStream_t st) {
    return dispatch_te(k.entry_bytes, [&](auto te) {
        return dispatch_tl(k.tile_bytes, [&](auto tl) {
            return dispatch_r(k.runs_per_lane, [&](auto r) {
                return dispatch_b(k.table_in_lds, [&](auto lds_t) {
                    auto fn = plain_kernel<decltype(te), decltype(tl), decltype(r)::value, decltype(lds_t)::value>;
                    if (grid == 0) { g_fn = reinterpret_cast<const void *>(fn); return hipSuccess; }
                    hipLaunchKernelGGL(fn, dim3(grid), dim3(k.block_threads), lds, st, a);
                    return hipGetLastError();
                });
            });
        });
    });
}

hipError_t launch_warm(const WarmArgs &a, const KernelShape &k, int grid, size_t lds, hipStream_t st) {
    return dispatch_te(k.entry_bytes, [&](auto te) {
        return dispatch_ta(k.alias_bytes, [&](auto ta) {
            return dispatch_r(k.runs_per_lane, [&](auto r) {
                return dispatch_b(k.table_in_lds, [&](auto lds_t) {
                    return dispatch_b(k.code_regs == 1, [&](auto one) {
                        constexpr int NQ = decltype(one)::value ? 1 : 4;
                        auto fn = warm_kernel<decltype(te), decltype(ta), decltype(r)::value, decltype(lds_t)::value, NQ>;
                        if (grid == 0) { g_fn = reinterpret_cast<const void *>(fn); return hipSuccess; }
                        hipLaunchKernelGGL(fn, dim3(grid), dim3(k.block_threads), lds, st, a);
                        return hipGetLastError();
                    });
                });
            });
        });
    });
}

size_t warm_lds_bytes(const KernelShape &k, uint32_t table_bytes, uint32_t L) {
    return (k.table_in_lds ? table_bytes : 0) + 512 + (L <= kStageStarts ? (size_t)L * 4 : 0);
}

hipError_t launch_long(const LongArgs &a, const KernelShape &k, int grid, size_t lds, hipStream_t st) {
    return dispatch_te(k.entry_bytes, [&](auto te) {
        return dispatch_r(k.runs_per_lane, [&](auto r) {
            return dispatch_b(k.table_in_lds, [&](auto lds_t) {
                auto fn = long_kernel<decltype(te), decltype(r)::value, decltype(lds_t)::value>;
                if (grid == 0) { g_fn = reinterpret_cast<const void *>(fn); return hipSuccess; }
                hipLaunchKernelGGL(fn, dim3(grid), dim3(k.block_threads), lds, st, a);
                return hipGetLastError();
            });
        });
    });
}

// Occupancy does not change for a kernel instance, its block size, LDS size
// and device: the answers are kept so that a call queries each shape once.
int blocks_per_cu(int which, const KernelShape &k, size_t lds) {
    static std::mutex mu;
    static std::unordered_map<uint64_t, int> known;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return 0;
    // fields: which 3 bits, entry/tile/alias bytes and runs per lane 3 bits
    // each (values <= 4), LDS flag, waves per block 5 bits, LDS bytes 18 bits
    // (<= 160 KiB), device 12 bits, warm-up code registers 3 bits
    const uint64_t key = (uint64_t)(which & 7) | (uint64_t)(k.entry_bytes & 7) << 3 |
                         (uint64_t)(k.tile_bytes & 7) << 6 | (uint64_t)(k.alias_bytes & 7) << 9 |
                         (uint64_t)(k.runs_per_lane & 7) << 12 | (uint64_t)(k.table_in_lds ? 1 : 0) << 15 |
                         (uint64_t)((k.block_threads / 64) & 31) << 16 | (uint64_t)(lds & 0x3ffff) << 21 |
                         (uint64_t)(device & 0xfff) << 39 | (uint64_t)(k.code_regs & 7) << 51;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = known.find(key);
        if (it != known.end()) return it->second;
    }
    std::lock_guard<std::mutex> lk(mu);
    g_fn = nullptr;
    hipError_t e = hipSuccess;
    if (which == 0) e = launch_plain(PlainArgs{}, k, 0, lds, nullptr);
    else if (which == 1) e = launch_warm(WarmArgs{}, k, 0, lds, nullptr);
    else e = launch_long(LongArgs{}, k, 0, lds, nullptr);
    if (e != hipSuccess || !g_fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, g_fn, k.block_threads, lds) != hipSuccess) return 0;
    if (nb > 0) known[key] = nb;
    return nb;
}

#define RI_DISPATCH_W(W_, CALL)                 \
    switch (W_) {                               \
    case 1: CALL(1); break;                     \
    case 2: CALL(2); break;                     \
    case 4: CALL(4); break;                     \
    case 8: CALL(8); break;                     \
    case 16: CALL(16); break;                   \
    case 32: CALL(32); break;                   \
    case 64: CALL(64); break;                   \
    default: return hipErrorInvalidValue;       \
    }

hipError_t launch_join0_rel(const JoinArgs &a, int W, hipStream_t s) {
    const uint32_t ngroups = (a.nchunks + a.G - 1) / a.G;
    const uint32_t nb = blocks_for((uint64_t)ngroups * a.L, 256);
    return with_view(a, [&](auto view) {
#define CALL0(w) hipLaunchKernelGGL((join0_rel_kernel<w, decltype(view)>), dim3(nb), dim3(256), 0, s, a, view);
        RI_DISPATCH_W(W, CALL0)
#undef CALL0
        return hipGetLastError();
    });
}

hipError_t launch_join0_tile(const JoinArgs &a, int W, hipStream_t s) {
    const uint32_t ngroups = a.grp_first ? a.ngroups : (a.nchunks + a.G - 1) / a.G;
    const size_t lds = (size_t)a.L * a.G * 4;
    return with_view(a, [&](auto view) {
        if (W == 0) {
            hipLaunchKernelGGL((join0_tile_kernel<0, decltype(view)>), dim3(ngroups), dim3(256), lds, s, a, view);
            return hipGetLastError();
        }
#define CALLT(w) hipLaunchKernelGGL((join0_tile_kernel<w, decltype(view)>), dim3(ngroups), dim3(256), lds, s, a, view);
        RI_DISPATCH_W(W, CALLT)
#undef CALLT
        return hipGetLastError();
    });
}

hipError_t launch_joinN_rel(const JoinArgs &a, int W, hipStream_t s) {
    const uint32_t ngroups = (a.nin + a.G - 1) / a.G;
    const uint32_t nb = blocks_for((uint64_t)ngroups * a.L, 256);
#define CALLN(w) hipLaunchKernelGGL((joinN_rel_kernel<w>), dim3(nb), dim3(256), 0, s, a);
    RI_DISPATCH_W(W, CALLN)
#undef CALLN
    return hipGetLastError();
}

hipError_t launch_join0_fun(const JoinArgs &a, hipStream_t s) {
    const uint32_t ngroups = a.grp_first ? a.ngroups : (a.nchunks + a.G - 1) / a.G;
    const uint32_t nb = blocks_for((uint64_t)ngroups * a.L, 256);
    return with_view(a, [&](auto view) {
        hipLaunchKernelGGL((join0_fun_kernel<decltype(view)>), dim3(nb), dim3(256), 0, s, a, view);
        return hipGetLastError();
    });
}

hipError_t launch_joinN_fun(const JoinArgs &a, hipStream_t s) {
    const uint32_t ngroups = a.grp_first ? a.ngroups : (a.nin + a.G - 1) / a.G;
    const uint32_t nb = blocks_for((uint64_t)ngroups * a.L, 256);
    hipLaunchKernelGGL(joinN_fun_kernel, dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_materialize(const JoinArgs &a, int32_t *out, hipStream_t s) {
    const uint32_t nb = blocks_for((uint64_t)a.L * a.nchunks, 256);
    return with_view(a, [&](auto view) {
        hipLaunchKernelGGL((materialize_kernel<decltype(view)>), dim3(nb), dim3(256), 0, s, a, view, out);
        return hipGetLastError();
    });
}

size_t cls_join_lds(const ClsJoinArgs &a, int W, int alias_bytes) {
    const uint32_t gs = alias_bytes == 1 ? tile_stride<uint8_t>(a.G) : tile_stride<uint16_t>(a.G);
    return (size_t)a.G * kClsStage * W * 4 + (size_t)a.G * 4 + (((size_t)a.L * gs * alias_bytes + 15) & ~(size_t)15);
}

hipError_t launch_join_cls(const ClsJoinArgs &a, int W, int alias_bytes, bool level0, hipStream_t s) {
    const uint32_t ngroups = a.grp_first ? a.ngroups : (a.nmembers + a.G - 1) / a.G;
    const size_t lds = cls_join_lds(a, W, alias_bytes);
    return dispatch_ta(alias_bytes, [&](auto ta) {
        return dispatch_b(level0, [&](auto l0) {
#define CALLC(w) hipLaunchKernelGGL((join_cls_kernel<w, decltype(ta), decltype(l0)::value>), dim3(ngroups), dim3(256), lds, s, a);
            RI_DISPATCH_W(W, CALLC)
#undef CALLC
            return hipGetLastError();
        });
    });
}

hipError_t launch_finalize_cls(const FinalArgs &f, const ClsJoinArgs &a, int W, int alias_bytes, hipStream_t s) {
    return dispatch_ta(alias_bytes, [&](auto ta) {
#define CALLFC(w) hipLaunchKernelGGL((finalize_cls_kernel<w, decltype(ta)>), dim3(1), dim3(64), 0, s, f, a);
        RI_DISPATCH_W(W, CALLFC)
#undef CALLFC
        return hipGetLastError();
    });
}

hipError_t launch_finalize_rel(const FinalArgs &a, int W, hipStream_t s) {
#define CALLF(w) hipLaunchKernelGGL((finalize_rel_kernel<w>), dim3(1), dim3(64), 0, s, a);
    RI_DISPATCH_W(W, CALLF)
#undef CALLF
    return hipGetLastError();
}

hipError_t launch_finalize_fun(const FinalArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(finalize_fun_kernel, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_hit_prod(const HitArgs &a, int W, int alias_bytes, bool level0, hipStream_t s) {
    const uint32_t ngroups = (a.nmembers + kWave - 1) / kWave;
    const uint32_t blocks = (ngroups + 3) / 4;
    if (!level0) {
        hipLaunchKernelGGL(hit_prodN_kernel, dim3(blocks), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    // next-chunk rows staged in LDS when 4 waves x 64 rows fit in 64 KiB
    const size_t stage = (size_t)4 * kWave * a.L * alias_bytes;
    const bool st = stage <= 65536;
    return dispatch_ta(alias_bytes, [&](auto ta) {
        return dispatch_b(st, [&](auto stg) {
            constexpr bool S = decltype(stg)::value;
            const size_t lds = S ? stage : 0;
            if (W == 0) {
                hipLaunchKernelGGL((hit_prod0_kernel<0, decltype(ta), S>), dim3(blocks), dim3(256), lds, s, a);
                return hipGetLastError();
            }
#define CALLH(w) hipLaunchKernelGGL((hit_prod0_kernel<w, decltype(ta), S>), dim3(blocks), dim3(256), lds, s, a);
            RI_DISPATCH_W(W, CALLH)
#undef CALLH
            return hipGetLastError();
        });
    });
}

hipError_t launch_finalize_hit(const FinalArgs &f, const HitArgs &a, int W, int alias_bytes, hipStream_t s,
                               int32_t *out, uint32_t prop_words) {
    if (a.nmembers > kHitTailMax || (out && prop_words > kPropMaxWords)) return hipErrorInvalidValue;
    const size_t lds = out ? (size_t)prop_words * 12 : 0;
    return dispatch_ta(alias_bytes, [&](auto ta) {
        if (W == 0) {
            hipLaunchKernelGGL((hit_tail_kernel<0, decltype(ta)>), dim3(1), dim3(kWave), lds, s, f, a, prop_words, out);
            return hipGetLastError();
        }
#define CALLFH(w) hipLaunchKernelGGL((hit_tail_kernel<w, decltype(ta)>), dim3(1), dim3(kWave), lds, s, f, a, prop_words, out);
        RI_DISPATCH_W(W, CALLFH)
#undef CALLFH
        return hipGetLastError();
    });
}

hipError_t launch_propagate(const FinalArgs &f, const HitArgs &a, uint32_t W, int alias_bytes, hipStream_t s) {
    if (W > kPropMaxWords) return hipErrorInvalidValue;
    return dispatch_ta(alias_bytes, [&](auto ta) {
        hipLaunchKernelGGL((propagate_kernel<decltype(ta)>), dim3(1), dim3(1024), (size_t)W * 12, s, f, a, W);
        return hipGetLastError();
    });
}

hipError_t launch_store_result(int32_t *out, int32_t accept, int32_t final_state, hipStream_t s) {
    hipLaunchKernelGGL(store_result_kernel, dim3(1), dim3(64), 0, s, out, accept, final_state);
    return hipGetLastError();
}

hipError_t launch_batch_final_cls(const BatchFinalArgs &b, const FinalArgs &f, const ClsJoinArgs &a, int W,
                                  int alias_bytes, hipStream_t s) {
    const uint32_t blocks = blocks_for(b.ntexts ? b.ntexts : 1, 256);
    return dispatch_ta(alias_bytes, [&](auto ta) {
#define CALLBC(w) hipLaunchKernelGGL((batch_final_cls_kernel<w, decltype(ta)>), dim3(blocks), dim3(256), 0, s, b, f, a);
        RI_DISPATCH_W(W, CALLBC)
#undef CALLBC
        return hipGetLastError();
    });
}

hipError_t launch_batch_final_fun(const BatchFinalArgs &b, const FinalArgs &f, uint32_t L, hipStream_t s) {
    hipLaunchKernelGGL(batch_final_fun_kernel, dim3(blocks_for(b.ntexts ? b.ntexts : 1, 256)), dim3(256), 0, s,
                       b, f, L);
    return hipGetLastError();
}

hipError_t launch_batch_fill(const BatchFinalArgs &b, hipStream_t s) {
    hipLaunchKernelGGL(batch_fill_kernel, dim3(blocks_for(b.ntexts ? b.ntexts : 1, 256)), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_mwarm(const MultiArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(mwarm_kernel, dim3(grid), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mlong(const MultiArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(mlong_kernel, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mhit(const MultiArgs &a, bool level0, hipStream_t s) {
    const uint32_t blocks = (a.ngroups + 3) / 4;
    if (blocks == 0) return hipSuccess;
    if (level0) hipLaunchKernelGGL(mhit_kernel<true>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(mhit_kernel<false>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mfinal(const MultiArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(mfinal_kernel, dim3(blocks_for(a.ntexts ? a.ntexts : 1, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mprop(const MultiArgs &a, uint32_t max_words, hipStream_t s) {
    if (max_words > kPropMaxWords) return hipErrorInvalidValue;
    if (a.ntexts == 0) return hipSuccess;
    hipLaunchKernelGGL(mprop_kernel, dim3(a.ntexts), dim3(1024), (size_t)max_words * 12, s, a);
    return hipGetLastError();
}

int multi_blocks_per_cu(int which) {
    static std::mutex mu;
    static std::unordered_map<int, int> known;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return 0;
    const int key = device * 4 + (which == 1);
    std::lock_guard<std::mutex> lk(mu);
    auto it = known.find(key);
    if (it != known.end()) return it->second;
    int n = 0;
    if (which == 1) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mwarm_kernel, 1024, 0);
    else (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mlong_kernel, 256, 0);
    if (n > 0) known[key] = n;
    return n;
}

}  // namespace ri
