// Device helpers shared by the kernel translation units: table staging,
// byte-code steps, text loads, warm-up and merging of one chunk, boolean
// 8 x 8 products, the final acceptance step and launch-time dispatch.
#pragma once

#include "kernels.hpp"

#include <type_traits>

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
    uint8_t *c8 = smem + off + 512;
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) {
        const uint16_t v = s.code[i];
        c[i] = v;
        c8[i] = (uint8_t)v;
    }
    cls = c;
}

template <typename TE, bool LDS>
__host__ __device__ constexpr uint32_t tables_lds(uint32_t table_bytes) {
    return (LDS ? table_bytes : 0u) + kCodeLdsBytes;
}

// One transition: st and c are byte offsets into the table.
template <typename TE>
__device__ __forceinline__ uint32_t next_state(const __attribute__((address_space(1))) TE *tab, uint32_t st,
                                               uint32_t c) {
    typedef const __attribute__((address_space(1))) uint8_t gb;
    typedef const __attribute__((address_space(1))) TE gt;
    return *reinterpret_cast<gt *>(reinterpret_cast<gb *>(tab) + st + c);
}
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

// Byte codes (class * entry bytes) of the 256 byte values, one u16 table.
struct CodeTab {
    const uint16_t *cls;
    __device__ __forceinline__ uint32_t operator()(uint32_t b) const { return cls[b]; }
};
// The codes as bytes (rows of at most 256 bytes), staged after the u16 ones.
struct CodeTab8 {
    const uint8_t *cls;
    __device__ __forceinline__ uint32_t operator()(uint32_t b) const { return cls[b]; }
};
// The same table in global memory (global loads, not flat ones).
struct CodeGlobal {
    const __attribute__((address_space(1))) uint16_t *cls;
    __device__ __forceinline__ uint32_t operator()(uint32_t b) const { return cls[b]; }
};

// 16 steps of R runs over R different 16-byte blocks (runs of R chunks).
template <typename TE, int R, class Code>
__device__ __forceinline__ void step16_each(uint32_t (&st)[R], const uint4 (&v)[R], const TE *tab,
                                            const Code &code) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t w = i < 4 ? v[r].x : i < 8 ? v[r].y : i < 12 ? v[r].z : v[r].w;
            const uint32_t c = code((w >> ((i & 3) * 8)) & 0xffu);
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

// The same with any byte-code lookup.  SINK: a run in one of the sink rows
// sink0/1 stays there, so it stops as at the dead row (checked every 16
// bytes); without SINK the rows are ignored.
template <typename TE, class Code, bool SINK = false, typename TP>
__device__ __forceinline__ uint32_t scan_lane_code(uint32_t st, uint64_t p, uint64_t vend, uint64_t end,
                                                   TP tab, const Code &code, uint32_t dead,
                                                   uint32_t sink0 = 0xFFFFFFFFu, uint32_t sink1 = 0xFFFFFFFFu) {
    auto going = [&]() { return st != dead && (!SINK || (st != sink0 && st != sink1)); };
    for (; p < vend && going(); p += 16) {
        const uint4 v = load16(at(p));
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 16; ++i) st = next_state<TE>(tab, st, code((w[i >> 2] >> ((i & 3) * 8)) & 0xffu));
    }
    for (p = p < vend ? vend : p; p < end && going(); ++p) st = next_state<TE>(tab, st, code(*at(p)));
    return st;
}

__device__ __forceinline__ uint32_t wave_ticket(uint32_t *counter) {
    uint32_t t = 0;
    if (threadIdx.x % kWave == 0) t = atomicAdd(counter, 1u);
    return __shfl(t, 0);
}

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

// LDS of the warm-up kernel: tables (tables_bytes), staged starts, then one
// merge table of kWarmMergeBytes per wave.
__host__ __device__ constexpr uint32_t warm_merge_offset(uint32_t tables_bytes, uint32_t L) {
    return (tables_bytes + (L <= kStageStarts ? L * 4u : 0u) + 15u) & ~15u;
}

// Warm-up of the start block at `base` over codes[0..wlen) (codes of bytes
// 64 q + lane in register q).
template <typename TE, int R, int NQ, typename TP>
__device__ __forceinline__ void warm_block(uint32_t (&st)[R], const uint32_t (&code)[NQ], uint32_t wlen,
                                           TP tab, uint32_t dead) {
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
template <typename TE, typename TA, int R, int NQ, typename TP>
__device__ __forceinline__ void warm_classes(TP tab, const StartList &starts, uint32_t L, uint32_t dead,
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
template <typename TE, typename TA, int R, int NQ, typename TP>
__device__ __forceinline__ void warm_records(TP tab, const StartList &starts, uint32_t L, uint32_t dead,
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
__device__ inline void decide_bits(const uint32_t *x, uint32_t nw, const FinalArgs &f, int32_t *res) {
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

__device__ inline void decide_lists(const ListUnion &u, const FinalArgs &f, int32_t *res) {
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

inline uint32_t blocks_for(uint64_t threads, uint32_t per) { return (uint32_t)((threads + per - 1) / per); }

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

}  // namespace
}  // namespace ri
