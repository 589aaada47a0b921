// HIP kernels of the recognizer for gfx950 (CDNA4, wave64).
//
// Reach phase (Sect. 2): for every chunk and every start state of the chunk
// automaton, one deterministic run over the chunk; its end state (or "no
// run") is the chunk map lambda_i.  Integer table lookups only; no MFMA work
// exists on this path.
//
//   plain_kernel  every (chunk, start) run to the chunk end or its death, as
//                 the paper's reach phase is stated.
//   warmg_kernel / warm_kernel + long_kernel
//                 the same chunk maps with state convergence, an optimization
//                 the paper names as compatible with the RI-DFA (Sect. 5):
//                 every run is scanned for a short warm-up; the runs of one
//                 chunk that are then in the same state have the same future
//                 (the chunk automaton is deterministic), so they are merged
//                 into one run that alone is scanned to the chunk end, and
//                 runs of a chunk that meet later are merged again there.
//                 For 65 to 256 starts the first warm-up bytes of a chunk
//                 are one walk in the transformation automaton of the
//                 starts (built on the host, every word up to a depth),
//                 whose state lists the runs every start has become.
//
// The join kernels are in k_join.hip.
#include "device.hpp"

#include <type_traits>

#include <mutex>
#include <unordered_map>

namespace ri {
namespace {

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
// Merging by hashing (interfaces of at most 64 R starts, one start block;
// automata with few states merge through a table indexed by state instead,
// see merge_direct).  Each wave owns a table of kMergeSlots slots in LDS; in
// a round every
// pending run writes its state into slot hash(state, round), reads it back
// and is settled when it finds its own state there (one state per slot and
// round); settled runs elect one representative per slot and the
// representatives number the classes in (register, lane) order.  A run whose
// slot was taken by another state tries the next round's hash.  Runs of one
// class get one class number whatever their register or lane.
constexpr uint32_t kMergeSlots = 256;   // plus one slot that takes the writes of lanes with nothing to write
constexpr uint32_t kMergeTrash = kMergeSlots;
constexpr uint32_t kMergeSplit = 8;    // bytes scanned by every start between merges while > 64 classes

// LDS pointers (address space 3, so the accesses are LDS instructions and
// not flat ones); volatile keeps every access in program order, since other
// lanes of the wave write what a lane reads.
typedef volatile __attribute__((address_space(3))) uint32_t lds_u32;
typedef volatile __attribute__((address_space(3))) uint8_t lds_u8;
struct MergeArea {
    lds_u32 *key;    // [kMergeSlots + 1] state offsets; then states by class
    lds_u8 *id;      // [kMergeSlots + 1] representative (register * 64 + lane)
    lds_u8 *rank;    // [kMergeSlots + 1] class number of the slot's state
};

// 8-bit slot of a state in a round (a 24 x 24-bit multiply: states that
// agree in their low 24 bits share every round's slot, and one of them
// settles per round, so merging still ends)
__device__ __forceinline__ uint32_t merge_hash(uint32_t st, uint32_t salt) {
    return ((((st ^ salt) & 0xFFFFFFu) * 0x9E3779u) >> 12) & (kMergeSlots - 1);
}

// Classes of the live runs st[0..R) of the wave: cls[r] in [0, D) or kNone
// for a dead run.  Returns D (wave-uniform).  Pending runs are kept as wave
// masks, so a register with nothing pending is skipped by a scalar branch;
// writes that a lane must not make go to the trash slot.
template <int R>
__device__ uint32_t merge_runs(const uint32_t (&st)[R], uint32_t dead, uint32_t lane, uint64_t lane_lt,
                               const MergeArea &m, uint32_t (&cls)[R]) {
    static_assert(kMergeSlots == 256 && R * kWave <= 256, "class numbers and slots are bytes");
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    uint64_t pend[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        cls[r] = kNone;
        pend[r] = __ballot(st[r] != dead);
    }
    uint32_t D = 0;
    for (uint32_t round = 0;; ++round) {
        uint64_t any = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) any |= pend[r];
        if (any == 0) break;
        const uint32_t salt = round * 0x5BD1E9u;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (pend[r]) {
                const bool p = (pend[r] >> lane) & 1;
                m.key[p ? merge_hash(st[r], salt) : kMergeTrash] = st[r];
            }
        __builtin_amdgcn_wave_barrier();
        uint64_t got[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            got[r] = 0;
            if (pend[r]) {
                const uint32_t h = merge_hash(st[r], salt);
                const bool g = ((pend[r] >> lane) & 1) && m.key[h] == st[r];
                got[r] = __ballot(g);
                m.id[g ? h : kMergeTrash] = (uint8_t)(r * kWave + lane);
            }
        }
        __builtin_amdgcn_wave_barrier();
        uint32_t base = D;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (got[r]) {
                const uint32_t h = merge_hash(st[r], salt);
                const bool lead = ((got[r] >> lane) & 1) && m.id[h] == (uint8_t)(r * kWave + lane);
                const uint64_t b = __ballot(lead);
                m.rank[lead ? h : kMergeTrash] = (uint8_t)(base + (uint32_t)__builtin_popcountll(b & lane_lt));
                base += (uint32_t)__builtin_popcountll(b);
            }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (got[r]) {
                const uint32_t v = m.rank[merge_hash(st[r], salt)];
                cls[r] = ((got[r] >> lane) & 1) ? v : cls[r];
                pend[r] &= ~got[r];
            }
        D = base;
        __builtin_amdgcn_wave_barrier();   // the next round writes the slots again
    }
    return D;
}

// Warm-up bytes [j0, j1) (wave-uniform) of the runs of G chunks, R registers
// each; chunk g stops at its own length wlen[g] (wave-uniform).  Codes of
// bytes 64 q + lane of chunk g in register code[g][q].  Stepping the G
// chunks together gives the wave G R independent lookup chains.  Leaves
// early when every run is dead.
template <typename TE, int R, int NQ, int G>
__device__ __forceinline__ void warm_steps(uint32_t (&st)[G][R], const uint32_t (&code)[G][NQ],
                                           const uint32_t (&wlen)[G], uint32_t j0, uint32_t j1, const TE *tab,
                                           uint32_t dead) {
#pragma unroll
    for (uint32_t q = 0; q < (uint32_t)NQ; ++q) {
        const uint32_t lo = j0 > q * kWave ? j0 : q * kWave;
        const uint32_t hi = j1 < q * kWave + kWave ? j1 : q * kWave + kWave;
        for (uint32_t j = lo; j < hi;) {
            bool alive = false;
#pragma unroll
            for (int g = 0; g < G; ++g) alive |= any_alive<R>(st[g], dead);
            if (__ballot(alive) == 0) return;
            const uint32_t e = hi - j < 16 ? hi : j + 16;
            bool full = e - j == 16;
#pragma unroll
            for (int g = 0; g < G; ++g) full &= e <= wlen[g];
            if (full) {
#pragma unroll
                for (uint32_t k = 0; k < 16; ++k) {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)code[g][q], (int)(j - q * kWave + k));
#pragma unroll
                        for (int r = 0; r < R; ++r) st[g][r] = next_state<TE>(tab, st[g][r], c);
                    }
                }
            } else {
                for (uint32_t k = j; k < e; ++k) {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        if (k >= wlen[g]) continue;
                        const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)code[g][q], (int)(k - q * kWave));
#pragma unroll
                        for (int r = 0; r < R; ++r) st[g][r] = next_state<TE>(tab, st[g][r], c);
                    }
                }
            }
            j = e;
        }
    }
}

// Warm-up and merging of G chunks whose starts fit one start block (L <= 64
// R), stepped together: every start runs kMergeSplit bytes, each chunk's
// runs are merged, and while a chunk has more than 64 classes the runs go on
// kMergeSplit bytes more; then each chunk's classes move to one register
// (class k in lane k) for the rest of the warm-up, and a last merge gives
// the chunk's runs.  cls[g][r]: class of start r * 64 + lane of chunk g
// (kNone: no run); D[g]: classes (runs) of chunk g.  The states of chunk g's
// classes are left to emit_runs (they are in `st`/`one`).
template <typename TE, int R, int NQ, int G>
__device__ __forceinline__ void warm_merge_chunks(const TE *tab, const StartList &starts, uint32_t L, uint32_t dead,
                                                  const bool (&ok)[G], const bool (&first)[G],
                                                  const uint32_t (&code)[G][NQ], const uint32_t (&wlen)[G],
                                                  uint32_t lane, uint64_t lane_lt, const MergeArea &m,
                                                  uint32_t (&cls)[G][R], uint32_t (&one)[G], uint32_t (&D)[G],
                                                  bool &compacted, uint32_t (&st)[G][R]) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    uint32_t W = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        W = wlen[g] > W ? wlen[g] : W;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t s = r * kWave + lane;
            st[g][r] = (ok[g] && s < L && (!first[g] || s == 0)) ? starts[s] : dead;
        }
    }
    uint32_t j = (R == 1 || W < kMergeSplit) ? W : kMergeSplit;
    warm_steps<TE, R, NQ, G>(st, code, wlen, 0, j, tab, dead);
    uint32_t Dmax = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        D[g] = merge_runs<R>(st[g], dead, lane, lane_lt, m, cls[g]);
        Dmax = D[g] > Dmax ? D[g] : Dmax;
    }
    while (j < W && Dmax > kWave) {
        const uint32_t e = W - j < kMergeSplit ? W : j + kMergeSplit;
        warm_steps<TE, R, NQ, G>(st, code, wlen, j, e, tab, dead);
        j = e;
        Dmax = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            D[g] = merge_runs<R>(st[g], dead, lane, lane_lt, m, cls[g]);
            Dmax = D[g] > Dmax ? D[g] : Dmax;
        }
    }
    compacted = j < W;
    if (!compacted) return;
    // at most 64 classes per chunk: class k's state in lane k, one register
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            m.key[cls[g][r] != kNone ? cls[g][r] : kMergeTrash] = st[g][r];
        __builtin_amdgcn_wave_barrier();
        one[g] = lane < D[g] ? m.key[lane] : dead;
        __builtin_amdgcn_wave_barrier();
    }
    uint32_t one2[G][1];
#pragma unroll
    for (int g = 0; g < G; ++g) one2[g][0] = one[g];
    warm_steps<TE, 1, NQ, G>(one2, code, wlen, j, W, tab, dead);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        one[g] = one2[g][0];
        uint32_t c2[1];
        D[g] = merge_runs<1>(one2[g], dead, lane, lane_lt, m, c2);
        // every lane takes part in the shuffle (a lane without a run still
        // holds a class's state for the others to read)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t v = (uint32_t)__shfl((int)c2[0], (int)(cls[g][r] == kNone ? 0u : cls[g][r]));
            cls[g][r] = cls[g][r] == kNone ? kNone : v;
        }
        // lane k of `one` holds class c2[k]'s state; keep it in class order
        __builtin_amdgcn_wave_barrier();
        m.key[c2[0] != kNone ? c2[0] : kMergeTrash] = one[g];
        __builtin_amdgcn_wave_barrier();
        one[g] = lane < D[g] ? m.key[lane] : dead;
        __builtin_amdgcn_wave_barrier();
    }
}

// Merging through a table indexed by state, for automata whose states fit
// the wave's merge area (one byte per state after a 65-entry key row): no
// hashing, so every merge is one pass.
constexpr uint32_t kDirectTrash = 64;   // key[0..63]: states by class; key[64] takes the dead writes

// Index s of a state from its row offset st = s * row_bytes: st converts to
// float exactly (st < 2^24) and the reciprocal, raised by 2^-21 relative,
// puts the product in [s, s + 1), so truncation gives s (checked for every
// s < 2^16 and row length 1..1024).
struct RowDiv {
    float inv;
    __device__ explicit RowDiv(uint32_t row_bytes) : inv((1.0f / (float)row_bytes) * (1.0f + 0x1p-21f)) {}
    __device__ __forceinline__ uint32_t operator()(uint32_t st) const { return (uint32_t)((float)st * inv); }
};

// Classes of the live runs st[0..R) of the wave in one pass: every live run
// writes its id (register * 64 + lane) into its state's byte slot[s] (the
// dead row's byte takes the dead runs' writes); the run that reads its own
// id back leads its class; leaders take class numbers in (register, lane)
// order and write them over the ids; then every run reads its class.
// cls[r]: class or kNone; idx[r]: state index; lead[r]: leaders (wave mask).
// Returns the number of classes (wave-uniform).
template <int R>
__device__ uint32_t merge_direct(const uint32_t (&st)[R], uint32_t dead, uint32_t lane, uint64_t lane_lt,
                                 lds_u8 *slot, const RowDiv &rd, uint32_t (&cls)[R], uint32_t (&idx)[R],
                                 uint64_t (&lead)[R]) {
    static_assert(R * kWave <= 256, "ids and class numbers are bytes");
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    const uint32_t trash = rd(dead);
    uint64_t live[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        live[r] = __ballot(st[r] != dead);
        idx[r] = rd(st[r]);
        cls[r] = kNone;
        lead[r] = 0;
        if (live[r]) slot[idx[r]] = (uint8_t)(r * kWave + lane);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (live[r]) lead[r] = __ballot(((live[r] >> lane) & 1) && slot[idx[r]] == (uint8_t)(r * kWave + lane));
    __builtin_amdgcn_wave_barrier();   // every id is read before a class number replaces it
    uint32_t D = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (lead[r]) {
            const bool l = (lead[r] >> lane) & 1;
            slot[l ? idx[r] : trash] = (uint8_t)(D + (uint32_t)__builtin_popcountll(lead[r] & lane_lt));
            D += (uint32_t)__builtin_popcountll(lead[r]);
        }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (live[r]) {
            const uint32_t v = slot[idx[r]];
            cls[r] = ((live[r] >> lane) & 1) ? v : kNone;
        }
    __builtin_amdgcn_wave_barrier();   // the next merge writes the slots again
    return D;
}

// Single-register warm-up steps [j0, j1) of G chunks with their byte codes
// broadcast from LDS instead of readlane: the codes are written once to the
// wave's key area (free between merges), u8 when every code is below 256,
// and read back 8 at a time by every lane (one address: no bank conflict),
// so a step costs one add and one lookup.  Every chunk must have all
// j1 - j0 bytes.  Leaves early when every run is dead.
template <typename TE, int NQ, int G, typename CT>
__device__ __forceinline__ void warm_steps_lds(uint32_t (&st)[G][1], const uint32_t (&code)[G][NQ], uint32_t j0,
                                               uint32_t j1, const TE *tab, uint32_t dead, lds_u32 *key, uint32_t lane) {
    typedef volatile __attribute__((address_space(3))) CT lds_ct;
    typedef unsigned int v2u __attribute__((ext_vector_type(2)));
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(3))) v2u lds_u2;
    typedef const __attribute__((address_space(3))) v4u lds_u4;
    const uint32_t n = j1 - j0;
    const uint32_t stride = (n * (uint32_t)sizeof(CT) + 15u) & ~15u;
    lds_ct *area = (lds_ct *)key;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (uint32_t q = 0; q < (uint32_t)NQ; ++q) {
            const uint32_t p = q * kWave + lane;
            if (p >= j0 && p < j1) area[(g * stride) / sizeof(CT) + (p - j0)] = (CT)code[g][q];
        }
    __builtin_amdgcn_wave_barrier();
    for (uint32_t k = 0; k < n; k += 8) {
        bool alive = false;
#pragma unroll
        for (int g = 0; g < G; ++g) alive |= st[g][0] != dead;
        if (__ballot(alive) == 0) break;
        uint32_t w[G][sizeof(CT) == 1 ? 2 : 4];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t off = g * stride + k * (uint32_t)sizeof(CT);
            if constexpr (sizeof(CT) == 1) {
                const v2u v = *(lds_u2 *)((const __attribute__((address_space(3))) uint8_t *)key + off);
                w[g][0] = v.x;
                w[g][1] = v.y;
            } else {
                const v4u v = *(lds_u4 *)((const __attribute__((address_space(3))) uint8_t *)key + off);
                w[g][0] = v.x;
                w[g][1] = v.y;
                w[g][2] = v.z;
                w[g][3] = v.w;
            }
        }
#pragma unroll
        for (uint32_t i = 0; i < 8; ++i)
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const uint32_t c = sizeof(CT) == 1 ? (w[g][i >> 2] >> ((i & 3) * 8)) & 0xffu
                                                   : (w[g][i >> 1] >> ((i & 1) * 16)) & 0xffffu;
                st[g][0] = next_state<TE>(tab, st[g][0], c);
            }
    }
    __builtin_amdgcn_wave_barrier();   // the key area is written again by the next chunks
}

// Single-register steps [j0, j1) of G chunks whose table sits in LDS
// (j1 - j0 a multiple of 8, every chunk full).  The byte codes of 16 bytes
// at a time, with the table's LDS offset added, are written as words to the
// wave's key area and read back 4 at a time by every lane at one address
// (a broadcast); the address is kept in a vector register so that the words
// stay vector operands, and a step is one add and one lookup.
template <typename TE, int NQ, int G>
__device__ __forceinline__ void warm_steps_lds32(uint32_t (&st)[G][1], const uint32_t (&code)[G][NQ], uint32_t j0,
                                                 uint32_t j1, const TE *tab, uint32_t dead, lds_u32 *key,
                                                 uint32_t lane) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(3))) v4u lds_u4;
    typedef const __attribute__((address_space(3))) TE lds_te;
    static_assert(G * 16 * 4 <= kDirectKeyBytes - 16, "code window");
    const uint32_t tb = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint8_t *)tab;
    for (uint32_t w0 = j0; w0 < j1; w0 += 16) {
        bool alive = false;
#pragma unroll
        for (int g = 0; g < G; ++g) alive |= st[g][0] != dead;
        if (__ballot(alive) == 0) break;
        const uint32_t nw = j1 - w0 < 16 ? j1 - w0 : 16;   // 8 or 16
        __builtin_amdgcn_wave_barrier();   // the previous window is read
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (uint32_t q = 0; q < (uint32_t)NQ; ++q) {
                const uint32_t p = q * kWave + lane;
                if (p >= w0 && p < w0 + nw) key[g * 16 + (p - w0)] = code[g][q] + tb;
            }
        __builtin_amdgcn_wave_barrier();
        uint32_t a = (uint32_t)(uintptr_t)key;
        asm volatile("" : "+v"(a));   // a per-lane register: the words are read into vector registers
        for (uint32_t k = 0; k < nw; k += 4) {
            v4u c[G];
#pragma unroll
            for (int g = 0; g < G; ++g) c[g] = *(lds_u4 *)(uintptr_t)(a + 4 * (g * 16 + k));
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int g = 0; g < G; ++g) st[g][0] = *(lds_te *)(uintptr_t)(st[g][0] + c[g][e]);
        }
    }
    __builtin_amdgcn_wave_barrier();   // the key area is written again by the next chunks
}

// Steps [j0, j1) of two chunks packed in one register (lanes 0..31 run
// chunk 0, lanes 32..63 chunk 1) whose table sits in LDS; as
// warm_steps_lds32, each half reads its own chunk's code words.
template <typename TE, int NQ>
__device__ __forceinline__ void warm_steps_pair32(uint32_t &st, const uint32_t (&code)[2][NQ], uint32_t j0,
                                                  uint32_t j1, const TE *tab, uint32_t dead, lds_u32 *key,
                                                  uint32_t lane) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(3))) v4u lds_u4;
    typedef const __attribute__((address_space(3))) TE lds_te;
    const uint32_t tb = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint8_t *)tab;
    for (uint32_t w0 = j0; w0 < j1; w0 += 16) {
        if (__ballot(st != dead) == 0) break;
        const uint32_t nw = j1 - w0 < 16 ? j1 - w0 : 16;   // 8 or 16
        __builtin_amdgcn_wave_barrier();   // the previous window is read
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (uint32_t q = 0; q < (uint32_t)NQ; ++q) {
                const uint32_t p = q * kWave + lane;
                if (p >= w0 && p < w0 + nw) key[g * 16 + (p - w0)] = code[g][q] + tb;
            }
        __builtin_amdgcn_wave_barrier();
        const uint32_t a = (uint32_t)(uintptr_t)key + (lane >> 5) * 64u;   // this half's chunk
        for (uint32_t k = 0; k < nw; k += 4) {
            const v4u c = *(lds_u4 *)(uintptr_t)(a + 4 * k);
#pragma unroll
            for (int e = 0; e < 4; ++e) st = *(lds_te *)(uintptr_t)(st + c[e]);
        }
    }
    __builtin_amdgcn_wave_barrier();   // the key area is written again by the next chunks
}

// Single-register steps [j0, j1) through LDS codes when they fit the key area
// and every chunk has all the bytes (as words when the table is in LDS, TL),
// else by readlane.
template <typename TE, int NQ, int G, bool TL = false>
__device__ __forceinline__ void warm_steps1(uint32_t (&st)[G][1], const uint32_t (&code)[G][NQ],
                                            const uint32_t (&wlen)[G], uint32_t j0, uint32_t j1, const TE *tab,
                                            uint32_t dead, lds_u32 *key, uint32_t lane, bool code8) {
    bool full = j1 > j0;
#pragma unroll
    for (int g = 0; g < G; ++g) full &= wlen[g] >= j1;
    const uint32_t n = j1 - j0;
    if constexpr (TL && G <= 4) {
        if (full && (n & 7u) == 0) {
            warm_steps_lds32<TE, NQ, G>(st, code, j0, j1, tab, dead, key, lane);
            return;
        }
    }
    if (full && (n & 7u) == 0 && code8 && G * ((n + 15u) & ~15u) <= kDirectKeyBytes - 16)
        warm_steps_lds<TE, NQ, G, uint8_t>(st, code, j0, j1, tab, dead, key, lane);
    else if (full && (n & 7u) == 0 && G * ((2 * n + 15u) & ~15u) <= kDirectKeyBytes - 16)
        warm_steps_lds<TE, NQ, G, uint16_t>(st, code, j0, j1, tab, dead, key, lane);
    else
        warm_steps<TE, 1, NQ, G>(st, code, wlen, j0, j1, tab, dead);
}

// The single-register end of the warm-up of G chunks: class k's state in
// lane k of one[g], start r * 64 + lane in class cl[g][r]; bytes [j, W) are
// scanned, the runs merged once more and handed to emit with every start's
// final class.
template <typename TE, int R, int NQ, int G, bool TL, class Emit>
__device__ __forceinline__ void warm_tail1(uint32_t (&one)[G][1], uint32_t (&cl)[G][R], uint32_t j, uint32_t W,
                                           const uint32_t (&code)[G][NQ], const uint32_t (&wlen)[G], const TE *tab,
                                           uint32_t dead, uint32_t lane, uint64_t lane_lt, lds_u32 *key, lds_u8 *slot,
                                           const RowDiv &rd, bool code8, Emit &emit) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    warm_steps1<TE, NQ, G, TL>(one, code, wlen, j, W, tab, dead, key, lane, code8);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        uint32_t c2[1], ix[1];
        uint64_t ld[1];
        const uint32_t d = merge_direct<1>(one[g], dead, lane, lane_lt, slot, rd, c2, ix, ld);
        // lane k holds the new class of old class k; every lane takes part
        // in the shuffle
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t v = (uint32_t)__shfl((int)c2[0], (int)(cl[g][r] == kNone ? 0u : cl[g][r]));
            cl[g][r] = cl[g][r] == kNone ? kNone : v;
        }
        emit(g, d, cl[g], ld, c2, ix);
    }
}

// warm_merge_chunks with direct merging; instead of returning the runs it
// hands each chunk's result to emit(g, D, acl, lead, ecl, eidx): acl[r] the
// class of start r * 64 + lane, and for each register of the last merge the
// leaders (lead), their class (ecl) and state index (eidx).
template <typename TE, int R, int NQ, int G, bool TL, class Emit>
__device__ __forceinline__ void warm_direct_chunks(const TE *tab, const StartList &starts, uint32_t L, uint32_t dead,
                                                   const bool (&ok)[G], const bool (&first)[G],
                                                   const uint32_t (&code)[G][NQ], const uint32_t (&wlen)[G],
                                                   uint32_t lane, uint64_t lane_lt, lds_u32 *key, lds_u8 *slot,
                                                   const RowDiv &rd, bool code8, Emit &&emit) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    uint32_t st[G][R], cl[G][R], D[G];
    uint32_t W = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        W = wlen[g] > W ? wlen[g] : W;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t s = r * kWave + lane;
            st[g][r] = (ok[g] && s < L && (!first[g] || s == 0)) ? starts[s] : dead;
        }
    }
    uint32_t j = (R == 1 || W < kMergeSplit) ? W : kMergeSplit;
    if constexpr (R == 1)
        warm_steps1<TE, NQ, G, TL>(st, code, wlen, 0, j, tab, dead, key, lane, code8);
    else
        warm_steps<TE, R, NQ, G>(st, code, wlen, 0, j, tab, dead);
    uint32_t Dmax = 0;
    if (j < W) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            uint32_t ix[R];
            uint64_t ld[R];
            D[g] = merge_direct<R>(st[g], dead, lane, lane_lt, slot, rd, cl[g], ix, ld);
            Dmax = D[g] > Dmax ? D[g] : Dmax;
        }
        while (j < W && Dmax > kWave) {
            const uint32_t e = W - j < kMergeSplit ? W : j + kMergeSplit;
            warm_steps<TE, R, NQ, G>(st, code, wlen, j, e, tab, dead);
            j = e;
            Dmax = 0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                uint32_t ix[R];
                uint64_t ld[R];
                D[g] = merge_direct<R>(st[g], dead, lane, lane_lt, slot, rd, cl[g], ix, ld);
                Dmax = D[g] > Dmax ? D[g] : Dmax;
            }
        }
    }
    if (j >= W) {
        // the warm-up is over with the starts in their own registers: the
        // last merge gives the runs
#pragma unroll
        for (int g = 0; g < G; ++g) {
            uint32_t ix[R];
            uint64_t ld[R];
            const uint32_t d = merge_direct<R>(st[g], dead, lane, lane_lt, slot, rd, cl[g], ix, ld);
            emit(g, d, cl[g], ld, cl[g], ix);
        }
        return;
    }
    // at most 64 classes per chunk: class k's state in lane k, one register
    uint32_t one[G][1];
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int r = 0; r < R; ++r) key[cl[g][r] != kNone ? cl[g][r] : kDirectTrash] = st[g][r];
        __builtin_amdgcn_wave_barrier();
        one[g][0] = lane < D[g] ? key[lane] : dead;
        __builtin_amdgcn_wave_barrier();
    }
    warm_tail1<TE, R, NQ, G, TL>(one, cl, j, W, code, wlen, tab, dead, lane, lane_lt, key, slot, rd, code8, emit);
}

// The walk of the transformation automaton stands for the first k bytes of
// every start of G chunks: prefix state f[g] with nrun[g] <= 64 live runs
// gives the chunk's runs (class k's state in lane k of one[g]) and every
// start's class (cl[g][r] for start r * 64 + lane).
template <int R, int G>
__device__ __forceinline__ void prefix_rows(const PrefixArgs &p, const uint32_t (&f)[G], const uint32_t (&nrun)[G],
                                            const bool (&ok)[G], uint32_t L, uint32_t dead, uint32_t row_bytes,
                                            uint32_t lane, uint32_t (&one)[G][1], uint32_t (&cl)[G][R]) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        one[g][0] = dead;
#pragma unroll
        for (int r = 0; r < R; ++r) cl[g][r] = kNone;
        if (!ok[g]) continue;
        if (lane < nrun[g]) one[g][0] = (uint32_t)p.tgt[(uint64_t)f[g] * kWave + lane] * row_bytes;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t s = r * kWave + lane;
            const uint32_t m = s < L ? (uint32_t)p.map[(uint64_t)f[g] * L + s] : 0xFFu;
            cl[g][r] = m == 0xFFu ? kNone : m;
        }
    }
}

// Direct merging after the walk: the rest of the warm-up is the
// single-register tail.
template <typename TE, int R, int NQ, int G, bool TL, class Emit>
__device__ __forceinline__ void warm_prefix_chunks(const TE *tab, const PrefixArgs &p, const uint32_t (&f)[G],
                                                   const uint32_t (&nrun)[G], uint32_t L, uint32_t dead,
                                                   uint32_t row_bytes, const bool (&ok)[G],
                                                   const uint32_t (&code)[G][NQ], const uint32_t (&wlen)[G],
                                                   uint32_t lane, uint64_t lane_lt, lds_u32 *key, lds_u8 *slot,
                                                   const RowDiv &rd, bool code8, Emit &&emit) {
    uint32_t one[G][1], cl[G][R];
    prefix_rows<R, G>(p, f, nrun, ok, L, dead, row_bytes, lane, one, cl);
    uint32_t W = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) W = wlen[g] > W ? wlen[g] : W;
    const uint32_t j = p.k < W ? p.k : W;
    if constexpr (TL && G == 2) {
        // two chunks of at most 32 runs each share one register: half the
        // lookups; each half is then merged on its own
        bool pack = W > j && ((W - j) & 7u) == 0;
#pragma unroll
        for (int g = 0; g < 2; ++g) pack = pack && (!ok[g] || (nrun[g] <= 32 && wlen[g] >= W));
        if (pack) {
            constexpr uint32_t kNone = 0xFFFFFFFFu;
            const uint32_t s0 = (uint32_t)__shfl((int)one[0][0], (int)(lane & 31u));
            const uint32_t s1 = (uint32_t)__shfl((int)one[1][0], (int)(lane & 31u));
            uint32_t st = lane < 32 ? s0 : s1;
            warm_steps_pair32<TE, NQ>(st, code, j, W, tab, dead, key, lane);
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                uint32_t h[1] = {(lane >> 5) == (uint32_t)g ? st : dead};
                uint32_t c2[1], ix[1];
                uint64_t ld[1];
                const uint32_t d = merge_direct<1>(h, dead, lane, lane_lt, slot, rd, c2, ix, ld);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t v =
                        (uint32_t)__shfl((int)c2[0], (int)(cl[g][r] == kNone ? 0u : 32u * g + cl[g][r]));
                    cl[g][r] = cl[g][r] == kNone ? kNone : v;
                }
                emit(g, d, cl[g], ld, c2, ix);
            }
            return;
        }
    }
    warm_tail1<TE, R, NQ, G, TL>(one, cl, j, W, code, wlen, tab, dead, lane, lane_lt, key, slot, rd, code8, emit);
}

// Hashed merging after the walk (as the single-register end of
// warm_merge_chunks): cls[g][r] the class of start r * 64 + lane, one[g]
// class k's state in lane k, D[g] the chunk's runs.
template <typename TE, int R, int NQ, int G, bool TL>
__device__ __forceinline__ void warm_prefix_hashed(const TE *tab, const PrefixArgs &p, const uint32_t (&f)[G],
                                                   const uint32_t (&nrun)[G], uint32_t L, uint32_t dead,
                                                   uint32_t row_bytes, const bool (&ok)[G],
                                                   const uint32_t (&code)[G][NQ], const uint32_t (&wlen)[G],
                                                   uint32_t lane, uint64_t lane_lt, const MergeArea &m,
                                                   uint32_t (&cls)[G][R], uint32_t (&one)[G], uint32_t (&D)[G]) {
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    uint32_t one2[G][1];
    prefix_rows<R, G>(p, f, nrun, ok, L, dead, row_bytes, lane, one2, cls);
    uint32_t W = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) W = wlen[g] > W ? wlen[g] : W;
    warm_steps1<TE, NQ, G, TL>(one2, code, wlen, p.k < W ? p.k : W, W, tab, dead, m.key, lane, false);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        one[g] = one2[g][0];
        uint32_t c2[1];
        D[g] = merge_runs<1>(one2[g], dead, lane, lane_lt, m, c2);
        // every lane takes part in the shuffle
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t v = (uint32_t)__shfl((int)c2[0], (int)(cls[g][r] == kNone ? 0u : cls[g][r]));
            cls[g][r] = cls[g][r] == kNone ? kNone : v;
        }
        // lane k of `one` holds class c2[k]'s state; keep it in class order
        __builtin_amdgcn_wave_barrier();
        m.key[c2[0] != kNone ? c2[0] : kMergeTrash] = one[g];
        __builtin_amdgcn_wave_barrier();
        one[g] = lane < D[g] ? m.key[lane] : dead;
        __builtin_amdgcn_wave_barrier();
    }
}

// Occupancy: a block is 16 waves (4 per SIMD), so two blocks per CU need 8
// waves per SIMD; without the attribute the kernel's SGPR use allows 7 and
// only one block fits (the SGPRs over the limit live in VGPR lanes).
//
// warm_kernel: interfaces of more than 64 R starts (several start blocks),
// one chunk per wave, classes by the leader loop of warm_classes.
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
    const uint64_t region = warm_region(blockIdx.x, gridDim.x, iters, L, kWarmWaves);
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

// warmg_kernel: interfaces of at most 64 R starts.  A wave takes G chunks
// at a time (G consecutive chunks of the block's a.cpi = 16 G) and steps
// their runs together, merging by hashing in its own LDS table.
template <typename TE, typename TA, int R, bool LDS, int NQ, bool DIRECT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) warmg_kernel(WarmArgs a) {
    constexpr int G = (int)warm_chunks_per_wave(true, DIRECT, R, NQ);
    constexpr uint32_t kNone = 0xFFFFFFFFu;
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
    uint8_t *marea = smem + warm_merge_offset(tables_lds<TE, LDS>(a.s.table_bytes), L) + wave * kWarmMergeBytes;
    const MergeArea merge{(lds_u32 *)(marea), (lds_u8 *)(marea + 4 * (kMergeSlots + 1)),
                          (lds_u8 *)(marea + 5 * (kMergeSlots + 1))};
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    // DIRECT: one byte per state fits the merge area (chosen by the host)
    const RowDiv rd(a.s.row_bytes);
    lds_u32 *const dkey = (lds_u32 *)marea;
    lds_u8 *const dslot = (lds_u8 *)(marea + kDirectKeyBytes);
    TA *alias = reinterpret_cast<TA *>(a.alias);
    const uint32_t cpi = kWarmWaves * G;
    const uint32_t iters = (a.s.nchunks + cpi - 1) / cpi;

    // the warm-up bytes of the wave's chunks in iteration `it` (raw, 64 per
    // register); loaded one iteration ahead
    auto fetch = [&](uint32_t it, uint32_t (&raw)[G][NQ], uint32_t (&wlen)[G], bool (&first)[G]) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t chunk = it * cpi + wave * G + g;
            uint64_t b = 0, e = 0;
            bool f = false;
            uint32_t w = 0;
            if (it < iters && chunk < a.s.nchunks) {
                chunk_bounds(a.s, chunk, b, e, f);
                w = (uint32_t)(e - b < a.warm ? e - b : a.warm);
            }
            b = wave_uniform(b);
            wlen[g] = wave_uniform(w);
            first[g] = wave_uniform((uint32_t)f) != 0;
#pragma unroll
            for (uint32_t q = 0; q < (uint32_t)NQ; ++q) {
                const uint32_t j = q * kWave + lane;
                raw[g][q] = j < wlen[g] ? (uint32_t)*at(b + j) : 0u;
            }
        }
    };
    uint32_t raw[G][NQ], wlen[G];
    bool first[G];
    fetch(blockIdx.x, raw, wlen, first);
    const uint64_t region = warm_region(blockIdx.x, gridDim.x, iters, L, cpi);
    // transformation-automaton walks of the wave's chunks, 64 / G iterations
    // at a time: lane t G + g walks chunk g of iteration pbase + t (kNone:
    // no walk, e.g. a chunk that begins its text)
    const uint32_t pk = R > 1 ? a.pfx.k : 0u;   // the host walks only starts of several registers
    constexpr uint32_t kPerWalk = kWave / G;
    uint32_t pf = kNone, pn = 0, pbase = 0;   // state reached and its live runs
    auto prewalk = [&](uint32_t t0) {
        pbase = t0;
        pf = kNone;
        pn = 0;
        const uint32_t t = t0 + lane / G, g = lane % G;
        const uint32_t it = blockIdx.x + t * gridDim.x;
        if (lane >= kPerWalk * G || it >= iters) return;
        const uint32_t chunk = it * cpi + wave * G + g;
        if (chunk >= a.s.nchunks) return;
        uint64_t b, e;
        bool fst;
        chunk_bounds(a.s, chunk, b, e, fst);
        if (fst) return;
        const uint32_t w = (uint32_t)(e - b < a.warm ? e - b : a.warm);
        const uint32_t m = w < pk ? w : pk;
        uint32_t f = 0;
#pragma unroll 8
        for (uint32_t j = 0; j < m; ++j) f = a.pfx.next[f * a.pfx.K + ((uint32_t)cls[*at(b + j)] >> a.pfx.shift)];
        pf = f;
        pn = a.pfx.count[f];
    };
    if (pk) prewalk(0);
    for (uint32_t it = blockIdx.x, t = 0; it < iters; it += gridDim.x, ++t) {
        const uint32_t chunk0 = it * cpi + wave * G;
        uint32_t code[G][NQ], cur_wlen[G];
        bool ok[G], cur_first[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            ok[g] = chunk0 + g < a.s.nchunks;
            cur_wlen[g] = wlen[g];
            cur_first[g] = first[g];
#pragma unroll
            for (uint32_t q = 0; q < (uint32_t)NQ; ++q) code[g][q] = q * kWave + lane < wlen[g] ? cls[raw[g][q]] : 0u;
        }
        fetch(it + gridDim.x, raw, wlen, first);   // next iteration's bytes, in flight meanwhile
        bool fast = pk != 0;
        uint32_t f[G], n[G];
        if (fast) {
            if (t - pbase >= kPerWalk) prewalk(t);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int src = (int)((t - pbase) * G + g);
                f[g] = (uint32_t)__builtin_amdgcn_readlane((int)pf, src);
                n[g] = (uint32_t)__builtin_amdgcn_readlane((int)pn, src);
                if (ok[g]) fast = fast && f[g] != kNone && n[g] <= kWave;
            }
        }
        if constexpr (DIRECT) {
            // a chunk's runs go to its region slots in class order, written
            // by the class leaders
            auto emit = [&](int g, uint32_t Dg, const uint32_t (&acl)[R], const auto &lead, const auto &ecl,
                            const auto &eidx) {
                constexpr int RE = (int)std::extent<std::remove_reference_t<decltype(lead)>>::value;
                const uint32_t chunk = chunk0 + g;
                uint32_t base = 0;
                if (lane == 0 && ok[g]) base = atomicAdd(&s_count, Dg);
                const uint32_t firstrun = (uint32_t)(region + (uint32_t)__shfl((int)base, 0));
                if (!ok[g]) return;
                if (lane == 0) {
                    a.run_base[chunk] = firstrun;
                    if (a.run_count) a.run_count[chunk] = Dg;
                    if (Dg > kRowCap) atomicOr(&a.counters[2], 1u);
                }
#pragma unroll
                for (int r = 0; r < RE; ++r)
                    if ((lead[r] >> lane) & 1) {
                        a.run_chunk[firstrun + ecl[r]] = chunk;
                        a.run_state[firstrun + ecl[r]] = eidx[r];
                    }
                TA *arow = alias + (uint64_t)chunk * L;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t k = r * kWave + lane;
                    if (k < L) arow[k] = acl[r] == kNone ? all_ones<TA>() : (TA)acl[r];
                }
            };
            if (fast)
                warm_prefix_chunks<TE, R, NQ, G, LDS>(tab, a.pfx, f, n, L, dead, a.s.row_bytes, ok, code, cur_wlen, lane,
                                                 lane_lt, dkey, dslot, rd, a.s.row_bytes <= 256, emit);
            else
                warm_direct_chunks<TE, R, NQ, G, LDS>(tab, starts, L, dead, ok, cur_first, code, cur_wlen, lane, lane_lt,
                                                 dkey, dslot, rd, a.s.row_bytes <= 256, emit);
        } else {
        uint32_t cl[G][R], one[G], D[G], st[G][R];
        bool compacted = true;
        if (fast)
            warm_prefix_hashed<TE, R, NQ, G, LDS>(tab, a.pfx, f, n, L, dead, a.s.row_bytes, ok, code, cur_wlen, lane,
                                                  lane_lt, merge, cl, one, D);
        else
            warm_merge_chunks<TE, R, NQ, G>(tab, starts, L, dead, ok, cur_first, code, cur_wlen, lane, lane_lt, merge,
                                            cl, one, D, compacted, st);
        // runs and alias rows, chunk by chunk: class k's state to lane k
        // (from the table when the runs were not compacted)
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t chunk = chunk0 + g;
            uint32_t fst[R];
            if (compacted) {
#pragma unroll
                for (int r = 0; r < R; ++r) fst[r] = r == 0 ? one[g] : dead;
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    merge.key[cl[g][r] != kNone ? cl[g][r] : kMergeTrash] = st[g][r];
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int r = 0; r < R; ++r) fst[r] = r * kWave + lane < D[g] ? merge.key[r * kWave + lane] : dead;
                __builtin_amdgcn_wave_barrier();
            }
            uint32_t base = 0;
            if (lane == 0 && ok[g]) base = atomicAdd(&s_count, D[g]);
            const uint32_t firstrun = (uint32_t)(region + (uint32_t)__shfl((int)base, 0));
            if (ok[g]) {
                if (lane == 0) {
                    a.run_base[chunk] = firstrun;
                    if (a.run_count) a.run_count[chunk] = D[g];
                    if (D[g] > kRowCap) atomicOr(&a.counters[2], 1u);
                }
                TA *arow = alias + (uint64_t)chunk * L;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t k = r * kWave + lane;
                    if (k < D[g]) {
                        a.run_chunk[firstrun + k] = chunk;
                        a.run_state[firstrun + k] = fst[r] / a.s.row_bytes;
                    }
                    if (k < L) arow[k] = cl[g][r] == kNone ? all_ones<TA>() : (TA)cl[g][r];
                }
            }
        }
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
                                             uint32_t cpi, uint32_t i) {
    uint32_t lo = 0, hi = G;   // pre[lo] <= i < pre[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (pre[mid] <= i) lo = mid;
        else hi = mid;
    }
    return (uint32_t)(warm_region(lo, G, iters, L, cpi) + (i - pre[lo]));
}

// One job of a wave: the runs in slots ri[r] (where ok[r]) from the end of
// their chunk's warm-up to the chunk end; byte codes through `code`.
// SINK: the automaton has sink rows (a.s.sink0/1); without them the checks
// are compiled out.
template <typename TE, int R, class Code, bool SINK = true>
__device__ __forceinline__ void long_job(const LongArgs &a, const TE *tab, const Code &code, const bool (&ok)[R],
                                         const uint32_t (&ri)[R]) {
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t dead = a.s.dead;
    const uint32_t sink0 = SINK ? a.s.sink0 : 0xFFFFFFFFu, sink1 = SINK ? a.s.sink1 : 0xFFFFFFFFu;
    {
        uint64_t p[R], vend[R], end[R];
        uint32_t st[R];
        uint32_t chk[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            p[r] = vend[r] = end[r] = 0;
            st[r] = dead;
            chk[r] = 0xFFFFFFFFu;
            if (ok[r]) {
                chk[r] = a.run_chunk[ri[r]];
                uint64_t b, e;
                bool first;
                chunk_bounds(a.s, chk[r], b, e, first);
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
        // One run per lane: the runs of a chunk sit in consecutive lanes and
        // advance in lockstep, so runs that reach the same state merge as they
        // go (Sect. 5, state convergence): every 4 blocks a lane compares its
        // run with the lane below; when both are live runs of one chunk in one
        // state the upper run stops and takes the lower one's end state.
        uint32_t tgt = lane;   // lane whose end state this lane's run takes
        uint32_t blk = 0;
        for (;;) {
            bool work = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // parked: no whole block left, or in a sink row (whose run
                // ends there; the remainder scan then stops at once)
                if (ok[r] && !pk[r] && (p[r] >= bend[r] || (SINK && (st[r] == sink0 || st[r] == sink1)))) {
                    parked[r] = st[r];
                    st[r] = dead;
                    pk[r] = true;
                }
            }
            if constexpr (R == 1) {
                if ((++blk & 3u) == 0) {
                    const bool live = ok[0] && !pk[0] && st[0] != dead;
                    const uint32_t key = live ? chk[0] : 0xFFFFFFFFu;
                    const uint32_t key_dn = (uint32_t)__shfl_up((int)key, 1);
                    const uint32_t st_dn = (uint32_t)__shfl_up((int)st[0], 1);
                    if (live && lane > 0 && key_dn == key && st_dn == st[0]) {
                        tgt = lane - 1;
                        st[0] = dead;
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) work |= ok[r] && !pk[r] && st[r] != dead;
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
                    step16_each<TE, R, Code>(st, v, tab, code);
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
        if constexpr (R == 1) {
            uint32_t f = ok[0] ? scan_lane_code<TE, Code, SINK>(st[0], p[0], vend[0], end[0], tab, code, dead, sink0,
                                                                sink1)
                               : dead;
            // merged runs take the end state at the root of their chain of
            // merges (targets are lower lanes; pointer jumping, 64 = 2^6)
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                f = (uint32_t)__shfl((int)f, (int)tgt);
                tgt = (uint32_t)__shfl((int)tgt, (int)tgt);
            }
            if (ok[0]) a.run_final[ri[0]] = f == dead ? kNoState : f / a.s.row_bytes;
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (ok[r]) {
                    const uint32_t f = scan_lane_code<TE, Code, SINK>(st[r], p[r], vend[r], end[r], tab, code,
                                                                      dead, sink0, sink1);
                    a.run_final[ri[r]] = f == dead ? kNoState : f / a.s.row_bytes;
                }
            }
        }
    }
}

// The jobs of one wave in the dense run numbering (prefix `pre`).
template <typename TE, int R, bool SINK, class Code>
__device__ __forceinline__ void long_jobs(const LongArgs &a, const TE *tab, const Code &code, const uint32_t *pre) {
    const uint32_t G = a.warm_blocks;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t iters = (a.s.nchunks + a.cpi - 1) / a.cpi;
    const uint32_t nruns = pre[G];
    const uint32_t per_job = kWave * R;
    const uint32_t njobs = (nruns + per_job - 1) / per_job;
    // jobs cost about the same (runs of one chunk length): static schedule,
    // dealt to the blocks in turn (job j to block j mod grid), so that every
    // block, and so every CU, gets an equal share however few jobs there are
    const uint32_t nwaves_grid = gridDim.x * (blockDim.x / kWave);
    for (uint32_t job = (threadIdx.x / kWave) * gridDim.x + blockIdx.x; job < njobs; job += nwaves_grid) {
        bool ok[R];
        uint32_t ri[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t i = job * per_job + r * kWave + lane;
            ok[r] = i < nruns;
            ri[r] = ok[r] ? run_slot(pre, G, iters, a.s.L, a.cpi, i) : 0u;
        }
        long_job<TE, R, Code, SINK>(a, tab, code, ok, ri);
    }
}

template <typename TE, int R, bool LDS, bool SINK>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(R == 1 ? 8 : 4))) long_kernel(LongArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const TE *tab;
    const uint16_t *cls;
    stage_tables<TE, LDS>(a.s, smem, tab, cls);
    uint32_t *pre = reinterpret_cast<uint32_t *>(smem + tables_lds<TE, LDS>(a.s.table_bytes));
    run_prefix(pre, a.block_count, a.warm_blocks);
    // every code is below a row's length: bytes when rows are <= 256 bytes
    if (a.s.row_bytes <= 256)
        long_jobs<TE, R, SINK>(a, tab, CodeTab8{reinterpret_cast<const uint8_t *>(cls) + 512}, pre);
    else
        long_jobs<TE, R, SINK>(a, tab, CodeTab{cls}, pre);
}

// Codes (and the table when `lds`) of one group of a queued batch in LDS,
// laid out as by stage_tables.
__device__ __forceinline__ void stage_group(const ScanArgs &s, bool lds, uint8_t *smem) {
    uint32_t off = 0;
    if (lds) {
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        const uint4 *src = reinterpret_cast<const uint4 *>(s.table);
        for (uint32_t i = threadIdx.x; i < s.table_bytes / 16; i += blockDim.x) dst[i] = src[i];
        off = s.table_bytes;
    }
    uint16_t *c = reinterpret_cast<uint16_t *>(smem + off);
    uint8_t *c8 = smem + off + 512;
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) {
        const uint16_t v = s.code[i];
        c[i] = v;
        c8[i] = (uint8_t)v;
    }
}

// One 64-run job of a queued group, with the group's entry width, table
// placement and code width chosen per item (wave-uniform branches).
template <typename TE, bool LDS>
__device__ __forceinline__ void queue_job(const LongArgs &a, uint8_t *smem, const bool (&ok)[1],
                                          const uint32_t (&ri)[1]) {
    const TE *tab = LDS ? reinterpret_cast<const TE *>(smem) : reinterpret_cast<const TE *>(a.s.table);
    const uint16_t *cls = reinterpret_cast<const uint16_t *>(smem + (LDS ? a.s.table_bytes : 0u));
    if (a.s.row_bytes <= 256)
        long_job<TE, 1>(a, tab, CodeTab8{reinterpret_cast<const uint8_t *>(cls) + 512}, ok, ri);
    else
        long_job<TE, 1>(a, tab, CodeTab{cls}, ok, ri);
}

__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) queue_long_kernel(QueueArgs q) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_left;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t g0 = (uint32_t)(((uint64_t)blockIdx.x * q.ngroups) / gridDim.x);
    for (uint32_t k = 0; k < q.ngroups; ++k) {
        const uint32_t g = g0 + k < q.ngroups ? g0 + k : g0 + k - q.ngroups;
        const QueueGroup &d = q.groups[g];
        const LongArgs &a = d.la;
        const uint32_t G = a.warm_blocks;
        // dense numbering of the group's runs (prefix of its warm-up blocks'
        // counts, after the tables); a job is 64 consecutive runs
        uint32_t *pre = reinterpret_cast<uint32_t *>(smem + (d.lds ? a.s.table_bytes : 0u) + kCodeLdsBytes);
        run_prefix(pre, a.block_count, G);
        const uint32_t nruns = pre[G];
        const uint32_t njobs = (nruns + kWave - 1) / kWave;
        // one thread looks whether the group has jobs left, for the block
        if (threadIdx.x == 0) s_left = *reinterpret_cast<volatile uint32_t *>(&q.counters[g]) < njobs ? 1u : 0u;
        __syncthreads();
        const bool left = s_left != 0;
        __syncthreads();
        if (!left) continue;
        stage_group(a.s, d.lds != 0, smem);
        __syncthreads();
        const uint32_t iters = (a.s.nchunks + a.cpi - 1) / a.cpi;
        for (;;) {
            uint32_t job = 0;
            if (lane == 0) job = atomicAdd(&q.counters[g], 1u);
            job = wave_uniform((uint32_t)__shfl((int)job, 0));
            if (job >= njobs) break;
            const uint32_t i = job * kWave + lane;
            const bool ok[1] = {i < nruns};
            const uint32_t ri[1] = {ok[0] ? run_slot(pre, G, iters, a.s.L, a.cpi, i) : 0u};
            if (d.lds) {
                if (d.entry_bytes == 1) queue_job<uint8_t, true>(a, smem, ok, ri);
                else if (d.entry_bytes == 2) queue_job<uint16_t, true>(a, smem, ok, ri);
                else queue_job<uint32_t, true>(a, smem, ok, ri);
            } else {
                if (d.entry_bytes == 1) queue_job<uint8_t, false>(a, smem, ok, ri);
                else if (d.entry_bytes == 2) queue_job<uint16_t, false>(a, smem, ok, ri);
                else queue_job<uint32_t, false>(a, smem, ok, ri);
            }
        }
        __syncthreads();   // every wave is done with the group's tables and prefix
    }
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
                        constexpr int R = decltype(r)::value;
                        using TE = decltype(te);
                        using TA = decltype(ta);
                        constexpr bool L_ = decltype(lds_t)::value;
                        auto fn = !k.hashed ? warm_kernel<TE, TA, R, L_, NQ>
                                  : k.direct ? warmg_kernel<TE, TA, R, L_, NQ, true>
                                             : warmg_kernel<TE, TA, R, L_, NQ, false>;
                        if (grid == 0) { g_fn = reinterpret_cast<const void *>(fn); return hipSuccess; }
                        hipLaunchKernelGGL(fn, dim3(grid), dim3(k.block_threads), lds, st, a);
                        return hipGetLastError();
                    });
                });
            });
        });
    });
}

hipError_t launch_queue_long(const QueueArgs &a, int grid, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(queue_long_kernel, dim3(grid), dim3(1024), lds, st, a);
    return hipGetLastError();
}

int queue_long_blocks_per_cu(size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(queue_long_kernel), 1024,
                                                     lds) != hipSuccess)
        return 0;
    return nb;
}

size_t warm_lds_bytes(const KernelShape &k, uint32_t table_bytes, uint32_t L) {
    const size_t merge = k.hashed ? (size_t)kWarmWaves * kWarmMergeBytes : 0;
    return warm_merge_offset((k.table_in_lds ? table_bytes : 0) + kCodeLdsBytes, L) + merge;
}

hipError_t launch_long(const LongArgs &a, const KernelShape &k, int grid, size_t lds, hipStream_t st) {
    return dispatch_te(k.entry_bytes, [&](auto te) {
        return dispatch_r(k.runs_per_lane, [&](auto r) {
            return dispatch_b(k.table_in_lds, [&](auto lds_t) {
                return dispatch_b(a.s.sink0 != 0xFFFFFFFFu, [&](auto sk) {
                    auto fn = long_kernel<decltype(te), decltype(r)::value, decltype(lds_t)::value,
                                          decltype(sk)::value>;
                    if (grid == 0) { g_fn = reinterpret_cast<const void *>(fn); return hipSuccess; }
                    hipLaunchKernelGGL(fn, dim3(grid), dim3(k.block_threads), lds, st, a);
                    return hipGetLastError();
                });
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
                         (uint64_t)(device & 0xfff) << 39 | (uint64_t)(k.code_regs & 7) << 51 |
                         (uint64_t)(k.hashed ? 1 : 0) << 54 | (uint64_t)(k.direct ? 1 : 0) << 55;
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

}  // namespace ri
