// Fused batches: many texts of many automata in one launch sequence.
#include "device.hpp"

#include <mutex>
#include <unordered_map>

namespace ri {
namespace {

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
            if (j < wlen) code[q] = ((const __attribute__((address_space(1))) uint16_t *)d.code)[*at(b + j)];
        }
        uint16_t *arow = a.alias + (ok ? a.alias_row[slot] : 0);
        uint32_t al[R], D = 0, cs = 0;
        bool spill = false;
        if (okl)
            with_entry(d.entry_bytes, [&](auto te) {
                using TE = decltype(te);
                warm_classes<TE, uint16_t, R, 4>((const __attribute__((address_space(1))) TE *)(d.table),
                                                 starts, d.L, d.dead, true,
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
                    warm_records<TE, uint16_t, R, 4>((const __attribute__((address_space(1))) TE *)(d.table),
                                                     starts, d.L, d.dead,
                                                  d.row_bytes, first, code, wlen, arow, lane, lane_lt, al, D, cs,
                                                  spill, firstrun, slot, a.run_chunk, a.run_state);
                });
        }
    }
}

// merged runs to the end of their chunks: one run per lane, grid-stride
__global__ void __launch_bounds__(256) mlong_kernel(MultiArgs a) {
    const uint32_t nruns = *reinterpret_cast<volatile uint32_t *>(&a.counters[1]);
    // runs dealt 64 at a time to the blocks in turn, so that every block gets
    // an equal share however few runs there are
    const uint32_t first = ((threadIdx.x / kWave) * gridDim.x + blockIdx.x) * kWave + threadIdx.x % kWave;
    for (uint32_t i = first; i < nruns; i += gridDim.x * blockDim.x) {
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
            const CodeGlobal code{(const __attribute__((address_space(1))) uint16_t *)d.code};
            f = scan_lane_code<TE, CodeGlobal, true>(a.run_state[i] * d.row_bytes, p, vend, e,
                                               (const __attribute__((address_space(1))) TE *)(d.table),
                                               code, d.dead, d.sink0, d.sink1);
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



}  // namespace

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
