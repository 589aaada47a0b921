// Join and finalize kernels (see k_reach.hip for the reach phase).
#include "device.hpp"

namespace ri {
namespace {

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

// One group `grp` of a class-join level, by the calling block (LDS at smem,
// cls_join_lds bytes).  Starts and ends by reading and writing LDS: a block
// that takes several groups synchronizes between them.
template <int W, typename TA, bool LEVEL0>
__device__ void cls_group(const ClsJoinArgs &a, uint32_t grp, uint8_t *smem) {
    uint32_t *scont = reinterpret_cast<uint32_t *>(smem);                    // [G][kClsStage][W]
    uint32_t *sncls = scont + (size_t)a.G * kClsStage * W;                    // [G]
    TA *salias = reinterpret_cast<TA *>(sncls + a.G);                         // [L][GS]
    const uint32_t G = a.G, L = a.L;
    const uint32_t GS = tile_stride<TA>(G);
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

template <int W, typename TA, bool LEVEL0>
__global__ void __launch_bounds__(256) join_cls_kernel(ClsJoinArgs a) {
    if (a.gate && *reinterpret_cast<const volatile uint32_t *>(a.gate) == 0) return;
    extern __shared__ __align__(16) uint8_t smem[];
    cls_group<W, TA, LEVEL0>(a, blockIdx.x, smem);
}

// The class join's levels lv[0 ..] and final step in one launch, for queued
// calls where it is gated on the hit join's flag: while the flag is clear
// every block returns at once.  Otherwise every block joins one group of
// lv[0] (level 0 when FIRST0); the last block to finish (a counter after a
// device-scope fence, so that it sees every group's output) joins the
// remaining levels group by group (a few groups: lv[0] is level 0 or 1) and
// takes the final step.
template <int W, typename TA, bool FIRST0>
__global__ void __launch_bounds__(256) cls_join_all_kernel(ClsJoinAll c) {
    if (*reinterpret_cast<const volatile uint32_t *>(c.lv[0].gate) == 0) return;
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint32_t s_last;
    cls_group<W, TA, FIRST0>(c.lv[0], blockIdx.x, smem);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(c.done, 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (uint32_t l = 1; l < c.nlevels; ++l) {
        const ClsJoinArgs &a = c.lv[l];
        const uint32_t ngroups = (a.nmembers + a.G - 1) / a.G;
        for (uint32_t grp = 0; grp < ngroups; ++grp) {
            cls_group<W, TA, false>(a, grp, smem);
            __syncthreads();
        }
        __threadfence();   // this level's output is read by the next one
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const ClsJoinArgs &a = c.lv[c.nlevels - 1];
        const TA c0 = reinterpret_cast<const TA *>(a.alias)[0];
        uint32_t x[W];
        load_row<W>(x, c0 != all_ones<TA>() ? c.final_rel + (uint64_t)c0 * W : nullptr);
        decide<W>(x, c.f, c.f.result);
        reset_counters(c.f.counters);
        *c.done = 0;
    }
}

// Level 0, fused with the hit rows: wave per group of 64 matrices; lane l
// builds M_k (k = 64 g + l) from the end states of chunk k's runs and the
// alias column of chunk k + 1.
template <int W, typename TA, bool STAGE>
__device__ __forceinline__ void hit_prod0_block(const HitArgs &a, uint32_t block, uint8_t *hsm) {
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t g = block * (blockDim.x / kWave) + threadIdx.x / kWave;
    const uint32_t ngroups = (a.nmembers + kWave - 1) / kWave;
    if (g >= ngroups) return;
    const uint32_t gn = g * kWave + kWave <= a.nmembers ? kWave : a.nmembers - g * kWave;
    const uint32_t k = g * kWave + lane;
    const TA *alias = reinterpret_cast<const TA *>(a.alias);
    // STAGE: the wave's next-chunk rows (chunks 64 g + 1 .. 64 g + gn, one
    // contiguous span of bytes [b0, b1)) are copied to LDS first: the LDS
    // image keeps the span's alignment (it starts at b0 rounded down to 16),
    // so the 16-byte-aligned interior moves as 16-byte words and only the
    // head and tail bytes one by one; nothing outside the span is read
    uint8_t *simg = hsm + (size_t)(threadIdx.x / kWave) * kHitStageBytes(a.L, sizeof(TA));
    TA *srow = nullptr;
    if constexpr (STAGE) {
        const uint8_t *gb = reinterpret_cast<const uint8_t *>(alias);
        const uint64_t b0 = (uint64_t)(g * kWave + 1) * a.L * sizeof(TA);
        const uint64_t b1 = b0 + (uint64_t)gn * a.L * sizeof(TA);
        const uint64_t base = b0 & ~(uint64_t)15;
        const uint64_t a0 = (b0 + 15) & ~(uint64_t)15, a1 = b1 & ~(uint64_t)15;
        if (a0 < a1) {
            for (uint64_t o = a0 + 16 * lane; o < a1; o += 16 * kWave)
                *reinterpret_cast<uint4 *>(simg + (o - base)) = *reinterpret_cast<const uint4 *>(gb + o);
            for (uint64_t o = b0 + lane; o < a0; o += kWave) simg[o - base] = gb[o];
            for (uint64_t o = a1 + lane; o < b1; o += kWave) simg[o - base] = gb[o];
        } else {
            for (uint64_t o = b0 + lane; o < b1; o += kWave) simg[o - base] = gb[o];
        }
        srow = reinterpret_cast<TA *>(simg + (b0 - base));
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

template <int W, typename TA, bool STAGE>
__global__ void __launch_bounds__(256) hit_prod0_kernel(HitArgs a) {
    extern __shared__ __align__(16) uint8_t hsm[];
    hit_prod0_block<W, TA, STAGE>(a, blockIdx.x, hsm);
}

// Queued calls: level 0 of the hit join in blocks [0, hit_blocks) and level
// 0 of the gated class join in the blocks after them, which return at once
// unless the warm-up flagged a chunk with more runs than a hit row holds (the
// flag is final once the warm-up has run).  The two write separate buffers.
template <int W, typename TA, bool STAGE>
__global__ void __launch_bounds__(256) hit_prod0_cls_kernel(HitArgs a, ClsJoinArgs c, uint32_t hit_blocks) {
    extern __shared__ __align__(16) uint8_t hcsm[];
    if (blockIdx.x < hit_blocks) {
        hit_prod0_block<W, TA, STAGE>(a, blockIdx.x, hcsm);
        return;
    }
    if (*reinterpret_cast<const volatile uint32_t *>(c.gate) == 0) return;
    cls_group<W, TA, true>(c, blockIdx.x - hit_blocks, hcsm);
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
    if (a.gate && *reinterpret_cast<const volatile uint32_t *>(a.gate) == 0) return;
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
__device__ uint32_t finalize_hit_one(const FinalArgs &f, const HitArgs &a, bool have, uint64_t prod, bool keep_flag) {
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
    if (!(flag && keep_flag)) reset_counters(f.counters);   // a kept flag gates the class join that follows
    return flag;
}

// The last level of the hit-matrix product (at most 64 products, a.nmembers
// of them in a.prod_in; 0 for a single chunk) and the final step, in one wave.
// With out != nullptr the result is also copied to out; when a chunk kept
// more runs than a hit row holds, the wave first joins again by propagation
// (prop_words words per set of N' states, 12 bytes per word of dynamic LDS),
// or, with gated_after, leaves the result and the flag to the gated class
// join enqueued after it.
template <int W, typename TA>
__global__ void __launch_bounds__(64) hit_tail_kernel(FinalArgs f, HitArgs a, uint32_t prop_words, int32_t *out,
                                                      uint32_t gated_after) {
    const uint32_t lane = threadIdx.x;
    const uint32_t nm = a.nmembers;
    uint64_t M = lane < nm ? a.prod_in[lane] : 0ull;
    if (nm > 1) wave_tree_product(M, lane, nm);
    uint32_t redo = 0;
    if (lane == 0) redo = finalize_hit_one<W, TA>(f, a, nm > 0, M, out && gated_after);
    if (!out) return;
    redo = (uint32_t)__shfl((int)redo, 0);
    if (redo && gated_after) return;
    if (redo) {
        extern __shared__ __align__(16) uint32_t tsm[];
        propagate_block<TA>(f, a, prop_words, tsm);   // ends with the result in f.result
    }
    if (lane == 0) {
        out[0] = f.result[0];
        out[1] = f.result[1];
    }
}

// Queued calls whose gated class join has run its level 0 already (inside
// the hit join's first launch): the last level of the hit-matrix product and
// the final step in wave 0 of block 0, and the class join's upper levels in
// the blocks after it, gated on the warm-up's flag.  Flag clear: block 0
// writes the result and clears the counters, the other blocks return at once.
// Flag set: block 0 writes nothing; every block, block 0 included, counts
// itself done, and the last one (so after block 0 has read the flag) joins
// the remaining levels group by group, takes the final step and clears the
// counters and the done count.
template <int W, typename TA>
__global__ void __launch_bounds__(256) hit_tail_cls_kernel(FinalArgs f, HitArgs a, int32_t *out, ClsJoinAll c) {
    extern __shared__ __align__(16) uint8_t tcsm[];
    __shared__ uint32_t s_flag, s_last;
    if (blockIdx.x == 0) {
        if (threadIdx.x < kWave) {
            const uint32_t lane = threadIdx.x;
            const uint32_t nm = a.nmembers;
            uint64_t M = lane < nm ? a.prod_in[lane] : 0ull;
            if (nm > 1) wave_tree_product(M, lane, nm);
            if (lane == 0) {
                const uint32_t flag = finalize_hit_one<W, TA>(f, a, nm > 0, M, true);
                if (!flag) {
                    out[0] = f.result[0];
                    out[1] = f.result[1];
                }
                s_flag = flag;
            }
        }
        __syncthreads();
        if (s_flag == 0) return;
    } else {
        if (threadIdx.x == 0) s_flag = *reinterpret_cast<const volatile uint32_t *>(c.lv[0].gate);
        __syncthreads();
        if (s_flag == 0) return;
        cls_group<W, TA, false>(c.lv[0], blockIdx.x - 1, tcsm);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(c.done, 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (uint32_t l = 1; l < c.nlevels; ++l) {
        const ClsJoinArgs &la = c.lv[l];
        const uint32_t ngroups = (la.nmembers + la.G - 1) / la.G;
        for (uint32_t grp = 0; grp < ngroups; ++grp) {
            cls_group<W, TA, false>(la, grp, tcsm);
            __syncthreads();
        }
        __threadfence();   // this level's output is read by the next one
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const ClsJoinArgs &la = c.lv[c.nlevels - 1];
        const TA c0 = reinterpret_cast<const TA *>(la.alias)[0];
        uint32_t x[W];
        load_row<W>(x, c0 != all_ones<TA>() ? c.final_rel + (uint64_t)c0 * W : nullptr);
        decide<W>(x, c.f, c.f.result);
        reset_counters(c.f.counters);
        *c.done = 0;
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

__global__ void zero_words_kernel(uint32_t *p, uint32_t n) {
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
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

}  // namespace

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

hipError_t launch_cls_join_all(const ClsJoinAll &c, int W, int alias_bytes, bool first0, hipStream_t s) {
    const ClsJoinArgs &a = c.lv[0];
    const uint32_t ngroups = (a.nmembers + a.G - 1) / a.G;
    size_t lds = 0;
    for (uint32_t l = 0; l < c.nlevels; ++l) lds = std::max(lds, cls_join_lds(c.lv[l], W, alias_bytes));
    return dispatch_ta(alias_bytes, [&](auto ta) {
        return dispatch_b(first0, [&](auto f0) {
#define CALLA(w) hipLaunchKernelGGL((cls_join_all_kernel<w, decltype(ta), decltype(f0)::value>), dim3(ngroups), dim3(256), lds, s, c);
            RI_DISPATCH_W(W, CALLA)
#undef CALLA
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

hipError_t launch_hit_prod_cls(const HitArgs &a, const ClsJoinArgs &c, int W, int alias_bytes, hipStream_t s) {
    if (W <= 0 || !c.gate) return hipErrorInvalidValue;
    const uint32_t ngroups = (a.nmembers + kWave - 1) / kWave;
    const uint32_t blocks = (ngroups + 3) / 4;
    const uint32_t cls_groups = (c.nmembers + c.G - 1) / c.G;
    const size_t stage = (size_t)4 * kHitStageBytes(a.L, alias_bytes);
    const bool st = stage <= 65536;
    const size_t lds = std::max(st ? stage : (size_t)0, cls_join_lds(c, W, alias_bytes));
    return dispatch_ta(alias_bytes, [&](auto ta) {
        return dispatch_b(st, [&](auto stg) {
            constexpr bool S = decltype(stg)::value;
#define CALLHC(w) hipLaunchKernelGGL((hit_prod0_cls_kernel<w, decltype(ta), S>), dim3(blocks + cls_groups), dim3(256), lds, s, a, c, blocks);
            RI_DISPATCH_W(W, CALLHC)
#undef CALLHC
            return hipGetLastError();
        });
    });
}

hipError_t launch_hit_prod(const HitArgs &a, int W, int alias_bytes, bool level0, hipStream_t s) {
    const uint32_t ngroups = (a.nmembers + kWave - 1) / kWave;
    const uint32_t blocks = (ngroups + 3) / 4;
    if (!level0) {
        hipLaunchKernelGGL(hit_prodN_kernel, dim3(blocks), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    // next-chunk rows staged in LDS when 4 waves x 64 rows fit in 64 KiB
    const size_t stage = (size_t)4 * kHitStageBytes(a.L, alias_bytes);
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
                               int32_t *out, uint32_t prop_words, bool gated_after) {
    const uint32_t ga = gated_after ? 1u : 0u;
    if (a.nmembers > kHitTailMax || (out && prop_words > kPropMaxWords)) return hipErrorInvalidValue;
    const size_t lds = out ? (size_t)prop_words * 12 : 0;
    return dispatch_ta(alias_bytes, [&](auto ta) {
        if (W == 0) {
            hipLaunchKernelGGL((hit_tail_kernel<0, decltype(ta)>), dim3(1), dim3(kWave), lds, s, f, a, prop_words, out, ga);
            return hipGetLastError();
        }
#define CALLFH(w) hipLaunchKernelGGL((hit_tail_kernel<w, decltype(ta)>), dim3(1), dim3(kWave), lds, s, f, a, prop_words, out, ga);
        RI_DISPATCH_W(W, CALLFH)
#undef CALLFH
        return hipGetLastError();
    });
}

hipError_t launch_hit_tail_cls(const FinalArgs &f, const HitArgs &a, int32_t *out, const ClsJoinAll &c, int W,
                               int alias_bytes, hipStream_t s) {
    if (W <= 0 || !out || a.nmembers > kHitTailMax || c.nlevels == 0 || !c.lv[0].gate) return hipErrorInvalidValue;
    const ClsJoinArgs &l0 = c.lv[0];
    const uint32_t ngroups = (l0.nmembers + l0.G - 1) / l0.G;
    size_t lds = 0;
    for (uint32_t l = 0; l < c.nlevels; ++l) lds = std::max(lds, cls_join_lds(c.lv[l], W, alias_bytes));
    return dispatch_ta(alias_bytes, [&](auto ta) {
#define CALLTC(w) hipLaunchKernelGGL((hit_tail_cls_kernel<w, decltype(ta)>), dim3(1 + ngroups), dim3(256), lds, s, f, a, out, c);
        RI_DISPATCH_W(W, CALLTC)
#undef CALLTC
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

hipError_t launch_zero_words(uint32_t *p, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
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

}  // namespace ri
