// HIP kernels of the recognizer for gfx950 (CDNA4, wave64).
//
// reach     -- the reach phase (Sect. 2): for every chunk and every start
//              state of the chunk automaton, one deterministic run over the
//              chunk; the end state (or "no run") is the chunk map lambda_i.
//              Integer table lookups only: no MFMA work exists on this path.
// join*     -- the join phase as an associative composition of chunk maps
//              over a tree of groups of G consecutive members.
//              Relations (RI-DFA, Sect. 3.2): row s of a chunk is the content
//              of lambda_i({s}), a set of interface states; composing two
//              chunks unions the rows of the second over the set bits of the
//              first, which is PLAS_i = lambda_i(if(PLAS_{i-1}) & PIS_i) taken
//              for every possible PLAS_{i-1} at once.
//              Functions (DFA, Sect. 2): lambda_i is a partial map Q -> Q and
//              composition is a gather.
// finalize  -- row 0 (the initial state) of the composition of all chunks:
//              acceptance test and the minimal-DFA state of the result.
#include "kernels.hpp"

namespace ri {
namespace {

constexpr int kWave = 64;

template <typename TL> __device__ __forceinline__ TL no_run() { return (TL)~(TL)0; }

// ---------------------------------------------------------------------------
// reach
// ---------------------------------------------------------------------------
//
// Work decomposition.  A job is 64 consecutive chunks x R consecutive starts;
// lane l of the wave scans chunk (64*cg + l) from the R starts (g*R .. g*R+R-1)
// at once, so the R runs share each byte and each class lookup and give the
// lane R independent lookup chains.  Jobs are numbered start-group-major and
// handed out by a global counter to persistent blocks, so that the groups
// whose runs survive whole chunks are spread over every CU first.  A wave
// leaves its job as soon as every run of every lane has died (wave vote).
//
// Table layout.  Row-major [state][class] entries holding the row offset of
// the next state (next * K), so a step is one add and one load; the dead row
// points to itself, so a dead run needs no branch.  The table and the byte
// class map sit in LDS when they fit.
template <typename TE, typename TL, int R, bool LDS_TABLE>
__global__ void __launch_bounds__(1024) reach_kernel(ReachArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const TE *tab;
    const uint8_t *cls;
    if constexpr (LDS_TABLE) {
        uint4 *dst = reinterpret_cast<uint4 *>(smem);
        const uint4 *src = reinterpret_cast<const uint4 *>(a.table);
        for (uint32_t i = threadIdx.x; i < a.table_bytes / 16; i += blockDim.x) dst[i] = src[i];
        uint8_t *c = smem + a.table_bytes;
        for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) c[i] = a.cls[i];
        __syncthreads();
        tab = reinterpret_cast<const TE *>(smem);
        cls = smem + a.table_bytes;
    } else {
        uint8_t *c = smem;
        for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) c[i] = a.cls[i];
        __syncthreads();
        tab = reinterpret_cast<const TE *>(a.table);
        cls = smem;
    }

    const uint32_t lane = threadIdx.x % kWave;
    TL *lam = reinterpret_cast<TL *>(a.lam);

    for (;;) {
        uint32_t job = 0;
        if (lane == 0) job = atomicAdd(a.job_counter, 1u);
        job = __shfl(job, 0);
        if (job >= a.njobs) break;
        const uint32_t g = job / a.chunk_groups;
        const uint32_t cg = job - g * a.chunk_groups;
        const uint32_t chunk = cg * kWave + lane;
        const bool chunk_ok = chunk < a.nchunks;
        uint64_t begin = 0, end = 0;
        if (chunk_ok) {
            begin = (uint64_t)chunk * a.cs;
            end = begin + a.cs < a.n ? begin + a.cs : a.n;
        }
        uint32_t st[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t s = g * R + r;
            // chunk 0 is scanned from the initial state only (I_1 = {q0})
            const bool on = chunk_ok && s < a.L && (chunk != 0 || s == 0);
            st[r] = on ? a.starts[s] : a.dead;
        }

        uint64_t p = begin;
        const uint64_t vend = begin + ((end - begin) & ~(uint64_t)15);
        for (;;) {
            bool alive = false;
#pragma unroll
            for (int r = 0; r < R; ++r) alive |= st[r] != a.dead;
            const bool work = alive && p < vend;
            if (__ballot(work) == 0) break;
            if (work) {
                const uint4 v = *reinterpret_cast<const uint4 *>(a.text + p);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const uint32_t c = cls[(w[i >> 2] >> ((i & 3) * 8)) & 0xffu];
#pragma unroll
                    for (int r = 0; r < R; ++r) st[r] = tab[st[r] + c];
                }
                p += 16;
            }
        }
        // ragged tail of the last chunk
        for (; p < end; ++p) {
            const uint32_t c = cls[a.text[p]];
#pragma unroll
            for (int r = 0; r < R; ++r) st[r] = tab[st[r] + c];
        }
        if (chunk_ok) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t s = g * R + r;
                if (s < a.L)
                    lam[(uint64_t)s * a.nchunks + chunk] =
                        st[r] == a.dead ? no_run<TL>() : (TL)(st[r] / a.K);
            }
        }
    }
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
template <int W, typename TL>
__global__ void __launch_bounds__(256) join0_rel_kernel(JoinArgs a) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ngroups = (a.nchunks + a.G - 1) / a.G;
    if (tid >= (uint64_t)ngroups * a.L) return;
    const uint32_t grp = (uint32_t)(tid / a.L), s = (uint32_t)(tid % a.L);
    const TL *lam = reinterpret_cast<const TL *>(a.lam);
    const uint32_t c0 = grp * a.G;
    const uint32_t c1 = c0 + a.G < a.nchunks ? c0 + a.G : a.nchunks;
    uint32_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = 0;
    {
        const TL v = lam[(uint64_t)s * a.nchunks + c0];
        if (v != no_run<TL>()) or_row<W>(x, a.content + (uint64_t)v * W);
    }
    for (uint32_t c = c0 + 1; c < c1 && !empty_row<W>(x); ++c) {
        uint32_t y[W];
#pragma unroll
        for (int w = 0; w < W; ++w) y[w] = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            for (uint32_t bits = x[w]; bits; bits &= bits - 1) {
                const uint32_t t = w * 32 + __builtin_ctz(bits);
                const TL v = lam[(uint64_t)t * a.nchunks + c];
                if (v != no_run<TL>()) or_row<W>(y, a.content + (uint64_t)v * W);
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = y[w];
    }
    uint32_t *out = reinterpret_cast<uint32_t *>(a.out) + tid * W;
#pragma unroll
    for (int w = 0; w < W; ++w) out[w] = x[w];
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

template <typename TL>
__global__ void __launch_bounds__(256) join0_fun_kernel(JoinArgs a) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ngroups = (a.nchunks + a.G - 1) / a.G;
    if (tid >= (uint64_t)ngroups * a.L) return;
    const uint32_t grp = (uint32_t)(tid / a.L), s = (uint32_t)(tid % a.L);
    const TL *lam = reinterpret_cast<const TL *>(a.lam);
    const uint32_t c0 = grp * a.G;
    const uint32_t c1 = c0 + a.G < a.nchunks ? c0 + a.G : a.nchunks;
    TL v = lam[(uint64_t)s * a.nchunks + c0];
    for (uint32_t c = c0 + 1; c < c1 && v != no_run<TL>(); ++c) v = lam[(uint64_t)v * a.nchunks + c];
    reinterpret_cast<int32_t *>(a.out)[tid] = v == no_run<TL>() ? -1 : (int32_t)v;
}

__global__ void __launch_bounds__(256) joinN_fun_kernel(JoinArgs a) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ngroups = (a.nin + a.G - 1) / a.G;
    if (tid >= (uint64_t)ngroups * a.L) return;
    const uint32_t grp = (uint32_t)(tid / a.L), s = (uint32_t)(tid % a.L);
    const int32_t *in = reinterpret_cast<const int32_t *>(a.in);
    const uint32_t k0 = grp * a.G;
    const uint32_t k1 = k0 + a.G < a.nin ? k0 + a.G : a.nin;
    int32_t v = in[(uint64_t)k0 * a.L + s];
    for (uint32_t k = k0 + 1; k < k1 && v >= 0; ++k) v = in[(uint64_t)k * a.L + v];
    reinterpret_cast<int32_t *>(a.out)[tid] = v;
}

// ---------------------------------------------------------------------------
// finalize
// ---------------------------------------------------------------------------

// FNV-1a over the words of a content bitset; the host fills the table with
// the same function.
template <int W>
__device__ __forceinline__ uint32_t hash_words(const uint32_t (&x)[W]) {
    uint32_t h = 2166136261u;
#pragma unroll
    for (int w = 0; w < W; ++w) { h ^= x[w]; h *= 16777619u; }
    return h;
}

template <int W>
__global__ void finalize_rel_kernel(FinalArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t *row = reinterpret_cast<const uint32_t *>(a.total);   // row 0
    uint32_t x[W];
    uint32_t acc = 0, any = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        x[w] = row[w];
        acc |= x[w] & a.fmask[w];
        any |= x[w];
    }
    int32_t fin = -1;
    if (any) {
        fin = -3;   // not found: cannot happen for a reachable subset
        uint32_t slot = hash_words<W>(x) & (a.hash_cap - 1);
        for (uint32_t probe = 0; probe < a.hash_cap; ++probe) {
            const uint32_t *e = a.hash + (uint64_t)slot * (W + 1);
            const int32_t val = (int32_t)e[W];
            if (val == -2) break;   // empty slot
            bool eq = true;
#pragma unroll
            for (int w = 0; w < W; ++w) eq &= e[w] == x[w];
            if (eq) { fin = val; break; }
            slot = (slot + 1) & (a.hash_cap - 1);
        }
    }
    a.result[0] = acc != 0;
    a.result[1] = fin;
    *a.job_counter = 0;
}

__global__ void finalize_fun_kernel(FinalArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int32_t t = reinterpret_cast<const int32_t *>(a.total)[0];
    a.result[0] = t >= 0 ? (int32_t)a.accept_of_state[t] : 0;
    a.result[1] = t >= 0 ? a.final_of_state[t] : -1;
    *a.job_counter = 0;
}

template <typename TE, typename TL, int R>
hipError_t launch_reach_t(const ReachArgs &a, bool lds, int grid, size_t lds_bytes, int block,
                          hipStream_t s) {
    if (lds)
        hipLaunchKernelGGL((reach_kernel<TE, TL, R, true>), dim3(grid), dim3(block), lds_bytes, s, a);
    else
        hipLaunchKernelGGL((reach_kernel<TE, TL, R, false>), dim3(grid), dim3(block), lds_bytes, s, a);
    return hipGetLastError();
}

template <typename TE, typename TL>
hipError_t launch_reach_r(const ReachArgs &a, const ReachConfig &c, int grid, size_t lds, hipStream_t s) {
    switch (c.runs_per_lane) {
    case 1: return launch_reach_t<TE, TL, 1>(a, c.table_in_lds, grid, lds, c.block_threads, s);
    case 2: return launch_reach_t<TE, TL, 2>(a, c.table_in_lds, grid, lds, c.block_threads, s);
    case 4: return launch_reach_t<TE, TL, 4>(a, c.table_in_lds, grid, lds, c.block_threads, s);
    case 8: return launch_reach_t<TE, TL, 8>(a, c.table_in_lds, grid, lds, c.block_threads, s);
    }
    return hipErrorInvalidValue;
}

template <typename TE>
hipError_t launch_reach_l(const ReachArgs &a, const ReachConfig &c, int grid, size_t lds, hipStream_t s) {
    if (c.lam_bytes == 2) return launch_reach_r<TE, uint16_t>(a, c, grid, lds, s);
    if (c.lam_bytes == 4) return launch_reach_r<TE, uint32_t>(a, c, grid, lds, s);
    return hipErrorInvalidValue;
}

template <typename TE, typename TL, int R>
const void *reach_fn(bool lds) {
    return lds ? reinterpret_cast<const void *>(&reach_kernel<TE, TL, R, true>)
               : reinterpret_cast<const void *>(&reach_kernel<TE, TL, R, false>);
}

template <typename TE, typename TL>
const void *reach_fn_r(const ReachConfig &c) {
    switch (c.runs_per_lane) {
    case 1: return reach_fn<TE, TL, 1>(c.table_in_lds);
    case 2: return reach_fn<TE, TL, 2>(c.table_in_lds);
    case 4: return reach_fn<TE, TL, 4>(c.table_in_lds);
    case 8: return reach_fn<TE, TL, 8>(c.table_in_lds);
    }
    return nullptr;
}

template <typename TE>
const void *reach_fn_l(const ReachConfig &c) {
    return c.lam_bytes == 2 ? reach_fn_r<TE, uint16_t>(c) : reach_fn_r<TE, uint32_t>(c);
}

const void *reach_function(const ReachConfig &c) {
    switch (c.entry_bytes) {
    case 1: return reach_fn_l<uint8_t>(c);
    case 2: return reach_fn_l<uint16_t>(c);
    case 4: return reach_fn_l<uint32_t>(c);
    }
    return nullptr;
}

uint32_t blocks_for(uint64_t threads, uint32_t per) { return (uint32_t)((threads + per - 1) / per); }

}  // namespace

hipError_t launch_reach(const ReachArgs &a, const ReachConfig &c, int grid, size_t lds, hipStream_t s) {
    switch (c.entry_bytes) {
    case 1: return launch_reach_l<uint8_t>(a, c, grid, lds, s);
    case 2: return launch_reach_l<uint16_t>(a, c, grid, lds, s);
    case 4: return launch_reach_l<uint32_t>(a, c, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

int reach_blocks_per_cu(const ReachConfig &c, size_t lds_bytes) {
    const void *fn = reach_function(c);
    if (!fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, c.block_threads, lds_bytes) != hipSuccess)
        return 0;
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
#define CALL0(w)                                                                                   \
    if (a.lam_bytes == 2)                                                                          \
        hipLaunchKernelGGL((join0_rel_kernel<w, uint16_t>), dim3(nb), dim3(256), 0, s, a);        \
    else                                                                                           \
        hipLaunchKernelGGL((join0_rel_kernel<w, uint32_t>), dim3(nb), dim3(256), 0, s, a);
    RI_DISPATCH_W(W, CALL0)
#undef CALL0
    return hipGetLastError();
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
    const uint32_t ngroups = (a.nchunks + a.G - 1) / a.G;
    const uint32_t nb = blocks_for((uint64_t)ngroups * a.L, 256);
    if (a.lam_bytes == 2)
        hipLaunchKernelGGL((join0_fun_kernel<uint16_t>), dim3(nb), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((join0_fun_kernel<uint32_t>), dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_joinN_fun(const JoinArgs &a, hipStream_t s) {
    const uint32_t ngroups = (a.nin + a.G - 1) / a.G;
    const uint32_t nb = blocks_for((uint64_t)ngroups * a.L, 256);
    hipLaunchKernelGGL(joinN_fun_kernel, dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
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

}  // namespace ri
