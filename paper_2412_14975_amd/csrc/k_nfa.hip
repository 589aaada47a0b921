// The NFA device of Sect. 2: chunked speculative recognition with the
// position NFA itself as chunk automaton (the third device of Fig. 1,
// compared in Tab. 3).  Chunk i is run from every single NFA state q (chunk
// 1 from q0 only); a run is a set of NFA states, moved on a byte b of class k
// to follow(S) & mask(k).  Its chunk map lambda_i(q) is the set reached at
// the chunk end (empty when every path died).  The join composes the
// relations: row q of (R1 R2) is the union of the rows R2(t) over t in R1(q).
#include "device.hpp"

namespace ri {
namespace {

template <int W>
__device__ __forceinline__ bool any_set(const uint64_t (&x)[W]) {
    uint64_t o = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) o |= x[w];
    return o != 0;
}

// One byte: S <- follow(S) & mask(class of b).  The loop over the members of
// S makes the work of a step the number of states in S (the NFA count of
// Fig. 1 counts the moves out of every active state).
template <int W>
__device__ __forceinline__ void nfa_step(uint64_t (&S)[W], uint32_t b, const uint64_t *follow, const uint64_t *mask,
                                         const uint8_t *cls) {
    uint64_t N[W];
#pragma unroll
    for (int w = 0; w < W; ++w) N[w] = 0;
#pragma unroll
    for (int w = 0; w < W; ++w)
        for (uint64_t bits = S[w]; bits; bits &= bits - 1) {
            const uint64_t *f = follow + (size_t)(w * 64 + __builtin_ctzll(bits)) * W;
#pragma unroll
            for (int v = 0; v < W; ++v) N[v] |= f[v];
        }
    const uint64_t *m = mask + (size_t)cls[b] * W;
#pragma unroll
    for (int w = 0; w < W; ++w) S[w] = N[w] & m[w];
}

// Job = 64 consecutive chunks (one per lane) x one start q; jobs are
// numbered start-major and handed out by a counter to persistent blocks.
// follow, mask and the byte classes are staged in LDS.
template <int W>
__global__ void __launch_bounds__(256) nfa_reach_kernel(NfaArgs a) {
    extern __shared__ __align__(16) uint64_t nsm[];
    uint64_t *follow = nsm;
    uint64_t *mask = follow + (size_t)a.L * W;
    uint8_t *cls = reinterpret_cast<uint8_t *>(mask + (size_t)a.K * W);
    for (uint32_t i = threadIdx.x; i < a.L * W; i += blockDim.x) follow[i] = a.follow[i];
    for (uint32_t i = threadIdx.x; i < a.K * W; i += blockDim.x) mask[i] = a.mask[i];
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) cls[i] = a.cls[i];
    __syncthreads();
    const uint32_t lane = threadIdx.x % kWave;
    for (;;) {
        const uint32_t job = wave_ticket(a.job_counter);
        if (job >= a.njobs) break;
        const uint32_t q = job / a.chunk_groups;
        const uint32_t chunk = (job - q * a.chunk_groups) * kWave + lane;
        const bool ok = chunk < a.nchunks;
        uint64_t p = 0, end = 0;
        uint64_t S[W];
#pragma unroll
        for (int w = 0; w < W; ++w) S[w] = 0;
        if (ok) {
            const uint64_t o = (uint64_t)chunk * a.cs;
            p = reinterpret_cast<uint64_t>(a.text) + o;
            end = reinterpret_cast<uint64_t>(a.text) + (o + a.cs < a.n ? o + a.cs : a.n);
            if (chunk != 0 || q == 0) {
#pragma unroll
                for (int w = 0; w < W; ++w) S[w] = (uint32_t)w == q / 64 ? 1ull << (q % 64) : 0ull;
            }
        }
        const uint64_t vend = p + ((end - p) & ~(uint64_t)15);
        // 16-byte blocks while any lane of the wave has a live set and bytes left
        for (;;) {
            const bool work = p < vend && any_set<W>(S);
            if (__ballot(work) == 0) break;
            if (work) {
                const uint4 v = load16(at(p));
                const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int i = 0; i < 16; ++i) nfa_step<W>(S, (wd[i >> 2] >> ((i & 3) * 8)) & 0xffu, follow, mask, cls);
                p += 16;
            }
        }
        for (p = p < vend ? vend : p; p < end && any_set<W>(S); ++p) nfa_step<W>(S, *at(p), follow, mask, cls);
        if (ok) {
            uint64_t *out = a.maps + ((uint64_t)chunk * a.L + q) * W;
#pragma unroll
            for (int w = 0; w < W; ++w) out[w] = S[w];
        }
    }
}

// Thread per (group of G consecutive relations, row q): X = row q of the
// first, then X <- union of row t of the next over t in X.
template <int W>
__global__ void __launch_bounds__(256) nfa_join_kernel(NfaJoinArgs a) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ngroups = (a.nin + a.G - 1) / a.G;
    if (tid >= (uint64_t)ngroups * a.L) return;
    const uint32_t grp = (uint32_t)(tid / a.L), q = (uint32_t)(tid % a.L);
    const uint32_t m0 = grp * a.G;
    const uint32_t m1 = m0 + a.G < a.nin ? m0 + a.G : a.nin;
    uint64_t X[W];
#pragma unroll
    for (int w = 0; w < W; ++w) X[w] = a.in[((uint64_t)m0 * a.L + q) * W + w];
    for (uint32_t m = m0 + 1; m < m1 && any_set<W>(X); ++m) {
        uint64_t Y[W];
#pragma unroll
        for (int w = 0; w < W; ++w) Y[w] = 0;
#pragma unroll
        for (int w = 0; w < W; ++w)
            for (uint64_t bits = X[w]; bits; bits &= bits - 1) {
                const uint64_t *row = a.in + ((uint64_t)m * a.L + w * 64 + __builtin_ctzll(bits)) * W;
#pragma unroll
                for (int v = 0; v < W; ++v) Y[v] |= row[v];
            }
#pragma unroll
        for (int w = 0; w < W; ++w) X[w] = Y[w];
    }
    uint64_t *out = a.out + tid * W;
#pragma unroll
    for (int w = 0; w < W; ++w) out[w] = X[w];
}

// Row q0 of the single remaining relation: acceptance and the canonical
// minimal-DFA state of the set (found among the powerset DFA's states by
// the hash of its members); the set as 2 W 32-bit words.
__global__ void nfa_final_kernel(FinalArgs f, const uint64_t *total, uint32_t W, int32_t *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    decide_bits(reinterpret_cast<const uint32_t *>(total), 2 * W, f, f.result);
    reset_counters(f.counters);
    if (out) {
        out[0] = f.result[0];
        out[1] = f.result[1];
    }
}

}  // namespace

hipError_t launch_nfa_reach(const NfaArgs &a, int grid, hipStream_t s) {
    const size_t lds = (size_t)(a.L + a.K) * a.W * 8 + 256;
    switch (a.W) {
    case 1: hipLaunchKernelGGL(nfa_reach_kernel<1>, dim3(grid), dim3(256), lds, s, a); break;
    case 2: hipLaunchKernelGGL(nfa_reach_kernel<2>, dim3(grid), dim3(256), lds, s, a); break;
    case 4: hipLaunchKernelGGL(nfa_reach_kernel<4>, dim3(grid), dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_nfa_join(const NfaJoinArgs &a, hipStream_t s) {
    const uint32_t ngroups = (a.nin + a.G - 1) / a.G;
    const uint32_t nb = blocks_for((uint64_t)ngroups * a.L, 256);
    switch (a.W) {
    case 1: hipLaunchKernelGGL(nfa_join_kernel<1>, dim3(nb), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(nfa_join_kernel<2>, dim3(nb), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(nfa_join_kernel<4>, dim3(nb), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_nfa_final(const FinalArgs &f, const uint64_t *total, uint32_t W, int32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(nfa_final_kernel, dim3(1), dim3(64), 0, s, f, total, W, out);
    return hipGetLastError();
}

}  // namespace ri
