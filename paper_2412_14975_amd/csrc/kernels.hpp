// Device kernels of the recognizer and their launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ri {

// Reach phase: every (chunk, start) run of the chunk automaton.
struct ReachArgs {
    const uint8_t *text;       // n bytes, 16-byte aligned
    uint64_t n;
    uint64_t cs;               // chunk size, multiple of 16
    uint32_t nchunks;
    const void *table;         // (nstates + 1) * K entries, row nstates = dead row
    uint32_t table_bytes;      // padded to 16
    const uint8_t *cls;        // byte -> class
    const uint32_t *starts;    // L start rows (entry offsets = state * K)
    uint32_t L;
    uint32_t K;
    uint32_t dead;             // entry offset of the dead row
    void *lam;                 // [L][nchunks] end state ids, all-ones = no run
    uint32_t *job_counter;     // zero on entry, zeroed again by finalize
    uint32_t njobs;
    uint32_t chunk_groups;     // ceil(nchunks / 64)
};

struct ReachConfig {
    int entry_bytes;           // 1, 2, 4
    int lam_bytes;             // 2, 4
    int runs_per_lane;         // 1, 2, 4, 8
    bool table_in_lds;
    int block_threads;         // 1024
};

hipError_t launch_reach(const ReachArgs &a, const ReachConfig &cfg, int grid_blocks,
                        size_t lds_bytes, hipStream_t s);
// blocks of the reach kernel that fit on one CU for this config
int reach_blocks_per_cu(const ReachConfig &cfg, size_t lds_bytes);

// Join phase.
struct JoinArgs {
    const void *lam;           // level 0: chunk maps [L][nchunks]
    int lam_bytes;
    uint32_t nchunks;
    const uint32_t *content;   // relations: content bitsets [nstates][W]
    const void *in;            // level >= 1: [nin][L] functions or [nin][L][W] relations
    uint32_t nin;
    void *out;                 // [nout][L] (int32) or [nout][L][W] (uint32)
    uint32_t L;
    uint32_t G;                // members per group
};

hipError_t launch_join0_rel(const JoinArgs &a, int W, hipStream_t s);
hipError_t launch_joinN_rel(const JoinArgs &a, int W, hipStream_t s);
hipError_t launch_join0_fun(const JoinArgs &a, hipStream_t s);
hipError_t launch_joinN_fun(const JoinArgs &a, hipStream_t s);

struct FinalArgs {
    const void *total;         // one relation [L][W] or one function [L]
    const uint32_t *fmask;     // relations: final N' states (W words)
    const uint32_t *hash;      // relations: cap slots of (W key words, 1 value word)
    uint32_t hash_cap;
    const int32_t *final_of_state;   // functions
    const uint8_t *accept_of_state;  // functions
    int32_t *result;           // [0] accept, [1] final state
    uint32_t *job_counter;     // reset to zero
};

hipError_t launch_finalize_rel(const FinalArgs &a, int W, hipStream_t s);
hipError_t launch_finalize_fun(const FinalArgs &a, hipStream_t s);

}  // namespace ri
