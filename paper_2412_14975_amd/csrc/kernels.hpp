// Device kernels of the recognizer and their launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ri {

constexpr uint32_t kNoState = 0xFFFFFFFFu;   // "no run" in run_final / materialized maps

// Text, chunking and chunk-automaton tables shared by every reach kernel.
// One text: chunk i = text[i*cs, min((i+1)*cs, n)).  A batch of texts:
// chunk_addr/chunk_len describe every chunk slot (absolute address, length
// in the low 31 bits, bit 31 = first chunk of its text; length 0 = unused).
struct ScanArgs {
    const uint8_t *text;       // n bytes, 16-byte aligned (one text)
    uint64_t n;
    uint64_t cs;               // chunk size, multiple of 16 (batch: the largest chunk)
    uint32_t nchunks;          // chunks (batch: slots)
    const uint64_t *chunk_addr;   // batch only, else nullptr
    const uint32_t *chunk_len;    // batch only
    const void *table;         // (nstates + 1) rows of K entries, row nstates = dead row;
                               // an entry is the BYTE offset of the next state's row
    uint32_t table_bytes;      // padded to 16
    const uint16_t *code;      // byte -> class * entry_bytes (byte offset within a row)
    const uint32_t *starts;    // L start rows (byte offsets = state * row_bytes)
    uint32_t L;
    uint32_t row_bytes;        // K * entry_bytes
    uint32_t dead;             // byte offset of the dead row
    // up to two sink rows (every class leads back to the state): a run that
    // enters one ends there, so the converging reach stops it; ~0 = none
    uint32_t sink0 = 0xFFFFFFFFu, sink1 = 0xFFFFFFFFu;
};

// LDS bytes of the byte-code tables staged after the transition table: the
// 256 codes as u16, then the same codes as u8 (used when every code is below
// 256, i.e. a row is at most 256 bytes: 256 bytes are 64 dwords, so two
// lanes that read different codes of ASCII text never share an LDS bank)
constexpr uint32_t kCodeLdsBytes = 768;

// Merge area of a warm-up wave (hashed merging): 257 slots of a u32 key, a
// u8 id and a u8 rank.  Direct merging uses it as a 65-entry u32 key row
// (272 bytes) and then one byte per state, the dead row's included.
constexpr uint32_t kWarmMergeBytes = (257 * 6 + 15) & ~15u;
constexpr uint32_t kDirectKeyBytes = 272;
__host__ __device__ constexpr bool warm_direct_fits(uint32_t nstates) {
    return kDirectKeyBytes + nstates + 1 <= kWarmMergeBytes;
}

struct KernelShape {
    int entry_bytes;           // table entry: 1, 2, 4
    int tile_bytes;            // state ids in chunk maps / tiles: 2, 4
    int alias_bytes;           // local run index: 1, 2
    int runs_per_lane;         // 1, 2, 4
    bool table_in_lds;
    int block_threads;         // 1024
    int code_regs = 4;         // warm-up: registers of 64 byte codes (1 when the warm-up is <= 64 bytes)
    bool hashed = false;       // warm-up: starts fit one start block (L <= 64 runs_per_lane), merging by hashing
    bool direct = false;       // hashed warm-up merging through a table indexed by state instead (warm_direct_fits)
};

// Chunks that one warm-up wave takes at a time: with merging by hashing the
// wave interleaves the runs of several chunks (independent lookup chains)
// within the same register budget; otherwise one.
__host__ __device__ constexpr uint32_t warm_chunks_per_wave(bool hashed, bool direct, int runs_per_lane,
                                                           int code_regs) {
    (void)direct;   // direct merging takes the same number (measured: fewer is slower)
    return !hashed || code_regs == 4 ? 1u : runs_per_lane == 4 ? 2u : 4u;
}

// ---- plain reach: every (chunk, start) run to the chunk end or its death ----
struct PlainArgs {
    ScanArgs s;
    void *lam;                 // [L][nchunks] state ids, all-ones = no run
    uint32_t *job_counter;     // zero on entry
    uint32_t njobs;
    uint32_t chunk_groups;     // ceil(nchunks / 64)
};
hipError_t launch_plain(const PlainArgs &a, const KernelShape &k, int grid, size_t lds, hipStream_t st);

// ---- converging reach, step 1: warm-up of every run, then merging of runs
// of one chunk that are in the same state (state convergence) ----
//
// Run slots: warm-up block b (of G, each taking cpi chunks per iteration of
// `iters`) owns the region of the run arrays that holds L runs for each of
// its chunks, starting at warm_region(b); it fills its region from the front
// and reports the count in block_count[b].  A block is kWarmChunksPerBlock
// waves; cpi = kWarmChunksPerBlock * warm_chunks_per_wave(...).
constexpr uint32_t kWarmChunksPerBlock = 16;
__host__ __device__ inline uint64_t warm_region(uint32_t b, uint32_t G, uint32_t iters, uint32_t L, uint32_t cpi) {
    const uint64_t q = iters / G, r = iters % G;
    return (uint64_t)cpi * L * ((uint64_t)b * q + (b < r ? b : r));
}
// The first bytes of the warm-up read by the transformation automaton of the
// starts (the simultaneous automaton of Sin'ya, Matsuzaki and Sassa, ICPP
// 2013): its state after a word u is the vector of the states that every
// start reaches on u, so one lookup per byte advances every start of a chunk
// at once.  The host expands every word of up to k bytes.
struct PrefixArgs {
    const uint16_t *next;      // [n][K] successor by byte class (only states of depth < k)
    const uint8_t *count;      // [n] distinct live states, kPrefixWide when more than 64
    const uint16_t *tgt;       // [n][64] those states (ids), in order of the first start reaching them
    const uint8_t *map;        // [n][L] start -> index into tgt, 0xFF = dead
    uint32_t k;                // bytes walked; 0 = no walk
    uint32_t K;                // classes
    uint32_t shift;            // class = byte code >> shift
};
constexpr uint8_t kPrefixWide = 0xFF;
struct WarmArgs {
    ScanArgs s;
    PrefixArgs pfx;            // used by the grouped warm-up (at most 256 starts)
    uint32_t warm;             // bytes scanned by every run before merging (<= 256)
    void *alias;               // [nchunks][L] class (merged run) of every start, all-ones = no run
    uint32_t *run_base;        // [nchunks] first run of the chunk
    uint32_t *run_count;       // [nchunks] runs of the chunk (nullptr: not needed)
    uint32_t *run_chunk;       // [cap]
    uint32_t *run_state;       // [cap] state id after the warm-up
    uint32_t *counters;        // [2] set to 1 when a chunk has more than kRowCap runs
    uint32_t *block_count;     // [grid] runs in each block's region
    uint32_t cpi;              // chunks per block iteration
};
hipError_t launch_warm(const WarmArgs &a, const KernelShape &k, int grid, size_t lds, hipStream_t st);
size_t warm_lds_bytes(const KernelShape &k, uint32_t table_bytes, uint32_t L);

// ---- converging reach, step 2: the merged runs to the chunk end ----
struct LongArgs {
    ScanArgs s;
    uint32_t warm;
    const uint32_t *run_chunk;
    const uint32_t *run_state;
    uint32_t *run_final;       // state id at the chunk end, kNoState if the run died
    const uint32_t *block_count;   // runs of each warm-up block's region
    uint32_t warm_blocks;      // grid of the warm-up kernel
    uint32_t cpi;              // chunks per warm-up block iteration
};
hipError_t launch_long(const LongArgs &a, const KernelShape &k, int grid, size_t lds, hipStream_t st);

// blocks of a kernel that fit on one CU: which = 0 plain, 1 warm, 2 long
int blocks_per_cu(int which, const KernelShape &k, size_t lds);

// ---- long runs of a grouped batch: one persistent work-queue launch ----
// An item is a job of 64 consecutive runs of one group (automaton) in the
// group's dense run numbering.  A workgroup takes the groups in turn,
// starting at group blockIdx * ngroups / grid; for each group that still has
// jobs it computes the group's run prefix and stages its byte codes (and its
// table when `lds`) in LDS, and its waves pull jobs from the group's counter
// until none is left.  Runs are stepped as by launch_long (one run per
// lane).
struct QueueGroup {
    LongArgs la;
    uint32_t entry_bytes;      // 1, 2, 4
    uint32_t lds;              // 1: the table is staged in LDS
};
struct QueueArgs {
    const QueueGroup *groups;
    uint32_t ngroups;
    uint32_t *counters;        // [ngroups] jobs taken; zero before the launch
};
hipError_t launch_queue_long(const QueueArgs &a, int grid, size_t lds, hipStream_t st);
int queue_long_blocks_per_cu(size_t lds);

// ---- join ----
struct JoinArgs {
    // level 0 input: either plain chunk maps or the converged form
    bool converged;
    const void *lam;           // plain: [L][nchunks]
    const void *alias;         // converged: [nchunks][L]
    const uint32_t *run_base;  // converged
    const uint32_t *run_final; // converged
    int tile_bytes;
    int alias_bytes;
    uint32_t nchunks;
    const uint32_t *content;   // relations: content bitsets [nstates][W]
    const void *in;            // level >= 1: [nin][L] functions or [nin][L][W] relations
    uint32_t nin;
    void *out;                 // [nout][L] (int32) or [nout][L][W] (uint32)
    uint32_t L;
    uint32_t G;                // members per group
    const uint32_t *grp_first;  // batch: explicit level-0 groups (see ClsJoinArgs), else nullptr
    const uint32_t *grp_count;
    uint32_t ngroups;
};
hipError_t launch_join0_rel(const JoinArgs &a, int W, hipStream_t s);
// level 0 with the group's chunk maps staged in LDS (L * G * 4 bytes); W = 0 for functions
hipError_t launch_join0_tile(const JoinArgs &a, int W, hipStream_t s);
hipError_t launch_joinN_rel(const JoinArgs &a, int W, hipStream_t s);
hipError_t launch_join0_fun(const JoinArgs &a, hipStream_t s);
hipError_t launch_joinN_fun(const JoinArgs &a, hipStream_t s);
// chunk maps as [L][nchunks] int32 (-1 = no run), for inspection
hipError_t launch_materialize(const JoinArgs &a, int32_t *out, hipStream_t s);

// Join over merged runs with class-partitioned relations (converging reach,
// relational chunk automata).  Level 0 members are chunks (span 1, classes =
// runs of the chunk); level >= 1 members are relations of the level below
// (span = chunks per member; classes of a member = runs of its first chunk).
struct ClsJoinArgs {
    const void *alias;         // [nchunks][L] local run index, all-ones = no run
    uint32_t nchunks;
    uint32_t L;
    uint32_t G;                // members per group
    uint32_t nmembers;
    uint64_t span;             // chunks per member
    const uint32_t *run_base;  // level 0
    const uint32_t *run_final; // level 0
    const uint32_t *content;   // level 0: content bitsets [nstates][W]
    const uint32_t *ncls_in;   // level >= 1: [nmembers]
    const uint32_t *cont_in;   // level >= 1: [nmembers][L][W]; finalize: the last relation
    uint32_t *ncls_out;        // [ngroups]
    uint32_t *cont_out;        // [ngroups][L][W]
    // batch: explicit groups (members [grp_first[g], grp_first[g] + grp_count[g]),
    // count <= G) and the first chunk of each member; nullptr = fixed groups of
    // G consecutive members, member m starting at chunk m * span
    const uint32_t *grp_first;
    const uint32_t *grp_count;
    const uint32_t *member_chunk;
    uint32_t ngroups;          // with explicit groups
    const uint32_t *gate;      // non-null: every kernel of the join returns at once while *gate == 0
};
size_t cls_join_lds(const ClsJoinArgs &a, int W, int alias_bytes);
hipError_t launch_join_cls(const ClsJoinArgs &a, int W, int alias_bytes, bool level0, hipStream_t s);

// Join over merged runs by products of hit matrices (converging reach,
// relational chunk automata).  M_k (chunk k -> k+1) has one row per run
// (class) of chunk k: the bitmask of classes of chunk k+1 hit by the content
// of the run's end state.  The text's relation restricted to the initial
// state is row a0 of M_0 M_1 ... M_{K-2}; products over 64 consecutive
// members are reduced as a tree of wave shuffles.  Valid while every chunk
// has at most kRowCap runs (counters[2] stays 0); otherwise the class join
// must be used.
constexpr uint32_t kRowCap = 8;
struct HitArgs {
    const void *alias;         // [nchunks][L]
    uint32_t L;
    uint32_t nchunks;          // K
    const uint32_t *run_base;
    const uint32_t *run_count;
    const uint32_t *run_final;
    const uint32_t *csr_off;   // member lists of the RI-DFA states (see FinalArgs)
    const uint32_t *csr_idx;
    const uint32_t *content;   // the same as [nstates][W] bitsets when W <= 64, else nullptr
    uint32_t nmembers;         // level 0: K - 1 matrices; level >= 1: products of the level below
    const uint64_t *prod_in;   // level >= 1 and the last level: [nmembers] products, 8 rows x 8 columns in one word
    const uint32_t *rows_in;   // level >= 1: [nmembers]
    uint64_t *prod_out;        // [ngroups] products (row r = byte r, column c = bit c of it)
    uint32_t *rows_out;        // [ngroups]
};
// W: words of the dense content bitsets, 0 = member lists
hipError_t launch_hit_prod(const HitArgs &a, int W, int alias_bytes, bool level0, hipStream_t s);
// level 0 of the hit join and, in the same launch, level 0 of the class join
// gated on c.gate (W > 0; c.grp_first unused)
hipError_t launch_hit_prod_cls(const HitArgs &a, const ClsJoinArgs &c, int W, int alias_bytes, hipStream_t s);
// LDS bytes of one wave's staged alias rows in hit_prod0 (64 rows, plus 16
// for the alignment of the image)
__host__ __device__ constexpr size_t kHitStageBytes(uint32_t L, size_t alias_bytes) {
    return (((size_t)64 * L * alias_bytes + 16) + 15) & ~(size_t)15;
}

struct FinalArgs {
    const void *total;         // one relation [L][W] or one function [L]
    const uint32_t *fmask;     // relations: final N' states (W words)
    const uint32_t *hash;      // relations: cap slots of (RI-DFA state, final id); state ~0 = empty;
                               // slot of a state = FNV-1a of its members in ascending order
    uint32_t hash_cap;
    const uint32_t *csr_off;   // relations: member list of RI-DFA state p = csr_idx[csr_off[p] ..
    const uint32_t *csr_idx;   //   csr_off[p + 1]), ascending
    const uint32_t *content;   // relations with W <= 64: the same as [nstates][W] bitsets, else nullptr
    const int32_t *final_of_state;   // functions
    const uint8_t *accept_of_state;  // functions
    int32_t *result;           // [0] accept, [1] final state
    uint32_t *counters;        // [0..3] reset to zero for the next call
};
hipError_t launch_finalize_rel(const FinalArgs &a, int W, hipStream_t s);
hipError_t launch_finalize_fun(const FinalArgs &a, hipStream_t s);
hipError_t launch_finalize_cls(const FinalArgs &f, const ClsJoinArgs &a, int W, int alias_bytes, hipStream_t s);
// Levels of the class join of a queued call and its final step in one
// launch, gated on *lv[0].gate: lv[0] (level 0 when first0, else level 1) one
// group per block, the remaining levels by the block that finishes lv[0]
// last, then the final step on final_rel, the relation rows the last level
// wrote.
constexpr uint32_t kMaxClsLevels = 8;
struct ClsJoinAll {
    ClsJoinArgs lv[kMaxClsLevels];
    uint32_t nlevels;
    const uint32_t *final_rel;
    FinalArgs f;
    uint32_t *done;            // zero before the launch, left zero
};
hipError_t launch_cls_join_all(const ClsJoinAll &c, int W, int alias_bytes, bool first0, hipStream_t s);
// queued calls: the hit join's last level and final step (result to `out`
// unless the flag c.lv[0].gate is set) and, in the same launch, the gated
// class join from its level 1 (c.lv[0]) up (W > 0)
hipError_t launch_hit_tail_cls(const FinalArgs &f, const HitArgs &a, int32_t *out, const ClsJoinAll &c, int W,
                               int alias_bytes, hipStream_t s);
// The last level (a.nmembers <= kHitTailMax products in a.prod_in, 0 for a
// single chunk) and the final step, in one launch.
// result[2] = counters[2] (1: the hit-matrix result is not valid).  With
// out != nullptr an invalid result is redone by propagation in the same
// launch (prop_words <= kPropMaxWords) and {accept, final} is copied to out;
// with gated_after the kernel instead leaves out untouched and counters[2]
// set, for a class join gated on counters[2] that the caller enqueues next.
constexpr uint32_t kHitTailMax = 64;
hipError_t launch_finalize_hit(const FinalArgs &f, const HitArgs &a, int W, int alias_bytes, hipStream_t s,
                               int32_t *out = nullptr, uint32_t prop_words = 0, bool gated_after = false);
// Join by propagating the set of N' states chunk after chunk (one block; any
// number of runs per chunk, any interface size up to kPropMaxWords * 32).
constexpr uint32_t kPropMaxWords = 1024;
hipError_t launch_propagate(const FinalArgs &f, const HitArgs &a, uint32_t W, int alias_bytes, hipStream_t s);
// out[0] = accept, out[1] = final_state, in stream order
hipError_t launch_store_result(int32_t *out, int32_t accept, int32_t final_state, hipStream_t s);
// p[0 .. n) = 0 in stream order (a kernel, so that a captured graph replays it)
hipError_t launch_zero_words(uint32_t *p, uint32_t n, hipStream_t s);

// Batch results, one per text, from the last join level (one group per
// text, in text order): a class-partitioned relation or a function.
struct BatchFinalArgs {
    uint32_t ntexts;
    const uint32_t *text_slot;   // first chunk slot of each text
    const uint32_t *text_out;    // result row of each text
    int32_t *results;            // [rows][2]: accept, final state
};
hipError_t launch_batch_final_cls(const BatchFinalArgs &b, const FinalArgs &f, const ClsJoinArgs &a, int W,
                                  int alias_bytes, hipStream_t s);
// f.total: [ntexts][L] functions
hipError_t launch_batch_final_fun(const BatchFinalArgs &b, const FinalArgs &f, uint32_t L, hipStream_t s);
// results of texts whose automaton accepts nothing: (0, -1)
hipError_t launch_batch_fill(const BatchFinalArgs &b, hipStream_t s);

// ---- NFA device: the position NFA as chunk automaton over sets of states ----
struct NfaArgs {
    const uint8_t *text;       // one text, 16-byte aligned
    uint64_t n, cs;            // length, chunk size (multiple of 16)
    uint32_t nchunks;
    const uint64_t *follow;    // [L][W] follow sets
    const uint64_t *mask;      // [K][W] states entered on class k
    const uint8_t *cls;        // byte -> class
    uint32_t L, K, W;          // NFA states, classes, 64-bit words of a set (1, 2, 4)
    uint64_t *maps;            // [nchunks][L][W] set reached from each single state
    uint32_t *job_counter;     // zero on entry
    uint32_t njobs;            // L * chunk_groups
    uint32_t chunk_groups;     // ceil(nchunks / 64)
};
hipError_t launch_nfa_reach(const NfaArgs &a, int grid, hipStream_t s);

// groups of G consecutive relations [nin][L][W] composed into [ngroups][L][W]
struct NfaJoinArgs {
    const uint64_t *in;
    uint32_t nin;
    uint64_t *out;
    uint32_t L, W, G;
};
hipError_t launch_nfa_join(const NfaJoinArgs &a, hipStream_t s);
// row q0 of total ([L][W], the last relation): f.result = {accept, final state}
// (f.fmask, f.hash, f.csr_* describe the powerset DFA's states as sets of N's
// states); out (may be null) receives a copy
hipError_t launch_nfa_final(const FinalArgs &f, const uint64_t *total, uint32_t W, int32_t *out, hipStream_t s);

// ---- fused batches: many automata in one launch sequence ----
//
// Every chunk slot names its automaton; tables stay in global memory (L2),
// entry widths are read at run time, alias rows are 16-bit.  Every automaton
// is joined by hit matrices over member lists: an RI-DFA state stands for
// its content, a DFA state s (functional automata) for {s}.
struct AutoDesc {
    const void *table;
    const uint16_t *code;          // byte -> class * entry_bytes
    const uint32_t *starts;        // row offsets of the L starts
    uint32_t L, row_bytes, dead, entry_bytes;
    uint32_t functional;           // 1: content(s) = {s}, results from the tables below
    uint32_t W;                    // words of a set of starts
    const uint32_t *csr_off, *csr_idx, *fmask, *hash;
    uint32_t hash_cap;
    const int32_t *final_of_state;
    const uint8_t *accept_of_state;
    uint32_t sink0 = 0xFFFFFFFFu, sink1 = 0xFFFFFFFFu;   // sink rows as in ScanArgs
};

struct MultiArgs {
    const AutoDesc *autos;
    uint32_t nslots, ntexts;
    const uint64_t *chunk_addr;    // per slot (see ScanArgs)
    const uint32_t *chunk_len;
    const uint32_t *slot_auto;     // automaton of each slot
    const uint32_t *slot_text;     // text of each slot
    const uint64_t *alias_row;     // per slot: first entry of its alias row (uint16 entries)
    uint16_t *alias;
    uint32_t warm;
    uint32_t *run_base, *run_count, *run_chunk, *run_state, *run_final;
    uint32_t *counters;            // [1] runs; reset by the final kernel
    uint32_t *text_flag;           // per text: 1 when a chunk kept more than kRowCap runs
    // texts
    const uint32_t *text_slot, *text_nslots, *text_auto, *text_out, *text_prod;
    int32_t *results;              // [rows][2]
    // hit products: every level in one buffer
    uint64_t *prod;                // [groups] products (row r = byte r, column c = bit c of it)
    uint32_t *prod_rows;           // [groups]
    const uint32_t *grp_first, *grp_count;   // the level being launched
    uint32_t ngroups;
    uint32_t prod_out;             // first product index of the level being launched
};
hipError_t launch_mwarm(const MultiArgs &a, int grid, hipStream_t s);
hipError_t launch_mlong(const MultiArgs &a, int grid, hipStream_t s);
hipError_t launch_mhit(const MultiArgs &a, bool level0, hipStream_t s);
hipError_t launch_mfinal(const MultiArgs &a, hipStream_t s);
hipError_t launch_mprop(const MultiArgs &a, uint32_t max_words, hipStream_t s);
int multi_blocks_per_cu(int which);

}  // namespace ri
