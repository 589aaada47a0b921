/*
 * ri.h -- reduced-interface speculative data-parallel recognizer (RID) for
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Borsotti, Breveglieri, Crespi Reghizzi, Morzenti, "Minimizing
 * speculation overhead in a parallel recognizer for regular texts",
 * arXiv 2412.14975.
 *
 * The problem (Sect. 2): given a regular language L, written as a regular
 * expression, and a text x of n bytes, decide whether x is in L.  The text is
 * cut into c non-empty chunks; every chunk is scanned independently by a
 * deterministic chunk automaton from each of its possible start states (the
 * reach phase), and the per-chunk start->end maps are joined to check
 * consistency and acceptance (the join phase).
 *
 * RI_ALGO_RID runs the chunk automaton of Sect. 3: an RI-DFA whose start
 * (interface) states are the singletons of an NFA for L, after the interface
 * reduction of Sect. 3.4.  RI_ALGO_DFA is the classic baseline of Sect. 2
 * (Fig. 2): the minimal DFA speculated from all of its states.
 * RI_ALGO_SUBSET speculates from all states of the unminimized powerset DFA
 * of the position NFA (a second baseline for languages whose minimal DFA is
 * trivially small).  RI_ALGO_NFA is the third device of Sect. 2 (Fig. 1):
 * the position NFA itself as chunk automaton, every NFA state speculated,
 * each run a set of NFA states; the chunk relations are composed and the
 * set reached from q0 decides acceptance.
 *
 * Every call returns RI_OK (0) or a negative RI_ERR_* code; ri_last_error()
 * then gives a message for the calling thread.  No C++ exception crosses
 * this interface.  All functions are thread-safe; calls that share a stream
 * are ordered by that stream.
 *
 * Streams are passed as `void *` and are hipStream_t values (NULL = the
 * null stream).  Device pointers are plain HIP device addresses (for
 * example `torch.Tensor.data_ptr()` of a CUDA/ROCm tensor).
 */
#ifndef RI_H
#define RI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define RI_OK          0
#define RI_ERR_PARSE  (-1)   /* malformed expression; the message gives the byte offset */
#define RI_ERR_LIMIT  (-2)   /* an automaton exceeds max_states, or a size limit of the
                                device path is exceeded (see ri_recognize_ex) */
#define RI_ERR_NOMEM  (-3)   /* host or device allocation failed */
#define RI_ERR_DEVICE (-4)   /* a HIP call failed (no device, launch error, ...) */
#define RI_ERR_ARG    (-5)   /* invalid argument: NULL pointer, bad algo, misaligned text */

/* ---- algorithms -------------------------------------------------------- */
#define RI_ALGO_RID     0    /* RI-DFA chunk automaton, reduced interface (Sects. 3.1-3.4) */
#define RI_ALGO_DFA     1    /* minimal DFA, all states speculated (Sect. 2, Fig. 2)      */
#define RI_ALGO_SUBSET  2    /* powerset DFA of the position NFA, all states speculated  */
#define RI_ALGO_NFA     3    /* the position NFA itself, every state speculated, runs are
                                sets of states (the NFA device of Sect. 2, Fig. 1; Tab. 3);
                                at most 256 NFA states, single texts only               */
#define RI_NUM_ALGOS    4

typedef struct ri_handle ri_handle;   /* opaque; immutable after ri_build */

typedef struct {
    uint32_t max_states;   /* cap on the states of any automaton built; 0 = 1<<20 */
    uint32_t flags;        /* reserved, must be 0 */
} ri_build_opts;

typedef struct {
    int32_t  accept;       /* 1 iff x is in L (Th. 1)                                  */
    int32_t  final_state;  /* state of the minimal, trimmed DFA after x, numbered
                              breadth-first from the initial state with bytes scanned
                              in ascending order; -1 when the run dies               */
    uint64_t n;            /* text length                                              */
    uint32_t chunks;       /* number of chunks c actually used                         */
    uint32_t chunk_size;   /* bytes per chunk (the last one may be shorter)            */
} ri_result;

typedef struct {
    uint32_t nfa_states;          /* |Q_N|: trimmed position NFA (Sect. 4.1)          */
    uint32_t interface_states;    /* |I^{B_min}| = states of the quotient NFA N'      */
    uint32_t ridfa_states;        /* |P'|: states of B' = RI-DFA(N')                  */
    uint32_t ridfa_full_states;   /* |P|: states of B = RI-DFA(N) before reduction   */
    uint32_t min_dfa_states;      /* |Q_min| of the trimmed minimal DFA               */
    uint32_t subset_dfa_states;   /* states of the powerset DFA of N                  */
    uint32_t classes;             /* K: byte classes                                  */
    uint32_t accepts_empty;       /* 1 iff the empty text is in L                     */
    uint32_t starts[RI_NUM_ALGOS];      /* speculative starts per chunk, per algo      */
    uint32_t entry_bytes[RI_NUM_ALGOS]; /* bytes per transition-table entry, per algo  */
    uint64_t table_bytes[RI_NUM_ALGOS]; /* device transition-table bytes, per algo     */
    uint32_t prefix_depth[RI_NUM_ALGOS];  /* warm-up bytes covered by the transformation
                                             automaton of the starts (0: none; see
                                             RI_OPT_PREFIX)                               */
    uint32_t prefix_states[RI_NUM_ALGOS]; /* its states                                 */
} ri_info_t;

/*
 * ri_build -- construct every automaton for the expression `re` (re_len
 * bytes; see the package documentation for the syntax) on the host:
 * position NFA N, RI-DFA B = RI-DFA(N) (Sect. 3.1), Nerode classes of B and
 * the interface reduction (Sect. 3.4), the quotient NFA N' whose states are
 * the surviving interface states, B' = RI-DFA(N'), the minimal DFA and the
 * powerset DFA, and for automata of at most 256 starts the transformation
 * automaton of the starts over the first bytes (RI_OPT_PREFIX).  No device
 * call is made; tables are uploaded to the current
 * device by the first recognition call on it.
 * opts may be NULL.  On success *out owns everything until ri_free.
 * Errors: RI_ERR_ARG (NULL re/out, flags != 0), RI_ERR_PARSE, RI_ERR_LIMIT,
 * RI_ERR_NOMEM.
 */
int ri_build(const char *re, size_t re_len, const ri_build_opts *opts, ri_handle **out);

/* ri_free -- release host and device memory of a handle; NULL is a no-op.
 * No call on the handle may be in flight. */
void ri_free(ri_handle *h);

/* ri_info -- sizes of the constructed automata (host only). */
int ri_info(const ri_handle *h, ri_info_t *out);

/*
 * ri_recognize -- recognize the device-resident text `text_dev` of n bytes
 * with RI_ALGO_RID and an automatically chosen chunk count.  Equivalent to
 * ri_recognize_ex(h, text_dev, n, stream, RI_ALGO_RID, 0, out).
 */
int ri_recognize(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream,
                 ri_result *out);

/*
 * ri_recognize_ex -- chunked speculative recognition (Sects. 2 and 3.2).
 *
 * text_dev : device pointer to n bytes, 16-byte aligned (RI_ERR_ARG otherwise);
 *            owned by the caller and read-only; must stay valid until return.
 * n        : text length; n = 0 decides whether the empty text is in L without
 *            touching the device.
 * stream   : hipStream_t on which all work is enqueued; the call synchronizes
 *            this stream (only) before it returns.
 * algo     : RI_ALGO_RID, RI_ALGO_DFA, RI_ALGO_SUBSET or RI_ALGO_NFA (NFAs of at
 *            most 256 states, RI_ERR_LIMIT otherwise; the reach options do
 *            not apply to it, only the chunk count).
 * chunks   : requested chunk count c (0 = choose automatically).  Chunks are
 *            ceil(n/c) bytes rounded up to a multiple of 16, so the count used
 *            (reported in out->chunks) can be smaller; c is clamped to n.
 * out      : result (host memory).
 * Chunk i covers bytes [i*s, min((i+1)*s, n)) with s = out->chunk_size.
 * Scratch memory is owned by the handle, cached per stream and reused.
 * Errors: RI_ERR_ARG, RI_ERR_LIMIT (interface too large for the device join,
 * table too large for the device path), RI_ERR_NOMEM, RI_ERR_DEVICE.
 */
int ri_recognize_ex(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream,
                    int algo, uint32_t chunks, ri_result *out);

/*
 * ri_recognize_async -- the recognition of ri_recognize_ex (chunking of
 * Sect. 2, reach, join and acceptance of Sect. 3.2), enqueued on `stream`
 * without a host wait; the result stays in device memory.
 *
 * result_dev : int32[2] in device memory, 4-byte aligned, owned by the
 *              caller; when the stream reaches the end of the call it holds
 *              {accept (0/1), final state} with the meaning of ri_result
 *              (final state -3: internal inconsistency).  Nothing else is
 *              written to it.
 * text_dev, n, algo, chunks : as for ri_recognize_ex; the text and result_dev
 *              must stay valid until the stream has passed the call.
 * Calls on one stream run in order and reuse that stream's scratch memory;
 * the handle's options and last tuning apply as for ri_recognize_ex;
 * profiling timings are not recorded.  Scratch that has to grow for a longer
 * text is reallocated with no synchronization at all: the buffer it replaces
 * may still be in use by earlier queued calls, so it is freed with the
 * handle.
 * Errors found before anything is enqueued (RI_ERR_ARG: NULL or misaligned
 * pointers; RI_ERR_LIMIT; RI_ERR_NOMEM) are returned and nothing is written;
 * a launch failure returns RI_ERR_DEVICE.  Faults during execution surface
 * at the caller's next synchronization.
 */
int ri_recognize_async(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream,
                       int algo, uint32_t chunks, int32_t *result_dev);

/*
 * ri_recognize_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops and harnesses that forbid
 * hipMalloc): the queued recognition of ri_recognize_async, with the same
 * arguments and result, that allocates nothing.
 *
 * Its scratch memory is one fixed device array of RI_NOALLOC_SCRATCH_BYTES
 * per GPU, held until the process ends and shared by every call of this
 * function on that GPU; it keeps the last call's contents.  Calls on one
 * GPU that overlap in time (different streams, or host threads) race on
 * it: order them on one stream.  Counters that must start at zero are
 * cleared by a kernel at the start of each call.
 *
 * chunks = 0 chooses the chunk count as ri_recognize_async does and then
 * halves it until the call fits the array; an explicit chunk count that
 * does not fit is rejected with RI_ERR_LIMIT (the message gives the bytes
 * needed).  The handle's tables must already be on the current device
 * (any earlier recognition call on it uploads them): RI_ERR_ARG otherwise.
 * Other errors as for ri_recognize_async.
 */
#define RI_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int ri_recognize_noalloc(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream,
                         int algo, uint32_t chunks, int32_t *result_dev);

/*
 * ri_chunk_maps -- the reach phase only, for inspection: like ri_recognize_ex,
 * and in addition copies the chunk maps lambda_i (Sects. 2 and 3.2) to the
 * host array maps[c * starts + s] (int32, caller-owned, `cap` entries), where
 * s indexes the algorithm's start list (ri_info starts[algo]) and the value
 * is the chunk automaton's end state, or -1 when the run dies (or, for chunk
 * 0, for every start but the initial one).  RI_ERR_ARG if cap is too small.
 */
int ri_chunk_maps(const ri_handle *h, const uint8_t *text_dev, size_t n, void *stream,
                  int algo, uint32_t chunks, int32_t *maps, size_t cap, ri_result *out);

/*
 * ri_state_content -- for RI_ALGO_RID, the content of RI-DFA state `state`
 * (the states of N' it stands for, Sect. 3.1), written in ascending order to
 * members[0..*count) (at most cap entries); start s of RI_ALGO_RID is the
 * singleton {s} of N'.  RI_ERR_ARG for RI_ALGO_NFA.  For RI_ALGO_DFA /
 * RI_ALGO_SUBSET, the minimal-DFA
 * state that the state stands for (one entry), or no entry for none.
 */
int ri_state_content(const ri_handle *h, int algo, uint32_t state, uint32_t *members,
                     uint32_t cap, uint32_t *count);

/*
 * ri_set_profiling / ri_last_timings -- when enabled, each recognition call
 * records HIP events on its stream around its kernels; ri_last_timings then
 * returns, for the last completed call on this handle, in milliseconds:
 * ms[0] reach phase (all reach kernels), ms[1] join and finalize kernels,
 * ms[2] whole enqueue-to-result, ms[3] the dominant reach kernel alone
 * (the plain reach kernel, or the long-run kernel of the converging reach),
 * ms[4] the warm-up kernel of the converging reach (0 for the plain one).
 */
int ri_set_profiling(ri_handle *h, int enable);
int ri_last_timings(const ri_handle *h, float ms[5]);

/*
 * ri_set_option / ri_get_option -- per-handle tuning of the reach phase;
 * a new value applies to calls that start after it is set.
 *   RI_OPT_CONVERGE       1 (default): every run is scanned for a warm-up of
 *                         RI_OPT_WARMUP_BYTES, then the runs of a chunk that
 *                         are in the same state are merged (state
 *                         convergence; the chunk maps are unchanged).
 *                         0: every run is scanned to the chunk end or to its
 *                         death, as the reach phase is stated.
 *   RI_OPT_WARMUP_BYTES   multiple of 16 in [16, 256]; default 64.
 *   RI_OPT_RUNS_PER_LANE  independent runs per GPU lane: 0 (automatic), 1, 2, 4.
 *   RI_OPT_CHUNK_TARGET   chunk count aimed at when chunks = 0; default 131072.
 *   RI_OPT_JOIN           join of the converging reach for RI_ALGO_RID:
 *                         0 (default): products of per-chunk hit matrices
 *                         (rows = merged runs of a chunk, columns = merged
 *                         runs of the next chunk), reduced as a tree; when a
 *                         chunk keeps more than 8 runs the call falls back
 *                         to 1.  1: class-partitioned relations composed
 *                         member by member within groups.  Results are
 *                         identical; only the speed differs.
 *   RI_OPT_PREFIX         1 (default): for 65 to 256 starts (the grouped
 *                         warm-up, more than one register of starts), the
 *                         first warm-up bytes of a chunk are read by the
 *                         transformation automaton of the starts, built by
 *                         ri_build (a state = the states every start reaches
 *                         on the bytes read so far; every word of up to
 *                         ri_info_t.prefix_depth bytes, at most 65535
 *                         states); the walk covers that depth rounded down to
 *                         a multiple of 8, at most the warm-up.  0: every
 *                         start steps byte by byte.  Results are identical.
 * Errors: RI_ERR_ARG for an unknown option or a value out of range.
 */
#define RI_OPT_CONVERGE       1
#define RI_OPT_WARMUP_BYTES   2
#define RI_OPT_RUNS_PER_LANE  3
#define RI_OPT_CHUNK_TARGET   4
#define RI_OPT_JOIN           5
#define RI_OPT_PREFIX         6
int ri_set_option(ri_handle *h, int option, int64_t value);
int ri_get_option(const ri_handle *h, int option, int64_t *value);

/*
 * ri_autotune -- pick the reach-phase settings for `algo` by timing a fixed
 * grid of them on the given device text (same arguments as ri_recognize_ex;
 * every trial is a full recognition whose result is checked against the
 * first one): the converging reach over chunk targets x warm-up bytes x runs
 * per lane, and the plain reach over chunk targets x runs per lane; a
 * setting the automaton does not support (RI_ERR_LIMIT, e.g. the plain reach
 * of an interface wider than its join takes) is skipped.  The
 * best setting is stored in the handle for that algorithm and used by later
 * calls with chunks = 0, until ri_set_option is called.  `out` (may be
 * NULL) receives the chosen values and the best time.  Must not run
 * concurrently with other calls on the same handle.
 */
typedef struct {
    uint32_t chunk_target;
    uint32_t warmup_bytes;
    uint32_t runs_per_lane;
    uint32_t trials;
    float best_ms;
    uint32_t converge;     /* 1: converging reach chosen; 0: plain reach */
} ri_tuning;
int ri_autotune(ri_handle *h, const uint8_t *text_dev, size_t n, void *stream, int algo,
                ri_tuning *out);

/* ---- batches ------------------------------------------------------------
 *
 * Many texts, each with its own automaton and algorithm, recognized by one
 * sequence of launches.  Requests are grouped by (handle, algo); within a
 * group every text is cut into chunks of the group's chunk size, and all
 * chunks of all texts of the group go through one converging reach
 * (RI_OPT_CONVERGE = 1 whatever the handle's setting) and one join tree
 * whose groups never span two texts, so each text's result is exactly the
 * one ri_recognize_ex gives for it (Th. 1 applies to every text alone).
 */
typedef struct ri_batch ri_batch;   /* opaque */

typedef struct {
    const ri_handle *h;        /* automaton; must stay alive while the batch exists  */
    const uint8_t *text_dev;   /* device pointer, 16-byte aligned; NULL allowed if n = 0 */
    uint64_t n;                /* text length (0 allowed)                             */
    int32_t algo;              /* RI_ALGO_RID, RI_ALGO_DFA or RI_ALGO_SUBSET (not NFA) */
    uint32_t reserved;         /* must be 0                                           */
} ri_request;

typedef struct {
    uint32_t texts;            /* requests                                            */
    uint32_t groups;           /* (handle, algo) groups                               */
    uint64_t slots;            /* chunks over all groups                              */
    uint64_t bytes;            /* text bytes over all requests                        */
    uint64_t device_bytes;     /* device memory held by the batch (not the tables)    */
    uint32_t kernels;          /* kernel launches per run                             */
    uint32_t captured;         /* 1 after a successful ri_batch_capture               */
    uint32_t fused;            /* 1: fused plan (RI_BATCH_FUSED), 0: grouped          */
    uint32_t queue;            /* grouped: 1 when the long runs of every group go to  */
                               /* one work-queue launch (RI_BATCH_QUEUE, or chosen by */
                               /* ri_batch_autotune for an RI_BATCH_AUTO batch)       */
} ri_batch_info;

typedef struct {
    const ri_handle *h;
    int32_t algo;
    uint32_t texts;
    uint32_t slots;            /* chunks of the group                                 */
    uint64_t bytes;
    uint32_t chunk_bytes;      /* chunk size used for every text of the group         */
    uint32_t warmup_bytes;
    uint32_t runs_per_lane;
    uint32_t join_levels;
    float tuned_ms;            /* best time found by ri_batch_autotune, else 0        */
} ri_batch_group;

typedef struct {
    uint32_t trials;           /* settings timed                                      */
    float best_ms;             /* sum over groups of the best group times             */
} ri_batch_tuning;

/*
 * ri_batch_create -- plan a batch of `count` requests on the current device:
 * build the chunk descriptors and join levels, upload the automata that are
 * not yet on the device and allocate every buffer the batch needs.  The
 * requests array is copied; the texts are read only by later runs, so they
 * must stay valid (and unchanged in place and size) until the last run.
 * chunk_bytes: multiple of 16, the chunk size of every group; 0 = chosen per
 * group from its total size (about 131072 chunks per group, 256 B to 1 MiB).
 * Synchronous.  Errors: RI_ERR_ARG (NULL pointers, misaligned text, bad
 * algo, chunk_bytes not a multiple of 16), RI_ERR_LIMIT (interface too large
 * for the device join, more than 2^31 chunk maps in a group), RI_ERR_NOMEM,
 * RI_ERR_DEVICE.
 */
int ri_batch_create(const ri_request *reqs, uint32_t count, uint32_t chunk_bytes, ri_batch **out);

/*
 * ri_batch_create_ex -- ri_batch_create with options (opts may be NULL):
 *   chunk_bytes   as for ri_batch_create;
 *   mode          RI_BATCH_GROUPED: one launch sequence per (handle, algo)
 *                 group, tables staged in LDS, per-group tuning (interfaces
 *                 up to 2048 states);
 *                 RI_BATCH_QUEUE: as GROUPED for the warm-up and the joins,
 *                 but the long runs of every group go to one persistent
 *                 work-queue launch: a job is 64 consecutive runs of one
 *                 group; a workgroup takes the groups in turn, stages the
 *                 group's table in LDS (when it fits, else it reads it from
 *                 L2) and its waves pull that group's jobs until none is
 *                 left (the paper's reach phase, Sect. 2, over many texts
 *                 at once);
 *                 RI_BATCH_FUSED: one launch sequence for every text of every
 *                 automaton: each chunk slot and text names its automaton,
 *                 tables are read from global memory (L2), every automaton
 *                 (RI-DFA, DFA, powerset DFA) is joined by hit matrices over
 *                 member lists, and texts whose chunks keep more than 8 runs
 *                 are joined by propagation.  A text gets at most 2^22
 *                 (start, chunk) pairs: its chunks grow beyond chunk_bytes when
 *                 needed;
 *                 RI_BATCH_AUTO (0): fused when an interface exceeds 2048 states
 *                 or the groups average less than 4 MiB of text, else grouped;
 *   warmup_bytes  0 (the handles' settings; 64 for fused) or a multiple of 16
 *                 in [16, 256];
 *   reserved      must be 0.
 */
#define RI_BATCH_AUTO     0
#define RI_BATCH_GROUPED  1
#define RI_BATCH_FUSED    2
#define RI_BATCH_QUEUE    3
typedef struct {
    uint32_t chunk_bytes;
    uint32_t mode;
    uint32_t warmup_bytes;
    uint32_t reserved;
} ri_batch_opts;
int ri_batch_create_ex(const ri_request *reqs, uint32_t count, const ri_batch_opts *opts, ri_batch **out);

/*
 * ri_batch_update -- re-plan a fused batch for a new set of requests (same
 * rules as ri_batch_create_ex), keeping its options and tuned chunk size and
 * warm-up and reusing its device buffers (they grow only when the new plan
 * needs more).  No run or graph launch of the batch may be in flight; a
 * captured graph is dropped.  Synchronous.  RI_ERR_ARG for a grouped batch.
 */
int ri_batch_update(ri_batch *b, const ri_request *reqs, uint32_t count);

/*
 * ri_request_footprint -- device bytes that one request (text of n bytes,
 * handle h, algo) occupies in a fused batch with this chunk_bytes (0 = the
 * fused default): the text itself plus its share of the batch's buffers.
 * Host only; for admission control.
 */
int ri_request_footprint(const ri_handle *h, int algo, uint64_t n, uint32_t chunk_bytes, uint64_t *bytes);

/* ri_batch_free -- release the batch (not the handles); NULL is a no-op.
 * No run or graph launch of the batch may be in flight. */
void ri_batch_free(ri_batch *b);

/*
 * ri_batch_run -- enqueue the whole batch on `stream` and return without
 * waiting.  results_dev: device array of 2 * count int32, written as
 * results_dev[2*i] = accept, results_dev[2*i+1] = final state of request i
 * (the values of ri_result).  Allocates nothing and makes no synchronous
 * call, so it may be captured into a HIP graph by the caller.  Runs of one
 * batch must not overlap (they share its buffers): order them on one stream.
 */
int ri_batch_run(ri_batch *b, void *stream, int32_t *results_dev);

/*
 * ri_batch_capture / ri_batch_launch -- capture one run of the batch into a
 * HIP graph kept by the batch (groups become independent branches that may
 * execute concurrently), writing to results_dev; ri_batch_launch then
 * launches that graph on `stream` (one call, no host work per text).  A
 * new capture replaces the previous graph; ri_batch_autotune drops it.
 */
int ri_batch_capture(ri_batch *b, int32_t *results_dev);
int ri_batch_launch(ri_batch *b, void *stream);

/* ri_batch_get_info / ri_batch_get_group -- sizes of the plan. */
int ri_batch_get_info(const ri_batch *b, ri_batch_info *out);
int ri_batch_get_group(const ri_batch *b, uint32_t index, ri_batch_group *out);

/*
 * ri_batch_autotune -- time the batch under a fixed grid of chunk sizes
 * (unless chunk_bytes was given at creation) and warm-up lengths and re-plan
 * with the fastest: per group for a grouped batch, for the whole batch for a
 * fused one.  A grouped batch created with RI_BATCH_AUTO then also times its
 * two placements of the long runs -- one launch sequence per group, or every
 * group's long runs in one work-queue launch (as RI_BATCH_QUEUE) -- and keeps
 * the faster (ri_batch_info.queue).  Every trial's results must equal the
 * first trial's (RI_ERR_DEVICE otherwise).  Synchronizes `stream`; allocates.
 * out may be NULL; out->best_ms is then the whole run's time for such a batch.
 */
int ri_batch_autotune(ri_batch *b, void *stream, ri_batch_tuning *out);

/* ri_last_error -- message of the last failing call on this thread. */
const char *ri_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RI_H */
