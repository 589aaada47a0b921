/*
 * Oracle: the reach phase of chunked speculative recognition with one POSIX
 * thread per chunk, the CPU scheme of the paper's experiments (Sect. 4).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU baseline
 * of the benchmark may load this library.
 *
 * The chunk automaton is a dense deterministic table (one row of 256 int32
 * entries per state, -1 for an undefined move).  Chunk i is
 * text[bounds[i], bounds[i+1]); it is scanned from starts[0] only when i = 0
 * (Sect. 2: the first chunk starts in the initial state) and from every one
 * of the nstarts starts otherwise.  maps[i * nstarts + s] receives the end
 * state of the run of chunk i from start s, or -1 when the run dies (or was
 * not made).  Every thread counts its transitions like oracle_scan (a failing
 * move counts zero); the total is returned in *transitions.  The join is left
 * to the caller.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

struct chunk_job {
    const int32_t *table;
    const int32_t *starts;
    int32_t nstarts;
    const uint8_t *text;
    int64_t begin, end;
    int first;
    int32_t *maps;
    int64_t transitions;
};

static void *chunk_reach(void *arg)
{
    struct chunk_job *j = (struct chunk_job *)arg;
    int32_t ns = j->first ? 1 : j->nstarts;
    int64_t k = 0;
    for (int32_t s = 0; s < j->nstarts; ++s)
        j->maps[s] = -1;
    for (int32_t s = 0; s < ns; ++s) {
        int32_t q = j->starts[s];
        for (int64_t p = j->begin; p < j->end && q >= 0; ++p) {
            int32_t t = j->table[(int64_t)q * 256 + j->text[p]];
            if (t >= 0)
                ++k;
            q = t;
        }
        j->maps[s] = q;
    }
    j->transitions = k;
    return 0;
}

/* Returns 0, or -1 when a thread could not be started. */
int oracle_threaded_reach(const int32_t *table, const int32_t *starts, int32_t nstarts,
                          const uint8_t *text, const int64_t *bounds, int32_t chunks,
                          int32_t *maps, int64_t *transitions)
{
    struct chunk_job *jobs = calloc((size_t)chunks, sizeof(*jobs));
    pthread_t *th = calloc((size_t)chunks, sizeof(*th));
    int rc = 0;
    int32_t started = 0;
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -1;
    }
    for (int32_t i = 0; i < chunks; ++i) {
        jobs[i].table = table;
        jobs[i].starts = starts;
        jobs[i].nstarts = nstarts;
        jobs[i].text = text;
        jobs[i].begin = bounds[i];
        jobs[i].end = bounds[i + 1];
        jobs[i].first = i == 0;
        jobs[i].maps = maps + (int64_t)i * nstarts;
        if (pthread_create(&th[i], 0, chunk_reach, &jobs[i]) != 0) {
            rc = -1;
            break;
        }
        ++started;
    }
    int64_t total = 0;
    for (int32_t i = 0; i < started; ++i) {
        pthread_join(th[i], 0);
        total += jobs[i].transitions;
    }
    *transitions = total;
    free(jobs);
    free(th);
    return rc;
}
