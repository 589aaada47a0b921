/*
 * Oracle: plain serial scan of a deterministic transition table.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU baseline
 * of the benchmark may load this library.
 *
 * The table is dense, one row of 256 int32 entries per state, entry -1 for an
 * undefined move.  oracle_scan runs one deterministic run over text[begin,end)
 * from state `start` (the serial operation of Sect. 2 when the range is the
 * whole text) and counts the transitions actually made: a failing move counts
 * zero and ends the run (the counting of Fig. 1).
 */
#include <stdint.h>

int32_t oracle_scan(const int32_t *table, int32_t start, const uint8_t *text,
                    int64_t begin, int64_t end, int64_t *transitions)
{
    int32_t s = start;
    int64_t k = 0;
    for (int64_t j = begin; j < end && s >= 0; ++j) {
        int32_t t = table[(int64_t)s * 256 + text[j]];
        if (t >= 0)
            ++k;
        s = t;
    }
    if (transitions)
        *transitions = k;
    return s;
}
