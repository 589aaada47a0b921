"""MI355X-native reduced-interface speculative data-parallel recognizer.

Implements the chunked recognizer of Borsotti, Breveglieri, Crespi Reghizzi
and Morzenti, "Minimizing speculation overhead in a parallel recognizer for
regular texts" (arXiv 2412.14975): an RI-DFA chunk automaton (Sect. 3) whose
reach and join phases run as HIP kernels on gfx950, behind the C ABI of
include/ri.h (libri.so).  ``binding`` is the ctypes layer with the C names.
"""

from .binding import (  # noqa: F401
    ALGOS, RIError, Recognizer, ri_build, ri_chunk_maps, ri_free, ri_info, ri_last_error,
    ri_last_timings, ri_recognize, ri_recognize_ex, ri_recognize_async, ri_set_profiling, ri_state_content,
    ri_set_option, ri_get_option, ri_autotune, Batch, ri_batch_create, ri_batch_free, ri_batch_run,
    ri_batch_capture, ri_batch_launch, ri_batch_get_info, ri_batch_get_group, ri_batch_autotune,
    ri_batch_create_ex, ri_batch_update, ri_request_footprint,
)
from . import serve  # noqa: F401,E402
