"""MI355X (gfx950) subsequence DTW for signal-level Read Until.

Python binding of the C ABI in ``include/sdtw.h`` (``libsdtw.so``, built by
``__graft_entry__.build()`` or ``python paper_2211_07340_amd/build.py``).
This module only marshals arguments: every step runs in the HIP library.
Device memory and streams come from PyTorch (``torch.cuda``).
"""
from .binding import (F32, I16, EventStates, Plan, Reference, SdtwError, Stream, align_batch, align_one,
                      align_one_wide, align_one_wide_noalloc, autotune, detect_events,
                      detect_events_prefix, library_path, load_library, prepare_queries,
                      prepare_queries_ex, prepare_reference, row_budget_info, row_pool_trim,
                      set_row_budget, set_stream_config, stream_best_two, stream_extend,
                      stream_extend_wide, use_tuned, version)

__all__ = ["F32", "I16", "EventStates", "Plan", "Reference", "SdtwError", "Stream", "align_batch",
           "align_one", "align_one_wide", "align_one_wide_noalloc", "autotune", "detect_events",
           "detect_events_prefix", "library_path", "load_library", "prepare_queries",
           "prepare_queries_ex", "prepare_reference", "row_budget_info", "row_pool_trim",
           "set_row_budget", "set_stream_config", "stream_best_two", "stream_extend",
           "stream_extend_wide", "use_tuned", "version"]
