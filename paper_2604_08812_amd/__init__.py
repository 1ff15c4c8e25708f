"""Greedy D-optimal sensor selection on MI355X (gfx950).

The selection runs in liboed.so (HIP kernels behind the C ABI of
``include/oed.h``); ``oed`` is its thin ctypes binding.
"""
from .oed import (  # noqa: F401
    EXPORTED,
    BatchSelector,
    Evaluator,
    oed_eval_create,
    oed_eval_destroy,
    oed_eval_run,
    oed_eval_stats,
    oed_batch_create,
    oed_batch_destroy,
    oed_batch_get_config,
    oed_batch_reset,
    oed_batch_run,
    oed_batch_stats,
    LIB_PATH,
    OedError,
    PRECISIONS,
    Selector,
    library,
    oed_create,
    oed_destroy,
    oed_device_bytes,
    oed_force,
    oed_get_config,
    oed_get_profile,
    oed_greedy,
    oed_greedy_noalloc,
    oed_pack_rows,
    oed_picks,
    oed_reset,
    oed_schur_block,
    oed_scores,
)
