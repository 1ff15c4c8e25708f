"""Helpers shared by the GPU parity tests (comparison rules, sub-matrix gathering)."""
from __future__ import annotations

import numpy as np

import oracle

# Gain tolerances: relative, with a floor of 1 nat, |g_gpu - g_or| <= RTOL * max(|g_or|, 1).
RTOL = {"fp64": 1e-10, "mixed_f32": 1e-4, "mixed_bf16x3": 1e-4}


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


def check_trajectory(K, N_s, N_t, s2, gpu_idx, gpu_gain, rtol, candidates=None):
    """Compare a GPU trajectory with the oracle replaying the GPU's own prefix.

    At every step the oracle scores all remaining candidates given the GPU's
    picks so far.  The GPU's pick must be the oracle's pick, except where the
    oracle's score of the GPU's pick is within tau = 2*rtol*max(|g_best|, 1) of
    the oracle's best score (a near-tie the precision cannot resolve).  The
    GPU's gains must match the oracle's scores of the same picks within rtol.
    Returns a dict with the per-step report.
    """
    B = len(gpu_idx)
    ref = oracle.greedy(K, N_s, N_t, s2, B, candidates=candidates, prefix=list(gpu_idx))
    assert len(ref["idx"]) == B
    assert list(ref["idx"]) == list(gpu_idx)
    err = rel_err(gpu_gain, ref["gain"])
    diverged = [k for k in range(B) if ref["best"][k] != gpu_idx[k]]
    for k in diverged:
        tau = 2.0 * rtol * max(abs(ref["best_gain"][k]), 1.0)
        assert ref["best_gain"][k] - ref["gain"][k] <= tau, (
            f"step {k}: GPU picked {gpu_idx[k]} (oracle score {ref['gain'][k]!r}), oracle best "
            f"{ref['best'][k]} ({ref['best_gain'][k]!r}), gap beyond tolerance {tau:.3e}")
    assert np.all(err <= rtol), f"max gain error {err.max():.3e} at step {int(np.argmax(err))} > {rtol}"
    return {"max_rel_err": float(err.max()) if B else 0.0, "diverged_steps": diverged, "ref": ref}


def lower_symmetric_sub(K, N_t, sensors):
    """Dense FP64 numpy block sub-matrix of K (device or host tensor) for the ordered sensor list."""
    from oed_inputs import k_sub_lower
    return k_sub_lower(K, N_t, sensors)
