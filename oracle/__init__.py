"""CPU oracle for greedy D-optimal sensor selection (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never calls it and has no fallback
to it.  It shares no code with the HIP path; inputs come from ``oed_inputs``.

Functions and the passage of the paper each one follows:

* ``greedy`` -- the greedy algorithm of Sec. III-D with the objective of
  Sec. III-C (isotropic noise, max form): at every step each remaining
  candidate j is scored by ``1/2 [logdet K_{A u j} - logdet K_A] - (N_t/2) ln
  sigma^2`` with both log-determinants factored from scratch (the "naive
  formulation" of Sec. IV-A); the first strictly largest score wins.  Runs in
  C (``oed_oracle.c``), FP64, OpenMP over candidates.
* ``gains`` -- the scores of one greedy step for a given prefix (same rule).
* ``subset_logdet`` / ``objective`` -- ``logdet K_SS`` and
  ``f(S) = 1/2 logdet(sigma^-2 K_SS)`` by a from-scratch Cholesky (Sec. III-C).
* ``logdet_lapack`` -- ``logdet`` of a large SPD matrix through LAPACK's
  Cholesky (numpy); used where the C factorisation would take too long.
* ``schur_complement`` -- the definition ``K_RR - K_RA K_AA^{-1} K_AR`` of the
  Schur complement whose diagonal blocks are the matrices M_s of Algorithm 1
  (Sec. III-D), via a library solve.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from .build import LIB, build as _build

_lib = None

ORC_STATUS = {0: "ok", 1: "bad argument", 2: "no candidate with a finite score", 3: "out of memory",
              4: "factorisation of K_A failed"}


class OracleError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"oracle status {code} ({ORC_STATUS.get(code, '?')}) {msg}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            _build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oedo_chol_logdet.argtypes = [dp, ctypes.c_int64, dp]
        L.oedo_subset_logdet.argtypes = [dp, ctypes.c_int64, ctypes.c_int, ip, ctypes.c_int, dp]
        L.oedo_gains.argtypes = [dp, ctypes.c_int64, ctypes.c_int, ctypes.c_double, dp, ip, ctypes.c_int,
                                 ip, ctypes.c_int, dp, ctypes.c_int]
        L.oedo_greedy.argtypes = [dp, ctypes.c_int64, ctypes.c_int, ctypes.c_double, dp, ip, ctypes.c_int,
                                  ip, ctypes.c_int, ctypes.c_int, ip, dp, dp, ip, dp, ip, ctypes.c_int]
        _lib = L
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _as_K(K):
    K = np.ascontiguousarray(np.asarray(K, dtype=np.float64))
    if K.ndim != 2 or K.shape[0] != K.shape[1]:
        raise ValueError("K must be square")
    return K


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _ints(x):
    return np.ascontiguousarray(np.asarray(list(x) if x is not None else [], dtype=np.int32))


def chol_logdet(M):
    """logdet of a dense SPD matrix by the oracle's Cholesky (None if not PD)."""
    A = np.array(M, dtype=np.float64, order="C", copy=True)
    out = ctypes.c_double()
    rc = lib().oedo_chol_logdet(_dp(A), A.shape[0], ctypes.byref(out))
    return None if rc != 0 else out.value


def subset_logdet(K, N_t, S):
    """logdet(K_SS) for the ordered sensor list S (None if not PD)."""
    K = _as_K(K)
    S = _ints(S)
    out = ctypes.c_double()
    rc = lib().oedo_subset_logdet(_dp(K), K.shape[1], N_t, _ip(S), len(S), ctypes.byref(out))
    if rc == 3:
        raise OracleError(3)
    return None if rc != 0 else out.value


def objective(K, N_t, sigma2, S, noise_hld=None):
    """f(S) = 1/2 logdet K_SS - sum_{j in S} h_j, h_j = (N_t/2) ln sigma2 (isotropic noise) or
    noise_hld[j] (1/2 logdet of sensor j's noise covariance block)."""
    ld = subset_logdet(K, N_t, S)
    if ld is None:
        return None
    if noise_hld is None:
        return 0.5 * ld - 0.5 * len(S) * N_t * math.log(sigma2)
    return 0.5 * ld - float(sum(noise_hld[j] for j in S))


def _hld(noise_hld):
    return None if noise_hld is None else np.ascontiguousarray(np.asarray(noise_hld, dtype=np.float64))


def gains(K, N_t, sigma2, A, cands, threads=None, noise_hld=None):
    """Scores of ``cands`` at the greedy step that follows the ordered prefix A (noise_hld: per
    sensor 1/2 logdet of its noise covariance block; None = isotropic sigma2)."""
    K = _as_K(K)
    A = _ints(A)
    c = _ints(cands)
    h = _hld(noise_hld)
    g = np.empty(len(c), dtype=np.float64)
    rc = lib().oedo_gains(_dp(K), K.shape[1], N_t, float(sigma2), _dp(h), _ip(A), len(A), _ip(c), len(c),
                          _dp(g), threads or default_threads())
    if rc != 0:
        raise OracleError(rc)
    return g


def greedy(K, N_s, N_t, sigma2, B, candidates=None, prefix=None, threads=None, raise_on_error=True, noise_hld=None):
    """Greedy selection of B sensors.

    Returns a dict with ``idx`` (picked sensors, pick order), ``gain`` (their
    scores), ``gap`` (best minus runner-up score at each step), ``best`` and
    ``best_gain`` (what the rule itself would pick at each step given the
    prefix; equal to idx/gain except at forced steps) and ``status``.
    """
    K = _as_K(K)
    if K.shape[0] < N_s * N_t:
        raise ValueError("K smaller than N_s*N_t")
    cand = _ints(range(N_s) if candidates is None else candidates)
    pre = _ints(prefix)
    idx = np.full(B, -1, dtype=np.int32)
    gain = np.full(B, np.nan)
    gap = np.full(B, np.nan)
    best = np.full(B, -1, dtype=np.int32)
    best_gain = np.full(B, np.nan)
    n = ctypes.c_int()
    h = _hld(noise_hld)
    if h is not None and len(h) < N_s:
        raise ValueError("noise_hld needs one entry per sensor")
    rc = lib().oedo_greedy(_dp(K), K.shape[1], N_t, float(sigma2), _dp(h), _ip(cand), len(cand), _ip(pre),
                           len(pre), int(B), _ip(idx), _dp(gain), _dp(gap), _ip(best), _dp(best_gain),
                           ctypes.byref(n),
                           threads or default_threads())
    if rc != 0 and raise_on_error:
        raise OracleError(rc, f"after {n.value} picks")
    m = n.value
    return {"idx": idx[:m].copy(), "gain": gain[:m].copy(), "gap": gap[:m].copy(), "best": best[:m].copy(),
            "best_gain": best_gain[:m].copy(), "status": rc}


def logdet_lapack(M):
    """logdet of an SPD matrix through numpy's (LAPACK) Cholesky."""
    L = np.linalg.cholesky(np.asarray(M, dtype=np.float64))
    return 2.0 * float(np.sum(np.log(np.diagonal(L))))


def block_index(N_t, S):
    """Row/column indices of K that belong to the ordered sensor list S."""
    S = np.asarray(list(S), dtype=np.int64)
    return (S[:, None] * N_t + np.arange(N_t)[None, :]).reshape(-1)


def symmetrize_lower(K):
    """The symmetric matrix whose lower triangle is that of K."""
    K = np.asarray(K, dtype=np.float64)
    L = np.tril(K)
    return L + np.tril(K, -1).T


def schur_complement(K, N_t, A, rest):
    """``K_RR - K_RA K_AA^{-1} K_AR`` for sensor lists A (conditioned on) and R=rest."""
    Ks = symmetrize_lower(K)
    ia = block_index(N_t, A)
    ir = block_index(N_t, rest)
    KRR = Ks[np.ix_(ir, ir)]
    if len(ia) == 0:
        return KRR
    KAA = Ks[np.ix_(ia, ia)]
    KAR = Ks[np.ix_(ia, ir)]
    return KRR - KAR.T @ np.linalg.solve(KAA, KAR)
