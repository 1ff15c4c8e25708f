"""Thin ctypes binding of liboed (the C ABI in include/oed.h).

Argument marshalling only: every step of the selection runs in the HIP
kernels of liboed.so.  torch is used for device memory (``K`` is a CUDA/HIP
tensor whose ``data_ptr()`` is handed over) and for the current stream.  If
liboed.so has not been built, importing this module raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboed.so")

OED_OK, OED_E_ARG, OED_E_NOT_SPD, OED_E_OOM, OED_E_HIP, OED_E_STATE, OED_E_UNSUPPORTED = range(7)
OED_F64, OED_F32 = 0, 1
PRECISIONS = {"fp64": 0, "mixed_f32": 1, "mixed_bf16x3": 2}
OED_FLAG_PROFILE = 1
OED_FLAG_AUTOTUNE = 4
OED_FLAG_DEFER_PACK = 8
OED_MAX_DELAY = 8
KERNELS = ("gain", "pick", "trsm", "syrk", "pack")


class oed_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("candidates", ctypes.POINTER(ctypes.c_int32)), ("n_candidates", ctypes.c_int32),
                ("delay", ctypes.c_int32), ("method", ctypes.c_int32), ("max_budget", ctypes.c_int32),
                ("noise_half_logdet", ctypes.POINTER(ctypes.c_double)), ("tune_cache", ctypes.c_char_p),
                ("max_device_bytes", ctypes.c_int64), ("tile_order", ctypes.c_int32),
                ("debug_fail_step", ctypes.c_int32), ("tile_size", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


TILE_ORDERS = {"auto": 0, "row8": 1, "col8": 2, "col4": 3, "col2": 4}


class oed_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 5), ("launches", ctypes.c_int64 * 5), ("syrk_flops", ctypes.c_double),
                ("syrk_bytes", ctypes.c_double)]


class oed_instance(ctypes.Structure):
    _fields_ = [("K_dev", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("N_s", ctypes.c_int32),
                ("N_t", ctypes.c_int32), ("budget", ctypes.c_int32), ("ld", ctypes.c_int64),
                ("sigma2", ctypes.c_double)]


OED_BATCH_NO_GRAPH = 2
OED_BATCH_AUTOTUNE = 0x10
OED_BATCH_LEFT_LOOKING = 0x20


class OedError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


_lib = None


def library() -> ctypes.CDLL:
    """Load liboed.so (raises if it is missing: build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"liboed.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    L.oed_options_init.argtypes = [ctypes.POINTER(oed_options)]
    L.oed_options_init.restype = None
    L.oed_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                             ctypes.c_double, vp, ctypes.POINTER(oed_options)]
    L.oed_reset.argtypes = [vp, vp]
    L.oed_pack_rows.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    L.oed_greedy.argtypes = [vp, ctypes.c_int32, ip, dp, ip]
    L.oed_force.argtypes = [vp, ctypes.c_int32, dp]
    L.oed_scores.argtypes = [vp, dp]
    L.oed_schur_block.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, dp]
    L.oed_picks.argtypes = [vp, ip, dp, ip]
    L.oed_get_profile.argtypes = [vp, ctypes.POINTER(oed_profile), ctypes.c_int32]
    L.oed_device_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.oed_get_config.argtypes = [vp, ip, ip, ip, dp]
    L.oed_destroy.argtypes = [vp]
    L.oed_last_error.argtypes = [vp]
    L.oed_last_error.restype = ctypes.c_char_p
    L.oed_status_string.argtypes = [ctypes.c_int32]
    L.oed_status_string.restype = ctypes.c_char_p
    L.oed_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(oed_instance), ctypes.c_int32, ctypes.c_int32,
                                   vp, ctypes.c_uint32]
    L.oed_batch_run.argtypes = [vp, ip, dp, ip, ip]
    L.oed_batch_reset.argtypes = [vp, ctypes.POINTER(oed_instance), ctypes.c_int32]
    L.oed_batch_stats.argtypes = [vp, dp, dp, dp]
    L.oed_batch_destroy.argtypes = [vp]
    L.oed_batch_get_config.argtypes = [vp, ip, ip, ip, dp]
    L.oed_batch_last_error.argtypes = [vp]
    L.oed_batch_last_error.restype = ctypes.c_char_p
    L.oed_eval_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                  ctypes.c_uint32]
    L.oed_eval_run.argtypes = [vp, ip, ctypes.c_int32, dp, dp]
    L.oed_eval_stats.argtypes = [vp, dp, dp, ctypes.POINTER(ctypes.c_int64), ip]
    L.oed_eval_destroy.argtypes = [vp]
    L.oed_eval_last_error.argtypes = [vp]
    L.oed_eval_last_error.restype = ctypes.c_char_p
    L.oed_greedy_noalloc.argtypes = [vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                                     vp, ctypes.c_char_p, ctypes.c_int32]
    for name in ("oed_create", "oed_reset", "oed_pack_rows", "oed_greedy", "oed_force", "oed_scores", "oed_schur_block", "oed_picks",
                 "oed_get_profile", "oed_device_bytes", "oed_destroy", "oed_batch_create", "oed_batch_run",
                 "oed_batch_reset", "oed_batch_stats", "oed_batch_destroy", "oed_batch_get_config", "oed_get_config",
                 "oed_eval_create", "oed_eval_run", "oed_eval_stats", "oed_eval_destroy", "oed_greedy_noalloc"):
        getattr(L, name).restype = ctypes.c_int32
    _lib = L
    return L


EXPORTED = ("oed_options_init", "oed_create", "oed_reset", "oed_pack_rows", "oed_greedy", "oed_force", "oed_scores",
            "oed_schur_block", "oed_picks", "oed_get_profile", "oed_device_bytes", "oed_get_config", "oed_destroy",
            "oed_last_error",
            "oed_status_string", "oed_batch_create", "oed_batch_run", "oed_batch_reset", "oed_batch_stats",
            "oed_batch_destroy", "oed_batch_last_error", "oed_batch_get_config", "oed_eval_create", "oed_eval_run",
            "oed_eval_stats", "oed_eval_destroy", "oed_eval_last_error", "oed_greedy_noalloc")
OED_NOALLOC_MAX_BYTES = 64 << 20


def _status_name(s):
    try:
        return library().oed_status_string(s).decode()
    except Exception:  # pragma: no cover - only when the library itself is unusable
        return f"status {s}"


def _check(h, st):
    if st != OED_OK:
        msg = library().oed_last_error(h).decode() if h else ""
        raise OedError(st, msg)


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


# ------------------------------------------------------------------ functions with the C names
def oed_create(K, N_s, N_t, sigma2, precision="fp64", candidates=None, profile=False, stream=None, delay=0,
               autotune=False, method="right", max_budget=0, noise_half_logdet=None, tile_order="auto",
               tune_cache=None, max_device_bytes=0, debug_fail_step=0, tile_size=0):
    """Create a handle for the device tensor K (2-D, float64/float32, row-major, lower triangle read).
    delay: downdate delay depth (0 automatic, 1..OED_MAX_DELAY); autotune: with delay 0, time the choices;
    method: "right" (downdate of all of R per pick), "left" (only the new block column per pick) or
    "auto" (left when max_budget <= half the candidates);
    max_budget: left-looking W history size (0: all candidates); noise_half_logdet: per-sensor
    1/2 logdet of the noise covariance blocks (None: isotropic sigma2); tile_order: the downdate's
    tile order ("auto", "row8", "col8", "col4", "col2"); tune_cache: autotuner cache file path;
    max_device_bytes: fail with OED_E_OOM instead of holding more (0: no limit); debug_fail_step:
    make that pick fail once (error-path tests); tile_size: downdate tile 128 or 256 (0: automatic).
    K = None: deferred packing (OED_FLAG_DEFER_PACK), the rows come through oed_pack_rows."""
    import torch
    L = library()
    if K is None:
        dtype, ld, kp = OED_F64, int(N_s) * int(N_t), None
    else:
        if not isinstance(K, torch.Tensor) or not K.is_cuda or K.dim() != 2 or K.stride(1) != 1:
            raise ValueError("K must be a 2-D row-major device tensor")
        dtype = {torch.float64: OED_F64, torch.float32: OED_F32}.get(K.dtype)
        if dtype is None:
            raise ValueError("K must be float64 or float32")
        if K.shape[0] < N_s * N_t or K.shape[1] < N_s * N_t:
            raise ValueError("K must have at least N_s*N_t rows and columns")
        ld, kp = K.stride(0), ctypes.c_void_p(K.data_ptr())
    opt = oed_options()
    L.oed_options_init(ctypes.byref(opt))
    opt.precision = PRECISIONS[precision]
    opt.flags = ((OED_FLAG_PROFILE if profile else 0) | (OED_FLAG_AUTOTUNE if autotune else 0) |
                 (OED_FLAG_DEFER_PACK if K is None else 0))
    opt.delay = int(delay)
    opt.method = {"right": 0, "left": 1, "auto": 2}[method]
    opt.max_budget = int(max_budget)
    opt.tile_order = TILE_ORDERS[tile_order]
    cache = None
    if tune_cache is not None:
        cache = os.fsencode(os.fspath(tune_cache))
        opt.tune_cache = cache
    opt.max_device_bytes = int(max_device_bytes)
    opt.debug_fail_step = int(debug_fail_step)
    opt.tile_size = int(tile_size)
    hld = None
    if noise_half_logdet is not None:
        hld = np.ascontiguousarray(np.asarray(noise_half_logdet, dtype=np.float64))
        if hld.shape != (int(N_s),):
            raise ValueError("noise_half_logdet needs one entry per sensor")
        opt.noise_half_logdet = _dp(hld)
    cand = None
    if candidates is not None:
        cand = np.ascontiguousarray(np.asarray(list(candidates), dtype=np.int32))
        opt.candidates = _ip(cand)
        opt.n_candidates = len(cand)
    h = ctypes.c_void_p()
    st = L.oed_create(ctypes.byref(h), kp, dtype, ld, int(N_s), int(N_t), float(sigma2), _stream_handle(stream),
                      ctypes.byref(opt))
    if st != OED_OK:
        raise OedError(st, L.oed_last_error(None).decode())
    # what oed_reset must be given again: the C side reuses the dtype and leading dimension of K
    _K_SIG[h.value] = None if K is None else _k_signature(K)
    return h


_K_SIG = {}


def _k_signature(K):
    return (K.dtype, K.stride(0), K.stride(1), tuple(K.shape), K.device)


def oed_reset(h, K):
    """K = None: a deferred-packing handle forgets its picks and its packed rows.  Otherwise K must be a
    device tensor of the dtype, strides, shape and device the handle was created with."""
    import torch
    if K is not None:
        if not isinstance(K, torch.Tensor) or not K.is_cuda:
            raise ValueError("K must be a device tensor")
        want = _K_SIG.get(h.value if isinstance(h, ctypes.c_void_p) else h)
        if want is not None and _k_signature(K) != want:
            raise ValueError(f"K (dtype, strides, shape, device) {_k_signature(K)} differs from creation {want}")
    _check(h, library().oed_reset(h, None if K is None else ctypes.c_void_p(K.data_ptr())))


def oed_pack_rows(h, K_rows, sensor0, n_sensors, N_t):
    """Pack the block rows of sensors sensor0 .. sensor0+n_sensors-1 from the device tensor K_rows
    (their rows of K, at least (sensor0+n_sensors)*N_t columns, row-major)."""
    import torch
    if not isinstance(K_rows, torch.Tensor) or not K_rows.is_cuda or K_rows.dim() != 2 or K_rows.stride(1) != 1:
        raise ValueError("K_rows must be a 2-D row-major device tensor")
    dtype = {torch.float64: OED_F64, torch.float32: OED_F32}.get(K_rows.dtype)
    if dtype is None:
        raise ValueError("K_rows must be float64 or float32")
    if K_rows.shape[0] < n_sensors * N_t or K_rows.shape[1] < (sensor0 + n_sensors) * N_t:
        raise ValueError("K_rows is smaller than the panel")
    _check(h, library().oed_pack_rows(h, ctypes.c_void_p(K_rows.data_ptr()), dtype, K_rows.stride(0),
                                      int(sensor0), int(n_sensors)))


def oed_greedy(h, budget, check=True):
    idx = np.full(max(budget, 1), -1, dtype=np.int32)
    gain = np.full(max(budget, 1), np.nan)
    n = ctypes.c_int32()
    st = library().oed_greedy(h, int(budget), _ip(idx), _dp(gain), ctypes.byref(n))
    if check:
        _check(h, st)
    return idx[:n.value].copy(), gain[:n.value].copy(), st


def oed_force(h, idx):
    g = ctypes.c_double()
    _check(h, library().oed_force(h, int(idx), ctypes.byref(g)))
    return g.value


def oed_scores(h, N_s):
    out = np.empty(N_s)
    _check(h, library().oed_scores(h, _dp(out)))
    return out


def oed_schur_block(h, i, j, N_t):
    out = np.empty((N_t, N_t))
    _check(h, library().oed_schur_block(h, int(i), int(j), _dp(out)))
    return out


def oed_picks(h, N_s):
    idx = np.empty(N_s, dtype=np.int32)
    gain = np.empty(N_s)
    n = ctypes.c_int32()
    _check(h, library().oed_picks(h, _ip(idx), _dp(gain), ctypes.byref(n)))
    return idx[:n.value].copy(), gain[:n.value].copy()


def oed_get_profile(h, reset=False):
    p = oed_profile()
    _check(h, library().oed_get_profile(h, ctypes.byref(p), 1 if reset else 0))
    return {"ms": {k: p.ms[i] for i, k in enumerate(KERNELS)},
            "launches": {k: int(p.launches[i]) for i, k in enumerate(KERNELS)},
            "syrk_flops": p.syrk_flops, "syrk_bytes": p.syrk_bytes}


def oed_device_bytes(h):
    b = ctypes.c_int64()
    _check(h, library().oed_device_bytes(h, ctypes.byref(b)))
    return b.value


def oed_get_config(h):
    """(delay, syrk_variant, autotuner per-pick ms for delay 1..OED_MAX_DELAY, tile order name)."""
    dl, var, to = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ms = np.zeros(OED_MAX_DELAY)
    _check(h, library().oed_get_config(h, ctypes.byref(dl), ctypes.byref(var), ctypes.byref(to), _dp(ms)))
    names = {v: k for k, v in TILE_ORDERS.items()}
    return dl.value, var.value, ms, names.get(to.value, str(to.value))


def oed_destroy(h):
    if h:
        _K_SIG.pop(h.value if isinstance(h, ctypes.c_void_p) else h, None)
        library().oed_destroy(h)


def oed_greedy_noalloc(K, N_s, N_t, sigma2, budget, idx_out, gain_out, status_out, precision="fp64", delay=0,
                       stream=None):
    """One whole selection without allocating (the library's static scratch array): K, idx_out (int32,
    length >= budget), gain_out (float64, length >= budget) and status_out (int32, length >= 2) are
    caller-owned device tensors.  Enqueued on the stream; returns without synchronising."""
    import torch
    if not isinstance(K, torch.Tensor) or not K.is_cuda or K.dim() != 2 or K.stride(1) != 1:
        raise ValueError("K must be a 2-D row-major device tensor")
    dtype = {torch.float64: OED_F64, torch.float32: OED_F32}.get(K.dtype)
    if dtype is None:
        raise ValueError("K must be float64 or float32")
    if K.shape[0] < N_s * N_t or K.shape[1] < N_s * N_t:
        raise ValueError("K must have at least N_s*N_t rows and columns")
    for t, dt, n in ((idx_out, torch.int32, budget), (gain_out, torch.float64, budget), (status_out, torch.int32, 2)):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous() or t.numel() < n:
            raise ValueError("outputs must be contiguous device tensors: idx int32, gain float64 (budget each), "
                             "status int32 (2)")
    err = ctypes.create_string_buffer(512)
    st = library().oed_greedy_noalloc(ctypes.c_void_p(K.data_ptr()), dtype, K.stride(0), int(N_s), int(N_t),
                                      float(sigma2), PRECISIONS[precision], int(delay), int(budget),
                                      _stream_handle(stream), ctypes.c_void_p(idx_out.data_ptr()),
                                      ctypes.c_void_p(gain_out.data_ptr()), ctypes.c_void_p(status_out.data_ptr()),
                                      err, len(err))
    if st != OED_OK:
        raise OedError(st, err.value.decode())


def _instances(items):
    """items: sequence of (K tensor, N_s, N_t, sigma2, budget)."""
    import torch
    arr = (oed_instance * len(items))()
    for q, (K, N_s, N_t, sigma2, budget) in enumerate(items):
        if not isinstance(K, torch.Tensor) or not K.is_cuda or K.dim() != 2 or K.stride(1) != 1:
            raise ValueError("K must be a 2-D row-major device tensor")
        if K.shape[0] < N_s * N_t or K.shape[1] < N_s * N_t:
            raise ValueError("K must have at least N_s*N_t rows and columns")
        dt = {torch.float64: OED_F64, torch.float32: OED_F32}.get(K.dtype)
        if dt is None:
            raise ValueError("K must be float64 or float32")
        arr[q] = oed_instance(K.data_ptr(), dt, int(N_s), int(N_t), int(budget), K.stride(0), float(sigma2))
    return arr


def _bcheck(b, st):
    if st != OED_OK:
        msg = library().oed_batch_last_error(b).decode() if b else ""
        raise OedError(st, msg)


def oed_batch_create(items, precision="fp64", profile=False, graph=True, stream=None, delay=0, autotune=False,
                     method="right", tile_order="auto", branches=0):
    arr = _instances(items)
    b = ctypes.c_void_p()
    flags = ((OED_FLAG_PROFILE if profile else 0) | (0 if graph else OED_BATCH_NO_GRAPH) | (int(delay) << 8) |
             (OED_BATCH_AUTOTUNE if autotune else 0) | (OED_BATCH_LEFT_LOOKING if method == "left" else 0) |
             (TILE_ORDERS[tile_order] << 12) | (int(branches) << 16))
    st = library().oed_batch_create(ctypes.byref(b), arr, len(items), PRECISIONS[precision], _stream_handle(stream),
                                    flags)
    _bcheck(None, st)
    return b


def oed_batch_run(b, budgets, check=True):
    tot = int(sum(budgets))
    idx = np.empty(max(tot, 1), dtype=np.int32)
    gain = np.empty(max(tot, 1))
    n = np.zeros(len(budgets), dtype=np.int32)
    status = np.zeros(len(budgets), dtype=np.int32)
    st = library().oed_batch_run(b, _ip(idx), _dp(gain), _ip(n), _ip(status))
    if check:
        _bcheck(b, st)
    out, o = [], 0
    for q, B in enumerate(budgets):
        out.append((idx[o:o + n[q]].copy(), gain[o:o + n[q]].copy(), int(status[q])))
        o += B
    return out, st


def oed_batch_reset(b, items):
    _bcheck(b, library().oed_batch_reset(b, _instances(items), len(items)))


def oed_batch_stats(b):
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _bcheck(b, library().oed_batch_stats(b, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)))
    return {"run_ms": ms.value, "syrk_flops": fl.value, "syrk_bytes": by.value}


def oed_batch_get_config(b):
    """(delay, autotuner run ms for delay 1..OED_MAX_DELAY, tile order name, launch sequences)."""
    dl, to, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ms = np.zeros(OED_MAX_DELAY)
    _bcheck(b, library().oed_batch_get_config(b, ctypes.byref(dl), ctypes.byref(to), ctypes.byref(nb), _dp(ms)))
    names = {v: k for k, v in TILE_ORDERS.items()}
    return dl.value, ms, names.get(to.value, str(to.value)), nb.value


def oed_batch_destroy(b):
    if b:
        library().oed_batch_destroy(b)


class BatchSelector:
    """Owns one batch.  ``BatchSelector([(K, N_s, N_t, sigma2, B), ...]).run()`` -> [(idx, gain, status)]."""

    def __init__(self, items, precision="fp64", profile=False, graph=True, stream=None, delay=0, autotune=False,
                 method="right", tile_order="auto", branches=0):
        self.budgets = [int(it[4]) for it in items]
        self.b = oed_batch_create(items, precision, profile, graph, stream, delay, autotune, method, tile_order,
                                  branches)

    def run(self, check=True):
        return oed_batch_run(self.b, self.budgets, check)[0]

    def reset(self, items):
        oed_batch_reset(self.b, items)

    def config(self):
        return oed_batch_get_config(self.b)

    def stats(self):
        return oed_batch_stats(self.b)

    def close(self):
        if self.b:
            oed_batch_destroy(self.b)
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _echeck(e, st):
    if st != OED_OK:
        msg = library().oed_eval_last_error(e).decode() if e else ""
        raise OedError(st, msg)


def oed_eval_create(K, N_s, N_t, sigma2, B, max_batch=0, precision="fp64", profile=False, graph=True, stream=None,
                    delay=0):
    import torch
    if not isinstance(K, torch.Tensor) or not K.is_cuda or K.dim() != 2 or K.stride(1) != 1:
        raise ValueError("K must be a 2-D row-major device tensor")
    if K.shape[0] < N_s * N_t or K.shape[1] < N_s * N_t:
        raise ValueError("K must have at least N_s*N_t rows and columns")
    dt = {torch.float64: OED_F64, torch.float32: OED_F32}.get(K.dtype)
    if dt is None:
        raise ValueError("K must be float64 or float32")
    e = ctypes.c_void_p()
    flags = (OED_FLAG_PROFILE if profile else 0) | (0 if graph else OED_BATCH_NO_GRAPH) | (int(delay) << 8)
    st = library().oed_eval_create(ctypes.byref(e), ctypes.c_void_p(K.data_ptr()), dt, K.stride(0), int(N_s),
                                   int(N_t), float(sigma2), int(B), int(max_batch), PRECISIONS[precision],
                                   _stream_handle(stream), flags)
    _echeck(None, st)
    return e


def oed_eval_run(e, designs, check=True):
    """designs: (n, B) int array.  Returns (objectives (n,), terms (n, B), status)."""
    d = np.ascontiguousarray(designs, dtype=np.int32)
    if d.ndim != 2:
        raise ValueError("designs must be a 2-D (n, B) array")
    n, B = d.shape
    obj = np.empty(max(n, 1))
    terms = np.empty((max(n, 1), B))
    st = library().oed_eval_run(e, _ip(d), n, _dp(obj), _dp(terms))
    if check:
        _echeck(e, st)
    return obj[:n].copy(), terms[:n].copy(), st


def oed_eval_stats(e):
    ms, fl = ctypes.c_double(), ctypes.c_double()
    ex, nb = ctypes.c_int64(), ctypes.c_int32()
    _echeck(e, library().oed_eval_stats(e, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(ex), ctypes.byref(nb)))
    return {"run_ms": ms.value, "syrk_flops": fl.value, "executed": ex.value, "batch": nb.value}


def oed_eval_destroy(e):
    if e:
        library().oed_eval_destroy(e)


class Evaluator:
    """Objective f(S) = 1/2 logdet(sigma^-2 K_SS) of given designs of B sensors:
    ``Evaluator(K, N_s, N_t, sigma2, B).run(designs)`` -> (objectives, per-block terms)."""

    def __init__(self, K, N_s, N_t, sigma2, B, max_batch=0, precision="fp64", profile=False, graph=True,
                 stream=None, delay=0):
        self.B = int(B)
        self.e = oed_eval_create(K, N_s, N_t, sigma2, B, max_batch, precision, profile, graph, stream, delay)

    def run(self, designs, check=True):
        obj, terms, _ = oed_eval_run(self.e, designs, check)
        return obj, terms

    def stats(self):
        return oed_eval_stats(self.e)

    def close(self):
        if self.e:
            oed_eval_destroy(self.e)
            self.e = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ convenience wrapper
class Selector:
    """Owns one handle.  ``Selector(K, N_s, N_t, sigma2).greedy(B)`` -> (indices, gains)."""

    def __init__(self, K, N_s, N_t, sigma2, precision="fp64", candidates=None, profile=False, stream=None,
                 delay=0, autotune=False, method="right", max_budget=0, noise_half_logdet=None, tile_order="auto",
                 tune_cache=None, max_device_bytes=0, debug_fail_step=0, tile_size=0):
        self.N_s, self.N_t = int(N_s), int(N_t)
        self.h = oed_create(K, N_s, N_t, sigma2, precision, candidates, profile, stream, delay, autotune, method,
                            max_budget, noise_half_logdet, tile_order, tune_cache, max_device_bytes,
                            debug_fail_step, tile_size)

    def greedy(self, budget):
        idx, gain, _ = oed_greedy(self.h, budget)
        return idx, gain

    def pack_rows(self, K_rows, sensor0, n_sensors):
        oed_pack_rows(self.h, K_rows, sensor0, n_sensors, self.N_t)

    def greedy_status(self, budget):
        return oed_greedy(self.h, budget, check=False)

    def force(self, idx):
        return oed_force(self.h, idx)

    def scores(self):
        return oed_scores(self.h, self.N_s)

    def schur_block(self, i, j):
        return oed_schur_block(self.h, i, j, self.N_t)

    def picks(self):
        return oed_picks(self.h, self.N_s)

    def reset(self, K):
        oed_reset(self.h, K)

    def profile(self, reset=False):
        return oed_get_profile(self.h, reset)

    def device_bytes(self):
        return oed_device_bytes(self.h)

    def config(self):
        return oed_get_config(self.h)

    def close(self):
        if self.h:
            oed_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
