"""Synthetic data-space matrices shaped like the paper's sensor-selection workload.

Recipe (the same for every size):

* ``N_d = N_s * N_t`` rows, sensor-major: row ``i*N_t + t`` is observation ``t``
  of sensor ``i`` (the block structure of K used in Sec. III-B/III-C, where K_S
  is the block-row/block-column subsample of K for the sensors in S).
* ``F`` is ``N_d x n_m``.  It is built from tiles of ``TILE x TILE`` standard
  normal draws; tile ``(rb, cb)`` is drawn by ``torch.randn`` from a
  ``torch.Generator`` on the forming device seeded with ``tile_seed(seed, rb, cb)``.
  Column ``m`` (0-based) is then scaled by ``(1 + m) ** -0.25`` so that the
  spectrum of ``F F^T`` decays.
* ``K = F F^T / n_m + sigma^2 I`` with
  ``sigma^2 = c * mean(diag(F F^T / n_m))`` (``c = 0.01`` unless stated),
  computed in FP64.  This is ``K = Gamma_noise + F Gamma_prior F^*`` with an
  identity prior covariance and isotropic noise (Sec. II-B and eq. for the
  isotropic-noise objective).

The random stream depends on the device type that forms K (torch's CPU and GPU
generators differ), so an instance is identified by (recipe, seed, device
type).  Parity never depends on it: every check hands the *same* K bits to the
oracle and to the HIP path.
"""
from __future__ import annotations

import math

import torch

TILE = 4096


def tile_seed(seed: int, rb: int, cb: int) -> int:
    """Seed of tile (rb, cb) of F for instance seed ``seed`` (63-bit mix)."""
    x = (seed * 0x9E3779B97F4A7C15 + rb * 0xBF58476D1CE4E5B9 + cb * 0x94D049BB133111EB + 1) & ((1 << 64) - 1)
    x ^= x >> 31
    x = (x * 0xD6E8FEB86659FD93) & ((1 << 64) - 1)
    x ^= x >> 32
    return x & ((1 << 63) - 1)


def f_tile(seed: int, rb: int, cb: int, rows: int, cols: int, device="cpu") -> torch.Tensor:
    """FP64 tile (rb, cb) of F, ``rows x cols`` (ragged at the edges), column-scaled."""
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(tile_seed(seed, rb, cb))
    x = torch.randn((rows, cols), generator=g, device=dev, dtype=torch.float64)
    m0 = cb * TILE
    scale = (1.0 + torch.arange(m0, m0 + cols, device=dev, dtype=torch.float64)) ** -0.25
    x *= scale
    return x


def f_column_chunk(seed: int, N_d: int, n_m: int, cb: int, device="cpu") -> torch.Tensor:
    """All rows of F for column tile ``cb``: an ``N_d x w`` FP64 tensor."""
    c0 = cb * TILE
    w = min(TILE, n_m - c0)
    parts = []
    for rb in range(math.ceil(N_d / TILE)):
        r0 = rb * TILE
        parts.append(f_tile(seed, rb, cb, min(TILE, N_d - r0), w, device))
    return torch.cat(parts, 0) if len(parts) > 1 else parts[0]


def make_K(N_s: int, N_t: int, n_m: int, seed: int, c: float = 0.01, device="cpu",
           dtype=torch.float64):
    """Form K (full symmetric, ``N_d x N_d``) and sigma^2 for a small instance.

    Accumulates ``F_c F_c^T`` over column tiles in FP64, then adds sigma^2 I.
    Returns ``(K, sigma2)``; K has dtype ``dtype`` on ``device``.
    """
    N_d = N_s * N_t
    G = torch.zeros((N_d, N_d), dtype=torch.float64, device=device)
    for cb in range(math.ceil(n_m / TILE)):
        Fc = f_column_chunk(seed, N_d, n_m, cb, device)
        G.addmm_(Fc, Fc.t())
    G /= n_m
    sigma2 = float(c * G.diagonal().mean().item())
    G.diagonal().add_(sigma2)
    return G.to(dtype), sigma2


def make_K_sensor_noise(N_s: int, N_t: int, n_m: int, seed: int, c_lo: float = 1e-3, c_hi: float = 1e-1,
                        device="cpu", dtype=torch.float64):
    """K = F F^T / n_m + diag(sigma_j^2) with a noise variance per sensor (independent,
    uncorrelated noise of uneven instruments): sigma_j^2 = c_j mean diag(F F^T / n_m), c_j
    log-uniform in [c_lo, c_hi] from ``numpy.random.default_rng(seed)``.  Returns
    ``(K, sigma2_per_sensor)`` (the latter a numpy array of length N_s).
    """
    import numpy as np
    N_d = N_s * N_t
    G = torch.zeros((N_d, N_d), dtype=torch.float64, device=device)
    for cb in range(math.ceil(n_m / TILE)):
        Fc = f_column_chunk(seed, N_d, n_m, cb, device)
        G.addmm_(Fc, Fc.t())
    G /= n_m
    scale = float(G.diagonal().mean().item())
    c = 10.0 ** np.random.default_rng(seed).uniform(np.log10(c_lo), np.log10(c_hi), N_s)
    var = scale * c
    G.diagonal().add_(torch.from_numpy(np.repeat(var, N_t)).to(device))
    return G.to(dtype), var


def make_K_weighted_noise(N_s: int, N_t: int, n_m: int, seed: int, c: float = 0.01, rho_max: float = 0.8,
                          w_lo: float = 1.0, w_hi: float = 30.0, device="cpu", dtype=torch.float64):
    """K = F F^T / n_m + W_c Gamma_noise with noise correlated in time within each sensor and a
    placement-cost weight per sensor (the weighted noise covariance of Sec. III-G, with a diagonal
    W_c): sensor j's noise block is ``w_j gamma^2 rho_j^|t-u|`` (a stationary AR(1) correlation of
    its N_t samples), ``gamma^2 = c mean diag(F F^T / n_m)``; ``rho_j`` uniform in [0, rho_max) and
    ``w_j`` log-uniform in [w_lo, w_hi] from ``numpy.random.default_rng(seed)``.  Sensors' noises
    are independent of each other, so W_c Gamma_noise is block-diagonal.  Returns
    ``(K, blocks)`` with ``blocks`` the FP64 noise blocks as a numpy array (N_s, N_t, N_t).
    """
    import numpy as np
    N_d = N_s * N_t
    G = torch.zeros((N_d, N_d), dtype=torch.float64, device=device)
    for cb in range(math.ceil(n_m / TILE)):
        Fc = f_column_chunk(seed, N_d, n_m, cb, device)
        G.addmm_(Fc, Fc.t())
    G /= n_m
    gamma2 = c * float(G.diagonal().mean().item())
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.0, rho_max, N_s)
    w = 10.0 ** rng.uniform(np.log10(w_lo), np.log10(w_hi), N_s)
    lag = np.abs(np.subtract.outer(np.arange(N_t), np.arange(N_t)))
    blocks = np.stack([w[j] * gamma2 * rho[j] ** lag for j in range(N_s)])
    for j in range(N_s):
        G[j * N_t:(j + 1) * N_t, j * N_t:(j + 1) * N_t] += torch.from_numpy(blocks[j]).to(device)
    return G.to(dtype), blocks


def make_K_lower_panels(N_s: int, N_t: int, n_m: int, seed: int, c: float = 0.01,
                        device="cuda", dtype=torch.float64, panel: int = 12800,
                        progress=None):
    """Form a large K on ``device`` with only its lower block-panels computed.

    Row panels of ``panel`` rows: panel p receives ``F_p F_{0..p}^T`` (columns up
    to the end of panel p), so the lower triangle (and the diagonal panel blocks
    in full) is valid; the strict upper part beyond the diagonal panels stays 0.
    The GEMMs run in ``dtype`` (FP64 for FP64 instances, FP32 for the large FP32
    instance).  sigma^2 is taken from the FP64 sum of the diagonal.
    Returns ``(K, sigma2)``.
    """
    N_d = N_s * N_t
    K = torch.zeros((N_d, N_d), dtype=dtype, device=device)
    n_cb = math.ceil(n_m / TILE)
    for cb in range(n_cb):
        Fc = f_column_chunk(seed, N_d, n_m, cb, device).to(dtype)
        for r0 in range(0, N_d, panel):
            r1 = min(N_d, r0 + panel)
            K[r0:r1, :r1].addmm_(Fc[r0:r1], Fc[:r1].t(), alpha=1.0 / n_m)
        del Fc
        if progress is not None:
            progress(cb + 1, n_cb)
    d = K.diagonal()
    sigma2 = float(c * d.to(torch.float64).mean().item())
    d.add_(sigma2)
    return K, sigma2


def f_matrix(N_d: int, n_m: int, seed: int, device="cuda", dtype=torch.float32, progress=None):
    """F itself (``N_d x n_m``), drawn by column tile in FP64 as above and stored in ``dtype``, with
    the FP64 mean of ``diag(F F^T) / n_m`` taken from the FP64 draws (the noise scale).
    Returns ``(F, scale)``; ``sigma^2 = c * scale``.  For K too large to be formed whole: its row
    panels come from ``k_row_panels``."""
    F = torch.empty((N_d, n_m), dtype=dtype, device=device)
    sq = torch.zeros(N_d, dtype=torch.float64, device=device)
    n_cb = math.ceil(n_m / TILE)
    for cb in range(n_cb):
        Fc = f_column_chunk(seed, N_d, n_m, cb, device)
        sq += (Fc * Fc).sum(1)
        F[:, cb * TILE:cb * TILE + Fc.shape[1]] = Fc.to(dtype)
        del Fc
        if progress is not None:
            progress(cb + 1, n_cb)
    return F, float(sq.mean().item()) / n_m


def k_row_panels(F: torch.Tensor, N_s: int, N_t: int, sigma2: float, panel_sensors: int):
    """Row panels of ``K = F F^T / n_m + sigma^2 I`` in F's dtype, one GEMM each: yields
    ``(sensor0, n, P)`` with ``P`` = rows ``sensor0*N_t .. (sensor0+n)*N_t - 1`` of K and its
    columns ``0 .. (sensor0+n)*N_t - 1`` (the panel's lower block triangle and diagonal blocks).
    Each panel is a new tensor; drop it before taking the next to keep one in memory."""
    n_m = F.shape[1]
    for s0 in range(0, N_s, panel_sensors):
        n = min(panel_sensors, N_s - s0)
        r0, r1 = s0 * N_t, (s0 + n) * N_t
        P = torch.matmul(F[r0:r1], F[:r1].t())
        P.mul_(1.0 / n_m)
        P[:, r0:r1].diagonal().add_(sigma2)
        yield s0, n, P
        del P


def k_sub_lower(K: torch.Tensor, N_t: int, sensors) -> "numpy.ndarray":
    """Dense FP64 host copy of the block sub-matrix of K for the ordered sensor list,
    every element taken from K's lower triangle (K may live on the GPU)."""
    idx = torch.as_tensor([int(s) * N_t + t for s in sensors for t in range(N_t)], device=K.device)
    sub = K.index_select(0, idx).index_select(1, idx)
    low = idx[:, None] >= idx[None, :]
    # element (a, b) with idx[a] < idx[b] lies in K's upper triangle: take (b, a) instead
    return torch.where(low, sub, sub.t()).to(torch.float64).cpu().numpy()
