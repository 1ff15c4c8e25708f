"""The seeded synthetic-input recipe (host only)."""
import numpy as np
import torch

from oed_inputs import CONFIGS, batched_instance_specs, f_tile, make_K, make_K_lower_panels, tile_seed


def test_K_recipe_properties():
    K, s2 = make_K(12, 4, 300, seed=3)
    K = K.numpy()
    assert K.shape == (48, 48)
    np.testing.assert_allclose(K, K.T, rtol=0, atol=1e-15)
    G = K - s2 * np.eye(48)
    np.testing.assert_allclose(s2, 0.01 * np.mean(np.diag(G)), rtol=1e-12)
    assert np.linalg.eigvalsh(K).min() >= 0.99 * s2


def test_deterministic_and_seed_dependent():
    a, sa = make_K(6, 3, 100, seed=1)
    b, sb = make_K(6, 3, 100, seed=1)
    c, _ = make_K(6, 3, 100, seed=2)
    assert torch.equal(a, b) and sa == sb
    assert not torch.equal(a, c)
    assert len({tile_seed(0, r, c) for r in range(20) for c in range(20)}) == 400


def test_column_scaling():
    x = f_tile(5, 0, 1, 2000, 64)   # columns 4096..4159
    s = x.std(0).numpy()
    expect = (1.0 + np.arange(4096, 4160)) ** -0.25
    np.testing.assert_allclose(s, expect, rtol=0.1)


def test_lower_panel_builder_matches_full_on_lower_triangle():
    full, s_full = make_K(10, 5, 333, seed=4)
    low, s_low = make_K_lower_panels(10, 5, 333, seed=4, device="cpu", panel=16)
    tri = torch.tril(torch.ones(50, 50, dtype=torch.bool))
    torch.testing.assert_close(low[tri], full[tri], rtol=1e-13, atol=1e-15)
    assert abs(s_full - s_low) <= 1e-15 * s_full


def test_config_table():
    assert CONFIGS["small_fp64_64x16"].N_d == 1024
    assert CONFIGS["mixed_600x128"].N_d == 76800
    specs = batched_instance_specs()
    assert len(specs) == 48
    for s in specs:
        assert 40 <= s.N_s <= 400 and s.N_t in (16, 32, 64)
        assert 1e-3 <= s.c <= 1e-1 and s.budget == s.N_s // 4 and s.n_m == 2 * s.N_d
    assert specs == batched_instance_specs()


def test_row_panels_are_the_lower_block_triangle_of_K():
    """k_row_panels (K formed by row panels from a resident F) gives exactly the rows and
    columns of K = F F^T / n_m + sigma^2 I that the panel covers, and f_matrix draws the F of
    make_K (same seed, same noise scale)."""
    import torch
    from oed_inputs import f_matrix, k_row_panels
    N_s, N_t, n_m = 7, 5, 300
    F, scale = f_matrix(N_s * N_t, n_m, 4, device="cpu", dtype=torch.float64)
    K = F @ F.t() / n_m
    assert abs(scale - K.diagonal().mean().item()) < 1e-12
    s2 = 0.01 * scale
    K.diagonal().add_(s2)
    seen = []
    for s0, n, P in k_row_panels(F, N_s, N_t, s2, 3):
        r0, r1 = s0 * N_t, (s0 + n) * N_t
        assert P.shape == (r1 - r0, r1)
        assert torch.allclose(P, K[r0:r1, :r1], rtol=0, atol=1e-13)
        seen.append((s0, n))
    assert seen == [(0, 3), (3, 3), (6, 1)]
    Kref, s2ref = make_K(N_s, N_t, n_m, seed=4)
    assert torch.allclose(Kref, K, rtol=0, atol=1e-12) and abs(s2ref - s2) <= 1e-14 * s2


def test_weighted_time_correlated_noise_recipe():
    """K = F F^T / n_m + blockdiag(w_j gamma^2 rho_j^|t-u|): the signal part is make_K's (same F),
    each noise block is a scaled AR(1) correlation (positive definite, Toeplitz, lag-1 ratio rho_j),
    weights and correlations in their ranges, nothing between sensors."""
    from oed_inputs import make_K_weighted_noise
    N_s, N_t, n_m, seed = 7, 5, 200, 9
    K, blocks = make_K_weighted_noise(N_s, N_t, n_m, seed, w_lo=2.0, w_hi=40.0, rho_max=0.7)
    K = K.numpy()
    K0, s2 = make_K(N_s, N_t, n_m, seed)
    G = K0.numpy() - s2 * np.eye(N_s * N_t)      # F F^T / n_m of the same F
    gamma2 = 0.01 * float(np.mean(np.diag(G)))
    D = K - G
    for j in range(N_s):
        for i in range(N_s):
            blk = D[i * N_t:(i + 1) * N_t, j * N_t:(j + 1) * N_t]
            if i != j:
                assert np.abs(blk).max() <= 1e-14
        B = blocks[j]
        np.testing.assert_allclose(D[j * N_t:(j + 1) * N_t, j * N_t:(j + 1) * N_t], B, rtol=1e-12, atol=1e-16)
        w = B[0, 0] / gamma2
        rho = B[0, 1] / B[0, 0]
        assert 2.0 <= w <= 40.0 and 0.0 <= rho < 0.7
        lag = np.abs(np.subtract.outer(np.arange(N_t), np.arange(N_t)))
        np.testing.assert_allclose(B, w * gamma2 * rho ** lag, rtol=1e-12)
        assert np.linalg.eigvalsh(B).min() > 0
