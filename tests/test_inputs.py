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
