"""GPU parity of deferred packing (the working copy filled block row by block row from panels of
K's rows, for K too large to be resident beside it): the selection must be bit-for-bit the one of
the same handle created from the whole K, for every precision and method, with candidate subsets,
uneven panels and N_t > 128; steps before every candidate row is packed are refused."""
import numpy as np
import pytest
import torch

from oed_inputs import make_K

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def pack_panels(sel, K, N_s, N_t, sizes):
    s0, q = 0, 0
    while s0 < N_s:
        n = min(sizes[q % len(sizes)], N_s - s0)
        # a view of K's rows: leading dimension N_d, columns up to the panel's end are read
        sel.pack_rows(K[s0 * N_t:(s0 + n) * N_t], s0, n)
        s0 += n
        q += 1


@pytest.mark.parametrize("prec", ["fp64", "mixed_f32", "mixed_bf16x3"])
@pytest.mark.parametrize("method", ["right", "left"])
def test_deferred_equals_whole_K(prec, method):
    from paper_2604_08812_amd import Selector
    N_s, N_t, B = 23, 24, 9
    K, s2 = make_K(N_s, N_t, 900, 501)
    Kd = K.to(DEV)
    cand = [q for q in range(N_s) if q % 5 != 2]
    with Selector(Kd, N_s, N_t, s2, precision=prec, method=method, candidates=cand) as a:
        i_a, g_a = a.greedy(B)
    with Selector(None, N_s, N_t, s2, precision=prec, method=method, candidates=cand) as b:
        pack_panels(b, Kd, N_s, N_t, [4, 1, 7])
        i_b, g_b = b.greedy(B)
        # reset forgets the rows; packing them again (other panel sizes, FP32 rows for FP32 paths
        # would change K, so the same FP64 rows) reproduces the selection
        b.reset(None)
        pack_panels(b, Kd, N_s, N_t, [N_s])
        i_c, g_c = b.greedy(B)
    assert list(i_a) == list(i_b) == list(i_c)
    assert np.array_equal(g_a, g_b) and np.array_equal(g_a, g_c)


def test_deferred_large_block_and_refusals():
    from paper_2604_08812_amd import OedError, Selector
    N_s, N_t, B = 7, 160, 4  # N_t > 128: factorisations in global scratch, no delay
    K, s2 = make_K(N_s, N_t, 2000, 502)
    Kd = K.to(DEV)
    with Selector(Kd, N_s, N_t, s2, precision="mixed_f32") as a:
        i_a, g_a = a.greedy(B)
    with Selector(None, N_s, N_t, s2, precision="mixed_f32") as b:
        b.pack_rows(Kd[0:3 * N_t], 0, 3)
        with pytest.raises(OedError):  # rows of sensors 3..6 missing
            b.greedy(1)
        with pytest.raises(OedError):
            b.scores()
        b.pack_rows(Kd[3 * N_t:], 3, 4)
        i_b, g_b = b.greedy(B)
        with pytest.raises(OedError):  # no packing once picks are made
            b.pack_rows(Kd[0:N_t], 0, 1)
        with pytest.raises(OedError):  # a deferred handle resets without K
            b.reset(Kd)
    assert list(i_a) == list(i_b) and np.array_equal(g_a, g_b)
