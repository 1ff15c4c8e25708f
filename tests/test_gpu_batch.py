"""GPU parity of the batched selection (many uneven designs in one graph launch).

Each instance of the batch must give exactly the picks and gains of the same instance
selected alone through oed_create/oed_greedy (same kernels, same tiles), and both must match
the oracle within the precision's tolerance.  Graph replays are checked against the eager run.
"""
import numpy as np
import pytest
import torch

from oed_inputs import make_K
from parity import RTOL, check_trajectory

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# (N_s, N_t, n_m, seed, c, budget): uneven sizes, block sizes 16/32/64/24/128, full budgets
SPECS = [(21, 16, 600, 201, 0.01, 5), (13, 32, 800, 202, 0.05, 13), (30, 64, 4000, 203, 0.002, 7),
         (17, 24, 900, 204, 0.03, 4), (9, 128, 2000, 205, 0.01, 3), (40, 16, 1500, 206, 0.001, 10),
         (11, 48, 1000, 207, 0.02, 11)]


@pytest.fixture(scope="module")
def insts():
    out = []
    for (N_s, N_t, n_m, seed, c, B) in SPECS:
        K, s2 = make_K(N_s, N_t, n_m, seed, c)
        out.append((K.numpy(), K.to(DEV), N_s, N_t, s2, B))
    return out


def items(insts, dtype=torch.float64):
    return [(Kd.to(dtype), N_s, N_t, s2, B) for (_, Kd, N_s, N_t, s2, B) in insts]


@pytest.mark.parametrize("delay", [1, 2, 4, 8])
@pytest.mark.parametrize("prec", ["fp64", "mixed_f32", "mixed_bf16x3"])
def test_batch_equals_single_and_oracle(insts, prec, delay):
    from paper_2604_08812_amd import BatchSelector, Selector
    with BatchSelector(items(insts), precision=prec, delay=delay) as bs:
        res = bs.run()
    for q, (K, Kd, N_s, N_t, s2, B) in enumerate(insts):
        idx, gain, st = res[q]
        assert st == 0 and len(idx) == B
        with Selector(Kd, N_s, N_t, s2, precision=prec, delay=delay) as sel:
            i1, g1 = sel.greedy(B)
        assert list(idx) == list(i1), q
        np.testing.assert_array_equal(gain, g1)
        check_trajectory(K, N_s, N_t, s2, idx, gain, RTOL[prec])


def test_graph_replays_match_eager(insts):
    from paper_2604_08812_amd import BatchSelector, OedError
    its = items(insts)
    with BatchSelector(its, precision="mixed_f32", graph=False) as eager:
        ref = eager.run()
    with BatchSelector(its, precision="mixed_f32", profile=True) as bs:
        for rep in range(3):
            res = bs.run()
            for (i0, g0, s0), (i1, g1, s1) in zip(ref, res):
                assert list(i0) == list(i1) and s0 == s1 == 0
                np.testing.assert_array_equal(g0, g1)
            with pytest.raises(OedError):
                bs.run()                      # already ran: needs a reset
            torch.cuda.synchronize()
            _ = torch.ones(1000, device=DEV).sum().item()   # eager work between replays
            bs.reset(its)
        st = bs.stats()
        assert st["run_ms"] > 0 and st["syrk_flops"] > 0


def test_batch_non_pd_instance_stops_alone(insts):
    from paper_2604_08812_amd import BatchSelector
    N_s, N_t = 8, 16
    K, s2 = make_K(N_s, N_t, 300, 301)
    K = K.clone()
    K[3 * N_t:4 * N_t, :] = 0.0
    K[:, 3 * N_t:4 * N_t] = 0.0
    its = items(insts[:2]) + [(K.to(DEV), N_s, N_t, s2, N_s)]
    with BatchSelector(its, precision="fp64") as bs:
        res = bs.run(check=False)
    assert res[0][2] == 0 and res[1][2] == 0
    idx, gain, st = res[2]
    assert st == 2 and len(idx) == N_s - 1 and 3 not in set(idx.tolist())


def test_batch_autotune(insts):
    from paper_2604_08812_amd import BatchSelector
    its = items(insts)
    with BatchSelector(its, precision="mixed_f32", autotune=True) as t:
        delay, ms, _, _ = t.config()
        res = t.run()
    assert np.all(ms > 0) and delay == int(np.argmin(ms)) + 1
    with BatchSelector(its, precision="mixed_f32", delay=delay) as f:
        ref = f.run()
    for (i0, g0, s0), (i1, g1, s1) in zip(ref, res):
        assert list(i0) == list(i1) and s0 == s1 == 0
        np.testing.assert_array_equal(g0, g1)


@pytest.mark.parametrize("prec", ["fp64", "mixed_f32", "mixed_bf16x3"])
def test_batch_left_looking(insts, prec):
    """Batched left-looking: each instance bitwise equal to a left-looking handle of its own, and
    to the oracle within tolerance; graph replays equal."""
    from paper_2604_08812_amd import BatchSelector, Selector
    its = items(insts)
    with BatchSelector(its, precision=prec, method="left") as bs:
        res = bs.run()
        bs.reset(its)
        res2 = bs.run()
    for q, (K, Kd, N_s, N_t, s2, B) in enumerate(insts):
        idx, gain, st = res[q]
        assert st == 0 and len(idx) == B
        assert list(idx) == list(res2[q][0])
        np.testing.assert_array_equal(gain, res2[q][1])
        with Selector(Kd, N_s, N_t, s2, precision=prec, method="left", max_budget=B) as sel:
            i1, g1 = sel.greedy(B)
        assert list(idx) == list(i1), q
        np.testing.assert_array_equal(gain, g1)
        check_trajectory(K, N_s, N_t, s2, idx, gain, RTOL[prec])


def test_batch_reset_is_ordered_after_the_caller_stream(insts):
    """K rewritten on the creation (torch) stream, behind a long matrix product, and oed_batch_reset
    called at once with no host synchronisation: the pack must see the rewritten K."""
    from paper_2604_08812_amd import BatchSelector
    alt = []
    for (N_s, N_t, n_m, seed, c, B) in SPECS:
        K, s2 = make_K(N_s, N_t, n_m, seed + 1000, c)
        alt.append((K.to(DEV), N_s, N_t, s2, B))
    with BatchSelector(alt, precision="mixed_f32") as ref_bs:
        ref = ref_bs.run()
    # working buffers that start as the original K and are overwritten with the alternative ones
    work = [(Kd.clone(), N_s, N_t, s2a, B) for (_, Kd, N_s, N_t, _, B), (_, _, _, s2a, _) in zip(insts, alt)]
    with BatchSelector(work, precision="mixed_f32") as bs:
        bs.run()
        a = torch.randn(8192, 8192, device=DEV)
        torch.cuda.synchronize()
        for _ in range(6):
            a = a @ a
            a = a / a.norm()
        for (Kw, *_), (Ka, *_) in zip(work, alt):
            Kw.copy_(Ka)
        bs.reset(work)
        res = bs.run()
    for (i0, g0, s0), (i1, g1, s1) in zip(ref, res):
        assert s0 == s1 == 0 and list(i0) == list(i1)
        np.testing.assert_array_equal(g0, g1)


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("method", ["right", "left"])
def test_branches_give_the_same_selection(insts, method, graph):
    """Splitting the batch into concurrent launch sequences (forked streams, parallel graph branches)
    changes nothing: every branch count gives bitwise the picks and gains of one sequence, on
    repeated runs."""
    from paper_2604_08812_amd import BatchSelector
    its = items(insts, torch.float32)
    with BatchSelector(its, precision="mixed_f32", method=method, branches=1) as one:
        ref = one.run()
    for nb in (2, 3, 4):
        with BatchSelector(its, precision="mixed_f32", method=method, branches=nb, graph=graph) as bs:
            assert bs.config()[3] == nb
            for rep in range(2):
                res = bs.run()
                for (i0, g0, s0), (i1, g1, s1) in zip(ref, res):
                    assert s0 == s1 == 0 and list(i0) == list(i1)
                    np.testing.assert_array_equal(g0, g1)
                torch.cuda.synchronize()
                bs.reset(its)
