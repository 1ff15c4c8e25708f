"""GPU parity of design evaluation (the objective of given sensor sets, as in the comparison of
the greedy design with random and uniform ones).

Every design's objective f(S) = 1/2 logdet(sigma^-2 K_SS) and its per-block terms
t_k = f(s_0..s_k) - f(s_0..s_{k-1}) must match the oracle's (plain Cholesky of K_SS and of its
leading blocks) within the precision's tolerance; the greedy design in pick order must
reproduce the greedy's gains term by term; the objective must not depend on the order.
"""
import numpy as np
import pytest
import torch

import oracle
from oed_inputs import make_K
from parity import RTOL, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PRECS = ("fp64", "mixed_f32", "mixed_bf16x3")


@pytest.fixture(scope="module", params=[(30, 16, 600, 401), (14, 24, 700, 402), (10, 128, 1500, 403)],
                ids=lambda p: f"{p[0]}x{p[1]}")
def inst(request):
    N_s, N_t, n_m, seed = request.param
    K, s2 = make_K(N_s, N_t, n_m, seed)
    return K.numpy(), K.to(DEV), N_s, N_t, s2


def random_designs(N_s, B, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(N_s)[:B] for _ in range(n)]).astype(np.int32)


def oracle_terms(K, N_t, s2, S):
    f = [0.0] + [oracle.objective(K, N_t, s2, S[:k + 1]) for k in range(len(S))]
    return np.diff(np.asarray(f))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("delay", [1, 4])
def test_eval_against_oracle(inst, prec, delay):
    from paper_2604_08812_amd import Evaluator
    Kh, Kd, N_s, N_t, s2 = inst
    B = min(7, N_s)
    designs = random_designs(N_s, B, 7, 11)  # unsorted designs, 7 = 3 + 3 + a short chunk of 1
    print(f"eval {N_s}x{N_t} B={B} {prec} delay {delay}", flush=True)
    with Evaluator(Kd, N_s, N_t, s2, B, max_batch=3, precision=prec, delay=delay) as ev:
        obj, terms = ev.run(designs)
        st = ev.stats()
    assert st["batch"] == 3 and st["executed"] == 9
    for r, S in enumerate(designs):
        ref = oracle_terms(Kh, N_t, s2, S.tolist())
        assert np.all(rel_err(terms[r], ref) <= RTOL[prec]), (r, terms[r], ref)
        assert rel_err(obj[r], ref.sum()) <= RTOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_eval_edge_designs(inst, prec):
    """B = 1 (a single block: f = 1/2 logdet(sigma^-2 K_jj)), B = N_s (all sensors, reversed),
    one design with a batch of one, and two runs in a row on one evaluator."""
    from paper_2604_08812_amd import Evaluator
    Kh, Kd, N_s, N_t, s2 = inst
    with Evaluator(Kd, N_s, N_t, s2, 1, max_batch=4, precision=prec) as ev:
        obj, _ = ev.run(np.array([[N_s - 1], [0], [N_s // 2]], dtype=np.int32))
        for j, o in zip((N_s - 1, 0, N_s // 2), obj):
            assert rel_err(o, oracle.objective(Kh, N_t, s2, [j])) <= RTOL[prec]
    full = np.arange(N_s - 1, -1, -1, dtype=np.int32)[None, :]
    with Evaluator(Kd, N_s, N_t, s2, N_s, max_batch=1, precision=prec, graph=False) as ev:
        obj, _ = ev.run(full)
        assert rel_err(obj[0], oracle.objective(Kh, N_t, s2, list(range(N_s)))) <= RTOL[prec]
    B = min(5, N_s)
    with Evaluator(Kd, N_s, N_t, s2, B, max_batch=2, precision=prec) as ev:
        for seed in (21, 22):
            d = random_designs(N_s, B, 3, seed)
            obj, _ = ev.run(d)
            for r, S in enumerate(d):
                assert rel_err(obj[r], oracle.objective(Kh, N_t, s2, S.tolist())) <= RTOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_eval_greedy_design_reproduces_gains(inst, prec):
    from paper_2604_08812_amd import Evaluator, Selector
    _, Kd, N_s, N_t, s2 = inst
    B = min(6, N_s)
    with Selector(Kd, N_s, N_t, s2, precision=prec) as sel:
        idx, gain = sel.greedy(B)
    with Evaluator(Kd, N_s, N_t, s2, B, precision=prec) as ev:
        rev = idx[::-1].copy()
        obj, terms = ev.run(np.stack([idx, rev]))
    assert np.all(rel_err(terms[0], gain) <= RTOL[prec])
    # the order changes the terms, not the objective
    assert rel_err(obj[1], obj[0]) <= RTOL[prec]


def test_eval_rejects_bad_designs(inst):
    from paper_2604_08812_amd import Evaluator, OedError
    _, Kd, N_s, N_t, s2 = inst
    with Evaluator(Kd, N_s, N_t, s2, 3, max_batch=2) as ev:
        for bad in ([[0, 1, 1]], [[0, 1, N_s]], [[-1, 0, 1]]):
            with pytest.raises(OedError):
                ev.run(np.array(bad, dtype=np.int32))
        obj, _ = ev.run(np.zeros((0, 3), dtype=np.int32))
        assert obj.shape == (0,)
