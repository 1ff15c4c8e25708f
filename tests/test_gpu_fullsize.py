"""Full-size parity on the 600-sensor x 128-observation instance (K = 76,800^2 FP64,
seed 1, budget 175), in the launch configuration the benchmark times.

The oracle cannot replay 175 full steps here, so the checks are
* sampled outputs: the scores of every candidate at early steps, and of sampled
  candidates at a late step, each computed by the oracle from K given the GPU's
  own prefix;
* properties that hold at any size: the telescoping identity
  sum(gains) = 1/2 logdet(sigma^-2 K_AA) (LAPACK Cholesky of the 22,400^2
  selected block), non-increasing gains, mixed vs FP64 agreement;
* the 100-sensor subsample (candidates 0..99 of the same K) replayed in full by
  the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from oed_inputs import CONFIGS, k_sub_lower, make_K_lower_panels
from parity import REGRESSION, RTOL, check_trajectory, rel_err

pytestmark = pytest.mark.gpu

PRECS = ("fp64", "mixed_f32", "mixed_bf16x3")


@pytest.fixture(scope="module")
def big():
    spec = CONFIGS["fp64_600x128"]
    print(f"forming K {spec.N_d}^2 FP64 (seed {spec.seed})", flush=True)
    K, s2 = make_K_lower_panels(spec.N_s, spec.N_t, spec.n_m, spec.seed, spec.c, device="cuda:0",
                                dtype=torch.float64)
    torch.cuda.synchronize()
    yield spec, K, s2
    del K
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def runs(big):
    from paper_2604_08812_amd import Selector
    spec, K, s2 = big
    out = {}
    for prec in PRECS:
        print(f"greedy {prec} B={spec.budget}", flush=True)
        # autotuned delay, as the benchmark runs it
        with Selector(K, spec.N_s, spec.N_t, s2, precision=prec, autotune=True) as sel:
            print(f"  delay {sel.config()[0]}", flush=True)
            out[prec] = sel.greedy(spec.budget)
    for prec in PRECS:
        print(f"greedy left-looking {prec} B={spec.budget}", flush=True)
        with Selector(K, spec.N_s, spec.N_t, s2, precision=prec, method="left", max_budget=spec.budget) as sel:
            out["left_" + prec] = sel.greedy(spec.budget)
    return out


@pytest.mark.timeout(900)
def test_fullsize_telescoping_and_monotone(big, runs):
    spec, K, s2 = big
    for prec in PRECS:
        idx, gain = runs[prec]
        assert len(set(idx.tolist())) == spec.budget
        rtol = RTOL[prec]
        assert np.all(gain[1:] <= gain[:-1] + rtol * np.maximum(1.0, np.abs(gain[:-1])))
        sub = k_sub_lower(K, spec.N_t, idx)
        total = 0.5 * oracle.logdet_lapack(sub) - 0.5 * len(idx) * spec.N_t * np.log(s2)
        err = abs(gain.sum() - total) / abs(total)
        print(f"{prec}: sum of gains {gain.sum():.12e} vs 1/2 logdet {total:.12e}, rel {err:.2e}")
        assert err <= rtol


@pytest.mark.timeout(900)
def test_fullsize_sampled_steps_against_oracle(big, runs):
    from paper_2604_08812_amd import Selector
    spec, K, s2 = big
    idx64, g64 = runs["fp64"]
    rng = np.random.default_rng(0)
    for prec in PRECS:
        with Selector(K, spec.N_s, spec.N_t, s2, precision=prec) as sel:
            done = 0
            for k in (0, 1, 2, 40):
                while done < k:
                    sel.force(int(idx64[done]))
                    done += 1
                g = sel.scores()
                prefix = list(idx64[:k])
                rest = [j for j in range(spec.N_s) if j not in prefix]
                if k <= 2:
                    # every candidate, from-scratch factorisations of K_{A u j}, in chunks of
                    # candidates so that only (k + 50) block rows of K are copied at a time
                    cand = rest
                    ref = np.concatenate([
                        oracle.gains(k_sub_lower(K, spec.N_t, prefix + rest[c0:c0 + 50]), spec.N_t, s2,
                                     list(range(k)), list(range(k, k + len(rest[c0:c0 + 50]))))
                        for c0 in range(0, len(rest), 50)])
                else:
                    # sampled candidates via the Schur complement of K_AA (library solve)
                    cand = sorted(set(rng.choice(rest, 6, replace=False).tolist()) | {int(idx64[k])})
                    sensors = prefix + cand
                    sub = k_sub_lower(K, spec.N_t, sensors)
                    S = oracle.schur_complement(sub, spec.N_t, list(range(k)), list(range(k, len(sensors))))
                    nt = spec.N_t
                    ref = np.array([0.5 * np.linalg.slogdet(S[p * nt:(p + 1) * nt, p * nt:(p + 1) * nt] / s2)[1]
                                    for p in range(len(cand))])
                err = rel_err(g[cand], ref)
                print(f"{prec} step {k}: {len(cand)} candidates, max rel err {err.max():.2e}")
                assert np.all(err <= RTOL[prec])
                if k <= 2:
                    best = rest[int(np.argmax(ref))]
                    top2 = np.sort(ref)[-2:]
                    assert best == int(idx64[k]) or top2[1] - top2[0] <= 2 * RTOL["fp64"] * abs(top2[1])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["mixed_f32", "mixed_bf16x3"])
def test_fullsize_mixed_vs_fp64(big, runs, prec):
    spec, K, s2 = big
    i64, g64 = runs["fp64"]
    i32, g32 = runs[prec]
    div = next((k for k in range(spec.budget) if i64[k] != i32[k]), None)
    upto = spec.budget if div is None else div
    err = rel_err(g32[:upto], g64[:upto]).max()
    print(f"{prec} vs fp64: first divergence {div}, max rel gain diff before it {err:.2e}")
    assert err <= RTOL[prec]
    # regression bounds at the achieved level: FP32 picks every FP64 pick on this instance (its
    # smallest FP64 top-two gap, 6.2e-8 relative, is several times its gain error), and both mixed
    # paths stay within REGRESSION of FP64 before any divergence
    assert err <= REGRESSION[prec], f"{prec}: gain difference to FP64 {err:.2e} > {REGRESSION[prec]}"
    if prec == "mixed_f32":
        assert div is None, f"mixed FP32 left the FP64 picks at step {div}"
    if div is not None:
        # a divergence must be a near-tie at that step for the FP64 scores
        from paper_2604_08812_amd import Selector
        with Selector(K, spec.N_s, spec.N_t, s2, precision="fp64") as sel:
            for k in range(div):
                sel.force(int(i64[k]))
            g = sel.scores()
        assert g[i64[div]] - g[i32[div]] <= 2 * RTOL[prec] * abs(g[i64[div]])


_SUB_CACHE = {}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", PRECS)
def test_subsample_100_against_oracle(big, prec):
    """Sensors 0..99 of the same K (its leading 12,800^2 block), budget 29 (175 scaled to 100 of
    600 sensors), replayed in full by the oracle."""
    from paper_2604_08812_amd import Selector
    spec, K, s2 = big
    n, B = 100, 29
    with Selector(K, spec.N_s, spec.N_t, s2, precision=prec, candidates=range(n)) as sel:
        idx, gain = sel.greedy(B)
    sub = k_sub_lower(K, spec.N_t, range(n))
    rep = check_trajectory(sub, n, spec.N_t, s2, idx, gain, RTOL[prec], cache=_SUB_CACHE,
                           progress="600x128 " + prec)
    print(f"{prec} subsample: picks {list(idx)}, max rel err {rep['max_rel_err']:.2e}")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", PRECS)
def test_fullsize_left_looking(big, runs, prec):
    """Left-looking selection at full size: the picks of the right-looking FP64 path, gains within
    the precision's tolerance, and the telescoping identity."""
    spec, K, s2 = big
    i64, g64 = runs["fp64"]
    il, gl = runs["left_" + prec]
    div = next((k for k in range(spec.budget) if i64[k] != il[k]), None)
    upto = spec.budget if div is None else div
    err = rel_err(gl[:upto], g64[:upto]).max()
    print(f"left {prec} vs right fp64: first divergence {div}, max rel gain diff {err:.2e}")
    assert err <= RTOL[prec]
    assert div is None or RTOL[prec] > 1e-9
    sub = k_sub_lower(K, spec.N_t, il)
    total = 0.5 * oracle.logdet_lapack(sub) - 0.5 * len(il) * spec.N_t * np.log(s2)
    assert abs(gl.sum() - total) / abs(total) <= RTOL[prec]


@pytest.fixture(scope="module")
def eval_designs(big, runs):
    """The FP64 greedy design in pick order, one random design and the uniformly spaced one, all
    of B = 175 sensors, with the oracle's objective of the last two (LAPACK Cholesky of the
    22,400^2 K_SS)."""
    spec, K, s2 = big
    B = spec.budget
    rng = np.random.default_rng(5)
    rand = rng.permutation(spec.N_s)[:B]
    unif = np.round(np.linspace(0, spec.N_s - 1, B)).astype(np.int64)
    ref = []
    for S in (rand, unif):
        sub = k_sub_lower(K, spec.N_t, S)
        ref.append(0.5 * oracle.logdet_lapack(sub) - 0.5 * B * spec.N_t * np.log(s2))
        del sub
    designs = np.stack([runs["fp64"][0], rand, unif]).astype(np.int32)
    return designs, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", PRECS)
def test_fullsize_design_evaluation(big, runs, eval_designs, prec):
    from paper_2604_08812_amd import Evaluator
    spec, K, s2 = big
    designs, ref = eval_designs
    print(f"design evaluation {prec}: 3 designs of {spec.budget} sensors", flush=True)
    with Evaluator(K, spec.N_s, spec.N_t, s2, spec.budget, max_batch=2, precision=prec) as ev:
        obj, terms = ev.run(designs)
    i_g, g_g = runs[prec]
    same = next((k for k in range(spec.budget) if i_g[k] != designs[0][k]), spec.budget)
    err_g = rel_err(terms[0][:same], g_g[:same]).max()
    err_r = rel_err(obj[1:], np.asarray(ref)).max()
    print(f"{prec}: greedy terms vs gains over {same} steps {err_g:.2e}; random/uniform objective "
          f"{obj[1]:.10e}/{obj[2]:.10e} vs {ref[0]:.10e}/{ref[1]:.10e}, rel {err_r:.2e}")
    assert err_g <= RTOL[prec]
    assert err_r <= RTOL[prec]
    assert obj[0] > obj[1] and obj[0] > obj[2]
