"""Full-size parity on the large single instance: 1500 candidate sensors x 96 observations
(N_d = 144,000), K formed and handed over in FP32 (83 GB; F is 144,000 x 40,000, seed 2), budget
175, in the launch configuration the benchmark times for it.

The oracle cannot replay 175 full steps, so the checks are
* sampled outputs: the score of every candidate at steps 0 and 1 (from-scratch factorisations of
  K_{A u j}), and of sampled candidates at a late step (Schur complement of K_AA), each computed by
  the oracle in FP64 from K's FP32 entries given the GPU's own prefix;
* properties that hold at any size: the telescoping identity sum(gains) = 1/2 logdet(sigma^-2 K_AA)
  (LAPACK Cholesky of the 16,800^2 selected block), non-increasing gains, mixed vs FP64 agreement
  up to a near-tie, and the left-looking method against the right-looking one.
"""
import numpy as np
import pytest
import torch

import oracle
from oed_inputs import CONFIGS, k_sub_lower, make_K_lower_panels
from parity import REGRESSION, RTOL, check_trajectory, rel_err

pytestmark = pytest.mark.gpu

PRECS = ("mixed_f32", "fp64", "mixed_bf16x3")


@pytest.fixture(scope="module")
def big():
    spec = CONFIGS["large_1500x96"]
    print(f"forming K {spec.N_d}^2 FP32 (n_m {spec.n_m}, seed {spec.seed})", flush=True)
    K, s2 = make_K_lower_panels(spec.N_s, spec.N_t, spec.n_m, spec.seed, spec.c, device="cuda:0",
                                dtype=torch.float32)
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
    print(f"greedy left-looking mixed_f32 B={spec.budget}", flush=True)
    with Selector(K, spec.N_s, spec.N_t, s2, precision="mixed_f32", method="left",
                  max_budget=spec.budget) as sel:
        out["left_mixed_f32"] = sel.greedy(spec.budget)
    return out


def half_logdet(K, spec, s2, idx):
    sub = k_sub_lower(K, spec.N_t, idx)
    return 0.5 * oracle.logdet_lapack(sub) - 0.5 * len(idx) * spec.N_t * np.log(s2)


@pytest.mark.timeout(900)
def test_large_telescoping_and_monotone(big, runs):
    spec, K, s2 = big
    totals = {}
    for name, (idx, gain) in runs.items():
        rtol = RTOL["fp64" if name == "fp64" else "mixed_f32"]
        assert len(set(idx.tolist())) == spec.budget
        assert np.all(gain[1:] <= gain[:-1] + rtol * np.maximum(1.0, np.abs(gain[:-1])))
        key = tuple(sorted(idx.tolist()))
        if key not in totals:
            totals[key] = half_logdet(K, spec, s2, idx)
        err = abs(gain.sum() - totals[key]) / abs(totals[key])
        print(f"{name}: sum of gains {gain.sum():.12e} vs 1/2 logdet {totals[key]:.12e}, rel {err:.2e}")
        assert err <= rtol


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", PRECS)
def test_large_sampled_steps_against_oracle(big, runs, prec):
    from paper_2604_08812_amd import Selector
    spec, K, s2 = big
    idx64, _ = runs["fp64"]
    rng = np.random.default_rng(2)
    nt = spec.N_t
    with Selector(K, spec.N_s, nt, s2, precision=prec) as sel:
        done = 0
        for k in (0, 1, 120):
            while done < k:
                sel.force(int(idx64[done]))
                done += 1
            g = sel.scores()
            prefix = [int(i) for i in idx64[:k]]
            rest = [j for j in range(spec.N_s) if j not in prefix]
            if k <= 1:
                # every candidate, from scratch, 100 candidates' block rows of K at a time
                cand = rest
                ref = np.concatenate([
                    oracle.gains(k_sub_lower(K, nt, prefix + rest[c0:c0 + 100]), nt, s2,
                                 list(range(k)), list(range(k, k + len(rest[c0:c0 + 100]))))
                    for c0 in range(0, len(rest), 100)])
            else:
                cand = sorted(set(rng.choice(rest, 6, replace=False).tolist()) | {int(idx64[k])})
                sub = k_sub_lower(K, nt, prefix + cand)
                S = oracle.schur_complement(sub, nt, list(range(k)), list(range(k, k + len(cand))))
                ref = np.array([0.5 * np.linalg.slogdet(S[p * nt:(p + 1) * nt, p * nt:(p + 1) * nt] / s2)[1]
                                for p in range(len(cand))])
            err = rel_err(g[cand], ref)
            print(f"{prec} step {k}: {len(cand)} candidates, max rel err {err.max():.2e}", flush=True)
            assert np.all(err <= RTOL[prec])
            if k <= 1:
                best = rest[int(np.argmax(ref))]
                top2 = np.sort(ref)[-2:]
                assert best == int(idx64[k]) or top2[1] - top2[0] <= 2 * RTOL["fp64"] * abs(top2[1])


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["mixed_f32", "mixed_bf16x3", "left_mixed_f32"])
def test_large_against_fp64(big, runs, name):
    """The mixed paths (and the left-looking one) pick the FP64 path's sensors up to the first
    step where FP64's own scores of the two picks are within the mixed tolerance, with gains
    within it before that."""
    from paper_2604_08812_amd import Selector
    spec, K, s2 = big
    i64, g64 = runs["fp64"]
    im, gm = runs[name]
    rtol = RTOL["mixed_f32"]
    div = next((k for k in range(spec.budget) if i64[k] != im[k]), None)
    upto = spec.budget if div is None else div
    err = rel_err(gm[:upto], g64[:upto]).max()
    print(f"{name} vs fp64: first divergence {div}, max rel gain diff before it {err:.2e}")
    assert err <= rtol
    # regression bound at the achieved level (the parity tolerance above stays 1e-4)
    reg = REGRESSION["mixed_bf16x3" if name == "mixed_bf16x3" else "mixed_f32"]
    assert err <= reg, f"{name}: gain difference to FP64 {err:.2e} > {reg}"
    if div is not None:
        with Selector(K, spec.N_s, spec.N_t, s2, precision="fp64") as sel:
            for k in range(div):
                sel.force(int(i64[k]))
            g = sel.scores()
        print(f"FP64 scores at step {div}: {g[i64[div]]:.12e} ({i64[div]}) vs {g[im[div]]:.12e} ({im[div]})")
        assert g[i64[div]] - g[im[div]] <= 2 * rtol * abs(g[i64[div]])


_SUB_CACHE = {}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", PRECS)
def test_large_subsample_100_against_oracle(big, prec):
    """Sensors 0..99 of the large instance's K (its leading 9,600^2 block), budget 29, replayed in
    full by the oracle from K's FP32 entries."""
    from paper_2604_08812_amd import Selector
    spec, K, s2 = big
    n, B = 100, 29
    with Selector(K, spec.N_s, spec.N_t, s2, precision=prec, candidates=range(n)) as sel:
        idx, gain = sel.greedy(B)
    sub = k_sub_lower(K, spec.N_t, range(n))
    rep = check_trajectory(sub, n, spec.N_t, s2, idx, gain, RTOL[prec], cache=_SUB_CACHE,
                           progress="1500x96 " + prec)
    print(f"{prec} subsample: picks {list(idx)}, max rel err {rep['max_rel_err']:.2e}, near-tie divergences "
          f"{rep['diverged_steps']}")
