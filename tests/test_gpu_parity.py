"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Each case runs the selection on cuda:0 through liboed and replays the GPU's
trajectory in the oracle (from-scratch FP64 Cholesky of every candidate test
matrix).  Sizes span several 128-row tiles with ragged tails and the padded
block sizes (N_t = 1, 24, 160 are not multiples of 16 or exceed the LDS path).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oed_inputs import make_K
from parity import RTOL, check_trajectory, rel_err

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def selector(*a, **k):
    from paper_2604_08812_amd import Selector
    return Selector(*a, **k)


def instance(N_s, N_t, n_m, seed, c=0.01):
    K, s2 = make_K(N_s, N_t, n_m, seed, c)
    return K.numpy(), K.to(DEV), s2


# (N_s, N_t, n_m, seed, budget)
CASES = [
    (64, 16, 4096, 0, 16),   # the 64 x 16 FP64 workload, budget 16
    (37, 16, 1024, 3, 12),   # 592 rows: 5 row tiles, ragged last tile, 8 sensors per tile
    (20, 128, 4000, 4, 8),   # one sensor per 128-row tile
    (23, 96, 3000, 5, 8),    # 96-row blocks straddle the 128-row tiles
    (30, 24, 1500, 6, 10),   # N_t padded 24 -> 32
    (50, 1, 200, 7, 30),     # N_t = 1 padded to 16
    (17, 48, 2000, 8, 9),
    (9, 160, 2000, 9, 5),    # N_t > 128: factorisations in global scratch
    (12, 144, 2500, 10, 6),  # N_tp = 144: the smallest block of the runtime-size LDS downdate
    (5, 420, 3000, 11, 4),   # the paper's block size, padded to 432
]


PRECS = ["fp64", "mixed_f32", "mixed_bf16x3"]


@pytest.mark.parametrize("delay", [1, 2, 4, 8])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:2])))
def test_greedy_matches_oracle(case, prec, delay):
    N_s, N_t, n_m, seed, B = case
    print(f"case N_s={N_s} N_t={N_t} seed={seed} B={B} prec={prec} delay={delay}", flush=True)
    K, Kd, s2 = instance(N_s, N_t, n_m, seed)
    with selector(Kd, N_s, N_t, s2, precision=prec, delay=delay) as sel:
        idx, gain = sel.greedy(B)
    rep = check_trajectory(K, N_s, N_t, s2, idx, gain, RTOL[prec])
    print(f"  max rel gain err {rep['max_rel_err']:.2e}, near-tie divergences {rep['diverged_steps']}")
    if prec == "fp64":
        assert rep["diverged_steps"] == [] or min(rep["ref"]["gap"]) < 1e-9


@pytest.mark.parametrize("prec", PRECS)
def test_blocks_beyond_the_blocked_factorisation(prec):
    """N_t = 1040 > 1024: the gains and the pick factor each block element-wise in global scratch,
    the downdate is the run-time-size kernel of the precision (33 tile rows, the last partial);
    delay 1, the only depth served there."""
    N_s, N_t, n_m, seed, B = 4, 1040, 3000, 12, 3
    print(f"N_t {N_t} {prec}", flush=True)
    K, Kd, s2 = instance(N_s, N_t, n_m, seed)
    with selector(Kd, N_s, N_t, s2, precision=prec, delay=1) as sel:
        idx, gain = sel.greedy(B)
    rep = check_trajectory(K, N_s, N_t, s2, idx, gain, RTOL[prec])
    print(f"  max rel gain err {rep['max_rel_err']:.2e}", flush=True)


@pytest.mark.parametrize("prefix", [[7, 0, 28, 13], [7, 0, 28]], ids=["even", "odd"])
@pytest.mark.parametrize("prec", PRECS)
def test_scores_and_schur_blocks_after_forced_prefix(prec, prefix):
    # odd prefix with the delayed downdate: the scores are taken with a block column held
    # (gain-kernel correction), the Schur blocks after applying it alone
    N_s, N_t = 29, 48
    K, Kd, s2 = instance(N_s, N_t, 2000, 21)
    A = list(prefix)
    rest = [j for j in range(N_s) if j not in A]
    # W hi + lo in BF16 represents w to about 2^-17 relative (lo * lo is dropped)
    tol = {"fp64": 1e-11, "mixed_f32": 2e-5, "mixed_bf16x3": 5e-5}[prec]
    with selector(Kd, N_s, N_t, s2, precision=prec) as sel:
        g0 = sel.scores()
        ref0 = oracle.gains(K, N_t, s2, [], range(N_s))
        assert np.all(rel_err(g0, ref0) <= RTOL[prec])
        for a in A:
            sel.force(a)
        g = sel.scores()
        ref = oracle.gains(K, N_t, s2, A, rest)
        assert np.all(np.isneginf(g[A]))
        assert np.all(rel_err(g[rest], ref) <= RTOL[prec])
        S = oracle.schur_complement(K, N_t, A, rest)
        scale = np.abs(S).max()
        for (i, j) in [(1, 1), (27, 3), (3, 27), (20, 19), (27, 27), (14, 12), (2, 1)]:
            if i in A or j in A:
                continue
            blk = sel.schur_block(i, j)
            pi, pj = rest.index(i), rest.index(j)
            ref_blk = S[pi * N_t:(pi + 1) * N_t, pj * N_t:(pj + 1) * N_t]
            assert np.abs(blk - ref_blk).max() <= tol * scale, (i, j)


def test_exact_ties_go_to_lowest_index():
    N_s, N_t, c, s2 = 40, 16, 3.0, 0.02
    K = c * torch.eye(N_s * N_t, dtype=torch.float64)
    for prec in PRECS:
        with selector(K.to(DEV), N_s, N_t, s2, precision=prec) as sel:
            idx, gain = sel.greedy(12)
        assert list(idx) == list(range(12))
        np.testing.assert_allclose(gain, 0.5 * N_t * math.log(c / s2), rtol=1e-12)


def test_non_pd_and_nan_candidates_are_never_picked():
    N_s, N_t = 12, 16
    K, s2 = make_K(N_s, N_t, 500, 31)
    K = K.clone()
    K[5 * N_t:6 * N_t, :] = 0.0      # sensor 5: zero block row (its Schur block stays 0)
    K[:, 5 * N_t:6 * N_t] = 0.0
    K[3 * N_t + 2, 3 * N_t + 1] = float("nan")   # sensor 3: NaN inside its diagonal block
    K[8 * N_t + 4, 0 * N_t + 7] = float("nan")   # sensor 8: NaN in its block column of sensor 0
    Kn = K.numpy()
    g_ref = oracle.gains(Kn, N_t, s2, [], range(N_s))
    assert np.isneginf(g_ref[5]) and np.isneginf(g_ref[3])
    ref = oracle.greedy(Kn, N_s, N_t, s2, N_s, raise_on_error=False)
    assert ref["status"] == 2
    # sensors 3 and 5 are never finite; once one of 0 and 8 is picked the other turns non-finite
    assert not ({3, 5} & set(ref["idx"].tolist())) and len({0, 8} & set(ref["idx"].tolist())) == 1
    for prec in PRECS:
        with selector(K.to(DEV), N_s, N_t, s2, precision=prec) as sel:
            g = sel.scores()
            assert np.isneginf(g[5]) and np.isneginf(g[3]) and np.isfinite(g[8])
            idx, gain, st = sel.greedy_status(N_s)
        assert st == 2  # OED_E_NOT_SPD once only non-PD candidates remain
        assert list(idx) == list(ref["idx"])
        assert np.all(rel_err(gain, ref["gain"]) <= RTOL[prec])


def test_upper_triangle_is_not_read():
    N_s, N_t = 21, 32
    K, s2 = make_K(N_s, N_t, 900, 41)
    Kn = K.clone()
    iu = torch.triu_indices(N_s * N_t, N_s * N_t, 1)
    Kn[iu[0], iu[1]] = float("nan")
    for prec in PRECS:
        with selector(K.to(DEV), N_s, N_t, s2, precision=prec) as a, \
                selector(Kn.to(DEV), N_s, N_t, s2, precision=prec) as b:
            ia, ga = a.greedy(8)
            ib, gb = b.greedy(8)
        assert list(ia) == list(ib)
        np.testing.assert_array_equal(ga, gb)


def test_candidate_subset():
    N_s, N_t = 45, 16
    K, Kd, s2 = instance(N_s, N_t, 1500, 51)
    cand = [44, 3, 17, 29, 8, 12, 40, 0, 21, 33, 5]
    for prec in PRECS:
        with selector(Kd, N_s, N_t, s2, precision=prec, candidates=cand) as sel:
            idx, gain = sel.greedy(6)
        assert set(idx.tolist()) <= set(cand)
        check_trajectory(K, N_s, N_t, s2, idx, gain, RTOL[prec], candidates=cand)


def test_force_then_greedy_and_split_calls():
    N_s, N_t = 33, 32
    K, Kd, s2 = instance(N_s, N_t, 1200, 61)
    with selector(Kd, N_s, N_t, s2) as a:
        ga = [a.force(5), a.force(2)]
        idx, gain = a.greedy(6)
    ref = oracle.greedy(K, N_s, N_t, s2, 8, prefix=[5, 2])
    assert list(ref["idx"][2:]) == list(idx)
    assert np.all(rel_err(np.r_[ga, gain], ref["gain"]) <= 1e-10)
    with selector(Kd, N_s, N_t, s2) as b, selector(Kd, N_s, N_t, s2) as c:
        i1, g1 = b.greedy(3)
        i2, g2 = b.greedy(5)
        i3, g3 = c.greedy(8)
        pi, pg = b.picks()
    assert list(np.r_[i1, i2]) == list(i3) == list(pi)
    np.testing.assert_array_equal(np.r_[g1, g2], g3)
    np.testing.assert_array_equal(pg, g3)


def test_reset_reproduces_bitwise():
    N_s, N_t = 40, 64
    _, Kd, s2 = instance(N_s, N_t, 3000, 71)
    for prec in PRECS:
        with selector(Kd, N_s, N_t, s2, precision=prec) as sel:
            i1, g1 = sel.greedy(10)
            sel.reset(Kd)
            i2, g2 = sel.greedy(10)
        assert list(i1) == list(i2)
        np.testing.assert_array_equal(g1, g2)


def test_float32_input_matrix():
    N_s, N_t = 26, 32
    K, s2 = make_K(N_s, N_t, 1500, 81)
    K32 = K.to(torch.float32)
    with selector(K32.to(DEV), N_s, N_t, s2, precision="mixed_f32") as sel:
        idx, gain = sel.greedy(7)
    check_trajectory(K32.to(torch.float64).numpy(), N_s, N_t, s2, idx, gain, RTOL["mixed_f32"])


def test_errors_and_states():
    from paper_2604_08812_amd import OedError
    N_s, N_t = 10, 16
    _, Kd, s2 = instance(N_s, N_t, 300, 91)
    with selector(Kd, N_s, N_t, s2) as sel:
        with pytest.raises(OedError):
            sel.greedy(11)
        sel.greedy(4)
        with pytest.raises(OedError):
            sel.greedy(7)          # only 6 remain
        picked = sel.picks()[0]
        with pytest.raises(OedError):
            sel.force(int(picked[0]))   # already picked
        with pytest.raises(OedError):
            sel.schur_block(int(picked[0]), 0)
        idx, gain = sel.greedy(6)   # exactly the rest
        assert len(idx) == 6
        g = sel.scores()
        assert np.all(np.isneginf(g))
    with pytest.raises(OedError):
        selector(Kd, N_s, N_t, -1.0)
    with pytest.raises(OedError):
        selector(Kd, N_s, N_t, s2, candidates=[1, 1, 2])


@pytest.mark.parametrize("delay", [2, 3, 4])
@pytest.mark.parametrize("prec", PRECS)
def test_delayed_downdate_matches_delay_one(prec, delay):
    """Holding block columns back changes the rounding only: same picks, gains equal to the
    precision's tolerance (FP64: 1e-12).  The split calls and the forced pick start with block
    columns held; the Schur-block query applies them."""
    N_s, N_t = 48, 64
    K, Kd, s2 = instance(N_s, N_t, 4000, 23)
    with selector(Kd, N_s, N_t, s2, precision=prec, delay=1) as a, \
            selector(Kd, N_s, N_t, s2, precision=prec, delay=delay) as b:
        i1, g1 = a.greedy(20)
        i2a, g2a = b.greedy(7)
        i2b, g2b = b.greedy(5)
        gf = b.force(int(i1[12]))
        blk = b.schur_block(int(i1[13]), int(i1[14]))
        i2c, g2c = b.greedy(7)
    assert list(i1) == list(np.r_[i2a, i2b, [i1[12]], i2c])
    tol = 1e-12 if prec == "fp64" else RTOL[prec]
    assert np.all(rel_err(np.r_[g2a, g2b, [gf], g2c], g1) <= tol)
    A = list(i1[:13])
    rest = [j for j in range(N_s) if j not in A]
    S = oracle.schur_complement(K, N_t, A, rest)
    p, q = rest.index(int(i1[13])), rest.index(int(i1[14]))
    ref = S[p * N_t:(p + 1) * N_t, q * N_t:(q + 1) * N_t]
    stol = {"fp64": 1e-11, "mixed_f32": 2e-5, "mixed_bf16x3": 5e-5}[prec]
    assert np.abs(blk - ref).max() <= stol * np.abs(S).max()


@pytest.mark.parametrize("prec", PRECS)
def test_autotuned_handle_selects_like_a_fixed_one(prec):
    """The autotuner times kernels on the packed working copy with zero W: it must leave R as
    packed, so the tuned handle gives bitwise the picks and gains of a handle created with the
    delay it chose; the choice is the depth of its least estimate (the shallowest on ties), and it is
    cached."""
    N_s, N_t = 70, 64
    K, Kd, s2 = instance(N_s, N_t, 5000, 29)
    with selector(Kd, N_s, N_t, s2, precision=prec, autotune=True) as t:
        delay, variant, ms, _ = t.config()
        it, gt = t.greedy(12)
    assert 1 <= delay <= 8 and variant in (0, 1, 2)
    assert np.all(ms > 0) and delay == int(np.argmin(ms)) + 1
    with selector(Kd, N_s, N_t, s2, precision=prec, delay=delay) as f:
        i_f, g_f = f.greedy(12)
    assert list(it) == list(i_f)
    np.testing.assert_array_equal(gt, g_f)
    check_trajectory(K, N_s, N_t, s2, it, gt, RTOL[prec])
    with selector(Kd, N_s, N_t, s2, precision=prec, autotune=True) as t2:
        d2, v2, ms2, _ = t2.config()
    assert (d2, v2) == (delay, variant)
    np.testing.assert_array_equal(ms2, ms)


LEFT_CASES = CASES  # N_t > 128: blocked global-scratch gain kernel with the diagonal update


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", LEFT_CASES, ids=lambda c: "x".join(map(str, c[:2])))
def test_left_looking_matches_oracle_and_right_looking(case, prec):
    N_s, N_t, n_m, seed, B = case
    print(f"left-looking N_s={N_s} N_t={N_t} seed={seed} B={B} prec={prec}", flush=True)
    K, Kd, s2 = instance(N_s, N_t, n_m, seed)
    with selector(Kd, N_s, N_t, s2, precision=prec, method="left", max_budget=B) as sel:
        idx, gain = sel.greedy(B)
    rep = check_trajectory(K, N_s, N_t, s2, idx, gain, RTOL[prec])
    print(f"  max rel gain err {rep['max_rel_err']:.2e}")
    with selector(Kd, N_s, N_t, s2, precision=prec, delay=1) as r:
        ir, gr = r.greedy(B)
    assert list(idx) == list(ir) or rep["diverged_steps"]
    if list(idx) == list(ir):
        assert np.all(rel_err(gain, gr) <= (1e-12 if prec == "fp64" else RTOL[prec]))


@pytest.mark.parametrize("prec", PRECS)
def test_left_looking_queries(prec):
    """Forced picks, scores, Schur blocks (diagonal and off-diagonal, formed on the host from K and
    the W history) and split calls in left-looking mode, against the oracle."""
    N_s, N_t = 31, 48
    K, Kd, s2 = instance(N_s, N_t, 2500, 37)
    A = [9, 2, 30]
    rest = [j for j in range(N_s) if j not in A]
    tol = {"fp64": 1e-11, "mixed_f32": 2e-5, "mixed_bf16x3": 5e-5}[prec]
    with selector(Kd, N_s, N_t, s2, precision=prec, method="left", max_budget=10) as sel:
        for a in A:
            sel.force(a)
        g = sel.scores()
        ref = oracle.gains(K, N_t, s2, A, rest)
        assert np.all(rel_err(g[rest], ref) <= RTOL[prec])
        S = oracle.schur_complement(K, N_t, A, rest)
        scale = np.abs(S).max()
        for (i, j) in [(1, 1), (28, 3), (3, 28), (20, 19), (29, 29), (0, 1)]:
            blk = sel.schur_block(i, j)
            pi, pj = rest.index(i), rest.index(j)
            assert np.abs(blk - S[pi * N_t:(pi + 1) * N_t, pj * N_t:(pj + 1) * N_t]).max() <= tol * scale, (i, j)
        i1, g1 = sel.greedy(4)
        i2, g2 = sel.greedy(3)
        with pytest.raises(Exception):
            sel.greedy(1)      # max_budget = 10 picks made
    ref = oracle.greedy(K, N_s, N_t, s2, 10, prefix=A)
    assert list(ref["idx"][3:]) == list(np.r_[i1, i2])
    assert np.all(rel_err(np.r_[g1, g2], ref["gain"][3:]) <= RTOL[prec])


def test_method_auto():
    """AUTO takes left-looking for a budget of at most half the candidates (N_t <= 128)."""
    N_s, N_t = 40, 32
    K, Kd, s2 = instance(N_s, N_t, 1500, 41)
    with selector(Kd, N_s, N_t, s2, precision="mixed_f32", method="auto", max_budget=12) as a:
        assert a.config()[1] == -1
        ia, ga = a.greedy(12)
    with selector(Kd, N_s, N_t, s2, precision="mixed_f32", method="auto") as b:
        assert b.config()[1] in (0, 1)
        ib, gb = b.greedy(12)
    assert list(ia) == list(ib)
    check_trajectory(K, N_s, N_t, s2, ia, ga, RTOL["mixed_f32"])


@pytest.mark.parametrize("method,delay", [("right", 1), ("right", 4), ("left", 0)])
@pytest.mark.parametrize("prec", PRECS)
def test_per_sensor_noise(prec, method, delay):
    """Noise variances differing by sensor (100x range): gains 1/2 logdet S_j - h_j with
    h_j = (N_t/2) ln sigma_j^2, against the oracle with the same per-sensor terms."""
    from oed_inputs import make_K_sensor_noise
    N_s, N_t, B = 36, 32, 10
    K, var = make_K_sensor_noise(N_s, N_t, 2000, 51)
    h = 0.5 * N_t * np.log(var)
    with selector(K.to(DEV), N_s, N_t, 1.0, precision=prec, method=method, delay=delay,
                  noise_half_logdet=h) as sel:
        idx, gain = sel.greedy(B)
    ref = oracle.greedy(K.numpy(), N_s, N_t, 1.0, B, noise_hld=h)
    div = next((k for k in range(B) if idx[k] != ref["idx"][k]), None)
    upto = B if div is None else div
    assert np.all(rel_err(gain[:upto], ref["gain"][:upto]) <= RTOL[prec])
    if div is not None:
        assert ref["gap"][div] <= 2 * RTOL[prec] * max(1.0, abs(ref["gain"][div])), (div, ref["gap"][div])


@pytest.mark.parametrize("method,delay", [("right", 1), ("right", 4), ("left", 0)])
@pytest.mark.parametrize("prec", PRECS)
def test_correlated_sensor_noise_with_cost_weights(prec, method, delay):
    """Sensor placement cost as a weighted noise covariance W_c Gamma_noise (Sec. III-G, diagonal
    W_c, weights over a 30x range) on noise correlated in time within each sensor (AR(1) blocks):
    K carries the weighted blocks and h_j = 1/2 logdet(w_j Gamma_jj); the HIP path against the
    oracle with the same per-sensor terms, on a ragged N_t."""
    from oed_inputs import make_K_weighted_noise
    N_s, N_t, B = 34, 24, 10
    K, blocks = make_K_weighted_noise(N_s, N_t, 2000, 52)
    h = np.array([0.5 * np.linalg.slogdet(b)[1] for b in blocks])
    print(f"weighted noise {prec} {method} delay {delay}", flush=True)
    with selector(K.to(DEV), N_s, N_t, 1.0, precision=prec, method=method, delay=delay,
                  noise_half_logdet=h) as sel:
        idx, gain = sel.greedy(B)
    ref = oracle.greedy(K.numpy(), N_s, N_t, 1.0, B, noise_hld=h)
    div = next((k for k in range(B) if idx[k] != ref["idx"][k]), None)
    upto = B if div is None else div
    assert np.all(rel_err(gain[:upto], ref["gain"][:upto]) <= RTOL[prec])
    if div is not None:
        assert ref["gap"][div] <= 2 * RTOL[prec] * max(1.0, abs(ref["gain"][div])), (div, ref["gap"][div])


@pytest.mark.parametrize("prec", PRECS)
def test_every_tile_order_gives_the_same_selection(prec):
    """The downdate's tile order changes which work-group computes a tile, never the arithmetic:
    at each delay every order gives bitwise the picks and gains of the others, on a ragged
    instance whose tile rows are not a multiple of any super-tile edge, and the oracle agrees."""
    N_s, N_t, B = 83, 48, 14   # 3,984 rows: 32 tile rows, the last one partial
    K, Kd, s2 = instance(N_s, N_t, 6000, 31)
    for delay in (1, 4, 7):
        outs = []
        for order in ("col4", "row8", "col8", "col2"):
            print(f"tile order {order} delay {delay} {prec}", flush=True)
            with selector(Kd, N_s, N_t, s2, precision=prec, delay=delay, tile_order=order) as sel:
                assert sel.config()[3] == order
                outs.append(sel.greedy(B))
        for i1, g1 in outs[1:]:
            assert list(i1) == list(outs[0][0])
            np.testing.assert_array_equal(g1, outs[0][1])
        check_trajectory(K, N_s, N_t, s2, outs[0][0], outs[0][1], RTOL[prec])


def test_tune_cache_file_round_trip(tmp_path):
    """With a tune-cache file the tuner appends its choice; a line edited in the file is what the
    next tuned handle of that shape takes (the file takes precedence over the process's cache)."""
    N_s, N_t = 37, 80
    K, Kd, s2 = instance(N_s, N_t, 4000, 33)
    path = tmp_path / "oed_tune.txt"
    with selector(Kd, N_s, N_t, s2, precision="mixed_f32", autotune=True, tune_cache=str(path)) as t:
        delay, variant, ms, order = t.config()
        i0, g0 = t.greedy(9)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("oedtune1 ")
    f = lines[0].split()
    assert int(f[6]) == delay and int(f[7]) == variant
    f[6], f[7], f[8] = "2", "1", "3"          # delay 2, LDS downdate, 8 x 8 down the columns
    path.write_text(" ".join(f) + "\n")
    with selector(Kd, N_s, N_t, s2, precision="mixed_f32", autotune=True, tune_cache=str(path)) as t2:
        d2, v2, _, o2 = t2.config()
        i2, g2 = t2.greedy(9)
    assert (d2, v2, o2) == (2, 1, "col8")
    with selector(Kd, N_s, N_t, s2, precision="mixed_f32", delay=2) as f2:
        i3, g3 = f2.greedy(9)
    assert list(i2) == list(i3) and list(i0) == list(i3)
    np.testing.assert_array_equal(g2, g3)


@pytest.mark.parametrize("method", ["right", "left"])
def test_injected_failure_stops_cleanly(method):
    """debug_fail_step = 5: the fifth pick fails once on the host before anything of it is
    enqueued.  The call returns OED_E_HIP with the picks made before it, the handle then refuses
    steps until it is reset, the reset selection equals a clean one, and destroying the handle
    returns all of its device memory."""
    from paper_2604_08812_amd import OedError
    N_s, N_t, B = 30, 32, 10
    K, Kd, s2 = instance(N_s, N_t, 3000, 35)
    kw = {"method": method, "max_budget": B} if method == "left" else {"delay": 3}
    with selector(Kd, N_s, N_t, s2, precision="mixed_f32", **kw) as clean:
        ic, gc = clean.greedy(B)
        need = clean.device_bytes()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    sel = selector(Kd, N_s, N_t, s2, precision="mixed_f32", debug_fail_step=5, **kw)
    assert sel.device_bytes() == need
    idx, gain, st = sel.greedy_status(B)
    assert st == 4 and len(idx) == 4
    assert list(idx) == list(ic[:4])
    np.testing.assert_array_equal(gain, gc[:4])
    from paper_2604_08812_amd import library
    assert "injected failure before pick 5" in library().oed_last_error(sel.h).decode()
    with pytest.raises(OedError):
        sel.greedy(1)
    with pytest.raises(OedError):
        sel.force(int(ic[5]))
    sel.reset(Kd)
    i2, g2 = sel.greedy(B)
    assert list(i2) == list(ic)
    np.testing.assert_array_equal(g2, gc)
    sel.close()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    # a limit of exactly what the handle holds is accepted; one byte less is OED_E_OOM
    selector(Kd, N_s, N_t, s2, precision="mixed_f32", max_device_bytes=need, **kw).close()
    with pytest.raises(OedError) as ei:
        selector(Kd, N_s, N_t, s2, precision="mixed_f32", max_device_bytes=need - 1, **kw)
    assert ei.value.status == 3 and str(need) in str(ei.value)


@pytest.mark.parametrize("N_t", [32, 48, 96, 128])
def test_bf16_big_tiles_equal_the_128_tiles(N_t):
    """The BF16 split-product downdate over 256 x 256 tiles (eight waves) accumulates every element
    in the order of the 128 x 128 kernel (slot, slice, then hi hi, hi lo, lo hi), so the selections
    are bitwise equal, at several delays and on ragged instances (the tile rows end mid-tile and, for
    N_t = 48 and 96, mid-block), and agree with the oracle."""
    N_s, B = {32: (61, 12), 48: (45, 10), 96: (27, 8), 128: (23, 8)}[N_t]
    K, Kd, s2 = instance(N_s, N_t, 5000, 40 + N_t)
    for delay in (1, 3, 8):
        print(f"bf16 big tiles N_t={N_t} delay={delay}", flush=True)
        with selector(Kd, N_s, N_t, s2, precision="mixed_bf16x3", delay=delay, tile_size=128) as a:
            assert a.config()[1] == 1
            ia, ga = a.greedy(B)
        with selector(Kd, N_s, N_t, s2, precision="mixed_bf16x3", delay=delay, tile_size=256) as b:
            assert b.config()[1] == 2
            ib, gb = b.greedy(B)
        assert list(ia) == list(ib)
        np.testing.assert_array_equal(ga, gb)
    check_trajectory(K, N_s, N_t, s2, ib, gb, RTOL["mixed_bf16x3"])
