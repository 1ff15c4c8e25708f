"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's own formula: values come from
brute force over subsets with an LU-based log-determinant, from closed forms
derived by hand (tests/golden/closed_forms.json), from LAPACK's pivoted
Cholesky, from the Schur-complement route of Algorithm 1 written independently,
and from invariants (telescoping sum, diminishing returns, (1-1/e) bound).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.linalg.lapack as lapack

import oracle
from oed_inputs import make_K

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")


def rand_spd_instance(rng, N_s, N_t, n_m=None, c=0.05):
    N_d = N_s * N_t
    n_m = n_m or 2 * N_d
    F = rng.standard_normal((N_d, n_m)) * (1.0 + np.arange(n_m)) ** -0.25
    G = F @ F.T / n_m
    s2 = c * float(np.mean(np.diag(G)))
    return G + s2 * np.eye(N_d), s2


def f_slogdet(K, N_t, sigma2, S):
    """f(S) = 1/2 logdet(sigma^-2 K_SS) with numpy's LU-based slogdet."""
    if len(S) == 0:
        return 0.0
    idx = oracle.block_index(N_t, S)
    sign, ld = np.linalg.slogdet(oracle.symmetrize_lower(K)[np.ix_(idx, idx)] / sigma2)
    assert sign > 0
    return 0.5 * ld


def brute_force_table(K, N_s, N_t, sigma2, B):
    table = {(): 0.0}
    for k in range(1, B + 1):
        for S in itertools.combinations(range(N_s), k):
            table[S] = f_slogdet(K, N_t, sigma2, S)
    return table


def greedy_from_table(table, N_s, B):
    A, gains, gaps = [], [], []
    for _ in range(B):
        base = table[tuple(sorted(A))]
        sc = [(table[tuple(sorted(A + [j]))] - base, j) for j in range(N_s) if j not in A]
        best = max(sc, key=lambda x: (x[0], -x[1]))
        rest = sorted((v for v, j in sc if j != best[1]), reverse=True)
        gaps.append(best[0] - rest[0] if rest else math.inf)
        A.append(best[1])
        gains.append(best[0])
    return A, gains, gaps


# --------------------------------------------------------------------------- factorisation
@pytest.mark.parametrize("n", [1, 2, 5, 17, 64, 130])
def test_chol_logdet_vs_lu(n):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n + 3))
    M = X @ X.T / n + 0.1 * np.eye(n)
    got = oracle.chol_logdet(M)
    sign, ref = np.linalg.slogdet(M)
    assert sign > 0
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))


def test_chol_logdet_rejects_non_pd():
    M = np.array([[1.0, 2.0], [2.0, 1.0]])
    assert oracle.chol_logdet(M) is None
    assert oracle.chol_logdet(np.array([[0.0]])) is None
    assert oracle.chol_logdet(np.array([[np.nan]])) is None
    assert oracle.chol_logdet(np.array([[1.0, 0.0], [np.inf, 1.0]])) is None


# --------------------------------------------------------------------------- brute force
@pytest.mark.parametrize("N_s,N_t,B,seed", [(6, 1, 3, 0), (7, 2, 3, 1), (8, 3, 4, 2), (10, 4, 4, 3),
                                            (9, 2, 4, 4), (10, 1, 4, 5)])
def test_greedy_matches_brute_force(N_s, N_t, B, seed):
    rng = np.random.default_rng(seed)
    K, s2 = rand_spd_instance(rng, N_s, N_t)
    table = brute_force_table(K, N_s, N_t, s2, B)
    A_ref, g_ref, gaps = greedy_from_table(table, N_s, B)
    assert min(gaps) > 1e-8, "instance has a near-tie; pick another seed"
    res = oracle.greedy(K, N_s, N_t, s2, B)
    assert list(res["idx"]) == A_ref
    np.testing.assert_allclose(res["gain"], g_ref, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(res["gap"], gaps, rtol=1e-8, atol=1e-10)
    # (1 - 1/e) guarantee for monotone submodular maximisation (Sec. III-H)
    opt = max(v for S, v in table.items() if len(S) == B)
    assert table[tuple(sorted(A_ref))] >= (1.0 - 1.0 / math.e) * opt - 1e-12


# --------------------------------------------------------------------------- closed forms
def _det22(a, b, c, d):
    return a * d - b * c


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_closed_form_golden(case):
    K = np.array(case["K"], dtype=np.float64)
    res = oracle.greedy(K, case["N_s"], case["N_t"], case["sigma2"], case["B"])
    assert list(res["idx"]) == case["idx"]
    expect = [eval(e, {"ln": math.log, "det22": _det22}) for e in case["gain_expr"]]
    np.testing.assert_allclose(res["gain"], expect, rtol=1e-14, atol=1e-15)


def test_scaled_identity_ties_go_to_lowest_index():
    N_s, N_t, c, s2 = 9, 3, 2.5, 0.1
    K = c * np.eye(N_s * N_t)
    res = oracle.greedy(K, N_s, N_t, s2, 5)
    assert list(res["idx"]) == [0, 1, 2, 3, 4]
    np.testing.assert_allclose(res["gain"], 0.5 * N_t * math.log(c / s2), rtol=1e-15)
    assert np.all(res["gap"] == 0.0)


def test_block_diagonal_picks_top_blocks():
    rng = np.random.default_rng(7)
    N_s, N_t, s2 = 8, 3, 0.2
    K = np.zeros((N_s * N_t, N_s * N_t))
    vals = []
    for i in range(N_s):
        X = rng.standard_normal((N_t, N_t + 2))
        blk = X @ X.T / N_t + 0.5 * np.eye(N_t)
        if i == 5:
            blk = K[3 * N_t:4 * N_t, 3 * N_t:4 * N_t].copy()  # exact copy of sensor 3: a tie
        K[i * N_t:(i + 1) * N_t, i * N_t:(i + 1) * N_t] = blk
        vals.append(0.5 * np.linalg.slogdet(blk / s2)[1])
    order = sorted(range(N_s), key=lambda i: (-vals[i], i))
    res = oracle.greedy(K, N_s, N_t, s2, 6)
    assert list(res["idx"]) == order[:6]
    np.testing.assert_allclose(res["gain"], [vals[i] for i in order[:6]], rtol=1e-12)


def test_nt1_is_diagonally_pivoted_cholesky():
    """With N_t = 1 the greedy is Cholesky with maximal-diagonal pivoting (LAPACK dpstrf)."""
    rng = np.random.default_rng(11)
    N_s, s2 = 30, 0.03
    K, _ = rand_spd_instance(rng, N_s, 1, n_m=60)
    K = K - np.diag(np.diag(K)) + np.diag(np.diag(K)) + s2 * np.eye(N_s)
    L, piv, rank, info = lapack.dpstrf(np.asfortranarray(K), lower=1, tol=-1.0)
    assert info == 0 and rank == N_s
    res = oracle.greedy(K, N_s, 1, s2, N_s)
    assert list(res["idx"]) == list(piv - 1)
    np.testing.assert_allclose(res["gain"], np.log(np.abs(np.diag(L))) - 0.5 * math.log(s2),
                               rtol=1e-12, atol=1e-13)


# --------------------------------------------------------------------------- identities / invariants
def _config0_like(seed=0):
    K, s2 = make_K(24, 8, 512, seed)
    return K.numpy(), s2


def test_telescoping_and_diminishing_returns():
    K, s2 = _config0_like()
    N_s, N_t, B = 24, 8, 10
    res = oracle.greedy(K, N_s, N_t, s2, B)
    total = f_slogdet(K, N_t, s2, list(res["idx"]))
    assert abs(res["gain"].sum() - total) <= 1e-11 * max(1.0, abs(total))
    g = res["gain"]
    assert np.all(g[1:] <= g[:-1] + 1e-12 * np.maximum(1.0, np.abs(g[:-1])))
    assert np.all(g > 0)


def test_scale_invariance():
    K, s2 = _config0_like(3)
    a = oracle.greedy(K, 24, 8, s2, 8)
    b = oracle.greedy(7.0 * K, 24, 8, 7.0 * s2, 8)
    assert list(a["idx"]) == list(b["idx"])
    np.testing.assert_allclose(a["gain"], b["gain"], rtol=1e-11)


def test_permutation_equivariance():
    K, s2 = _config0_like(4)
    N_s, N_t, B = 24, 8, 8
    perm = np.random.default_rng(5).permutation(N_s)
    idx = oracle.block_index(N_t, perm)
    Ks = oracle.symmetrize_lower(K)
    Kp = Ks[np.ix_(idx, idx)]
    a = oracle.greedy(K, N_s, N_t, s2, B)
    b = oracle.greedy(Kp, N_s, N_t, s2, B)
    assert min(a["gap"]) > 1e-9
    assert list(perm[b["idx"]]) == list(a["idx"])
    np.testing.assert_allclose(a["gain"], b["gain"], rtol=1e-11)


def test_only_lower_triangle_is_read():
    K, s2 = _config0_like(6)
    Kn = K.copy()
    Kn[np.triu_indices_from(Kn, 1)] = np.nan
    a = oracle.greedy(K, 24, 8, s2, 6)
    b = oracle.greedy(Kn, 24, 8, s2, 6)
    assert list(a["idx"]) == list(b["idx"])
    np.testing.assert_array_equal(a["gain"], b["gain"])


def test_schur_route_equals_from_scratch_scores():
    """Scores equal 1/2 logdet(sigma^-2 M_s), M_s the Schur block of Algorithm 1 (Sec. III-D)."""
    K, s2 = _config0_like(8)
    N_s, N_t = 24, 8
    A = [5, 17, 2]
    rest = [j for j in range(N_s) if j not in A]
    g = oracle.gains(K, N_t, s2, A, rest)
    S = oracle.schur_complement(K, N_t, A, rest)
    for p, j in enumerate(rest):
        blk = S[p * N_t:(p + 1) * N_t, p * N_t:(p + 1) * N_t]
        ref = 0.5 * np.linalg.slogdet(blk / s2)[1]
        assert abs(g[p] - ref) <= 1e-11 * max(1.0, abs(ref))


def _left_looking_greedy(K, N_s, N_t, s2, B):
    """Greedy by the block Cholesky update of Sec. III-D, written independently:
    a growing lower factor L of K_AA, a triangular solve for each candidate's
    block column, the Schur block, its Cholesky, and a block-row append."""
    Ks = oracle.symmetrize_lower(K)
    A, gains = [], []
    L = np.zeros((0, 0))
    for _ in range(B):
        best = None
        for j in range(N_s):
            if j in A:
                continue
            jj = oracle.block_index(N_t, [j])
            Kjj = Ks[np.ix_(jj, jj)]
            if A:
                KAj = Ks[np.ix_(oracle.block_index(N_t, A), jj)]
                Y = scipy.linalg.solve_triangular(L, KAj, lower=True)
                M = Kjj - Y.T @ Y
            else:
                Y, M = None, Kjj
            Lm = np.linalg.cholesky(M)
            d = 2.0 * np.sum(np.log(np.diag(Lm)))
            if best is None or d > best[0]:
                best = (d, j, Y, Lm)
        d, j, Y, Lm = best
        n = L.shape[0]
        Ln = np.zeros((n + N_t, n + N_t))
        Ln[:n, :n] = L
        if n:
            Ln[n:, :n] = Y.T
        Ln[n:, n:] = Lm
        L = Ln
        A.append(j)
        gains.append(0.5 * d - 0.5 * N_t * math.log(s2))
    return A, gains


def test_left_looking_update_agrees():
    K, s2 = _config0_like(9)
    A, g = _left_looking_greedy(K, 24, 8, s2, 8)
    res = oracle.greedy(K, 24, 8, s2, 8)
    assert min(res["gap"]) > 1e-9
    assert list(res["idx"]) == A
    np.testing.assert_allclose(res["gain"], g, rtol=1e-11)


# --------------------------------------------------------------------------- edge cases
def test_non_pd_candidate_scores_minus_inf_and_all_fail_stops():
    rng = np.random.default_rng(12)
    N_s, N_t = 5, 2
    K, s2 = rand_spd_instance(rng, N_s, N_t)
    K[4 * N_t:, :] = 0.0          # sensor 4: zero block row -> not positive definite
    g = oracle.gains(K, N_t, s2, [], range(N_s))
    assert g[4] == -np.inf and np.all(np.isfinite(g[:4]))
    res = oracle.greedy(K, N_s, N_t, s2, 4)
    assert 4 not in list(res["idx"])
    res = oracle.greedy(K, N_s, N_t, s2, 5, raise_on_error=False)
    assert res["status"] == 2 and len(res["idx"]) == 4


def test_candidates_subset_and_forced_prefix():
    K, s2 = _config0_like(10)
    cand = [3, 19, 7, 11, 0, 22, 15]
    res = oracle.greedy(K, 24, 8, s2, 4, candidates=cand)
    assert set(res["idx"]) <= set(cand)
    # the restricted instance is the principal submatrix of those sensors
    sub = oracle.symmetrize_lower(K)[np.ix_(oracle.block_index(8, sorted(cand)),
                                            oracle.block_index(8, sorted(cand)))]
    r2 = oracle.greedy(sub, len(cand), 8, s2, 4)
    assert [sorted(cand)[i] for i in r2["idx"]] == list(res["idx"])
    np.testing.assert_allclose(r2["gain"], res["gain"], rtol=1e-12)
    # forcing a prefix reproduces the scores of gains() on that prefix
    forced = oracle.greedy(K, 24, 8, s2, 3, prefix=[11, 3])
    assert list(forced["idx"][:2]) == [11, 3]
    g0 = oracle.gains(K, 8, s2, [], [11])[0]
    g1 = oracle.gains(K, 8, s2, [11], [3])[0]
    np.testing.assert_allclose(forced["gain"][:2], [g0, g1], rtol=1e-14)


def test_argument_errors():
    K = np.eye(4)
    with pytest.raises(oracle.OracleError):
        oracle.greedy(K, 4, 1, 0.0, 2)
    with pytest.raises(oracle.OracleError):
        oracle.greedy(K, 4, 1, 1.0, 5)
    with pytest.raises(oracle.OracleError):
        oracle.greedy(K, 4, 1, 1.0, 0)


def test_thread_count_does_not_change_results():
    K, s2 = _config0_like(13)
    a = oracle.greedy(K, 24, 8, s2, 6, threads=1)
    b = oracle.greedy(K, 24, 8, s2, 6, threads=4)
    assert list(a["idx"]) == list(b["idx"])
    np.testing.assert_array_equal(a["gain"], b["gain"])


def test_small_fp64_config_properties():
    """The 64 x 16 FP64 instance (n_m = 4096, seed 0, budget 16)."""
    from oed_inputs import CONFIGS
    sp = CONFIGS["small_fp64_64x16"]
    K, s2 = make_K(sp.N_s, sp.N_t, sp.n_m, sp.seed)
    K = K.numpy()
    res = oracle.greedy(K, sp.N_s, sp.N_t, s2, sp.budget)
    assert len(set(res["idx"])) == sp.budget
    g = res["gain"]
    assert np.all(g[1:] <= g[:-1] + 1e-12 * np.abs(g[:-1]))
    total = 0.5 * oracle.logdet_lapack(
        oracle.symmetrize_lower(K)[np.ix_(oracle.block_index(16, res["idx"]),
                                          oracle.block_index(16, res["idx"]))] / s2)
    assert abs(g.sum() - total) <= 1e-10 * abs(total)


# --------------------------------------------------------------------------- per-sensor noise
def sensor_noise_instance(rng, N_s, N_t, n_m=None):
    """K = F F^T / n_m + blockdiag(D_j), D_j a random SPD noise covariance per sensor; returns K,
    the blocks D_j and h_j = 1/2 logdet D_j (from eigenvalues)."""
    N_d = N_s * N_t
    n_m = n_m or 2 * N_d
    F = rng.standard_normal((N_d, n_m)) * (1.0 + np.arange(n_m)) ** -0.25
    G = F @ F.T / n_m
    scale = float(np.mean(np.diag(G)))
    K = G.copy()
    D, h = [], np.empty(N_s)
    for j in range(N_s):
        Q = rng.standard_normal((N_t, N_t))
        Dj = scale * (0.01 * 10 ** rng.uniform(-1, 1)) * (np.eye(N_t) + 0.3 * Q @ Q.T / N_t)
        K[j * N_t:(j + 1) * N_t, j * N_t:(j + 1) * N_t] += Dj
        D.append(Dj)
        h[j] = 0.5 * float(np.sum(np.log(np.linalg.eigvalsh(Dj))))
    return K, D, h


def test_sensor_noise_greedy_matches_brute_force():
    """f(S) = 1/2 logdet K_S - sum_{j in S} h_j, the computable objective with independent
    per-sensor noise: the oracle follows the greedy trajectory of the brute-force value table."""
    rng = np.random.default_rng(11)
    N_s, N_t, B = 8, 3, 4
    K, _, h = sensor_noise_instance(rng, N_s, N_t)
    table = {(): 0.0}
    for k in range(1, B + 1):
        for S in itertools.combinations(range(N_s), k):
            idx = oracle.block_index(N_t, S)
            sign, ld = np.linalg.slogdet(K[np.ix_(idx, idx)])
            table[S] = 0.5 * ld - float(sum(h[list(S)]))
    A, g, _ = greedy_from_table(table, N_s, B)
    res = oracle.greedy(K, N_s, N_t, 1.0, B, noise_hld=h)
    assert list(res["idx"]) == A
    np.testing.assert_allclose(res["gain"], g, rtol=1e-11, atol=1e-11)


def test_sensor_noise_block_diagonal_is_single_sensor_information():
    """With no coupling between sensors each gain is the single sensor's information
    1/2 logdet(I + D^-1 P) = 1/2 sum ln(1 + lambda_i) (generalised eigenvalues of (P, D)), whatever
    was picked before; picks are the top blocks (ties to the lowest index).  A candidate subset
    checks that h is taken by sensor index."""
    rng = np.random.default_rng(12)
    N_s, N_t, B = 9, 4, 5
    K = np.zeros((N_s * N_t, N_s * N_t))
    info, h = np.empty(N_s), np.empty(N_s)
    for j in range(N_s):
        X = rng.standard_normal((N_t, 2 * N_t))
        P = X @ X.T / (2 * N_t) * 10 ** rng.uniform(-1, 1)
        Dj = np.diag(10 ** rng.uniform(-2, 0, N_t))
        K[j * N_t:(j + 1) * N_t, j * N_t:(j + 1) * N_t] = P + Dj
        lam = scipy.linalg.eigh(P, Dj, eigvals_only=True)
        info[j] = 0.5 * float(np.sum(np.log1p(lam)))
        h[j] = 0.5 * float(np.sum(np.log(np.diag(Dj))))
    cand = [8, 1, 5, 3, 0, 7]
    res = oracle.greedy(K, N_s, N_t, 1.0, B, candidates=cand, noise_hld=h)
    order = sorted(cand, key=lambda j: (-info[j], j))[:B]
    assert list(res["idx"]) == order
    np.testing.assert_allclose(res["gain"], info[order], rtol=1e-10)


def test_sensor_noise_telescoping_and_isotropic_special_case():
    rng = np.random.default_rng(13)
    N_s, N_t, B = 12, 4, 7
    K, _, h = sensor_noise_instance(rng, N_s, N_t)
    res = oracle.greedy(K, N_s, N_t, 1.0, B, noise_hld=h)
    A = list(res["idx"])
    idx = oracle.block_index(N_t, A)
    total = 0.5 * oracle.logdet_lapack(K[np.ix_(idx, idx)]) - float(sum(h[A]))
    assert abs(res["gain"].sum() - total) <= 1e-10 * abs(total)
    # equal noise blocks s2 I: identical to the isotropic objective
    K2, s2 = rand_spd_instance(rng, N_s, N_t)
    iso = oracle.greedy(K2, N_s, N_t, s2, B)
    eq = oracle.greedy(K2, N_s, N_t, 1.0, B, noise_hld=np.full(N_s, 0.5 * N_t * math.log(s2)))
    assert list(iso["idx"]) == list(eq["idx"])
    np.testing.assert_allclose(iso["gain"], eq["gain"], rtol=1e-13, atol=1e-13)


def test_sensor_cost_weight_scales_only_that_sensors_information():
    """Placement cost as a weighted noise covariance W_c Gamma_noise (Sec. III-G, diagonal W_c) on
    noise correlated in time within each sensor: scaling sensor j's noise block by w changes K's
    diagonal block j and h_j = 1/2 logdet(w Gamma_jj).  At a fixed prefix A (j not in A) j's gain is
    then 1/2 sum ln(1 + lambda_i / w) over the generalised eigenvalues of (P_j, Gamma_jj), P_j the
    signal part of j's Schur complement: it falls strictly with w and tends to 0 (a sensor with
    unbounded noise carries no information), while every other candidate's gain stays bitwise the
    same (j's noise enters no other block)."""
    from oed_inputs import make_K_weighted_noise
    N_s, N_t = 10, 4
    K0, blocks = make_K_weighted_noise(N_s, N_t, 300, 41)
    K0 = K0.numpy()
    A, j = [3, 7], 5
    cand = [c for c in range(N_s) if c not in A]
    bj = slice(j * N_t, (j + 1) * N_t)
    ia = oracle.block_index(N_t, A)
    # signal part of j's Schur complement at A (the noise of j is not coupled to A)
    Gjj = K0[bj, bj] - blocks[j]
    P = Gjj - K0[bj, ia] @ np.linalg.solve(K0[np.ix_(ia, ia)], K0[ia, bj])
    lam = scipy.linalg.eigh(P, blocks[j], eigvals_only=True)
    assert lam.min() > 0
    h0 = np.array([0.5 * np.linalg.slogdet(b)[1] for b in blocks])
    prev, others = None, None
    for w in (1.0, 4.0, 64.0, 1e6, 1e12):
        K = K0.copy()
        K[bj, bj] += (w - 1.0) * blocks[j]
        h = h0.copy()
        h[j] += 0.5 * N_t * math.log(w)
        g = oracle.gains(K, N_t, 1.0, A, cand, noise_hld=h)
        gj = g[cand.index(j)]
        ref = 0.5 * float(np.sum(np.log1p(lam / w)))
        assert abs(gj - ref) <= 1e-9 * max(ref, 1e-6) + 1e-12, (w, gj, ref)
        if prev is not None:
            assert gj < prev, (w, gj, prev)
        prev = gj
        rest = np.delete(g, cand.index(j))
        if others is None:
            others = rest
        np.testing.assert_array_equal(rest, others)
    assert prev < 1e-9


# --------------------------------------------------------------------------- objective f(S)
@pytest.mark.parametrize("N_s,N_t,B,seed", [(6, 1, 3, 20), (7, 2, 3, 21), (8, 3, 4, 22)])
def test_objective_matches_lu_table_for_every_subset(N_s, N_t, B, seed):
    """f(S) = 1/2 logdet(sigma^-2 K_SS) (Sec. III-C, isotropic noise) for every subset of up to B
    sensors, against numpy's LU-based slogdet; the value does not depend on the order of S."""
    rng = np.random.default_rng(seed)
    K, s2 = rand_spd_instance(rng, N_s, N_t)
    assert abs(math.log(s2)) > 1.0  # the noise term is far from zero, so its count and sign matter
    table = brute_force_table(K, N_s, N_t, s2, B)
    assert oracle.objective(K, N_t, s2, []) == 0.0
    for S, ref in table.items():
        if not S:
            continue
        got = oracle.objective(K, N_t, s2, list(S))
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (S, got, ref)
        rev = oracle.objective(K, N_t, s2, list(S)[::-1])
        assert abs(rev - ref) <= 1e-12 * max(1.0, abs(ref)), (S, rev, ref)


def test_objective_is_sum_of_greedy_gains():
    """Telescoping: the gains of the greedy trajectory add up to f(A_B), isotropic and per-sensor."""
    K, s2 = _config0_like(14)
    N_s, N_t, B = 24, 8, 9
    res = oracle.greedy(K, N_s, N_t, s2, B)
    for k in range(1, B + 1):
        f = oracle.objective(K, N_t, s2, list(res["idx"][:k]))
        assert abs(f - res["gain"][:k].sum()) <= 1e-11 * max(1.0, abs(f)), k
    rng = np.random.default_rng(15)
    Kn, _, h = sensor_noise_instance(rng, 12, 4)
    rn = oracle.greedy(Kn, 12, 4, 1.0, 6, noise_hld=h)
    f = oracle.objective(Kn, 4, 1.0, list(rn["idx"]), noise_hld=h)
    assert abs(f - rn["gain"].sum()) <= 1e-11 * max(1.0, abs(f))


def test_objective_parameter_space_and_generalised_eigenvalues():
    """With K = F F^T / n_m + D (D block-diagonal, the noise covariance of sensors independent of each
    other), the computable objective f(S) = 1/2 logdet K_SS - sum_{j in S} 1/2 logdet D_j equals the
    expected information gain in the parameter space, 1/2 logdet(I + F_S^T D_S^-1 F_S / n_m)
    (Sylvester's determinant identity), and 1/2 sum ln(lambda) over the generalised eigenvalues of
    (K_SS, D_SS).  Isotropic D = sigma^2 I is checked the same way."""
    rng = np.random.default_rng(16)
    N_s, N_t, n_m = 7, 3, 40
    N_d = N_s * N_t
    F = rng.standard_normal((N_d, n_m)) * (1.0 + np.arange(n_m)) ** -0.25
    D = np.zeros((N_d, N_d))
    h = np.empty(N_s)
    for j in range(N_s):
        Q = rng.standard_normal((N_t, N_t))
        Dj = 0.02 * 10 ** rng.uniform(-1, 1) * (np.eye(N_t) + 0.3 * Q @ Q.T / N_t)
        D[j * N_t:(j + 1) * N_t, j * N_t:(j + 1) * N_t] = Dj
        h[j] = 0.5 * float(np.sum(np.log(np.linalg.eigvalsh(Dj))))
    K = F @ F.T / n_m + D
    s2 = 0.013
    Kiso = F @ F.T / n_m + s2 * np.eye(N_d)
    for S in ([3], [0, 5], [6, 1, 4], [2, 0, 6, 3, 5]):
        idx = oracle.block_index(N_t, S)
        FS, DS = F[idx], D[np.ix_(idx, idx)]
        eig = 0.5 * np.linalg.slogdet(np.eye(n_m) + FS.T @ np.linalg.solve(DS, FS) / n_m)[1]
        lam = scipy.linalg.eigh(K[np.ix_(idx, idx)], DS, eigvals_only=True)
        got = oracle.objective(K, N_t, 1.0, S, noise_hld=h)
        assert abs(got - eig) <= 1e-11 * max(1.0, abs(eig)), (S, got, eig)
        assert abs(got - 0.5 * float(np.sum(np.log(lam)))) <= 1e-11 * max(1.0, abs(eig)), S
        eig_iso = 0.5 * np.linalg.slogdet(np.eye(n_m) + FS.T @ FS / (n_m * s2))[1]
        got_iso = oracle.objective(Kiso, N_t, s2, S)
        assert abs(got_iso - eig_iso) <= 1e-11 * max(1.0, abs(eig_iso)), (S, got_iso, eig_iso)


def test_step_replay_helper_matches_the_oracle_greedy():
    """The GPU tests replay a trajectory step by step with oracle.gains; on the oracle's own picks
    that replay must reproduce oracle.greedy exactly (picks, gains, its own argmax), with and
    without a candidate subset, and a planted wrong pick must be reported."""
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from parity import check_trajectory
    N_s, N_t, B = 12, 3, 6
    K, s2 = make_K(N_s, N_t, 60, 77)
    K = K.numpy()
    for cand in (None, [0, 2, 3, 5, 7, 8, 10, 11]):
        ref = oracle.greedy(K, N_s, N_t, s2, B, candidates=cand)
        rep = check_trajectory(K, N_s, N_t, s2, ref["idx"], ref["gain"], 1e-12, candidates=cand)
        assert list(rep["ref"]["best"]) == list(ref["idx"]) and rep["diverged_steps"] == []
        np.testing.assert_array_equal(rep["ref"]["gain"], ref["gain"])
    bad = list(ref["idx"])
    bad[2], bad[3] = bad[3], bad[2]   # not a near-tie: the replay must reject it
    with pytest.raises(AssertionError):
        check_trajectory(K, N_s, N_t, s2, bad, ref["gain"], 1e-12, candidates=cand)
