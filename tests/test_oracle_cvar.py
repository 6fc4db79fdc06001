"""Pins of the oracle's Monte-Carlo CVaR (Eq. 10-13) and risk scaling (Eq. 18-19).

The estimator is pinned by its limits (alpha -> 0 gives the mean, alpha -> 1
the maximum), by the Gaussian closed form CVaR_alpha = mu + sigma *
phi(Phi^-1(alpha)) / (1 - alpha) on a million draws, by brute force straight
from the definitions (VaR as the smallest t with P(L <= t) >= alpha, Eq. 11;
the mean of the draws with L >= VaR, Eq. 12-13), and by the affine identity of
the scaling, CVaR(L_a) = Lbar + B (CVaR(L) - Lbar) for B > 0.
"""
import json
import os

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_tail_sizes():
    # k_alpha = ceil(alpha M); n_tail = M - k_alpha + 1
    assert oracle.tail_size(0.9, 16) == (15, 2)
    assert oracle.tail_size(0.9, 64) == (58, 7)
    assert oracle.tail_size(0.9, 128) == (116, 13)
    assert oracle.tail_size(0.5, 16) == (8, 9)
    assert oracle.tail_size(1e-6, 10) == (1, 10)
    assert oracle.tail_size(0.999999, 10) == (10, 1)
    # float32 alpha = 0.9 on the paper's 300 draws keeps the 31 largest
    assert oracle.tail_size(float(np.float32(0.9)), 300) == (270, 31)


def test_alpha_to_zero_is_the_mean():
    rng = np.random.default_rng(0)
    for M in (1, 2, 7, 16, 128):
        L = rng.normal(3.0, 2.0, size=M)
        assert oracle.cvar(L, 0.5 / M) == pytest.approx(L.mean(), rel=1e-13, abs=1e-13)


def test_alpha_to_one_is_the_max():
    rng = np.random.default_rng(1)
    for M in (1, 2, 7, 16, 128, 300):
        L = rng.exponential(5.0, size=M)
        assert oracle.cvar(L, 1.0 - 0.5 / M) == L.max()


def _brute_force_cvar(L, alpha):
    """Eq. 11: VaR = min{t : #(L <= t)/M >= alpha}, scanning every candidate t
    (the optimum is attained at a sample).  Eq. 12-13: average of the draws
    with L >= VaR, N_o of them."""
    M = len(L)
    var = None
    for t in sorted(L):
        if sum(1 for x in L if x <= t) / M >= alpha:
            var = t
            break
    tail = [x for x in L if x >= var]
    return sum(tail) / len(tail), var, len(tail)


def test_brute_force_definition_on_small_inputs():
    rng = np.random.default_rng(2)
    for trial in range(300):
        M = int(rng.integers(1, 13))
        alpha = float(rng.uniform(0.01, 0.99))
        # keep alpha * M away from integers so both sides read the same VaR
        if abs(alpha * M - round(alpha * M)) < 1e-6:
            continue
        L = rng.normal(0, 1, size=M) * rng.uniform(0.1, 10) + rng.uniform(-5, 5)
        ref, var, n_o = _brute_force_cvar(list(L), alpha)
        ka, nt = oracle.tail_size(alpha, M)
        assert nt == n_o
        assert oracle.cvar(L, alpha) == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_ties_take_the_n_tail_largest():
    # with ties at VaR the literal ">= VaR" rule would average more values;
    # the reading keeps exactly n_tail of them, which is tie-independent
    L = np.array([1.0, 2.0, 2.0, 2.0, 5.0])
    # alpha = 0.7: k_alpha = 4, VaR = 2, n_tail = 2 -> mean(5, 2)
    assert oracle.cvar(L, 0.7) == pytest.approx(3.5)


def test_tied_var_is_where_the_reading_leaves_the_literal_rule():
    # Eq. 12-13 read literally average every draw with L >= VaR (N_o of them);
    # the reading averages the n_tail largest.  Brute force on rows drawn from
    # a few values (many ties): the two agree exactly when N_o == n_tail (no
    # draw below the k_alpha-th order statistic equals it), and otherwise the
    # literal mean is the reading's n_tail values plus N_o - n_tail further
    # copies of VaR, averaged over N_o.
    rng = np.random.default_rng(5)
    n_differ = 0
    for trial in range(400):
        M = int(rng.integers(2, 40))
        alpha = float(rng.uniform(0.05, 0.95))
        if abs(alpha * M - round(alpha * M)) < 1e-6:
            continue
        L = rng.integers(0, 4, size=M).astype(np.float64) * rng.uniform(0.5, 3.0)
        lit, var, n_o = _brute_force_cvar(list(L), alpha)
        ka, nt = oracle.tail_size(alpha, M)
        got = oracle.cvar(L, alpha)
        if n_o == nt:
            assert got == pytest.approx(lit, rel=1e-12, abs=1e-12)
        else:
            n_differ += 1
            assert n_o > nt
            assert (got * nt + (n_o - nt) * var) / n_o == pytest.approx(lit, rel=1e-12, abs=1e-12)
    assert n_differ > 50
    # the structural case of impulse disturbances: draws with no jump follow
    # one trajectory and tie; one jumped draw above 15 tied ones (M = 16,
    # alpha = 0.9: k_alpha = 15, n_tail = 2)
    L = np.array([4.0] * 15 + [10.0])
    lit, var, n_o = _brute_force_cvar(list(L), 0.9)
    assert (var, n_o) == (4.0, 16) and lit == pytest.approx((10.0 + 15 * 4.0) / 16)
    assert oracle.cvar(L, 0.9) == pytest.approx((10.0 + 4.0) / 2)


@pytest.mark.parametrize("alpha,const", [(0.7, 1.1589753807), (0.9, 1.7549833193), (0.95, 2.0627128075)])
def test_gaussian_closed_form(alpha, const):
    # CVaR_alpha of N(mu, sigma^2) = mu + sigma phi(Phi^-1(alpha)) / (1 - alpha)
    assert stats.norm.pdf(stats.norm.ppf(alpha)) / (1 - alpha) == pytest.approx(const, abs=1e-9)
    mu, sigma = 4.0, 2.5
    rng = np.random.default_rng(3)
    n, nb = 1_000_000, 20
    L = rng.normal(mu, sigma, size=n)
    full = oracle.cvar(L, alpha)
    batches = np.array([oracle.cvar(b, alpha) for b in L.reshape(nb, -1)])
    se = batches.std(ddof=1) / np.sqrt(nb)
    assert abs(full - (mu + sigma * const)) < 3 * se, (full, mu + sigma * const, se)


@pytest.mark.parametrize("B", [0.5, 1.0, 2.0, 7.5])
def test_scaling_is_affine(B):
    rng = np.random.default_rng(4)
    for M in (4, 16, 64, 300):
        L = rng.gamma(2.0, 3.0, size=M)
        mean = L.mean()
        for alpha in (0.3, 0.9):
            got = oracle.cvar(L, alpha, B)
            ref = mean + B * (oracle.cvar(L, alpha, 1.0) - mean)
            assert got == pytest.approx(ref, rel=1e-12, abs=1e-12)
    La = oracle.scale_risk(L, B)
    assert La.mean() == pytest.approx(L.mean(), rel=1e-12)
    assert La.std() == pytest.approx(B * L.std(), rel=1e-12)


def test_invariants():
    rng = np.random.default_rng(5)
    for _ in range(50):
        M = int(rng.integers(2, 200))
        L = rng.lognormal(1.0, 1.0, size=M)
        c = oracle.cvar(L, 0.9)
        assert L.mean() - 1e-12 <= c <= L.max()
        assert oracle.cvar(rng.permutation(L), 0.9) == c
        cs = [oracle.cvar(L, a) for a in np.linspace(0.01, 0.99, 25)]
        assert np.all(np.diff(cs) >= -1e-12)


def test_batch_matches_single():
    rng = np.random.default_rng(6)
    L = rng.normal(size=(9, 33))
    out = oracle.cvar_batch(L, 0.8, 1.0)
    for k in range(9):
        assert out[k] == oracle.cvar(L[k], 0.8)


def test_filtered_cost():
    # Eq. 14-16: J_C = A CVaR if CVaR > C_u (strict), else 0
    assert oracle.filtered_cost(3.0, 2.0, 10.0, 1.0) == 23.0
    assert oracle.filtered_cost(3.0, 1.0, 10.0, 1.0) == 3.0
    assert oracle.filtered_cost(3.0, 0.5, 10.0, 1.0) == 3.0
    assert oracle.filtered_cost(3.0, 2.0, 0.0, 1.0) == 3.0


def test_paper_preset_matches_the_printed_setup():
    from paper_2209_12842_amd import workloads as W
    g = json.load(open(os.path.join(HERE, "golden", "paper_controller_setup.json")))
    p = W.PRESETS["p0"]
    assert p["T"] == g["horizon_T"] and p["K"] == g["samples_K"] and p["M"] == g["draws_M"]
    assert p["K"] * p["M"] == g["total_disturbed_trajectories"]
    assert p["lam"] == g["lambda"] and p["eta"] == g["eta"] and p["A"] == g["A"]
    assert (p["c_bdry"], p["c_obs"], p["c_dev"]) == (g["c1_boundary"], g["c2_obstacle"], g["c3_deviation"])
    assert (p["c4"], p["c5"]) == (g["c4_terminal"], g["c5_terminal"])
    assert p["alpha"] in g["alpha_grid_examples"] and p["C_u"] in g["C_u_examples"]
    assert 2 * p["track"][4] == pytest.approx(g["track_width_m"])
    # the elliptic stand-in for the paper's track has about its centreline length
    a, b = p["track"][2], p["track"][3]
    from scipy.special import ellipe
    perim = 4 * a * ellipe(1 - (b / a) ** 2)
    assert perim == pytest.approx(g["centreline_length_m"], rel=0.01)
    w = W.make_world("p0")
    assert w["obstacles"].shape == (g["n_obstacles"], 3)
    assert np.allclose(w["obstacles"][:, 2], g["obstacle_radius_m"])
