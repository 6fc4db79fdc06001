"""Pins of the oracle's disturbance forms (Eq. 6-7 with the forms of the
paper's robustness experiments: Gaussian, uniform, impulse).

Every form must be zero-mean (Eq. 7: the nominal model is the mean of the
disturbed one).  Gaussian: covariance Sigma_w.  Uniform: support [-h, h] with
h = sqrt(3 Sigma_w) and the same covariance.  Impulse: a jump of exactly the
given length with the given probability, in a uniformly random planar
direction, and nothing on the heading and speed.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2209_12842_amd import workloads as W

N = 1 << 17


def _ctr(n=N):
    c = np.zeros((n, 4), dtype=np.uint32)
    c[:, 0] = np.arange(n) % 64
    c[:, 1] = np.arange(n) // 64
    c[:, 2] = 5
    c[:, 3] = 9
    return c


def _p(**kw):
    p = dict(W.PRESETS["c1"])
    p.update(kw)
    return p


def test_gaussian_form_matches_the_scaled_normals():
    p = _p(noise_kind=0)
    w = oracle.disturbance_batch(p, _ctr(1000))
    z = oracle.normals_batch(_ctr(1000), p["seed"])
    sw = np.sqrt(np.float32(p["sigma_w"]).astype(np.float64))
    np.testing.assert_allclose(w, z * sw, rtol=0, atol=1e-15)


def test_uniform_form_support_and_moments():
    var = np.float32(W.PRESETS["c1"]["sigma_w"]).astype(np.float64)
    w = oracle.disturbance_batch(_p(noise_kind=1), _ctr())
    h = np.sqrt(3 * var)
    assert np.all(np.abs(w) < h)
    assert np.all(np.abs(w.mean(axis=0)) < 5 * np.sqrt(var / N))
    np.testing.assert_allclose(w.var(axis=0), var, rtol=0.02)
    for i in range(4):
        assert stats.kstest(w[:, i], "uniform", args=(-h[i], 2 * h[i])).pvalue > 1e-4


@pytest.mark.parametrize("prob,size", [(0.02, 0.45), (0.3, 1.5)])
def test_impulse_form(prob, size):
    w = oracle.disturbance_batch(_p(noise_kind=2, jump_prob=prob, jump_size=size), _ctr())
    jumped = np.any(w != 0.0, axis=1)
    frac = jumped.mean()
    assert abs(frac - prob) < 5 * math.sqrt(prob * (1 - prob) / N)
    size32 = float(np.float32(size))
    np.testing.assert_allclose(np.hypot(w[jumped, 0], w[jumped, 1]), size32, rtol=1e-12)
    assert np.all(w[:, 2:] == 0.0)
    ang = np.arctan2(w[jumped, 1], w[jumped, 0])
    assert stats.kstest(ang, "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-4
    # zero mean (Eq. 7)
    se = size32 * math.sqrt(prob / N)
    assert np.all(np.abs(w[:, :2].mean(axis=0)) < 5 * se)


def test_no_jump_and_zero_width_reproduce_the_nominal_cost():
    for kw in (dict(noise_kind=2, jump_prob=0.0, jump_size=0.45), dict(noise_kind=1, sigma_w=(0, 0, 0, 0))):
        w = W.make_world("c1", K=8, T=10, M=6, gamma=0.0, **kw)
        r = oracle.step(w["params"], w["obstacles"], w["x0"], w["V0"], 0)
        assert np.all(r["L"] == r["S"][:, None])


def test_forms_change_only_the_risk_costs():
    w = W.make_world("c1", K=16, T=10, M=8)
    base = oracle.step(w["params"], w["obstacles"], w["x0"], w["V0"], 2)
    for kw in (dict(noise_kind=1), dict(noise_kind=2, jump_prob=0.2, jump_size=0.45)):
        r = oracle.step(dict(w["params"], **kw), w["obstacles"], w["x0"], w["V0"], 2)
        assert np.array_equal(r["S"], base["S"]) and np.array_equal(r["u"], base["u"])
        assert not np.array_equal(r["L"], base["L"])
