"""Pins of the oracle's noise: Philox4x32-10 and the Box-Muller transform.

The paper names no generator; the reading is Philox4x32-10 (Salmon et al.,
SC'11) with Box-Muller normals.  No known-answer vectors are available here,
so the generator is pinned by (a) special counters that expose the round
structure, the multipliers and the Weyl key schedule, with the Weyl constants
derived from their mathematical definitions, (b) mixing (avalanche) and
distribution statistics, and (c) closed-form Box-Muller values and moments.
"""
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

import oracle

M0_PUBLISHED = 0xD2511F53   # Philox4x32 multipliers as published with the generator (Salmon et al. 2011)
M1_PUBLISHED = 0xCD9E8D57


def _weyl_constants():
    """floor(2^32 * (golden ratio - 1)) and floor(2^32 * (sqrt(3) - 1))."""
    getcontext().prec = 60
    phi_frac = (Decimal(5).sqrt() - 1) / 2
    s3_frac = Decimal(3).sqrt() - 1
    return int(phi_frac * (1 << 32)), int(s3_frac * (1 << 32))


def test_weyl_constants_from_definition():
    w0, w1 = _weyl_constants()
    consts = oracle.philox_constants()
    assert consts[2] == w0
    assert consts[3] == w1
    assert consts[0] == M0_PUBLISHED and consts[1] == M1_PUBLISHED


def test_one_round_exposes_multipliers_and_word_order():
    # counter (1, 0, 1, 0), key 0: the products are the multipliers themselves
    # (high words 0), so one round returns (0, M1, 0, M0).
    out = oracle.philox([1, 0, 1, 0], [0, 0], rounds=1)
    assert list(out) == [0, M1_PUBLISHED, 0, M0_PUBLISHED]


def test_one_round_xors_key_into_the_right_words():
    rng = np.random.default_rng(0)
    for _ in range(20):
        c1, c3, k0, k1 = (int(v) for v in rng.integers(0, 2**32, size=4, dtype=np.uint64))
        out = oracle.philox([0, c1, 0, c3], [k0, k1], rounds=1)
        assert list(out) == [c1 ^ k0, 0, c3 ^ k1, 0]


def test_two_rounds_expose_the_key_schedule():
    # With counter (0, k0, 0, k1) the first round returns all zeros, so the
    # second round returns (k0 + W0, 0, k1 + W1, 0).
    w0, w1 = _weyl_constants()
    rng = np.random.default_rng(1)
    for _ in range(20):
        k0, k1 = (int(v) for v in rng.integers(0, 2**32, size=2, dtype=np.uint64))
        out = oracle.philox([0, k0, 0, k1], [k0, k1], rounds=2)
        assert list(out) == [(k0 + w0) & 0xFFFFFFFF, 0, (k1 + w1) & 0xFFFFFFFF, 0]


def test_batch_is_ten_rounds():
    rng = np.random.default_rng(2)
    ctr = rng.integers(0, 2**32, size=(16, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x0123456789ABCDEF
    key = [seed & 0xFFFFFFFF, seed >> 32]
    out = oracle.philox_batch(ctr, seed)
    for i in range(16):
        assert np.array_equal(out[i], oracle.philox(ctr[i], key, rounds=10))
        assert not np.array_equal(out[i], oracle.philox(ctr[i], key, rounds=9))


def _popcount(a: np.ndarray) -> np.ndarray:
    a = a.astype(np.uint64)
    c = np.zeros(a.shape, dtype=np.int64)
    for b in range(32):
        c += ((a >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return c


def test_avalanche():
    # flipping any single counter or key bit changes each output bit with
    # probability 1/2 (10 rounds are far past full diffusion)
    rng = np.random.default_rng(3)
    n = 200
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x5EED0003
    base = oracle.philox_batch(ctr, seed)
    dist = []
    for word in range(4):
        for bit in range(0, 32, 3):
            c2 = ctr.copy()
            c2[:, word] ^= np.uint32(1 << bit)
            out = oracle.philox_batch(c2, seed)
            dist.append(_popcount(out ^ base).sum(axis=1))
    for bit in (0, 17, 31, 40, 63):
        out = oracle.philox_batch(ctr, seed ^ (1 << bit))
        dist.append(_popcount(out ^ base).sum(axis=1))
    d = np.concatenate(dist).astype(np.float64)
    # 128 output bits, Binomial(128, 1/2): mean 64, sd 5.66
    assert abs(d.mean() - 64.0) < 0.3
    assert abs(d.std() - np.sqrt(32.0)) < 0.3


def test_uniform_words_statistics():
    n = 1 << 18
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint32)
    ctr[:, 1] = 7
    ctr[:, 2] = 12345
    ctr[:, 3] = 3
    out = oracle.philox_batch(ctr, 0x5EED0001)
    # distinct outputs for distinct counters (a bijection for a fixed key)
    flat = out.view(np.dtype([("a", "<u4"), ("b", "<u4"), ("c", "<u4"), ("d", "<u4")])).ravel()
    assert np.unique(flat).size == n
    # byte histogram chi-square, each of the 4 words
    for w in range(4):
        bytes_ = np.ascontiguousarray(out[:, w]).view(np.uint8)
        hist = np.bincount(bytes_, minlength=256)
        chi2, p = stats.chisquare(hist)
        assert p > 1e-4, (w, p)
    # each of the 128 bit positions is balanced
    for w in range(4):
        for b in range(32):
            frac = ((out[:, w] >> np.uint32(b)) & 1).mean()
            assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(n)
    # no lag-1 correlation between consecutive counters
    u = out[:, 0].astype(np.float64) / 2**32
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5 / np.sqrt(n)


def test_uniform_mapping_endpoints_and_exactness():
    assert oracle.uniform(0) == 2.0 ** -24
    assert oracle.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert oracle.uniform(0x80000000) == 0.5 + 2.0 ** -24
    rng = np.random.default_rng(4)
    for r in rng.integers(0, 2**32, size=2000, dtype=np.uint64):
        u = oracle.uniform(int(r))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u  # exactly representable in float32


def test_box_muller_closed_form():
    # u0 = exp(-1/2) gives radius 1; u1 = 1/8 is the angle pi/4
    z0, z1 = oracle.box_muller(np.exp(-0.5), 0.125)
    assert z0 == pytest.approx(np.sqrt(0.5), abs=1e-15)
    assert z1 == pytest.approx(np.sqrt(0.5), abs=1e-15)
    # u0 = exp(-2) gives radius 2; u1 = 1/2 is the angle pi
    z0, z1 = oracle.box_muller(np.exp(-2.0), 0.5)
    assert z0 == pytest.approx(-2.0, abs=1e-14)
    assert z1 == pytest.approx(0.0, abs=1e-14)


def test_normals4_uses_the_philox_words_in_order():
    ctr = [5, 9, 11, 13]
    seed = 0x5EED0002
    r = oracle.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32])
    z = oracle.normals4(ctr, seed)
    a = oracle.box_muller(oracle.uniform(int(r[0])), oracle.uniform(int(r[1])))
    b = oracle.box_muller(oracle.uniform(int(r[2])), oracle.uniform(int(r[3])))
    assert list(z) == [a[0], a[1], b[0], b[1]]


def test_normals_distribution():
    n = 1 << 17
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n) % 100
    ctr[:, 1] = np.arange(n) // 100
    ctr[:, 2] = 77
    ctr[:, 3] = 1
    z = oracle.normals_batch(ctr, 0x5EED0001)
    flat = z.ravel()
    N = flat.size
    assert abs(flat.mean()) < 5 / np.sqrt(N)
    assert abs(flat.var() - 1.0) < 5 * np.sqrt(2.0 / N)
    # fourth moment of N(0, 1) is 3
    assert abs((flat ** 4).mean() - 3.0) < 5 * np.sqrt(96.0 / N)
    for col in range(4):
        assert stats.kstest(z[:, col], "norm").pvalue > 1e-4
    # the four normals of one counter are uncorrelated
    c = np.corrcoef(z.T)
    off = c[~np.eye(4, dtype=bool)]
    assert np.all(np.abs(off) < 5 / np.sqrt(n))
