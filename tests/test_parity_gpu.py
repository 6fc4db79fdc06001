"""Parity of the HIP path (through the C ABI) with the FP64 oracle on MI355X.

Noise: Philox words bit-exact; Box-Muller normals to FP32 rounding.  Stages:
the CVaR kernel against the oracle's estimator on the same inputs, and
against the Gaussian closed form.  Full step: the flip-aware protocol of
parity_helpers on the small, paper-preset and receding-horizon workloads at
their full sizes, on the largest workload through sampled rollouts and
stage-wise checks, plus invariants, determinism and edge shapes.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2209_12842_amd import workloads as W

from parity_helpers import check_step, gpu_step, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2209_12842_amd as R  # noqa: E402


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _threads():
    oracle.set_threads(min(16, max(1, len(__import__("os").sched_getaffinity(0)))))
    yield


# ------------------------------------------------------------- noise ----

def test_philox_bit_exact():
    rng = np.random.default_rng(0)
    n = 1 << 20
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:64] = np.array([[0, 0, 0, 0], [0xFFFFFFFF] * 4, [0, 0xFFFFFFFF, 0, 0xFFFFFFFF],
                         [0xFFFFFFFF, 0, 0xFFFFFFFF, 0]] * 16, dtype=np.uint32)
    for seed in (0, 0x5EED0003, 0xFFFFFFFFFFFFFFFF, 0x0123456789ABCDEF):
        _log("philox seed %x" % seed)
        g = R.philox(seed, torch.from_numpy(ctr.view(np.int32)).cuda()).cpu().numpy().view(np.uint32)
        o = oracle.philox_batch(ctr, seed)
        assert np.array_equal(g, o)


def test_normals_match_oracle():
    rng = np.random.default_rng(1)
    n = 1 << 18
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    g = R.normals(0x5EED0002, torch.from_numpy(ctr.view(np.int32)).cuda()).cpu().numpy().astype(np.float64)
    o = oracle.normals_batch(ctr, 0x5EED0002)
    err = np.abs(g - o)
    assert err.max() <= 4e-6 * max(1.0, np.abs(o).max()), err.max()
    assert np.median(err) <= 1e-7


# -------------------------------------------------------------- CVaR ----

@pytest.mark.parametrize("K,M,alpha,B", [(1000, 16, 0.9, 1.0), (333, 64, 0.9, 1.0), (77, 128, 0.9, 1.0),
                                         (50, 300, 0.9, 1.0), (9, 1024, 0.5, 1.0), (500, 7, 0.7, 1.0),
                                         (300, 1, 0.9, 1.0), (257, 100, 0.95, 2.0), (64, 16, 0.05, 0.5)])
def test_cvar_stage(K, M, alpha, B):
    rng = np.random.default_rng(K * 1000 + M)
    L = (rng.gamma(2.0, 5.0, size=(K, M)) + rng.integers(0, 3, size=(K, M)) * 1e4).astype(np.float32)
    g = R.cvar(torch.from_numpy(L).cuda(), alpha, B).cpu().numpy().astype(np.float64)
    o = oracle.cvar_batch(L.astype(np.float64), float(np.float32(alpha)), float(np.float32(B)))
    assert np.all(rel_err(g, o) <= 1e-5), rel_err(g, o).max()


@pytest.mark.parametrize("M", [8, 64, 128, 256, 48])
def test_cvar_ties(M):
    # many equal costs: the tail order (larger first, then smaller draw index)
    # is unique, so the sorted path (powers of two, within and across waves)
    # and the rank count (M = 48) pick the oracle's tail; its sum is an exact
    # small integer, so the FP32 mean is the oracle's mean rounded to FP32
    row = np.resize(np.array([1.0, 2.0, 2.0, 2.0, 5.0, 2.0, 2.0, 0.0], dtype=np.float32), M)
    rng = np.random.default_rng(M)
    L = np.stack([rng.permutation(row) for _ in range(40)]).astype(np.float32)
    g = R.cvar(torch.from_numpy(L).cuda(), 0.7).cpu().numpy()
    o = oracle.cvar_batch(L.astype(np.float64), float(np.float32(0.7)))
    assert np.array_equal(g, o.astype(np.float32))


def test_cvar_gaussian_closed_form():
    from scipy import stats
    mu, sigma, alpha = 4.0, 2.5, 0.9
    rng = np.random.default_rng(7)
    K, M = 4000, 1000
    L = rng.normal(mu, sigma, size=(K, M)).astype(np.float32)
    g = R.cvar(torch.from_numpy(L).cuda(), alpha).cpu().numpy().astype(np.float64)
    o = oracle.cvar_batch(L.astype(np.float64), float(np.float32(alpha)))
    assert np.all(rel_err(g, o) <= 1e-5)
    # the per-row estimator at M = 1000 averages the 101 largest of 1000 draws;
    # its mean is within a small bias of the closed form
    ref = mu + sigma * stats.norm.pdf(stats.norm.ppf(alpha)) / (1 - alpha)
    se = g.std(ddof=1) / np.sqrt(K)
    assert abs(g.mean() - ref) < 3 * se + 0.01 * sigma, (g.mean(), ref, se)


# --------------------------------------------------------- full step ----

def _world(name, **kw):
    w = W.make_world(name, **kw)
    return w["params"], w["obstacles"], w["x0"], w["V0"]


# worlds built so that many rollouts cross obstacle edges (the paper preset's
# 0.6 m wide oval with its discs, the dense fields): up to 3 % of the disturbed
# rollouts pass within 1e-3 m of an edge there, against at most about 0.5 %
# on the other workloads
COLLISION_HEAVY = 0.03


def _run(p, obs, x0, V0, step_idx, shift=False, strict=True, allow_zero=False, split=False, tag="",
         max_near_edge=None):
    tag = tag or "%s K=%d T=%d M=%d n_obs=%d" % (p.get("config_id"), p["K"], p["T"], p["M"], len(obs))
    _log("step %s idx=%d split=%d" % (tag, step_idx, split))
    ctl = R.Controller(p, obs, debug=True, allow_zero_noise=allow_zero, split_update=split)
    g = gpu_step(ctl, x0, V0, step_idx)
    o = oracle.step(p, obs, x0, V0, step_idx)
    kw = {} if max_near_edge is None else dict(max_near_edge=max_near_edge)
    rep = check_step(p, g, o, shift=shift, strict_e2e=strict, tag=tag + (" split" if split else ""), **kw)
    _log("  " + ", ".join("%s=%s" % kv for kv in rep.items()))
    ctl.close()
    return g, o, rep


def test_step_c1():
    p, obs, x0, V0 = _world("c1")
    _run(p, obs, x0, V0, 0, tag="c1")
    _run(p, obs, x0, W.random_V(p["T"], 5, scale=(2.0, 0.4)), 3, tag="c1 random V")


def test_step_c2():
    p, obs, x0, V0 = _world("c2")
    _run(p, obs, x0, V0, 0, shift=True, tag="c2 shift")


def test_step_c2_many_weighted_samples():
    # at lambda = 0.5 one sample carries nearly all the weight; a large
    # temperature spreads it over hundreds of samples, so that V+ is a true
    # weighted average (Eq. 4) at the full size
    p, obs, x0, V0 = _world("c2", lam=400.0)
    _, _, rep = _run(p, obs, x0, W.random_V(p["T"], 12, scale=(1.0, 0.2)), 5, shift=True, tag="c2 lambda=400")
    assert rep["n_weighted"] >= 100, rep


def test_step_paper_preset_m128_and_m300():
    p, obs, x0, V0 = _world("p0", M=128)
    _run(p, obs, x0, W.random_V(p["T"], 6, scale=(1.0, 0.3)), 2, tag="p0 M=128", max_near_edge=COLLISION_HEAVY)
    p, obs, x0, V0 = _world("p0")
    _run(p, obs, x0, V0, 1, tag="p0 M=300", max_near_edge=COLLISION_HEAVY)


def test_step_c3_full():
    # the largest workload (K=16384, T=100, M=128, 200 obstacles, 2.1e8
    # disturbed state steps): every sample's S, L, CVaR and S~ and the
    # end-to-end V+ against a complete oracle step
    p, obs, x0, V0 = _world("c3")
    _run(p, obs, x0, V0, 0, tag="c3")


def test_step_c3_full_many_weighted_samples():
    # the same world at a temperature (and control-cost weight gamma = lambda)
    # at which hundreds of samples carry weight
    p, obs, x0, V0 = _world("c3", lam=20000.0)
    _, _, rep = _run(p, obs, x0, W.random_V(p["T"], 13, scale=(1.0, 0.2)), 1, tag="c3 lambda=20000")
    assert rep["n_weighted"] >= 100, rep


def test_closed_loop_c2_steps():
    # receding horizon with shift: each device step is checked against the
    # oracle run from the same state and the same incoming mean sequence
    p, obs, x0, V0 = _world("c2", K=512)
    ctl = R.Controller(p, obs, debug=True)
    V = ctl.new_V(V0)
    x = np.asarray(x0, dtype=np.float64)
    for j in range(4):
        Vin = V.detach().cpu().numpy().copy()
        u0 = ctl.step(x.astype(np.float32), V, j)
        torch.cuda.synchronize()
        d = ctl.debug()
        g = {k: v.detach().cpu().numpy().astype(np.float64) for k, v in d.items()}
        g["u"] = np.transpose(g["u"], (1, 0, 2))
        g["V_next"] = V.detach().cpu().numpy().astype(np.float64)
        g["u0_host"] = u0.astype(np.float64)
        o = oracle.step(p, obs, x.astype(np.float32), Vin, j)
        rep = check_step(p, g, o, shift=True, tag="c2 K=512 closed loop %d" % j)
        _log("  loop %d: %s" % (j, rep))
        # host plant: the nominal model plus a Philox disturbance
        z = oracle.normals4(W.plant_noise_counter(j), p["seed"])
        x = oracle.dynamics(x, u0.astype(np.float64), float(np.float32(p["dt"])),
                            float(np.float32(p["wheelbase"])))
        x = x + np.sqrt(np.float32(p["sigma_w"]).astype(np.float64)) * z
    ctl.close()


def test_determinism():
    p, obs, x0, V0 = _world("c1")
    ctl = R.Controller(p, obs, debug=True)
    a = gpu_step(ctl, x0, V0, 4)
    b = gpu_step(ctl, x0, V0, 4)
    for k in ("S", "L", "cvar", "S_tilde", "w_hat", "V_next", "u"):
        assert np.array_equal(a[k], b[k]), k
    c = gpu_step(ctl, x0, V0, 5)
    assert not np.array_equal(a["L"], c["L"])
    ctl.close()


def test_zero_disturbance_matches_nominal_on_device():
    p, obs, x0, V0 = _world("c1", sigma_w=(0.0, 0.0, 0.0, 0.0), gamma=0.0)
    ctl = R.Controller(p, obs, debug=True)
    g = gpu_step(ctl, x0, V0, 0)
    assert np.all(rel_err(g["L"], g["S"][:, None]) <= 1e-6)
    frac_exact = float((g["L"] == g["S"][:, None]).mean())
    _log("bitwise-equal fraction %.4f" % frac_exact)
    assert np.all(rel_err(g["cvar"], g["S"]) <= 1e-6)
    ctl.close()


def test_zero_control_noise_returns_clamped_mean_on_device():
    p, obs, x0, _ = _world("c1", sigma_eps=(0.0, 0.0), gamma=0.0)
    V0 = W.random_V(p["T"], 9, scale=(4.0, 0.8))
    ctl = R.Controller(p, obs, debug=True, allow_zero_noise=True)
    g = gpu_step(ctl, x0, V0, 0)
    Vc = np.clip(V0.astype(np.float64), p["u_lo"], p["u_hi"])
    assert np.abs(g["V_next"] - Vc).max() <= 1e-6
    ctl.close()


def test_plain_mppi_ignores_disturbances_on_device():
    p, obs, x0, V0 = _world("c1", A=0.0)
    a = gpu_step(R.Controller(p, obs, debug=True), x0, V0, 2)
    b = gpu_step(R.Controller(dict(p, M=32, sigma_w=(0.5, 0.5, 0.1, 1.0)), obs, debug=True), x0, V0, 2)
    assert np.array_equal(a["V_next"], b["V_next"])
    assert np.array_equal(a["S_tilde"], a["S"])


@pytest.mark.parametrize("kw", [dict(K=1, M=1, T=1), dict(K=257, M=16, T=7), dict(K=33, M=7, T=5),
                                dict(K=20, M=300, T=6), dict(K=5, M=1024, T=4), dict(K=300, M=64, T=3, n_obs=0),
                                dict(K=64, M=16, T=9, eta=0.5, B=3.0, C_u=60.0, lam=20.0),
                                dict(K=600, M=64, T=300, lam=50.0)])
@pytest.mark.parametrize("split", [False, True], ids=["one-launch", "split"])
def test_edge_shapes(kw, split):
    kw = dict(kw)
    n_obs = kw.pop("n_obs", None)
    p, obs, x0, _ = _world("c1", **kw)
    if n_obs is not None:
        obs = obs[:n_obs]
    V0 = W.random_V(p["T"], 3, scale=(1.0, 0.2))
    _run(p, obs, x0, V0, 1, split=split, tag="edge %s" % ",".join("%s=%s" % kv for kv in sorted(kw.items())))


def _dense_obstacles(n, seed, x0, r=(0.1, 0.5)):
    """n discs scattered around x0 over a square of half side
    max(25, 25 sqrt(n / 300)) m (the first one on the start heading, 4 m
    ahead, radius 0.6 m), so that many rollouts end up inside discs."""
    half = max(25.0, 25.0 * np.sqrt(n / 300.0))
    rng = np.random.default_rng(seed)
    c = np.asarray(x0[:2], dtype=np.float64) + rng.uniform(-half, half, size=(n, 2))
    rr = rng.uniform(r[0], r[1], size=n)
    c[0] = np.asarray(x0[:2], dtype=np.float64) + 4.0 * np.array([np.cos(x0[2]), np.sin(x0[2])])
    rr[0] = 0.6
    return np.column_stack([c, rr]).astype(np.float32)


@pytest.mark.parametrize("n_obs,M", [(1, 64), (63, 64), (64, 48), (65, 16), (300, 64), (1024, 128), (200, 300)])
def test_dense_obstacle_fields(n_obs, M):
    # obstacle counts when many rollouts pass through discs: every group size
    # of the obstacle table (1, 63, 64, 65, 300, 1024 entries) and waves that
    # hold one sample (M >= 64) or several (M = 16, 48)
    p, _, x0, _ = _world("c1", K=256, M=M, T=30, lam=50.0)
    obs = _dense_obstacles(n_obs, 11 + n_obs, x0)
    V0 = W.random_V(p["T"], 7, scale=(1.0, 0.2))
    g, o, rep = _run(p, obs, x0, V0, 2, strict=False, tag="dense n_obs=%d M=%d" % (n_obs, M),
                     max_near_edge=COLLISION_HEAVY)
    hits = float((o["L"] >= float(np.float32(p["c_obs"]))).mean())
    _log("  fraction of disturbed rollouts with a collision: %.3f" % hits)
    assert hits > 0.02


@pytest.mark.parametrize("name,kw", [("c1", {}), ("c2", {}), ("p0", dict(M=128)), ("c1", dict(K=257, M=48, T=9)),
                                     ("c1", dict(K=700, M=7, T=5, B=2.0, eta=0.3)),
                                     # M > 256: the two-launch step lays its disturbed lanes out as
                                     # 256 consecutive (sample, draw) pairs per workgroup and forms
                                     # the CVaR in a separate pass (ragged: 300 pairs per sample,
                                     # and M = 512 with the sort of power-of-two M)
                                     ("c1", dict(K=300, M=300)), ("c1", dict(K=129, M=512, T=12, B=2.0)),
                                     ("c1", dict(K=70, M=600, T=8, B=0.5))])
def test_one_launch_step_equals_split_update(name, kw):
    # the step as one launch (the update run by the workgroups that finish
    # each chunk) and as two launches give the same bits, over several calls
    # (the chunk and merge counters reset themselves between launches)
    p, obs, x0, _ = _world(name, **kw)
    p = dict(p, shift=True)
    V0 = W.random_V(p["T"], 9, scale=(1.0, 0.2))
    a = R.Controller(p, obs, debug=True)
    b = R.Controller(p, obs, debug=True, split_update=True)
    Va, Vb = a.new_V(V0), b.new_V(V0)
    for j in range(4):
        ua = a.step(x0, Va, 3 + j)
        ub = b.step(x0, Vb, 3 + j)
        torch.cuda.synchronize()
        assert np.array_equal(ua, ub)
        assert torch.equal(Va, Vb)
        da, db = a.debug(), b.debug()
        for k in ("u", "S", "L", "cvar", "S_tilde", "w_hat", "u0"):
            assert torch.equal(da[k], db[k]), (j, k)
    a.close()
    b.close()


@pytest.mark.parametrize("name,kw", [("c2", {}), ("c2", dict(lam=50.0)), ("c2", dict(lam=1.0e4, K=1000)),
                                     ("c1", dict(K=700, M=7, T=5, B=2.0, eta=0.3, lam=1.0e4))])
def test_steps_without_stored_controls(name, kw):
    # without the debug flag no step stores its sampled controls: the chunk
    # updates draw the controls of the weighted samples again; V+ and the
    # first command of the one-launch and the two-launch step equal those of
    # the two-launch step in debug mode (which stores the controls and reads
    # them), also when every weight is non-zero (large lambda)
    p, obs, x0, _ = _world(name, **kw)
    p = dict(p, shift=True)
    V0 = W.random_V(p["T"], 5, scale=(1.0, 0.2))
    a = R.Controller(p, obs)
    b = R.Controller(p, obs, split_update=True)
    c = R.Controller(p, obs, split_update=True, debug=True)
    Va, Vb, Vc = a.new_V(V0), b.new_V(V0), c.new_V(V0)
    for j in range(3):
        ua = a.step(x0, Va, 11 + j, want_u0=True)
        ub = b.step(x0, Vb, 11 + j, want_u0=True)
        uc = c.step(x0, Vc, 11 + j, want_u0=True)
        torch.cuda.synchronize()
        assert np.array_equal(ua, uc) and np.array_equal(ub, uc), (j, ua, ub, uc)
        assert torch.equal(Va, Vc) and torch.equal(Vb, Vc), j
    a.close()
    b.close()
    c.close()


@pytest.mark.parametrize("turns", [0, 17, -160])
def test_start_heading_far_from_zero(turns):
    # the same start heading plus whole turns: beyond 100 rad the library
    # reduces it modulo 2 pi before the rollouts (the hardware sine and cosine
    # then see small arguments); the oracle takes it as given in FP64
    p, obs, x0, V0 = _world("c1")
    x0 = np.array(x0, dtype=np.float32)
    x0[2] = np.float32(float(x0[2]) + 2.0 * np.pi * turns)
    _run(p, obs, x0, V0, 1, tag="c1 heading %+d turns (%.4f rad)" % (turns, float(x0[2])))


def test_shift_and_first_command():
    p, obs, x0, V0 = _world("c1", shift=True)
    g, o, rep = _run(p, obs, x0, V0, 0, shift=True, tag="c1 shift")
    assert np.abs(g["u0_host"] - o["u0"]).max() <= 1e-3


@pytest.mark.parametrize("name,kw", [("c1", dict(noise_kind=1)),
                                     ("c1", dict(noise_kind=2, jump_prob=0.02, jump_size=0.45)),
                                     ("c2", dict(noise_kind=2, jump_prob=0.02, jump_size=0.45, K=512)),
                                     ("p0", dict(noise_kind=1, M=64, K=256))])
def test_step_disturbance_forms(name, kw):
    # the paper's uniform and impulse disturbances (robustness experiments)
    p, obs, x0, V0 = _world(name, **kw)
    _run(p, obs, x0, W.random_V(p["T"], 8, scale=(1.0, 0.2)), 1, shift=bool(p.get("shift")),
         tag="%s noise_kind=%d" % (name, kw["noise_kind"]), max_near_edge=COLLISION_HEAVY if name == "p0" else None)


def test_disturbance_forms_stage_parity():
    # the disturbed rollouts of a controller with zero control noise are pure
    # functions of the disturbance draws: compare L against the oracle draw by draw
    for kw in (dict(noise_kind=1), dict(noise_kind=2, jump_prob=0.3, jump_size=0.45)):
        p, obs, x0, V0 = _world("c1", K=32, M=16, T=12, sigma_eps=(0.0, 0.0), gamma=0.0, **kw)
        ctl = R.Controller(p, obs, debug=True, allow_zero_noise=True)
        g = gpu_step(ctl, x0, V0, 3)
        o = oracle.step(p, obs, x0, V0, 3)
        ok = (o["obs_margin"] >= 1e-3) & (o["obs_cond"] >= 0.25)
        assert np.all(rel_err(g["L"], o["L"])[ok] <= 1e-4)
        ctl.close()
