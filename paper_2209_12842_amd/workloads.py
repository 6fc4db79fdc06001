"""Seeded synthetic workloads for the RA-MPPI control step.

This module only generates inputs: parameter presets, obstacle tables, the
initial state and the initial mean control sequence.  It holds none of the
method's arithmetic, and both the device path and the FP64 oracle take their
inputs from here.

The paper measured on its own race track and car; no track file, vehicle log
or dataset exists here.  These worlds stand in for that workload and keep its
shape: circular obstacles scattered along a closed track (the paper uses 10
obstacles on a 0.6 m track with a 10.9 m centreline), Gaussian state
disturbances, and 1e5-5e5 disturbed trajectories per control step.

Presets (sizes in the notation K samples, T horizon steps, M draws per sample):
  c1   K=256,   T=20,  M=16,  10 obstacles, small 40 x 40 m world
  c2   K=2048,  T=50,  M=64,  50 obstacles along a 100 x 40 m oval, receding horizon
  c3   K=16384, T=100, M=128, 200 obstacles along the c2 oval (largest plain step)
  c4   K=4096,  T=50,  M=64,  50 obstacles (the differentiation workload)
  p0   the paper's own controller settings (T=30, K=1024, M=300, lambda=0.35,
       eta=0.2, A=10, alpha=0.9, C_u=0.5, running-cost weights 2 / 1 / 0.1,
       terminal weights 0.6 / 2) on a 0.6 m wide oval with a 10.9 m centreline
  make_batch  64 controllers of uneven size (K multiple of 256 up to 8192,
       T 20-100, M 8-128, 10-200 obstacles) for batched serving
All floating values are rounded to float32 by both consumers.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Settings shared by c1-c4 (the paper fixes none of these numbers for a
# kinematic bicycle; they are the synthetic workloads' own recipe).
COMMON = dict(
    dt=0.05, wheelbase=2.5,
    u_lo=(-3.0, -0.5), u_hi=(3.0, 0.5),
    sigma_eps=(1.0, 0.1),                   # control-noise variances (accel, steer)
    sigma_w=(0.01, 0.01, 0.002, 0.05),      # state-disturbance variances (x, y, psi, v)
    alpha=0.9, eta=0.0, A=10.0, B=1.0, C_u=0.0,
    c_bdry=0.0, c_obs=1.0e4, c_dev=1.0, c_v=1.0, c4=0.0, c5=0.0,
    shift=False,
)

SEED_BASE = 0x5EED0000


def _preset(config_id: int, **kw) -> dict:
    p = copy.deepcopy(COMMON)
    p.update(kw)
    p["gamma"] = kw.get("gamma", p["lam"])  # gamma = lambda (classic MPPI weighting)
    p["seed"] = SEED_BASE + config_id
    p["config_id"] = config_id
    return p


PRESETS = {
    "c1": _preset(1, K=256, T=20, M=16, lam=1.0, v_ref=5.0, track=(0.0, 0.0, 15.0, 10.0, 3.0)),
    "c2": _preset(2, K=2048, T=50, M=64, lam=0.5, v_ref=8.0, track=(0.0, 0.0, 50.0, 20.0, 3.0), shift=True),
    "c3": _preset(3, K=16384, T=100, M=128, lam=1.0, v_ref=8.0, track=(0.0, 0.0, 50.0, 20.0, 3.0)),
    "c4": _preset(4, K=4096, T=50, M=64, lam=0.5, v_ref=8.0, track=(0.0, 0.0, 50.0, 20.0, 3.0)),
    "p0": _preset(0, K=1024, T=30, M=300, lam=0.35, eta=0.2, A=10.0, alpha=0.9, C_u=0.5,
                  c_bdry=2.0, c_obs=1.0, c_dev=0.1, c_v=0.0, v_ref=0.0, c4=0.6, c5=2.0,
                  wheelbase=0.1, track=(0.0, 0.0, 2.27, 1.1, 0.3),
                  sigma_w=(1.0e-4, 1.0e-4, 2.0e-5, 5.0e-4)),
}

WORLD = {
    "c1": dict(world_seed=1, n_obs=10, kind="box", x0=(15.0, 0.0, math.pi / 2, 5.0)),
    "c2": dict(world_seed=2, n_obs=50, kind="oval", x0=(50.0, 0.0, math.pi / 2, 5.0),
               lateral=3.0, r=(0.5, 1.5), clear_ahead=15.0),
    "c3": dict(world_seed=3, n_obs=200, kind="oval", x0=(50.0, 0.0, math.pi / 2, 5.0),
               lateral=3.0, r=(0.5, 1.5), clear_ahead=15.0),
    "c4": dict(world_seed=4, n_obs=50, kind="oval", x0=(50.0, 0.0, math.pi / 2, 5.0),
               lateral=3.0, r=(0.5, 1.5), clear_ahead=15.0),
    "p0": dict(world_seed=10, n_obs=10, kind="oval", x0=(2.27, 0.0, math.pi / 2, 1.5),
               lateral=0.2, r=(0.1, 0.1), clear_ahead=1.0),
}


def _seg_dist(px, py, ax, ay, bx, by) -> float:
    vx, vy = bx - ax, by - ay
    t = max(0.0, min(1.0, ((px - ax) * vx + (py - ay) * vy) / (vx * vx + vy * vy)))
    return math.hypot(px - (ax + t * vx), py - (ay + t * vy))


def _arc_length(a: float, b: float, th0: float, th1: float, n: int = 2048) -> float:
    """Arc length of the ellipse (a cos th, b sin th) from th0 to th1 >= th0."""
    th = np.linspace(th0, th1, n + 1)
    sp = np.sqrt((a * np.sin(th)) ** 2 + (b * np.cos(th)) ** 2)
    return float(np.trapezoid(sp, th))


def _box_obstacles(rng, n, x0) -> np.ndarray:
    """Radii U[0.5, 1.5] m, centres uniform in [-20, 20]^2; discs that come
    within 2 m of the first 10 m of the start heading ray are redrawn."""
    ax, ay, psi = x0[0], x0[1], x0[2]
    bx, by = ax + 10.0 * math.cos(psi), ay + 10.0 * math.sin(psi)
    out = []
    while len(out) < n:
        r = rng.uniform(0.5, 1.5)
        cx, cy = rng.uniform(-20.0, 20.0, size=2)
        if _seg_dist(cx, cy, ax, ay, bx, by) - r < 2.0:
            continue
        out.append((cx, cy, r))
    return np.asarray(out, dtype=np.float32)


def _oval_obstacles(rng, n, x0, track, lateral, rr, clear_ahead) -> np.ndarray:
    """Centreline parameter U[0, 2 pi), lateral offset U[-lateral, lateral]
    along the outward normal, radius U[rr]; obstacles less than `clear_ahead`
    metres of arc ahead of the start, or whose disc covers the start point,
    are redrawn."""
    ox, oy, a, b = track[0], track[1], track[2], track[3]
    th_start = math.atan2((x0[1] - oy) / b, (x0[0] - ox) / a)
    out = []
    while len(out) < n:
        th = rng.uniform(0.0, 2.0 * math.pi)
        off = rng.uniform(-lateral, lateral)
        r = rng.uniform(rr[0], rr[1]) if rr[1] > rr[0] else rr[0]
        dth = (th - th_start) % (2.0 * math.pi)
        if _arc_length(a, b, th_start, th_start + dth) < clear_ahead:
            continue
        px, py = ox + a * math.cos(th), oy + b * math.sin(th)
        nx, ny = math.cos(th) / a, math.sin(th) / b
        nn = math.hypot(nx, ny)
        cx, cy = px + off * nx / nn, py + off * ny / nn
        if math.hypot(cx - x0[0], cy - x0[1]) < r + 0.5 * lateral:
            continue
        out.append((cx, cy, r))
    return np.asarray(out, dtype=np.float32)


def make_world(name: str, **overrides) -> dict:
    """Parameters, obstacles (n x 3: cx, cy, r), x0 (4) and V0 (T x 2 zeros).

    `overrides` replace preset entries (e.g. K, M, sigma_w); the obstacle table
    and start state depend only on the world recipe and its seed."""
    p = copy.deepcopy(PRESETS[name])
    w = WORLD[name]
    p.update(overrides)
    if "lam" in overrides and "gamma" not in overrides:
        p["gamma"] = p["lam"]
    rng = np.random.default_rng(w["world_seed"])
    x0 = np.asarray(w["x0"], dtype=np.float32)
    n_obs = int(overrides.get("n_obs", w["n_obs"]))
    if w["kind"] == "box":
        obs = _box_obstacles(rng, n_obs, w["x0"])
    else:
        obs = _oval_obstacles(rng, n_obs, w["x0"], p["track"], w["lateral"], w["r"], w["clear_ahead"])
    obs = obs.reshape(-1, 3)
    V0 = np.zeros((int(p["T"]), 2), dtype=np.float32)
    return dict(name=name, params=p, obstacles=obs, x0=x0, V0=V0)


def random_V(T: int, seed: int, scale=(1.0, 0.2)) -> np.ndarray:
    """A non-zero mean sequence for tests: uniform within +-scale."""
    rng = np.random.default_rng(seed)
    V = np.stack([rng.uniform(-scale[0], scale[0], size=T), rng.uniform(-scale[1], scale[1], size=T)], axis=1)
    return V.astype(np.float32)


def plant_noise_counter(j: int) -> tuple[int, int, int, int]:
    """Philox counter of the host plant's disturbance at closed-loop step j."""
    return (0, 0xFFFFFFFE, 0xFFFFFFFF, j & 0xFFFFFFFF)


def make_batch(n: int = 64, seed: int = 5, k_range=(256, 8192), t_range=(20, 100), m_range=(8, 128),
               obs_range=(10, 200)) -> list[dict]:
    """Worlds of n independent controllers of uneven size (batched serving):
    K a multiple of 256 in k_range, T in t_range, M in m_range and n_obs in
    obs_range, each uniform; every controller drives its own obstacle field on
    the 100 x 40 m oval from its own start angle, with its own Philox key."""
    rng = np.random.default_rng(seed)
    worlds = []
    for i in range(n):
        K = 256 * int(rng.integers(k_range[0] // 256, k_range[1] // 256 + 1))
        T = int(rng.integers(t_range[0], t_range[1] + 1))
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        n_obs = int(rng.integers(obs_range[0], obs_range[1] + 1))
        th = float(rng.uniform(0.0, 2.0 * math.pi))
        a, b = 50.0, 20.0
        x0 = (a * math.cos(th), b * math.sin(th),
              math.atan2(b * math.cos(th), -a * math.sin(th)), float(rng.uniform(3.0, 8.0)))
        p = _preset(1000 + i, K=K, T=T, M=M, lam=0.5, v_ref=8.0, track=(0.0, 0.0, a, b, 3.0), shift=True)
        wrng = np.random.default_rng(seed * 1000 + i)
        obs = _oval_obstacles(wrng, n_obs, x0, p["track"], 3.0, (0.5, 1.5), 15.0)
        worlds.append(dict(name="batch%d" % i, params=p, obstacles=obs.reshape(-1, 3),
                           x0=np.asarray(x0, dtype=np.float32), V0=np.zeros((T, 2), dtype=np.float32)))
    return worlds
