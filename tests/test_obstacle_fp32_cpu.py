"""FP32 error band of the device's obstacle test (Eq. 22) against the 1e-3 m
margin of the parity protocol (CPU only).

The device decides "inside a disc" in the frame centred on the start
position with the expanded form |p|^2 - 2 c.p < r^2 - |c|^2: the table holds
(-2 cx, -2 cy, r^2 - |c|^2), each point's |p|^2 is one fused multiply-add,
and the test is two more.  Its rounding error grows with |c|^2 and |p|^2,
i.e. with the distance from the start, so it is largest on the largest
workload (horizon 100, about 50 m of reach on the 100 m x 40 m oval).  Here
that arithmetic is restated in numpy FP32 (a fused multiply-add is the exact
FP64 product and sum rounded once to FP32) for points placed at known signed
distances from every disc of the large workload's world, and from a disc of
the smallest radius at the farthest reach; the largest distance from an
edge at which the FP32 decision disagrees with the exact one is the decision
band (about 3.2e-4 m at 60 m from the start for a 0.5 m disc, growing about
with the square of the distance).  The FP32 rollout positions themselves
drift from the oracle's FP64 ones; a numpy FP32 Euler integration of the
bicycle at the same horizon measures that drift (about 7e-5 m).  Band plus
drift must stay below half the margin, so that a rollout the protocol keeps
(oracle margin >= 1e-3 m) cannot change its collision count on the device.
"""
import numpy as np

from paper_2209_12842_amd import workloads as W

MARGIN = 1e-3     # the parity protocol's margin (tests/parity_helpers.py)


def fma32(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(np.float32)


def device_inside(px, py, cxw, cyw, r, fx, fy):
    """The device's decision: table entry from the FP32 world disc and frame
    origin, then the two fused multiply-adds against the point's |p|^2."""
    f32 = np.float32
    cx = (f32(cxw) - f32(fx)).astype(f32)
    cy = (f32(cyw) - f32(fy)).astype(f32)
    c2 = fma32(cx, cx, (cy * cy).astype(f32))
    a, b = f32(-2.0) * cx, f32(-2.0) * cy
    z = fma32(r, r, -c2)
    rho = fma32(px, px, (py * py).astype(f32))
    return fma32(a, px, fma32(b, py, rho)) < z


def exact_distance(px, py, cxw, cyw, r, fx, fy):
    """Signed distance of the FP32 point from the disc edge, in FP64 from the
    same FP32 inputs (the frame shift is exact in FP64)."""
    cx = np.float64(np.float32(cxw)) - np.float64(np.float32(fx))
    cy = np.float64(np.float32(cyw)) - np.float64(np.float32(fy))
    return np.hypot(px.astype(np.float64) - cx, py.astype(np.float64) - cy) - np.float64(np.float32(r))


def _band(discs, fx, fy, n=4000, spread=4e-3, seed=0):
    """Largest |signed distance| at which the FP32 decision is wrong, over n
    points per disc within +-spread of its edge."""
    rng = np.random.default_rng(seed)
    worst = 0.0
    wrong = 0
    for cxw, cyw, r in discs:
        th = rng.uniform(0, 2 * np.pi, n)
        d = rng.uniform(-spread, spread, n)
        cx, cy = np.float64(np.float32(cxw)) - fx, np.float64(np.float32(cyw)) - fy
        px = (cx + (r + d) * np.cos(th)).astype(np.float32)
        py = (cy + (r + d) * np.sin(th)).astype(np.float32)
        got = device_inside(px, py, cxw, cyw, np.float32(r), fx, fy)
        ex = exact_distance(px, py, cxw, cyw, r, fx, fy)
        bad = got != (ex < 0)
        wrong += int(bad.sum())
        if bad.any():
            worst = max(worst, float(np.abs(ex[bad]).max()))
    return worst, wrong


def test_expanded_form_error_band_on_the_large_workload():
    w = W.make_world("c3")
    fx, fy = np.float32(w["x0"][0]), np.float32(w["x0"][1])
    obs = w["obstacles"].astype(np.float64)
    # every disc the rollouts can reach (a horizon of 100 steps of 0.05 s at
    # up to about 12 m/s: 60 m from the start), plus the worst case: the
    # smallest radius at 60 m in each quadrant
    far = [(fx + 60.0 * np.cos(a), fy + 60.0 * np.sin(a), 0.5) for a in np.linspace(0, 2 * np.pi, 8, endpoint=False)]
    reach = np.hypot(obs[:, 0] - fx, obs[:, 1] - fy) <= 60.0
    discs = [tuple(o) for o in obs[reach]] + far
    worst, wrong = _band(discs, fx, fy)
    print("discs %d, wrong decisions %d, widest band %.2e m" % (len(discs), wrong, worst))
    assert wrong > 0            # the band exists: the test does probe it
    drift = _euler_drift()
    print("band %.2e m + drift %.2e m against the margin %.0e m" % (worst, drift, MARGIN))
    assert worst + drift <= MARGIN / 2, (worst, drift)


def test_expanded_form_error_band_grows_with_distance():
    # the same disc moved away from the frame origin: the band widens with
    # |c| (the rounding of |c|^2 and |p|^2, over the 2 r slope of the edge),
    # here about with its square
    fx = fy = np.float32(0.0)
    bands = [_band([(d, 0.0, 0.5)], fx, fy, n=20000, spread=2e-3, seed=3)[0] for d in (5.0, 20.0, 60.0)]
    print("bands at 5, 20, 60 m: %s" % bands)
    assert bands[0] < bands[1] < bands[2]
    assert bands[2] <= MARGIN / 2


def _euler_drift():
    """Largest distance between FP32 and FP64 forward-Euler bicycle positions
    with the same controls and disturbances over 100 steps (the large
    workload's horizon, dt = 0.05, speeds near 8 m/s, its disturbance
    variances)."""
    rng = np.random.default_rng(5)
    n, T, dt, wb = 4096, 100, 0.05, 2.5
    sw = np.sqrt(np.array([0.01, 0.01, 0.002, 0.05]))
    a = rng.uniform(-3, 3, (T, n))
    dl = rng.uniform(-0.5, 0.5, (T, n))
    wn = rng.standard_normal((T, 4, n)) * sw[None, :, None]
    x64 = np.zeros((4, n))
    x64[2], x64[3] = np.pi / 2, 8.0
    x32 = x64.astype(np.float32)
    f32 = np.float32
    worst = 0.0
    for t in range(T):
        k64 = np.tan(dl[t]) / wb
        x64 = x64 + np.stack([dt * x64[3] * np.cos(x64[2]), dt * x64[3] * np.sin(x64[2]),
                              dt * x64[3] * k64, dt * a[t]]) + wn[t]
        k32 = (np.tan(dl[t].astype(f32)).astype(f32) / f32(wb)).astype(f32)
        dv = (f32(dt) * x32[3]).astype(f32)
        c, s = np.cos(x32[2]).astype(f32), np.sin(x32[2]).astype(f32)
        x32 = np.stack([fma32(dv, c, x32[0]), fma32(dv, s, x32[1]), fma32(dv, k32, x32[2]),
                        (x32[3] + (f32(dt) * a[t].astype(f32)).astype(f32)).astype(f32)])
        x32 = (x32 + wn[t].astype(f32)).astype(f32)
        worst = max(worst, float(np.hypot(x32[0] - x64[0], x32[1] - x64[1]).max()))
    return worst
