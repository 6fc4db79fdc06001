"""Benchmark of the RA-MPPI control step on one MI355X.

Default workload (c2, the receding-horizon loop): K = 2048 samples, T = 50,
M = 64 draws, 50 obstacles along a 100 m x 40 m oval, alpha = 0.9,
lambda = 0.5, consecutive mppi_step calls with the shifted mean sequence,
the first command read back every step and a host FP64 plant closing the
loop.  Synthetic seeded inputs.  One JSON line on stdout:

  value        rollout-steps/s (K M T per step) over the timed steps
  roofline     the rollout kernel: model FP32 FLOPs per launch / its average
               HIP-event duration on the step's stream, against the FP32
               vector peak
  cpu_baseline the FP64 oracle on a bounded sample of the same workload,
               timed on this host's cores

    python bench.py [--steps K] [--warmup W] [--workload c2|c3|c1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2209_12842_amd import workloads as W  # noqa: E402

PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector peak (256 CU x 256 FLOP/clk x 2.4 GHz)
PEAK_HBM_GBS = 8000.0


def model_flops(p: dict, n_obs: int) -> float:
    """FP32 FLOPs of one rollout launch: 80 + 7 n_obs per disturbed state
    step (K M T of them) and 60 + 7 n_obs per nominal state step (K T)."""
    K, T, M = p["K"], p["T"], p["M"]
    return K * M * T * (80.0 + 7.0 * n_obs) + K * T * (60.0 + 7.0 * n_obs)


def model_bytes(p: dict, n_obs: int) -> float:
    """Algorithmic HBM bytes of one rollout launch: read V and the obstacle
    table, write the K x T x 2 controls, S and CVaR."""
    K, T = p["K"], p["T"]
    return 8.0 * T + 16.0 * n_obs + 8.0 * K * T + 8.0 * K


def plant_step(x, u, dt, wb, w):
    """Host FP64 plant: the nominal bicycle plus an additive disturbance."""
    px, py, psi, v = x
    return [px + dt * v * math.cos(psi) + w[0], py + dt * v * math.sin(psi) + w[1],
            psi + dt * v * math.tan(float(u[1])) / wb + w[2], v + dt * float(u[0]) + w[3]]


def cpu_baseline(world: dict, budget_s: float = 10.0) -> dict:
    """The FP64 oracle as it stands, on every host core: complete control
    steps of the same workload (same world, consecutive step indices) until
    about `budget_s` seconds of work have run."""
    import oracle
    p = world["params"]
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.step(p, world["obstacles"], world["x0"], world["V0"], n, diagnostics=False)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s:
            break
    steps = n * p["K"] * p["M"] * p["T"]
    return {"value": steps / dt, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
            "sample": "%d complete control steps of the workload (K=%d, M=%d, T=%d) in %.1f s, FP64, %d threads"
                      % (n, p["K"], p["M"], p["T"], dt, cores)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy a MIB-sized device buffer 3 times (a plain copy kernel of "
                         "known size for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2209_12842_amd as R

    world = W.make_world(args.workload)
    p = dict(world["params"])
    p["shift"] = True                      # receding horizon: V <- shifted V+
    obs = world["obstacles"]
    n_obs = len(obs)
    K, T, M = p["K"], p["T"], p["M"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctl = R.Controller(p, obs, device=dev)
    V = ctl.new_V(world["V0"])
    dt32, wb32 = float(np.float32(p["dt"])), float(np.float32(p["wheelbase"]))
    sw = np.sqrt(np.float32(p["sigma_w"]).astype(np.float64))
    n_total = args.warmup + args.steps
    plant_w = (np.random.default_rng(12345).standard_normal((n_total, 4)) * sw).tolist()
    x = [float(v) for v in world["x0"]]

    def one_step(j):
        nonlocal x
        u0 = ctl.step(x, V, j, want_u0=True)
        x = plant_step(x, u0, dt32, wb32, plant_w[j])
        return u0

    for j in range(args.warmup):
        one_step(j)
    torch.cuda.synchronize()
    ctl.timing_enable(True)
    lat = np.empty(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(args.steps):
        s0 = time.perf_counter()
        one_step(args.warmup + j)
        lat[j] = time.perf_counter() - s0
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    roll_ms, upd_ms, n_timed = ctl.timing_read()
    ctl.timing_enable(False)
    assert np.all(np.isfinite(V.cpu().numpy())) and np.all(np.isfinite(np.asarray(x)))

    steps_per_call = K * M * T
    value = steps_per_call * args.steps / elapsed
    roll_avg_s = roll_ms / max(n_timed, 1) * 1e-3
    flops = model_flops(p, n_obs)
    achieved_tf = flops / roll_avg_s / 1e12
    out = {
        "metric": "rollout-steps/s (K*M*T per mppi_step), receding-horizon loop",
        "value": value,
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded world: %d obstacles on an elliptic track, Philox noise)" % n_obs,
        "config": {"workload": "%s: K=%d T=%d M=%d n_obs=%d alpha=%g lambda=%g, shift + first-command readback"
                               % (args.workload, K, T, M, n_obs, p["alpha"], p["lam"]),
                   "K": K, "T": T, "M": M, "n_obs": n_obs, "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "kernel_ms": {"rollout": roll_avg_s * 1e3, "update": upd_ms / max(n_timed, 1)},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "k_rollout", "model_flops_per_launch": flops},
    }
    if args.calibrate_copy > 0:
        n = args.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = n
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(world)
        out["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)
    ctl.close()


if __name__ == "__main__":
    main()
