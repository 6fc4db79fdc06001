"""Benchmark of the RA-MPPI control step on one MI355X.

Default workload (c3, the large plain step): K = 16384 samples, T = 100,
M = 128 draws (2.1e8 disturbed state steps per control step), 200 obstacles
along a 100 m x 40 m oval, alpha = 0.9, lambda = 1, consecutive mppi_step
calls with the shifted mean sequence, the first command read back every step
and a host FP64 plant closing the loop.  Synthetic seeded inputs.  One JSON
line on stdout:

  value        rollout-steps/s (K M T per step) over the timed steps
  roofline     the rollout kernel: the FP32 FLOPs of its rollouts per launch
               (with the broad-phase candidates counted on the device over
               the timed steps) / its average HIP-event duration on the
               step's stream (events on every fourth step of the timed
               loop), against the FP32 vector peak; the
               brute-force-equivalent rate (every obstacle tested at every
               state) is given beside it.  When the whole grid is resident
               the step is one launch whose duration also covers the update
               (about 3 % of the FLOPs, not counted); valu_issue gives, over
               the same duration and from the committed rocprofv3 counters
               (profiles/k_rollout_valu_counters.md), the VALU
               instructions per SIMD per clock, the wave-cycles spent in
               VALU instructions per SIMD-cycle (about 1: the vector ALU is
               what bounds the kernel) and the share of them that two
               waves issued together
  serving      the same loop (same number of steps) through a persistent
               serving session (mppi_serve_*: one resident launch, one
               request per step): rollout-steps/s, ms per step and latency
  c2_receding_horizon  the latency configuration (K = 2048, T = 50, M = 64,
               50 obstacles, 200 steps of the same loop): rate, latency
               p50 / p99, kernel times, and the persistent serving loop
  paper_shape  the paper's own sample counts (K = 1024, T = 30, M = 300,
               10 obstacles on the 0.6 m paper-preset oval): update rate in Hz
               beside the paper's
  c5_batched   the batched-serving leg (--workload c5) in short: 64
               controllers per step call, rate, latency, kernel times and the
               64 sequential steps beside it
  c4_gradient  the gradient leg (--grad) in short: dJ/dV evaluations per
               second, cost against a plain step, equal-wall-time comparison
  paper        the paper's update rate with its hardware (context only)
  cpu_baseline the FP64 oracle on a bounded sample of the same workload,
               timed on this host's cores (all of them, and one thread on a
               subset of the samples), with the CPU model

    python bench.py [--steps K] [--warmup W] [--workload c3|c2|c1|c4|p0]

With --workload (c3 included) the line carries that workload only.

Other legs (one JSON line each, not the default):
  --workload c5   batched serving: 64 independent controllers of uneven size
                  in one step call (persistent work-queue kernel replayed
                  from a HIP graph, autotuned grid), closed loop through the
                  host plant; compared with 64 sequential single-controller
                  steps of the same controllers
  --grad          the free-energy gradient dJ/dV on the workload (default
                  c4: K = 4096, T = 50, M = 64): evaluations per second, its
                  cost relative to a plain step, and gradient-corrected steps
                  against plain steps at equal wall time
  --study         closed loop on the p0 oval (the paper's controller settings,
                  0.6 m track, ten 0.1 m obstacles): RA-MPPI (A = 10) against
                  plain MPPI (A = 0) under the same seeded plant disturbances,
                  collisions and track-boundary violations per lap; a synthetic
                  stand-in for the paper's collision study that shows only the
                  direction of the effect
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

# The paper's update rate for its middle sample count (Sec. V-A, the
# computation-time paragraph): 44.3 Hz with 1024 samples x 300 disturbance
# draws (3.072e5 trajectories) over a 30-step horizon on an NVIDIA RTX 3090,
# a tyre-model vehicle and unstated precision.  Context, not a target.
PAPER_RATE = {"update_rate_hz": 44.3, "trajectories": 3.072e5, "K": 1024, "M": 300, "T": 30,
              "rollout_steps_per_s": 44.3 * 3.072e5 * 30, "hardware": "NVIDIA GeForce RTX 3090",
              "note": "the paper's vehicle has tyre dynamics and its precision is not stated; "
                      "its rate covers its whole control loop"}


def model_flops(p: dict, n_obs: int) -> float:
    """Brute-force-equivalent FP32 FLOPs of one rollout launch: 80 + 7 n_obs
    per disturbed state step (K M T of them) and 60 + 7 n_obs per nominal
    state step (K T), every obstacle tested at every state."""
    K, T, M = p["K"], p["T"], p["M"]
    return K * M * T * (80.0 + 7.0 * n_obs) + K * T * (60.0 + 7.0 * n_obs)


def disturbed_waves(p: dict, block: int | None = None) -> int:
    """Waves of the disturbed workgroups of one rollout launch (workgroups of
    `block` threads; by default the single-controller size)."""
    K, M = p["K"], p["M"]
    spb = 1 if M >= 256 else 256 // M
    if block is None:
        block = (spb * M + 63) // 64 * 64
    return (K + spb - 1) // spb * (block // 64)


# Steps of the timed loop whose kernels are timed with HIP events (one in
# TIMING_EVERY): recording three events per step costs a few microseconds of
# host time, which would otherwise be charged to every step of the loop.
TIMING_EVERY = 4

# Time steps whose points share one broad-phase box in the rollout kernel
# (kCullSteps of the device code; a CPU test keeps the two equal).
CULL_STEPS = 6


def executed_flops(p: dict, n_obs: int, candidates: float, group_tests: float, block: int | None = None) -> float:
    """FP32 FLOPs the rollout kernel executes in one launch (FMA = 2,
    compares count one): 80 per disturbed state step and 60 per nominal state
    step for dynamics, noise and the smooth costs; per lane (disturbed and
    nominal) 4 per state step for the extent of the broad-phase box and, with
    more than one table group, 4 per box (one per CULL_STEPS steps) for the
    group-box compares; 17 per lane for each group test that ran
    (`group_tests` counted on the device, per wave); 5 per lane for each
    exact test of a (state step, candidate disc) pair (`candidates` counted
    on the device, per wave)."""
    K, T, M = p["K"], p["T"], p["M"]
    n_grp = (n_obs + 63) // 64
    boxes = -(-T // CULL_STEPS)
    spb = 1 if M >= 256 else 256 // M
    if block is None:
        block = (spb * M + 63) // 64 * 64
    lanes = 64 * disturbed_waves(p, block) + (K + block - 1) // block * block
    mask = 4.0 * boxes if n_grp > 1 else 0.0
    if n_grp == 0:
        return 80.0 * K * M * T + 60.0 * K * T
    return (80.0 * K * M * T + 60.0 * K * T + (4.0 * T + mask) * lanes + 17.0 * 64 * group_tests
            + 5.0 * 64 * candidates)


def kernel_sources_sha256() -> str:
    """Hash of the HIP sources and the C header (the code the counters measured)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_12842_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".h")))
    for path in files + [os.path.join(ROOT, "include", "ramppi.h")]:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per rollout launch from the committed counter summary
    (profiles/k_rollout_<workload>_traffic.md): FETCH_SIZE and WRITE_SIZE,
    each scaled by the same counter's reading for a plain copy of known size.
    None when there is no summary or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "k_rollout_%s_traffic.md" % workload)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel sources sha256") != kernel_sources_sha256():
        return None
    return float(vals["fetch bytes per launch"]) + float(vals["write bytes per launch"])


# MI355X: 256 CUs x 4 SIMDs at a 2.4 GHz engine clock.  A SIMD issues a
# wave64 FP32 VALU instruction in two clocks when the instructions of two
# waves pair in one four-clock cycle (the FP32 vector peak, 157.3 TFLOP/s),
# in four when they do not; transcendental and 64-bit integer instructions
# take longer (measured: about 8 and 6 clocks per wave).
N_SIMD = 1024
CLOCK_HZ = 2.4e9


def _counter_record(workload: str):
    """Fields of the committed VALU counter summary
    (profiles/k_rollout_valu_counters.md) when the kernel sources still hash
    to the recorded value, else None."""
    path = os.path.join(ROOT, "profiles", "k_rollout_valu_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel sources sha256") != kernel_sources_sha256():
        return None
    return vals


def measured_valu(workload: str):
    """VALU instructions per rollout launch (SQ_INSTS_VALU, whole device) from
    the committed counter summary, or None when there is none for the
    workload or the kernel sources changed."""
    vals = _counter_record(workload)
    if vals is None:
        return None
    v = vals.get("%s VALU instructions per launch" % workload)
    return float(v) if v is not None else None


def valu_issue(workload: str, seconds_per_launch: float):
    """How the rollout kernel uses its SIMDs over the measured launch
    duration, from the committed counters: VALU instructions issued per SIMD
    per clock; valu_busy, the wave-cycles spent in VALU instructions
    (SQ_ACTIVE_INST_VALU, summed over the waves) per SIMD-cycle; and the share
    of those cycles in which two waves issued together (SQ_ACTIVE_INST_VALU2).
    None without a record."""
    vals = _counter_record(workload)
    n = measured_valu(workload)
    if vals is None or n is None or not seconds_per_launch > 0:
        return None
    simd_cycles = seconds_per_launch * CLOCK_HZ * N_SIMD
    out = {"insts_per_launch": n, "per_simd_per_clock": n / simd_cycles}
    act = vals.get("%s active VALU quad-cycles per launch" % workload)
    dual = vals.get("%s dual-issue quad-cycles per launch" % workload)
    if act is not None:
        out["valu_busy"] = 4.0 * float(act) / simd_cycles
        if dual is not None:
            out["dual_issue_frac"] = float(dual) / float(act)
    return out


def plant_step(x, u, dt, wb, w):
    """Host FP64 plant: the nominal bicycle plus an additive disturbance."""
    px, py, psi, v = x
    return [px + dt * v * math.cos(psi) + w[0], py + dt * v * math.sin(psi) + w[1],
            psi + dt * v * math.tan(float(u[1])) / wb + w[2], v + dt * float(u[0]) + w[3]]


def cpu_model() -> str:
    """The host CPU's model string (/proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(world: dict, budget_s: float = 10.0, single_k: int = 256) -> dict:
    """The FP64 oracle as it stands, timed on this host: (a) on every host
    core, complete control steps of the same workload (same world,
    consecutive step indices) until about `budget_s` seconds have run (at
    least one step); (b) on one thread, the first `single_k` samples of a step
    (the same rollouts: every sample's draws depend only on its own index),
    scaled to rollout-steps/s."""
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
    out = {"value": steps / dt, "unit": "rollout-steps/s", "cores": cores, "kind": "oracle",
           "sample": "%d complete control steps of the workload (K=%d, M=%d, T=%d) in %.1f s, FP64, %d threads"
                     % (n, p["K"], p["M"], p["T"], dt, cores),
           "cpu_model": cpu_model()}
    ks = min(single_k, int(p["K"]))
    ps = dict(p, K=ks)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.step(ps, world["obstacles"], world["x0"], world["V0"], 0,
                diagnostics=False)
    dt1 = time.perf_counter() - t0
    out["single_thread"] = {"value": ks * p["M"] * p["T"] / dt1, "unit": "rollout-steps/s", "cores": 1,
                            "sample": "the first %d of %d samples of one step (K=%d, M=%d, T=%d) in %.2f s, "
                                      "FP64, 1 thread; a full step extrapolates to %.0f s"
                                      % (ks, p["K"], ks, p["M"], p["T"], dt1, dt1 * p["K"] / ks)}
    oracle.set_threads(cores)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default=None, choices=["c1", "c2", "c3", "c4", "c5", "p0"])
    ap.add_argument("--grad", action="store_true")
    ap.add_argument("--study", action="store_true")
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="leave the batched (c5) and gradient (c4) legs out of the default line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy a MIB-sized device buffer 3 times (a plain copy kernel of "
                         "known size for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2209_12842_amd as R

    if args.grad:
        print(json.dumps(run_grad(args, R, torch)), flush=True)
        return
    if args.study:
        return run_study(args, R, torch)
    if args.workload == "c5":
        print(json.dumps(run_batch(args, R, torch)), flush=True)
        return
    headline = args.workload is None
    if headline:
        args.workload = "c3"
    out = run_plain(R, torch, args.workload, args.steps, args.warmup)
    if headline:
        # the latency configuration and the paper's own sample counts, as
        # extra keys beside the headline (their own warm-up and step counts)
        c2 = run_plain(R, torch, "c2", 200, 10)
        out["c2_receding_horizon"] = {k: c2[k] for k in ("value", "ms_per_step", "latency_ms", "kernel_ms",
                                                         "serving")}
        out["c2_receding_horizon"]["config"] = c2["config"]["workload"]
        out["c2_receding_horizon"]["roofline_frac"] = c2["roofline"]["frac"]
        out["c2_receding_horizon"]["valu_issue"] = c2["roofline"]["valu_issue"]
        ps = run_plain(R, torch, "p0", 200, 10, serving=False)
        out["paper_shape"] = {
            "config": ps["config"]["workload"], "value": ps["value"], "ms_per_step": ps["ms_per_step"],
            "update_rate_hz": 1e3 / ps["ms_per_step"], "latency_ms": ps["latency_ms"],
            "paper": PAPER_RATE}
        if not args.no_extra_legs:
            # the batched-serving and gradient legs (their own lines with
            # --workload c5 / --grad), summarised beside the headline
            b5 = run_batch(argparse.Namespace(steps=30, warmup=5), R, torch)
            out["c5_batched"] = {k: b5[k] for k in ("metric", "value", "unit", "ms_per_step", "latency_ms",
                                                     "sequential", "speedup_vs_sequential", "kernel_ms")}
            out["c5_batched"]["config"] = b5["config"]["workload"]
            out["c5_batched"]["roofline_frac"] = b5["roofline"]["frac"]
            g4 = run_grad(argparse.Namespace(steps=50, warmup=5, workload=None), R, torch)
            out["c4_gradient"] = {k: g4[k] for k in ("metric", "value", "unit", "ms_per_step", "plain_step_ms",
                                                      "gradient_over_step", "equal_wall_time")}
            out["c4_gradient"]["config"] = g4["config"]["workload"]
    out["paper"] = PAPER_RATE
    if args.calibrate_copy > 0:
        dev = torch.device("cuda", 0)
        n = args.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = n
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W.make_world(args.workload))
        out["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


def run_plain(R, torch, workload: str, steps: int, warmup: int, serving: bool = True) -> dict:
    """Consecutive receding-horizon steps of one controller (shift, first
    command read back, host FP64 plant): the bench line of the workload."""
    world = W.make_world(workload)
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
    n_total = warmup + steps
    plant_w = (np.random.default_rng(12345).standard_normal((n_total, 4)) * sw).tolist()
    x = [float(v) for v in world["x0"]]

    def one_step(j):
        nonlocal x
        u0 = ctl.step(x, V, j, want_u0=True)
        x = plant_step(x, u0, dt32, wb32, plant_w[j])
        return u0

    for j in range(warmup):
        one_step(j)
    torch.cuda.synchronize()
    ctl.timing_enable(True)   # clear, then time every TIMING_EVERY-th step of the timed
    ctl.timing_enable(False)  # region (three events per timed step cost host time)
    lat = np.empty(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(steps):
        s0 = time.perf_counter()
        timed = j % TIMING_EVERY == 0
        if timed:
            ctl.timing_enable(True, resume=True)
        one_step(warmup + j)
        if timed:
            ctl.timing_enable(False)
        lat[j] = time.perf_counter() - s0
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    roll_ms, upd_ms, n_timed = ctl.timing_read()
    cand, gtests = (v / max(n_timed, 1) for v in ctl.timing_work())
    ctl.timing_enable(False)
    assert np.all(np.isfinite(V.cpu().numpy())) and np.all(np.isfinite(np.asarray(x)))

    steps_per_call = K * M * T
    value = steps_per_call * steps / elapsed
    roll_avg_s = roll_ms / max(n_timed, 1) * 1e-3
    flops = executed_flops(p, n_obs, cand, gtests)
    achieved_tf = flops / roll_avg_s / 1e12
    brute_tf = model_flops(p, n_obs) / roll_avg_s / 1e12
    out = {
        "metric": "rollout-steps/s (K*M*T per mppi_step), receding-horizon loop",
        "value": value,
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded world: %d obstacles on an elliptic track, Philox noise)" % n_obs,
        "config": {"workload": "%s: K=%d T=%d M=%d n_obs=%d alpha=%g lambda=%g, shift + first-command readback"
                               % (workload, K, T, M, n_obs, p["alpha"], p["lam"]),
                   "K": K, "T": T, "M": M, "n_obs": n_obs, "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "kernel_ms": {"rollout": roll_avg_s * 1e3, "update": upd_ms / max(n_timed, 1)},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / PEAK_FP32_TFLOPS, "traffic": measured_traffic(workload),
                     "kernel": "k_rollout", "executed_flops_per_launch": flops,
                     "broad_phase_candidates_per_launch": cand, "broad_phase_group_tests_per_launch": gtests,
                     "brute_force_equivalent_tflops": brute_tf,
                     "valu_issue": valu_issue(workload, roll_avg_s)},
    }
    # the same loop through a persistent serving session (mppi_serve_*):
    # one resident launch for all the steps, the same computation per step
    if not serving:
        ctl.close()
        return out
    try:
        ctl.serve_start(V, idle_ms=5000)
    except R.MppiError as e:  # the step does not run as one launch
        out["serving"] = {"available": False, "reason": str(e)}
        out["kernel_ms"]["launches"] = "two: rollouts, then the update"
    else:
        # "update" is then the gap between the events after the one launch
        out["kernel_ms"]["launches"] = "one: the update runs in the rollout launch"
        base = n_total
        lat_s = np.empty(steps)
        for j in range(warmup):
            u0 = ctl.serve_step(x, base + j)
            x = plant_step(x, u0, dt32, wb32, plant_w[j])
        t0 = time.perf_counter()
        for j in range(steps):
            s0 = time.perf_counter()
            u0 = ctl.serve_step(x, base + warmup + j)
            x = plant_step(x, u0, dt32, wb32, plant_w[(warmup + j) % n_total])
            lat_s[j] = time.perf_counter() - s0
        el_s = time.perf_counter() - t0
        ctl.serve_stop()
        assert np.all(np.isfinite(V.cpu().numpy())) and np.all(np.isfinite(np.asarray(x)))
        out["serving"] = {"available": True, "value": steps_per_call * steps / el_s,
                          "ms_per_step": el_s / steps * 1e3,
                          "latency_ms": {"p50": float(np.percentile(lat_s, 50) * 1e3),
                                         "p99": float(np.percentile(lat_s, 99) * 1e3)}}
    ctl.close()
    return out


def run_batch(args, R, torch):
    """64 independent controllers (workloads.make_batch) per step call."""
    ws = W.make_batch(64)
    n = len(ws)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    work = sum(w["params"]["K"] * w["params"]["M"] * w["params"]["T"] for w in ws)
    brute = sum(model_flops(w["params"], len(w["obstacles"])) for w in ws)
    dt32 = np.array([float(np.float32(w["params"]["dt"])) for w in ws])
    wb32 = np.array([float(np.float32(w["params"]["wheelbase"])) for w in ws])
    sw = np.stack([np.sqrt(np.float32(w["params"]["sigma_w"]).astype(np.float64)) for w in ws])
    n_total = args.warmup + args.steps
    plant_w = np.random.default_rng(12345).standard_normal((n_total, n, 4)) * sw

    def plant(x, u, j):
        px, py, psi, v = x[:, 0], x[:, 1], x[:, 2], x[:, 3]
        u = u.astype(np.float64)
        return np.stack([px + dt32 * v * np.cos(psi), py + dt32 * v * np.sin(psi),
                         psi + dt32 * v * np.tan(u[:, 1]) / wb32, v + dt32 * u[:, 0]], axis=1) + plant_w[j]

    x0 = np.stack([w["x0"] for w in ws]).astype(np.float64)

    # 64 sequential single-controller steps per round (no readback between
    # them; one synchronisation and one gather of the 64 commands per round)
    ctls = [R.Controller(w["params"], w["obstacles"], device=dev) for w in ws]
    Vs = [c.new_V() for c in ctls]
    u0v = [c.debug()["u0"] for c in ctls]
    x = x0.copy()

    def seq_round(j):
        nonlocal x
        for i, c in enumerate(ctls):
            c.step(x[i], Vs[i], j, want_u0=False)
        u = torch.stack(u0v).cpu().numpy()
        x = plant(x, u, j)

    for j in range(args.warmup):
        seq_round(j)
    torch.cuda.synchronize()
    seq_lat = np.empty(args.steps)
    t0 = time.perf_counter()
    for j in range(args.steps):
        s0 = time.perf_counter()
        seq_round(args.warmup + j)
        seq_lat[j] = time.perf_counter() - s0
    seq_elapsed = time.perf_counter() - t0
    for c in ctls:
        c.close()
    del ctls, Vs, u0v
    torch.cuda.empty_cache()

    b = R.Batch([w["params"] for w in ws], [w["obstacles"] for w in ws], device=dev)
    x = x0.copy()
    b.step(x, 0, want_u0=True)
    wg, order = b.autotune(3)
    x = x0.copy()
    for j in range(args.warmup):
        x = plant(x, b.step(x, j, want_u0=True), j)
    torch.cuda.synchronize()
    lat = np.empty(args.steps)
    t0 = time.perf_counter()
    for j in range(args.steps):
        s0 = time.perf_counter()
        jj = args.warmup + j
        x = plant(x, b.step(x, jj, want_u0=True), jj)
        lat[j] = time.perf_counter() - s0
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert np.all(np.isfinite(x))
    # kernel durations: the same kernels launched directly with HIP events
    n_k = min(args.steps, 50)
    b.timing_enable(True)
    for j in range(n_k):
        b.step(x, n_total + j, want_u0=False)
    roll_ms, upd_ms, n_timed = b.timing_read()
    cand, gtests = (v / max(n_timed, 1) for v in b.timing_work())
    b.timing_enable(False)
    b.close()

    roll_avg_s = roll_ms / max(n_timed, 1) * 1e-3
    flops = (sum(executed_flops(w["params"], len(w["obstacles"]), 0.0, 0.0, block=256) for w in ws)
             + 5.0 * 64 * cand + 17.0 * 64 * gtests)
    achieved_tf = flops / roll_avg_s / 1e12
    brute_tf = brute / roll_avg_s / 1e12
    value = work * args.steps / elapsed
    seq_value = work * args.steps / seq_elapsed
    out = {
        "metric": "rollout-steps/s (sum of K*M*T over 64 controllers per batched step), closed loop",
        "value": value, "unit": "rollout-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (64 seeded worlds: 10-200 obstacles each on a 100 x 40 m oval, Philox noise)",
        "config": {"workload": "c5: 64 controllers, K multiple of 256 in [256, 8192], T in [20, 100], "
                               "M in [8, 128]; %d rollout-steps per batched step" % work,
                   "controllers": n, "autotune": {"wg_per_cu": wg, "order": order}, "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "sequential": {"value": seq_value, "ms_per_step": seq_elapsed / args.steps * 1e3,
                       "p50_ms": float(np.percentile(seq_lat, 50) * 1e3),
                       "p99_ms": float(np.percentile(seq_lat, 99) * 1e3)},
        "speedup_vs_sequential": value / seq_value,
        "kernel_ms": {"rollout": roll_avg_s * 1e3, "update": upd_ms / max(n_timed, 1),
                      "measured_over": "%d direct launches after the timed steps" % n_timed},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tf / PEAK_FP32_TFLOPS, "traffic": None, "kernel": "k_batch_rollout",
                     "executed_flops_per_launch": flops, "broad_phase_candidates_per_launch": cand,
                     "broad_phase_group_tests_per_launch": gtests,
                     "brute_force_equivalent_tflops": brute_tf},
    }
    return out


def run_grad(args, R, torch):
    """dJ/dV of the free energy on the workload (default c4)."""
    name = args.workload or "c4"
    world = W.make_world(name)
    p = dict(world["params"])
    p["shift"] = False
    obs = world["obstacles"]
    K, T, M = p["K"], p["T"], p["M"]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    x0 = world["x0"]
    ctl = R.Controller(p, obs, device=dev, grad=True)
    V = ctl.new_V(W.random_V(T, 4, scale=(1.0, 0.2)))

    def timed(fn, n):
        for j in range(args.warmup):
            fn(j)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for j in range(n):
            fn(args.warmup + j)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    g_ms = timed(lambda j: ctl.free_energy(x0, V, j), args.steps)
    Vs = V.clone()
    s_ms = timed(lambda j: ctl.step(x0, Vs, j, want_u0=False), args.steps)

    # equal wall time: from V = 0 at the start state, plain steps against
    # rounds of (step, gradient, backtracking correction), each on fresh
    # noise, for the same wall-clock budget; both final sequences are scored
    # by the mean free energy over 16 held-out call indices (lower is better)
    def score(Vf):
        js = [ctl.free_energy(x0, Vf, 1_000_000 + i)[0] for i in range(16)]
        return float(torch.stack(js).mean().item())

    def grad_round(Vg, j):
        ctl.step(x0, Vg, 10_000 + j, want_u0=False)
        J0, g = ctl.free_energy(x0, Vg, 20_000 + j)
        gn = g / g.abs().max().clamp_min(1e-30)
        for tau in (0.3, 0.1, 0.03, 0.01):  # Armijo-style backtracking on the gradient's own noise
            Vt = (Vg - tau * gn).contiguous()
            if ctl.free_energy(x0, Vt, 20_000 + j)[0].item() < J0.item():
                Vg.copy_(Vt)
                break

    Vw = ctl.new_V()
    for j in range(3):  # warm-up of the torch elementwise kernels used above
        grad_round(Vw, 90_000 + j)
    budget_s = 0.25
    Vp = ctl.new_V()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_plain = 0
    while time.perf_counter() - t0 < budget_s:
        ctl.step(x0, Vp, 10_000 + n_plain, want_u0=True)
        n_plain += 1
    t_plain = time.perf_counter() - t0
    Vg = ctl.new_V()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_grad = 0
    while time.perf_counter() - t0 < budget_s:
        grad_round(Vg, n_grad)
        n_grad += 1
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    out = {
        "metric": "free-energy gradient evaluations/s (dJ/dV, K=%d T=%d M=%d)" % (K, T, M),
        "value": 1e3 / g_ms, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": g_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded world: %d obstacles on an elliptic track, Philox noise)" % len(obs),
        "config": {"workload": "%s: K=%d T=%d M=%d n_obs=%d lambda=%g, mppi_grad (forward + adjoint)"
                               % (name, K, T, M, len(obs), p["lam"]), "parallelism": "single GPU"},
        "plain_step_ms": s_ms, "gradient_over_step": g_ms / s_ms,
        "equal_wall_time": {"budget_s": budget_s, "plain_steps": n_plain, "plain_s": t_plain,
                            "grad_rounds": n_grad, "grad_s": t_grad, "J_plain": score(Vp),
                            "J_grad_corrected": score(Vg)},
    }
    ctl.close()
    return out


def run_study(args, R, torch):
    """Closed-loop collisions of RA-MPPI and plain MPPI on the p0 oval."""
    world = W.make_world("p0")
    base = dict(world["params"], shift=True)
    obs = np.asarray(world["obstacles"], dtype=np.float64)
    a, b, hw = base["track"][2], base["track"][3], base["track"][4]
    dt32, wb32 = float(np.float32(base["dt"])), float(np.float32(base["wheelbase"]))
    sw = np.sqrt(np.float32(base["sigma_w"]).astype(np.float64))
    n_steps = args.steps
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    def run(A, seed):
        p = dict(base, A=A)
        ctl = R.Controller(p, world["obstacles"], device=dev)
        V = ctl.new_V()
        w = np.random.default_rng(1000 + seed).standard_normal((n_steps, 4)) * sw
        x = [float(v) for v in world["x0"]]
        th_prev = math.atan2(x[1] / b, x[0] / a)
        turned, coll, out, dist, t0 = 0.0, 0, 0, 0.0, time.perf_counter()
        for j in range(n_steps):
            u0 = ctl.step(x, V, (seed << 16) + j, want_u0=True)
            xp = x
            x = plant_step(x, u0, dt32, wb32, w[j])
            dist += math.hypot(x[0] - xp[0], x[1] - xp[1])
            d2 = (obs[:, 0] - x[0]) ** 2 + (obs[:, 1] - x[1]) ** 2
            coll += int(np.any(d2 < obs[:, 2] ** 2))
            G = (x[0] / a) ** 2 + (x[1] / b) ** 2 - 1.0
            e = G / math.hypot(2 * x[0] / a ** 2, 2 * x[1] / b ** 2)
            out += int(abs(e) > hw)
            th = math.atan2(x[1] / b, x[0] / a)
            turned += (th - th_prev + math.pi) % (2 * math.pi) - math.pi
            th_prev = th
        ctl.close()
        return dict(laps=turned / (2 * math.pi), collisions=coll, outside=out, dist=dist,
                    s=time.perf_counter() - t0)

    res = {A: [run(A, s) for s in range(args.seeds)] for A in (0.0, 10.0)}

    def per(rs, key, unit):
        return np.array([r[key] / max(r[unit], 1e-9) for r in rs])

    def mse(v):
        return float(v.mean()), float(v.std(ddof=1) / math.sqrt(len(v))) if len(v) > 1 else 0.0

    summary = {}
    for A, rs in res.items():
        name = "ra_mppi" if A > 0 else "mppi"
        cm, cse = mse(per(rs, "collisions", "laps"))
        om, ose = mse(per(rs, "outside", "laps"))
        dm, dse = mse(per(rs, "collisions", "dist"))
        summary[name] = {"collision_steps_per_lap": cm, "collision_se": cse, "outside_steps_per_lap": om,
                         "outside_se": ose, "collision_steps_per_m": dm, "collision_per_m_se": dse,
                         "laps_mean": float(np.mean([r["laps"] for r in rs])),
                         "metres_mean": float(np.mean([r["dist"] for r in rs])),
                         "collision_steps_total": int(sum(r["collisions"] for r in rs)),
                         "ms_per_step": 1e3 * float(np.mean([r["s"] for r in rs])) / n_steps}
    # paired by seed (both controllers see the same plant disturbances):
    # MPPI minus RA-MPPI, per lap and per metre
    for key, unit in (("per_lap", "laps"), ("per_m", "dist")):
        d = per(res[0.0], "collisions", unit) - per(res[10.0], "collisions", unit)
        m, se = mse(d)
        summary["paired_difference_" + key] = {"mean": m, "se": se, "seeds": len(d)}
    out = {
        "metric": "collision steps per lap (plant inside an obstacle), closed loop on the p0 oval",
        "value": summary["ra_mppi"]["collision_steps_per_lap"], "unit": "steps/lap", "n_gpus": 1,
        "steps": n_steps, "warmup": 0, "higher_is_better": False, "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (p0 world, %d seeds of Gaussian plant disturbances shared by both controllers)"
                % args.seeds,
        "config": {"workload": "p0: K=%d T=%d M=%d lambda=%g alpha=%g C_u=%g, A=10 vs A=0, %d steps of %g s"
                               % (base["K"], base["T"], base["M"], base["lam"], base["alpha"], base["C_u"],
                                  n_steps, base["dt"]), "parallelism": "single GPU"},
        "study": summary,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
