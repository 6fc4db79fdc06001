"""Host logic of the benchmark: the FLOP models, the traffic record and its
guard against a changed kernel (CPU only)."""
import bench
from paper_2209_12842_amd import workloads as W


def test_brute_force_model_matches_the_survey_counts():
    # 80 + 7 n_obs per disturbed and 60 + 7 n_obs per nominal state step
    p = W.make_world("c2")["params"]
    assert bench.model_flops(p, 50) == 2048 * 64 * 50 * 430 + 2048 * 50 * 410
    p3 = W.make_world("c3")["params"]
    assert abs(bench.model_flops(p3, 200) - 3.13e11) / 3.13e11 < 0.01


def test_executed_model_counts_waves_groups_and_candidates():
    p = dict(K=256, T=10, M=64)
    # 256 samples of 64 draws: 4 samples per workgroup of 256 threads, 64
    # workgroups of 4 waves, and one nominal workgroup of 256 lanes
    assert bench.disturbed_waves(p) == 256
    base = bench.executed_flops(p, 10, 0.0, 0.0)
    lanes = 64 * 256 + 256
    assert base == 80.0 * 256 * 64 * 10 + 60.0 * 256 * 10 + 4.0 * 10 * lanes
    assert bench.executed_flops(p, 10, 3.0, 0.0) - base == 5.0 * 64 * 3.0
    assert bench.executed_flops(p, 10, 0.0, 2.0) - base == 17.0 * 64 * 2.0
    # with more than one table group every box also runs the group-box compares
    boxes = -(-10 // bench.CULL_STEPS)
    assert bench.executed_flops(p, 100, 0.0, 0.0) - base == 4.0 * boxes * lanes
    # no obstacles: no box at all
    assert bench.executed_flops(p, 0, 0.0, 0.0) == 80.0 * 256 * 64 * 10 + 60.0 * 256 * 10
    # the batched path runs workgroups of 256 threads whatever M is
    q = dict(K=256, T=10, M=129)
    assert bench.disturbed_waves(q) == 256 * 3 and bench.disturbed_waves(q, block=256) == 256 * 4


def test_cull_steps_match_the_kernel():
    import os
    import re
    path = os.path.join(os.path.dirname(bench.__file__), "paper_2209_12842_amd", "csrc", "step_device.h")
    m = re.search(r"constexpr int kCullSteps = (\d+);", open(path).read())
    assert m and int(m.group(1)) == bench.CULL_STEPS


def test_traffic_record_is_used_only_for_the_kernel_it_measured(monkeypatch):
    for wl in ("c2", "c3"):
        t = bench.measured_traffic(wl)
        assert t is None or t > 0
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
    assert bench.measured_traffic("c2") is None and bench.measured_traffic("c3") is None
    assert bench.measured_traffic("c1") is None  # nothing measured


def test_valu_record_is_used_only_for_the_kernel_it_measured(monkeypatch):
    for wl in ("c2", "c3"):
        n = bench.measured_valu(wl)
        assert n is None or n > 0
    assert bench.measured_valu("c1") is None  # nothing measured
    r = bench.valu_issue("c3", 0.8e-3)
    if r is not None:
        cycles = 0.8e-3 * 2.4e9 * 1024
        assert abs(r["per_simd_per_clock"] - r["insts_per_launch"] / cycles) < 1e-12
        assert 0.0 < r["valu_busy"] < 2.0 and 0.0 <= r["dual_issue_frac"] <= 1.0
    assert bench.valu_issue("c3", 0.0) is None
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
    assert bench.measured_valu("c2") is None and bench.valu_issue("c3", 1e-3) is None
