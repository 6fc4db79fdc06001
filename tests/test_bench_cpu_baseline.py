"""The benchmark's CPU baseline leg on a tiny workload (CPU only): the
oracle timed on every host core and on one thread, with the CPU model."""
import bench
from paper_2209_12842_amd import workloads as W


def test_cpu_baseline_reports_all_cores_one_thread_and_model():
    w = W.make_world("c1", K=64, T=5, M=4)
    out = bench.cpu_baseline(w, budget_s=0.01, single_k=16)
    assert out["kind"] == "oracle" and out["unit"] == "rollout-steps/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert isinstance(out["cpu_model"], str) and out["cpu_model"]
    st = out["single_thread"]
    assert st["cores"] == 1 and st["value"] > 0
    assert "16 of 64 samples" in st["sample"]


def test_paper_rate_is_the_papers_middle_sample_count():
    r = bench.PAPER_RATE
    assert r["K"] * r["M"] == r["trajectories"]
    assert abs(r["rollout_steps_per_s"] - 44.3 * 3.072e5 * 30) < 1.0
