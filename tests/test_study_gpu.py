"""The closed-loop study (synthetic stand-in for the paper's collision
comparison, Sec. V-B): plain MPPI (A = 0) against RA-MPPI (A = 10) on the
paper-preset oval under the same seeded plant disturbances.  The paper
reports fewer collisions with the risk term; the test asserts that
direction over 8 seeds of 300 steps, paired by seed, per metre driven
(RA-MPPI drives more slowly, so per lap alone would flatter it) and per lap,
with the paired difference at least two standard errors above zero per
metre."""
import argparse
import io
import json
import contextlib

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)


def test_closed_loop_study_direction():
    import bench
    import paper_2209_12842_amd as R
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        bench.run_study(argparse.Namespace(steps=300, seeds=8), R, torch)
    out = json.loads(buf.getvalue().strip().splitlines()[-1])
    s = out["study"]
    print(json.dumps(s), flush=True)
    for name in ("mppi", "ra_mppi"):
        assert s[name]["laps_mean"] > 0.1          # the car moves forward along the oval
        assert s[name]["collision_steps_per_lap"] >= 0.0 and s[name]["outside_steps_per_lap"] >= 0.0
    assert s["mppi"]["collision_steps_total"] > 0  # the world is hard enough to show a difference
    assert s["ra_mppi"]["collision_steps_total"] <= s["mppi"]["collision_steps_total"]
    assert s["ra_mppi"]["collision_steps_per_lap"] <= s["mppi"]["collision_steps_per_lap"]
    d = s["paired_difference_per_m"]
    assert d["seeds"] == 8
    assert d["mean"] - 2.0 * d["se"] > 0.0, d
