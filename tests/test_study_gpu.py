"""The closed-loop study leg runs end to end on the device (a few steps)."""
import argparse
import io
import json
import contextlib

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)


def test_closed_loop_study_runs():
    import bench
    import paper_2209_12842_amd as R
    buf = io.StringIO()
    with contextlib.redirect_stdout(buf):
        bench.run_study(argparse.Namespace(steps=40, seeds=2), R, torch)
    out = json.loads(buf.getvalue().strip().splitlines()[-1])
    for name in ("mppi", "ra_mppi"):
        s = out["study"][name]
        assert s["laps_mean"] > 0.02          # the car moves forward along the oval
        assert s["collision_steps_per_lap"] >= 0.0 and s["outside_steps_per_lap"] >= 0.0
