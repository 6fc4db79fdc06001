"""mppi_step_noalloc (the step without a handle or workspace, on the
library's static scratch) through the C ABI against mppi_step with the same
inputs: the same kernels run, so V+ and the first command must agree bit for
bit, on two calls in a row, the second with a smaller problem (fewer
samples, draws, steps and obstacles), then once more at the first size."""
import sys

import numpy as np
import pytest

from paper_2209_12842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2209_12842_amd as R  # noqa: E402


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _reference(p, obs, x0, V0, idx):
    ctl = R.Controller(p, obs)
    V = ctl.new_V(V0)
    u0 = ctl.step(x0, V, idx, want_u0=True)
    torch.cuda.synchronize()
    out = V.cpu().numpy().copy(), np.asarray(u0, dtype=np.float32)
    ctl.close()
    return out


def _noalloc(p, obs, x0, V0, idx):
    dev = torch.device("cuda", 0)
    V = torch.as_tensor(np.asarray(V0, dtype=np.float32)).to(dev).contiguous()
    o = torch.as_tensor(np.asarray(obs, dtype=np.float32).reshape(-1, 3)).to(dev).contiguous()
    u0 = torch.full((2,), float("nan"), dtype=torch.float32, device=dev)
    R.step_noalloc(p, o if o.shape[0] else None, x0, V, idx, u0=u0)
    torch.cuda.synchronize()
    return V.cpu().numpy().copy(), u0.cpu().numpy().copy()


CASES = [
    ("c2 shift", "c2", dict(), 3),
    ("smaller: K=300 T=17 M=24, 7 obstacles", "c1", dict(K=300, T=17, M=24, lam=20.0, shift=True), 4),
    ("c2 again", "c2", dict(), 5),
    # M = 300: the handle's two-launch step takes the flattened layout, the
    # no-alloc step the per-sample one; both give the same bits
    ("paper shape: K=1024 T=30 M=300", "p0", dict(), 6),
]


@pytest.mark.parametrize("case", [CASES])
def test_noalloc_step_equals_step(case):
    torch.cuda.set_device(0)
    for tag, name, kw, idx in case:
        w = W.make_world(name, **kw)
        p, obs, x0 = w["params"], w["obstacles"], w["x0"]
        if name == "c1":
            obs = obs[:7]
        V0 = W.random_V(int(p["T"]), 11, scale=(1.0, 0.2))
        _log("no-alloc step %s: K=%d T=%d M=%d n_obs=%d" % (tag, p["K"], p["T"], p["M"], len(obs)))
        Vr, ur = _reference(p, obs, x0, V0, idx)
        Vn, un = _noalloc(p, obs, x0, V0, idx)
        assert np.array_equal(Vn, Vr), (tag, np.abs(Vn - Vr).max())
        assert np.array_equal(un, ur), (tag, un, ur)


def test_noalloc_rejects_what_it_cannot_hold():
    w = W.make_world("c3", K=65536)      # a 52 MB workspace: beyond the 32 MiB scratch
    V = torch.zeros((w["params"]["T"], 2), dtype=torch.float32, device="cuda:0")
    o = torch.as_tensor(w["obstacles"]).cuda().contiguous()
    with pytest.raises(R.MppiError, match="scratch"):
        R.step_noalloc(w["params"], o, w["x0"], V, 0)
