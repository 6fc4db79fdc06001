"""Persistent serving of the receding-horizon loop (mppi_serve_*) on MI355X
through the C ABI.

A served step must give exactly what a launched step gives from the same
state, call index and mean sequence (the same device code runs in both), over
a session of consecutive steps; the session must end on request, by its idle
limit, and when the handle is destroyed, after which launched steps work as
before.
"""
import sys
import time

import numpy as np
import pytest

from paper_2209_12842_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2209_12842_amd as R  # noqa: E402

EINVAL, EUNSUPPORTED, EDEVICE = -1, -4, -3


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _states(x0, n):
    # a deterministic drift of the measured state, the same for both handles
    x0 = np.asarray(x0, dtype=np.float64)
    return [[float(x0[0] + 0.11 * j), float(x0[1] - 0.03 * j), float(x0[2] + 0.004 * j),
             float(x0[3] + 0.02 * (j % 5))] for j in range(n)]


@pytest.mark.parametrize("wl,n,kw", [("c1", 40, {}), ("c2", 25, {}),
                                     ("c1", 20, dict(K=300, M=300, noise_kind=1)),
                                     ("c1", 20, dict(M=48, noise_kind=2, jump_prob=0.1, jump_size=0.45, B=2.0)),
                                     # T = 45: the 90 values of V+ are stored by two waves of the merging
                                     # workgroup, and 90 is not a multiple of 64
                                     ("c2", 30, dict(K=1024, T=45, M=32))])
def test_served_steps_equal_launched_steps(wl, n, kw):
    w = W.make_world(wl, **kw)
    p = dict(w["params"], shift=True)
    _log("serve vs launch %s K=%d T=%d M=%d, %d steps" % (wl, p["K"], p["T"], p["M"], n))
    a = R.Controller(p, w["obstacles"])
    b = R.Controller(p, w["obstacles"])
    Va, Vb = a.new_V(), b.new_V()
    xs = _states(w["x0"], n)
    ua = []
    a.serve_start(Va, idle_ms=5000)
    try:
        for j, x in enumerate(xs):
            ua.append(a.serve_step(x, 7 + j))
    finally:
        a.serve_stop()
    ub = [b.step(x, Vb, 7 + j, want_u0=True) for j, x in enumerate(xs)]
    torch.cuda.synchronize()
    for j in range(n):
        assert np.array_equal(ua[j], ub[j]), (j, ua[j], ub[j])
    assert torch.equal(Va, Vb)
    a.close()
    b.close()


def test_session_restarts_and_launched_steps_follow():
    w = W.make_world("c1")
    p = dict(w["params"], shift=True)
    a = R.Controller(p, w["obstacles"])
    b = R.Controller(p, w["obstacles"])
    Va, Vb = a.new_V(), b.new_V()
    xs = _states(w["x0"], 12)
    out_a, out_b = [], []
    a.serve_start(Va)
    out_a += [a.serve_step(x, j) for j, x in enumerate(xs[:4])]
    with pytest.raises(R.MppiError) as e:  # no launched step while serving
        a.step(xs[4], Va, 4, want_u0=True)
    assert e.value.status == EINVAL
    with pytest.raises(R.MppiError):  # one session at a time
        a.serve_start(Va)
    a.serve_stop()
    a.serve_stop()  # nothing to stop
    out_a += [a.step(x, Va, 4 + j, want_u0=True) for j, x in enumerate(xs[4:8])]
    a.serve_start(Va)
    out_a += [a.serve_step(x, 8 + j) for j, x in enumerate(xs[8:])]
    a.serve_stop()
    out_b = [b.step(x, Vb, j, want_u0=True) for j, x in enumerate(xs)]
    torch.cuda.synchronize()
    for j in range(len(xs)):
        assert np.array_equal(out_a[j], out_b[j]), j
    assert torch.equal(Va, Vb)


def test_session_ends_by_its_idle_limit():
    w = W.make_world("c1")
    a = R.Controller(dict(w["params"], shift=True), w["obstacles"])
    V = a.new_V()
    a.serve_start(V, idle_ms=20)
    u = a.serve_step(w["x0"], 0)
    assert np.all(np.isfinite(u))
    time.sleep(0.5)  # far past the limit: the kernel has left
    with pytest.raises(R.MppiError) as e:
        a.serve_step(w["x0"], 1)
    assert e.value.status == EDEVICE
    a.serve_stop()  # the handle no longer serves: nothing to do
    u1 = a.step(w["x0"], V, 1, want_u0=True)
    assert np.all(np.isfinite(u1))
    torch.cuda.synchronize()


def test_destroy_ends_the_session():
    w = W.make_world("c1")
    a = R.Controller(dict(w["params"], shift=True), w["obstacles"])
    V = a.new_V()
    a.serve_start(V)
    a.serve_step(w["x0"], 0)
    a.close()
    torch.cuda.synchronize()  # the kernel has left: the device is free
    z = torch.ones(4, device="cuda") * 2
    assert float(z.sum().item()) == 8.0


def test_serving_needs_the_one_launch_step():
    w = W.make_world("c1")
    a = R.Controller(dict(w["params"], shift=True), w["obstacles"], split_update=True)
    V = a.new_V()
    with pytest.raises(R.MppiError) as e:
        a.serve_start(V)
    assert e.value.status == EUNSUPPORTED
    with pytest.raises(R.MppiError) as e:
        a.serve_step(w["x0"], 0)
    assert e.value.status == EINVAL
    with pytest.raises(R.MppiError) as e:
        a.serve_start(V, idle_ms=0)
    assert e.value.status == EINVAL
