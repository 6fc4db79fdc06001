"""Batched serving (many controllers per step) on MI355X through the C ABI.

Every controller of a batch must produce exactly what a single-controller
step produces with the same parameters and inputs (the same device code runs
in both), with the step replayed from a HIP graph or launched directly, after
autotuning, and over several receding-horizon steps; one controller is also
checked against the FP64 oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2209_12842_amd import workloads as W

from parity_helpers import check_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU hosts
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2209_12842_amd as R  # noqa: E402


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed_worlds():
    ws = W.make_batch(6, seed=11, k_range=(256, 1024), t_range=(8, 30), m_range=(7, 64), obs_range=(0, 40))
    # make the set uneven on purpose: ragged K, odd M, no obstacles, other noise forms
    ws[0]["params"].update(K=300)
    ws[1]["params"].update(M=7)
    ws[2]["obstacles"] = ws[2]["obstacles"][:0]
    ws[3]["params"].update(noise_kind=1)
    ws[4]["params"].update(noise_kind=2, jump_prob=0.05, jump_size=0.45)
    ws[5]["params"].update(M=256, K=256, eta=0.3, B=2.0)
    for w in ws:
        w["V0"] = W.random_V(w["params"]["T"], 3, scale=(1.0, 0.2))
    return ws


def _plain(ws, x0s, Vs, idx):
    out = []
    for w, x0, V0, j in zip(ws, x0s, Vs, idx):
        ctl = R.Controller(w["params"], w["obstacles"], debug=True)
        V = ctl.new_V(V0)
        u0 = ctl.step(x0, V, int(j))
        d = {k: v.detach().cpu().numpy().copy() for k, v in ctl.debug().items()}
        d["V"] = V.cpu().numpy().copy()
        d["u0h"] = u0
        out.append(d)
        ctl.close()
    return out


def _batch_state(b, i):
    d = {k: v.detach().cpu().numpy().copy() for k, v in b.debug(i).items()}
    d["V"] = b.V[i].cpu().numpy().copy()
    return d


KEYS = ("u", "S", "L", "cvar", "S_tilde", "w_hat", "V")


def _same(a, b, where):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (where, k, np.abs(a[k] - b[k]).max())


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_single_controller_steps(graph):
    ws = _mixed_worlds()
    n = len(ws)
    b = R.Batch([w["params"] for w in ws], [w["obstacles"] for w in ws], debug=True, V0=[w["V0"] for w in ws])
    b.set_graph(graph)
    x0s = np.stack([w["x0"] for w in ws])
    Vin = [w["V0"] for w in ws]
    for step in range(3):
        idx = np.arange(n, dtype=np.uint32) + 7 * step
        _log("batch step %d graph=%s" % (step, graph))
        u0 = b.step(x0s, idx)
        torch.cuda.synchronize()
        ref = _plain(ws, x0s, Vin, idx)
        for i in range(n):
            got = _batch_state(b, i)
            _same(got, ref[i], (step, i))
            assert np.array_equal(u0[i], ref[i]["u0h"])
        Vin = [b.V[i].cpu().numpy().copy() for i in range(n)]
        x0s = x0s + np.float32(0.1)
    b.close()


@pytest.mark.parametrize("kind", [1, 2])
def test_single_form_batch_equals_single_controller_steps(kind):
    # every controller with the same disturbance form: the batch runs the
    # rollout kernel compiled for that form alone (the Gaussian form is the
    # 64-controller batch's)
    ws = W.make_batch(4, seed=20 + kind, k_range=(256, 1024), t_range=(8, 30), m_range=(7, 64), obs_range=(0, 40))
    for w in ws:
        w["params"].update(noise_kind=kind)
        if kind == 2:
            w["params"].update(jump_prob=0.05, jump_size=0.45)
        w["V0"] = W.random_V(w["params"]["T"], 4, scale=(1.0, 0.2))
    n = len(ws)
    b = R.Batch([w["params"] for w in ws], [w["obstacles"] for w in ws], debug=True, V0=[w["V0"] for w in ws])
    x0s = np.stack([w["x0"] for w in ws])
    idx = np.arange(n, dtype=np.uint32) + 9
    _log("single-form batch, noise kind %d" % kind)
    u0 = b.step(x0s, idx)
    torch.cuda.synchronize()
    ref = _plain(ws, x0s, [w["V0"] for w in ws], idx)
    for i in range(n):
        _same(_batch_state(b, i), ref[i], i)
        assert np.array_equal(u0[i], ref[i]["u0h"])
    b.close()


def test_batch_autotune_keeps_results_and_state():
    ws = _mixed_worlds()
    n = len(ws)
    x0s = np.stack([w["x0"] for w in ws])
    idx = np.arange(n, dtype=np.uint32)
    b = R.Batch([w["params"] for w in ws], [w["obstacles"] for w in ws], debug=True, V0=[w["V0"] for w in ws])
    b.step(x0s, idx)
    torch.cuda.synchronize()
    before = [b.V[i].cpu().numpy().copy() for i in range(n)]
    wg, order = b.autotune(trials=2)
    _log("autotune: %d workgroups per CU, order %d" % (wg, order))
    assert wg >= 1 and order in (0, 1)
    for i in range(n):
        assert np.array_equal(b.V[i].cpu().numpy(), before[i])   # the tuner restored V
    b.step(x0s, idx + 1)
    torch.cuda.synchronize()
    ref = _plain(ws, x0s, before, idx + 1)
    for i in range(n):
        _same(_batch_state(b, i), ref[i], i)
    b.close()


def test_batch_controller_against_oracle():
    ws = _mixed_worlds()
    b = R.Batch([w["params"] for w in ws], [w["obstacles"] for w in ws], debug=True, V0=[w["V0"] for w in ws])
    x0s = np.stack([w["x0"] for w in ws])
    idx = np.arange(len(ws), dtype=np.uint32) + 3
    u0 = b.step(x0s, idx)
    torch.cuda.synchronize()
    oracle.set_threads(8)
    for i in (0, 1, 4):
        w = ws[i]
        d = _batch_state(b, i)
        g = {k: d[k].astype(np.float64) for k in ("S", "L", "cvar", "S_tilde", "w_hat", "u0")}
        g["u"] = np.transpose(d["u"], (1, 0, 2)).astype(np.float64)
        g["V_next"] = d["V"].astype(np.float64)
        g["u0_host"] = u0[i].astype(np.float64)
        o = oracle.step(w["params"], w["obstacles"], w["x0"], w["V0"], int(idx[i]))
        rep = check_step(w["params"], g, o, shift=True, tag="mixed batch controller %d" % i)
        _log("controller %d: %s" % (i, rep))


def test_full_serving_batch_matches_sampled_single_steps():
    ws = W.make_batch(64)
    n = len(ws)
    b = R.Batch([w["params"] for w in ws], [w["obstacles"] for w in ws], debug=True)
    x0s = np.stack([w["x0"] for w in ws])
    idx = np.full(n, 2, dtype=np.uint32)
    u0 = b.step(x0s, idx)
    torch.cuda.synchronize()
    for i in (0, 17, 40, 63):
        ref = _plain([ws[i]], [ws[i]["x0"]], [ws[i]["V0"]], [2])[0]
        _same(_batch_state(b, i), ref, i)
        assert np.array_equal(u0[i], ref["u0h"])
    b.close()


def test_c5_batch_controllers_against_oracle():
    # the 64-controller serving batch at its own shapes: the controller with
    # the most obstacle tests (K=7680, T=68, M=124, 150 obstacles), the one
    # with the most state steps (K=8192, T=90, M=100), the one with 200
    # obstacles and the one with the largest M among the large fields
    # (M=126, 191 obstacles), each checked against a complete oracle step
    ws = W.make_batch(64)
    n = len(ws)
    b = R.Batch([w["params"] for w in ws], [w["obstacles"] for w in ws], debug=True)
    x0s = np.stack([w["x0"] for w in ws])
    idx = np.arange(n, dtype=np.uint32) + 5
    u0 = b.step(x0s, idx)
    torch.cuda.synchronize()
    oracle.set_threads(min(16, max(1, len(__import__("os").sched_getaffinity(0)))))
    picks = {31: (7680, 68, 124, 150), 27: (8192, 90, 100, 63), 2: (256, 23, 26, 200), 13: (3840, 49, 126, 191)}
    for i, shape in picks.items():
        w = ws[i]
        p = w["params"]
        assert (p["K"], p["T"], p["M"], len(w["obstacles"])) == shape, (i, shape)
        _log("c5 controller %d: K=%d T=%d M=%d n_obs=%d" % ((i,) + shape))
        d = _batch_state(b, i)
        g = {k: d[k].astype(np.float64) for k in ("S", "L", "cvar", "S_tilde", "w_hat", "u0")}
        g["u"] = np.transpose(d["u"], (1, 0, 2)).astype(np.float64)
        g["V_next"] = d["V"].astype(np.float64)
        g["u0_host"] = u0[i].astype(np.float64)
        o = oracle.step(p, w["obstacles"], w["x0"], w["V0"], int(idx[i]))
        rep = check_step(p, g, o, shift=bool(p.get("shift")), tag="c5 controller %d" % i)
        _log("  " + ", ".join("%s=%s" % kv for kv in rep.items()))
    b.close()
