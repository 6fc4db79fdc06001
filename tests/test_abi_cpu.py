"""C-ABI contract tests that need no GPU.

The library loads, exports every function include/ramppi.h declares, and
rejects bad arguments with the documented status before any device call.
Only host-side validation is exercised here (no compute call is made).
"""
import ctypes

import numpy as np
import pytest

import paper_2209_12842_amd as R
from paper_2209_12842_amd import workloads as W
from paper_2209_12842_amd._binding import (MPPI_EDEVICE, MPPI_EINVAL, MPPI_EUNSUPPORTED, MPPI_OK, DebugPtrs,
                                           Params)


@pytest.fixture(scope="module")
def L():
    return R.lib()


def test_exports_every_declared_function(L):
    names = R.header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


def test_params_struct_layout_matches_the_header():
    # int32 x 4, 37 floats, a uint64 (8-aligned), two uint32 and two floats: 168 bytes
    assert ctypes.sizeof(Params) == 168
    assert Params.seed.offset == 144 and Params.flags.offset == 152
    assert Params.noise_kind.offset == 156 and Params.jump_size.offset == 164
    assert Params.track.offset == 120


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "p0"])
def test_presets_validate(L, name):
    w = W.make_world(name)
    p = R.make_params(w["params"], len(w["obstacles"]))
    assert L.mppi_validate(ctypes.byref(p)) == MPPI_OK, R.last_error()
    nb = L.mppi_workspace_bytes(ctypes.byref(p))
    K, T, M = p.K, p.T, p.M
    assert nb >= 8 * K * T + 4 * K * M + 16 * K
    assert nb % 256 == 0


BAD = [
    dict(K=0), dict(T=0), dict(M=0), dict(dt=0.0), dict(dt=float("nan")), dict(wheelbase=-1.0),
    dict(u_lo=(3.0, -0.5), u_hi=(-3.0, 0.5)), dict(u_lo=(-3.0, 0.5), u_hi=(3.0, 0.5)),
    dict(sigma_eps=(0.0, 0.1)), dict(sigma_eps=(-1.0, 0.1)), dict(sigma_w=(0.01, -0.01, 0.0, 0.0)),
    dict(alpha=0.0), dict(alpha=1.0), dict(alpha=1.5), dict(lam=0.0), dict(lam=float("inf")),
    dict(gamma=-0.1), dict(gamma=2.0), dict(eta=-0.1), dict(eta=1.1), dict(A=-1.0), dict(B=-1.0),
    dict(C_u=float("nan")), dict(c_obs=float("inf")), dict(c_v=-1.0), dict(track=(0.0, 0.0, 0.0, 10.0, 3.0)),
    dict(track=(0.0, 0.0, 15.0, 10.0, -1.0)), dict(noise_kind=3), dict(noise_kind=2, jump_prob=1.5),
    dict(noise_kind=2, jump_size=-0.1),
]


@pytest.mark.parametrize("bad", BAD, ids=[str(b) for b in BAD])
def test_invalid_parameters_are_rejected(L, bad):
    w = W.make_world("c1")
    p = dict(w["params"])
    p.update(bad)
    s = R.make_params(p, len(w["obstacles"]))
    assert L.mppi_validate(ctypes.byref(s)) == MPPI_EINVAL
    assert R.last_error() != ""
    assert L.mppi_workspace_bytes(ctypes.byref(s)) == 0


def test_unknown_flags_and_negative_obstacles(L):
    w = W.make_world("c1")
    s = R.make_params(w["params"], len(w["obstacles"]), flags=0x100)
    assert L.mppi_validate(ctypes.byref(s)) == MPPI_EINVAL
    s = R.make_params(w["params"], -1)
    assert L.mppi_validate(ctypes.byref(s)) == MPPI_EINVAL
    assert L.mppi_validate(None) == MPPI_EINVAL


def test_zero_noise_needs_the_flag_and_gamma_zero(L):
    w = W.make_world("c1")
    p = dict(w["params"], sigma_eps=(0.0, 0.0))
    s = R.make_params(p, 10)
    assert L.mppi_validate(ctypes.byref(s)) == MPPI_EINVAL
    s = R.make_params(p, 10, flags=R.MPPI_F_ALLOW_ZERO_NOISE)
    assert L.mppi_validate(ctypes.byref(s)) == MPPI_EINVAL          # gamma = lambda != 0
    s = R.make_params(dict(p, gamma=0.0), 10, flags=R.MPPI_F_ALLOW_ZERO_NOISE)
    assert L.mppi_validate(ctypes.byref(s)) == MPPI_OK


@pytest.mark.parametrize("kw", [dict(M=1025), dict(n_obs=1025), dict(T=4097), dict(K=(1 << 20) + 1),
                                dict(K=16, M=16, T=3000)])
def test_limits_are_unsupported(L, kw):
    w = W.make_world("c1")
    p = dict(w["params"])
    n_obs = kw.pop("n_obs", 10)
    p.update(kw)
    s = R.make_params(p, n_obs)
    assert L.mppi_validate(ctypes.byref(s)) == MPPI_EUNSUPPORTED, R.last_error()


def test_workspace_grows_with_sizes(L):
    w = W.make_world("c1")
    a = R.make_params(dict(w["params"], K=256), 10)
    b = R.make_params(dict(w["params"], K=512), 10)
    c = R.make_params(dict(w["params"], K=256, M=32), 10)
    na, nb, nc = (L.mppi_workspace_bytes(ctypes.byref(x)) for x in (a, b, c))
    assert nb > na and nc > na


def test_create_rejects_bad_arguments_before_any_device_call(L):
    w = W.make_world("c1")
    s = R.make_params(w["params"], 10)
    obs = np.ascontiguousarray(w["obstacles"], dtype=np.float32)
    optr = obs.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    nb = L.mppi_workspace_bytes(ctypes.byref(s))
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: every case fails validation first
    assert L.mppi_create(ctypes.byref(s), optr, fake, nb, None, None) == MPPI_EINVAL
    assert L.mppi_create(ctypes.byref(s), None, fake, nb, None, ctypes.byref(h)) == MPPI_EINVAL
    assert L.mppi_create(ctypes.byref(s), optr, None, nb, None, ctypes.byref(h)) == MPPI_EINVAL
    assert L.mppi_create(ctypes.byref(s), optr, ctypes.c_void_p((1 << 20) + 4), nb, None,
                         ctypes.byref(h)) == MPPI_EINVAL
    assert L.mppi_create(ctypes.byref(s), optr, fake, nb - 256, None, ctypes.byref(h)) == MPPI_EINVAL
    bad = obs.copy()
    bad[3, 2] = 0.0
    assert L.mppi_create(ctypes.byref(s), bad.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), fake, nb, None,
                         ctypes.byref(h)) == MPPI_EINVAL
    assert "radius" in R.last_error()
    assert not h.value


def test_create_without_a_device_reports_edevice(L):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present; this case is for hosts without one")
    w = W.make_world("c1")
    s = R.make_params(w["params"], 10)
    obs = np.ascontiguousarray(w["obstacles"], dtype=np.float32)
    nb = L.mppi_workspace_bytes(ctypes.byref(s))
    h = ctypes.c_void_p()
    st = L.mppi_create(ctypes.byref(s), obs.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                       ctypes.c_void_p(1 << 20), nb, None, ctypes.byref(h))
    assert st == MPPI_EDEVICE
    assert not h.value


def test_step_and_views_reject_null(L):
    x0 = (ctypes.c_float * 4)(0, 0, 0, 1)
    assert L.mppi_step(None, x0, ctypes.c_void_p(1 << 20), 0, None, None) == MPPI_EINVAL
    assert L.mppi_destroy(None) == MPPI_OK
    d = DebugPtrs()
    assert L.mppi_debug_view(None, ctypes.byref(d)) == MPPI_EINVAL
    assert L.mppi_timing_enable(None, 1) == MPPI_EINVAL
    u0 = (ctypes.c_float * 2)()
    assert L.mppi_serve_start(None, ctypes.c_void_p(1 << 20), 100, None) == MPPI_EINVAL
    assert L.mppi_serve_step(None, x0, 0, u0) == MPPI_EINVAL
    assert L.mppi_serve_stop(None) == MPPI_EINVAL


def test_stage_entries_validate_first(L):
    fake = ctypes.c_void_p(1 << 20)
    assert L.mppi_philox(1, fake, fake, -1, None) == MPPI_EINVAL
    assert L.mppi_philox(1, None, fake, 5, None) == MPPI_EINVAL
    assert L.mppi_philox(1, fake, fake, 0, None) == MPPI_OK        # nothing to do
    assert L.mppi_normals(1, fake, None, 5, None) == MPPI_EINVAL
    assert L.mppi_cvar(fake, 4, 0, 0.9, 1.0, fake, None) == MPPI_EINVAL
    assert L.mppi_cvar(fake, 4, 1025, 0.9, 1.0, fake, None) == MPPI_EUNSUPPORTED
    assert L.mppi_cvar(fake, 4, 16, 1.0, 1.0, fake, None) == MPPI_EINVAL
    assert L.mppi_cvar(fake, 4, 16, 0.9, -2.0, fake, None) == MPPI_EINVAL
    assert L.mppi_cvar(None, 4, 16, 0.9, 1.0, fake, None) == MPPI_EINVAL
    assert L.mppi_cvar(fake, 0, 16, 0.9, 1.0, fake, None) == MPPI_OK


def test_batch_validation_before_any_device_call(L):
    ws = W.make_batch(4, k_range=(256, 512), t_range=(10, 20))
    P = (R.Params * 4)(*[R.make_params(w["params"], len(w["obstacles"])) for w in ws])
    nb = L.mppi_batch_workspace_bytes(4, P)
    assert nb > 0 and nb % 256 == 0
    assert L.mppi_batch_workspace_bytes(0, P) == 0
    bad = (R.Params * 1)(R.make_params(dict(ws[0]["params"], M=300), 5))
    assert L.mppi_batch_workspace_bytes(1, bad) == 0
    assert "exceeds 256" in R.last_error()
    bad = (R.Params * 1)(R.make_params(dict(ws[0]["params"], alpha=2.0), 5))
    assert L.mppi_batch_workspace_bytes(1, bad) == 0
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)
    assert L.mppi_batch_create(4, P, None, None, fake, nb, None, ctypes.byref(h)) == MPPI_EINVAL
    assert L.mppi_batch_create(4, P, None, None, fake, nb, None, None) == MPPI_EINVAL
    assert L.mppi_batch_step(None, None, None, None, None) == MPPI_EINVAL
    assert L.mppi_batch_destroy(None) == MPPI_OK
    assert L.mppi_batch_autotune(None, 1, None, None, None) == MPPI_EINVAL


def test_batch_workspace_covers_every_controller(L):
    ws = W.make_batch(8)
    P = (R.Params * 8)(*[R.make_params(w["params"], len(w["obstacles"])) for w in ws])
    total = L.mppi_batch_workspace_bytes(8, P)
    single = sum(L.mppi_workspace_bytes(ctypes.byref(P[i])) for i in range(8))
    assert total > single
