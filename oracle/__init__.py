"""FP64 CPU oracle for one RA-MPPI control step (ctypes wrapper of oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  Nothing in the product package
imports this module, and this module imports nothing from the product package.

Every function follows the paper's definitions (arXiv 2209.12842):
  philox / normals   noise generator and Gaussian transform (the paper names
                     none; Philox4x32-10 and Box-Muller are the chosen reading)
  dynamics           Eq. 1 (kinematic bicycle, forward Euler: a reading)
  running_cost       Eq. 20-22 on an elliptic track (reading)
  terminal_cost      Eq. 23
  cvar               Eq. 10-13 with the scaling of Eq. 18-19
  filtered_cost      Eq. 14-16
  weights            Eq. 5 and Eq. 17
  update             Eq. 4
  step               Algorithm 1, one iteration

Parameters arrive as a plain dict; every floating value is rounded to float32
first and then widened, so the oracle sees exactly the inputs an FP32 device
path sees.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32), ("T", ctypes.c_int32), ("M", ctypes.c_int32), ("n_obs", ctypes.c_int32),
        ("dt", ctypes.c_double), ("wheelbase", ctypes.c_double),
        ("u_lo", ctypes.c_double * 2), ("u_hi", ctypes.c_double * 2),
        ("sigma_eps", ctypes.c_double * 2), ("sigma_w", ctypes.c_double * 4),
        ("alpha", ctypes.c_double), ("lam", ctypes.c_double), ("gamma", ctypes.c_double),
        ("eta", ctypes.c_double), ("A", ctypes.c_double), ("B", ctypes.c_double), ("C_u", ctypes.c_double),
        ("c_bdry", ctypes.c_double), ("c_obs", ctypes.c_double), ("c_dev", ctypes.c_double),
        ("c_v", ctypes.c_double), ("v_ref", ctypes.c_double), ("c4", ctypes.c_double), ("c5", ctypes.c_double),
        ("track", ctypes.c_double * 5),
        ("seed", ctypes.c_uint64),
        ("shift", ctypes.c_int32),
        ("noise_kind", ctypes.c_int32),
        ("jump_prob", ctypes.c_double), ("jump_size", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        D = ctypes.c_double
        P = ctypes.POINTER
        lib.orc_philox4x32.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), ctypes.c_int, P(ctypes.c_uint32)]
        lib.orc_philox_batch.argtypes = [P(ctypes.c_uint32), ctypes.c_int64, ctypes.c_uint64, P(ctypes.c_uint32)]
        lib.orc_philox_constants.argtypes = [P(ctypes.c_uint32)]
        lib.orc_uniform.argtypes = [ctypes.c_uint32]
        lib.orc_uniform.restype = D
        lib.orc_box_muller.argtypes = [D, D, P(D), P(D)]
        lib.orc_normals4.argtypes = [P(ctypes.c_uint32), ctypes.c_uint64, P(D)]
        lib.orc_normals_batch.argtypes = [P(ctypes.c_uint32), ctypes.c_int64, ctypes.c_uint64, P(D)]
        lib.orc_dynamics.argtypes = [P(D), P(D), D, D, P(D)]
        lib.orc_disturbance.argtypes = [P(_Params), P(ctypes.c_uint32), P(D)]
        lib.orc_disturbance_batch.argtypes = [P(_Params), P(ctypes.c_uint32), ctypes.c_int64, P(D)]
        lib.orc_track_terms.argtypes = [P(_Params), P(D), P(D), P(D)]
        lib.orc_boundary_cost.argtypes = [D]
        lib.orc_boundary_cost.restype = D
        lib.orc_obstacle_count.argtypes = [P(D), ctypes.c_int, D, D]
        lib.orc_obstacle_count.restype = ctypes.c_int
        lib.orc_obstacle_margin.argtypes = [P(D), ctypes.c_int, D, D]
        lib.orc_obstacle_margin.restype = D
        lib.orc_running_cost.argtypes = [P(_Params), P(D), P(D)]
        lib.orc_running_cost.restype = D
        lib.orc_progress.argtypes = [P(_Params), P(D), P(D)]
        lib.orc_progress.restype = D
        lib.orc_terminal_cost.argtypes = [P(_Params), P(D), P(D)]
        lib.orc_terminal_cost.restype = D
        lib.orc_tail_size.argtypes = [D, ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int)]
        lib.orc_n_warm.argtypes = [D, ctypes.c_int]
        lib.orc_n_warm.restype = ctypes.c_int
        lib.orc_scale_risk.argtypes = [P(D), ctypes.c_int, D, P(D)]
        lib.orc_cvar.argtypes = [P(D), ctypes.c_int64, D, D]
        lib.orc_cvar.restype = D
        lib.orc_cvar_batch.argtypes = [P(D), ctypes.c_int, ctypes.c_int, D, D, P(D)]
        lib.orc_filtered_cost.argtypes = [D, D, D, D]
        lib.orc_filtered_cost.restype = D
        lib.orc_weights.argtypes = [P(D), ctypes.c_int, D, P(D), P(D)]
        lib.orc_update.argtypes = [P(D), P(D), ctypes.c_int, ctypes.c_int, P(D)]
        lib.orc_shift.argtypes = [P(D), ctypes.c_int, P(D)]
        lib.orc_controls.argtypes = [P(_Params), P(D), ctypes.c_uint32, P(D)]
        lib.orc_nominal_cost.argtypes = [P(_Params), P(D), P(D), P(D), P(D), P(D), P(D)]
        lib.orc_nominal_cost.restype = D
        lib.orc_disturbed_cost.argtypes = [P(_Params), P(D), P(D), P(D), ctypes.c_int, ctypes.c_int,
                                           ctypes.c_uint32, P(D), P(D)]
        lib.orc_disturbed_cost.restype = D
        lib.orc_running_cost_grad.argtypes = [P(_Params), P(D), P(D)]
        lib.orc_terminal_cost_grad.argtypes = [P(_Params), P(D), P(D)]
        lib.orc_free_energy.argtypes = [P(_Params), P(D), P(D), P(D), ctypes.c_uint32, P(D)]
        lib.orc_free_energy.restype = D
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_get_threads.restype = ctypes.c_int
        lib.orc_step.argtypes = [P(_Params), P(D), P(D), P(D), ctypes.c_uint32] + [P(D)] * 12
        lib.orc_track_radius.argtypes = [P(_Params), P(D)]
        lib.orc_track_radius.restype = D
        lib.orc_step.restype = ctypes.c_int
        lib.orc_rollout_subset.argtypes = [P(_Params), P(D), P(D), P(D), ctypes.c_uint32, ctypes.c_int,
                                           ctypes.c_int, P(D), P(D)]
        lib.orc_rollout_subset.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f32(x) -> float:
    return float(np.float32(x))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u32ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _as_f64(a) -> np.ndarray:
    """float32-round then widen (inputs are FP32-representable by construction)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).astype(np.float64))


def make_params(p: dict, n_obs: int) -> _Params:
    s = _Params()
    s.K, s.T, s.M, s.n_obs = int(p["K"]), int(p["T"]), int(p["M"]), int(n_obs)
    s.dt, s.wheelbase = _f32(p["dt"]), _f32(p["wheelbase"])
    for i in range(2):
        s.u_lo[i] = _f32(p["u_lo"][i])
        s.u_hi[i] = _f32(p["u_hi"][i])
        s.sigma_eps[i] = _f32(p["sigma_eps"][i])
    for i in range(4):
        s.sigma_w[i] = _f32(p["sigma_w"][i])
    for name in ("alpha", "lam", "gamma", "eta", "A", "B", "C_u",
                 "c_bdry", "c_obs", "c_dev", "c_v", "v_ref", "c4", "c5"):
        setattr(s, name, _f32(p[name]))
    for i in range(5):
        s.track[i] = _f32(p["track"][i])
    s.seed = int(p["seed"]) & 0xFFFFFFFFFFFFFFFF
    s.shift = 1 if p.get("shift", False) else 0
    s.noise_kind = int(p.get("noise_kind", 0))
    s.jump_prob = _f32(p.get("jump_prob", 0.0))
    s.jump_size = _f32(p.get("jump_size", 0.0))
    return s


# ---------------------------------------------------------------- noise ----

def philox_constants() -> tuple[int, int, int, int]:
    out = (ctypes.c_uint32 * 4)()
    _load().orc_philox_constants(out)
    return tuple(int(v) for v in out)


def philox(ctr, key, rounds: int = 10) -> np.ndarray:
    """Philox4x32-`rounds` of one counter (4 words) under key (2 words)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32(_u32ptr(c), _u32ptr(k), int(rounds), _u32ptr(out))
    return out


def philox_batch(ctr: np.ndarray, seed: int) -> np.ndarray:
    """Philox4x32-10 of n counters (n x 4 uint32) under the key of `seed`."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    out = np.empty_like(c)
    _load().orc_philox_batch(_u32ptr(c), c.shape[0], int(seed) & 0xFFFFFFFFFFFFFFFF, _u32ptr(out))
    return out


def uniform(r: int) -> float:
    return _load().orc_uniform(int(r) & 0xFFFFFFFF)


def box_muller(u0: float, u1: float) -> tuple[float, float]:
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    _load().orc_box_muller(float(u0), float(u1), ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


def normals4(ctr, seed: int) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    z = np.zeros(4)
    _load().orc_normals4(_u32ptr(c), int(seed) & 0xFFFFFFFFFFFFFFFF, _dptr(z))
    return z


def normals_batch(ctr: np.ndarray, seed: int) -> np.ndarray:
    """Four Box-Muller normals per Philox counter (n x 4 uint32 -> n x 4)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    z = np.empty((c.shape[0], 4))
    _load().orc_normals_batch(_u32ptr(c), c.shape[0], int(seed) & 0xFFFFFFFFFFFFFFFF, _dptr(z))
    return z


def disturbance_batch(p: dict, ctr: np.ndarray) -> np.ndarray:
    """Disturbances w (n x 4) of n Philox counters under the form p['noise_kind']."""
    s = make_params(p, 0)
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    w = np.empty((c.shape[0], 4))
    _load().orc_disturbance_batch(ctypes.byref(s), _u32ptr(c), c.shape[0], _dptr(w))
    return w


# --------------------------------------------------------- model pieces ----

def dynamics(x, u, dt: float, wheelbase: float) -> np.ndarray:
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    ua = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    out = np.zeros(4)
    _load().orc_dynamics(_dptr(xa), _dptr(ua), float(dt), float(wheelbase), _dptr(out))
    return out


def track_terms(p: dict, x) -> tuple[float, float]:
    s = make_params(p, 0)
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    e, d = ctypes.c_double(), ctypes.c_double()
    _load().orc_track_terms(ctypes.byref(s), _dptr(xa), ctypes.byref(e), ctypes.byref(d))
    return e.value, d.value


def boundary_cost(d: float) -> float:
    return _load().orc_boundary_cost(float(d))


def obstacle_count(obs, px: float, py: float) -> int:
    o = np.ascontiguousarray(np.asarray(obs, dtype=np.float64).reshape(-1, 3))
    return _load().orc_obstacle_count(_dptr(o), o.shape[0], float(px), float(py))


def obstacle_margin(obs, px: float, py: float) -> float:
    o = np.ascontiguousarray(np.asarray(obs, dtype=np.float64).reshape(-1, 3))
    return _load().orc_obstacle_margin(_dptr(o), o.shape[0], float(px), float(py))


def running_cost(p: dict, obs, x) -> float:
    o = np.ascontiguousarray(np.asarray(obs, dtype=np.float64).reshape(-1, 3))
    s = make_params(p, o.shape[0])
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return _load().orc_running_cost(ctypes.byref(s), _dptr(o), _dptr(xa))


def track_radius(p: dict, x) -> float:
    s = make_params(p, 0)
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return _load().orc_track_radius(ctypes.byref(s), _dptr(xa))


def progress(p: dict, x0, x) -> float:
    s = make_params(p, 0)
    a0 = np.ascontiguousarray(np.asarray(x0, dtype=np.float64))
    a1 = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return _load().orc_progress(ctypes.byref(s), _dptr(a0), _dptr(a1))


def terminal_cost(p: dict, x0, x) -> float:
    s = make_params(p, 0)
    a0 = np.ascontiguousarray(np.asarray(x0, dtype=np.float64))
    a1 = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return _load().orc_terminal_cost(ctypes.byref(s), _dptr(a0), _dptr(a1))


def tail_size(alpha: float, M: int) -> tuple[int, int]:
    ka, nt = ctypes.c_int(), ctypes.c_int()
    _load().orc_tail_size(float(alpha), int(M), ctypes.byref(ka), ctypes.byref(nt))
    return ka.value, nt.value


def n_warm(eta: float, K: int) -> int:
    return _load().orc_n_warm(float(eta), int(K))


def scale_risk(L, B: float) -> np.ndarray:
    La = np.ascontiguousarray(np.asarray(L, dtype=np.float64))
    out = np.zeros_like(La)
    _load().orc_scale_risk(_dptr(La), La.size, float(B), _dptr(out))
    return out


def cvar(L, alpha: float, B: float = 1.0) -> float:
    La = np.ascontiguousarray(np.asarray(L, dtype=np.float64).ravel())
    return _load().orc_cvar(_dptr(La), La.size, float(alpha), float(B))


def cvar_batch(L: np.ndarray, alpha: float, B: float = 1.0) -> np.ndarray:
    La = np.ascontiguousarray(np.asarray(L, dtype=np.float64))
    K, M = La.shape
    out = np.zeros(K)
    _load().orc_cvar_batch(_dptr(La), K, M, float(alpha), float(B), _dptr(out))
    return out


def filtered_cost(S: float, cv: float, A: float, C_u: float) -> float:
    return _load().orc_filtered_cost(float(S), float(cv), float(A), float(C_u))


def weights(St, lam: float) -> tuple[np.ndarray, np.ndarray]:
    s = np.ascontiguousarray(np.asarray(St, dtype=np.float64))
    w = np.zeros_like(s)
    wh = np.zeros_like(s)
    _load().orc_weights(_dptr(s), s.size, float(lam), _dptr(w), _dptr(wh))
    return w, wh


def update(w_hat, u: np.ndarray) -> np.ndarray:
    """V+ (T x 2) from normalised weights (K) and controls (K x T x 2)."""
    wh = np.ascontiguousarray(np.asarray(w_hat, dtype=np.float64))
    ua = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    K, T = ua.shape[0], ua.shape[1]
    out = np.zeros((T, 2))
    _load().orc_update(_dptr(wh), _dptr(ua), K, T, _dptr(out))
    return out


def shift(Vplus) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(Vplus, dtype=np.float64))
    out = np.zeros_like(v)
    _load().orc_shift(_dptr(v), v.shape[0], _dptr(out))
    return out


def controls(p: dict, V, step_idx: int) -> np.ndarray:
    s = make_params(p, 0)
    Va = _as_f64(V).reshape(-1)
    out = np.zeros((s.K, s.T, 2))
    _load().orc_controls(ctypes.byref(s), _dptr(Va), int(step_idx) & 0xFFFFFFFF, _dptr(out))
    return out


def nominal_cost(p: dict, obs, x0, V, uk) -> tuple[float, float, float]:
    """(S, obstacle margin, minimum normalised track radius) of one sample."""
    o = _as_f64(obs).reshape(-1, 3)
    s = make_params(p, o.shape[0])
    a0 = _as_f64(x0)
    Va = _as_f64(V).reshape(-1)
    ua = np.ascontiguousarray(np.asarray(uk, dtype=np.float64).reshape(-1))
    mg, cd = ctypes.c_double(), ctypes.c_double()
    S = _load().orc_nominal_cost(ctypes.byref(s), _dptr(o), _dptr(a0), _dptr(Va), _dptr(ua), ctypes.byref(mg),
                                 ctypes.byref(cd))
    return S, mg.value, cd.value


def disturbed_cost(p: dict, obs, x0, uk, k: int, m: int, step_idx: int) -> tuple[float, float, float]:
    """(L, obstacle margin, minimum normalised track radius) of one draw."""
    o = _as_f64(obs).reshape(-1, 3)
    s = make_params(p, o.shape[0])
    a0 = _as_f64(x0)
    ua = np.ascontiguousarray(np.asarray(uk, dtype=np.float64).reshape(-1))
    mg, cd = ctypes.c_double(), ctypes.c_double()
    L = _load().orc_disturbed_cost(ctypes.byref(s), _dptr(o), _dptr(a0), _dptr(ua), int(k), int(m),
                                   int(step_idx) & 0xFFFFFFFF, ctypes.byref(mg), ctypes.byref(cd))
    return L, mg.value, cd.value


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return _load().orc_get_threads()


def step(p: dict, obs, x0, V, step_idx: int, diagnostics: bool = True) -> dict:
    """One RA-MPPI iteration (Algorithm 1).  Returns every intermediate; the
    margin and conditioning diagnostics are computed only when asked for."""
    o = _as_f64(obs).reshape(-1, 3)
    s = make_params(p, o.shape[0])
    K, T, M = s.K, s.T, s.M
    a0 = _as_f64(x0)
    Va = _as_f64(V).reshape(-1)
    out = {
        "u": np.zeros((K, T, 2)), "S": np.zeros(K), "L": np.zeros((K, M)), "cvar": np.zeros(K),
        "S_tilde": np.zeros(K), "w_hat": np.zeros(K), "V_plus": np.zeros((T, 2)),
        "V_next": np.zeros((T, 2)), "obs_margin": np.zeros((K, M)), "nom_margin": np.zeros(K),
        "obs_cond": np.zeros((K, M)), "nom_cond": np.zeros(K),
    }
    rc = _load().orc_step(ctypes.byref(s), _dptr(o), _dptr(a0), _dptr(Va), int(step_idx) & 0xFFFFFFFF,
                          _dptr(out["u"]), _dptr(out["S"]), _dptr(out["L"]), _dptr(out["cvar"]),
                          _dptr(out["S_tilde"]), _dptr(out["w_hat"]), _dptr(out["V_plus"]),
                          _dptr(out["V_next"]), *(
                              (_dptr(out["obs_margin"]), _dptr(out["nom_margin"]), _dptr(out["obs_cond"]),
                               _dptr(out["nom_cond"])) if diagnostics else (None, None, None, None)))
    if rc != 0:
        raise ValueError("oracle step rejected its arguments")
    out["u0"] = out["V_plus"][0].copy()
    return out


def rollout_subset(p: dict, obs, x0, V, step_idx: int, k0: int, nk: int) -> tuple[np.ndarray, np.ndarray]:
    """Nominal costs and risk costs of samples k0..k0+nk-1 only (timing helper)."""
    o = _as_f64(obs).reshape(-1, 3)
    s = make_params(p, o.shape[0])
    a0 = _as_f64(x0)
    Va = _as_f64(V).reshape(-1)
    S = np.zeros(nk)
    L = np.zeros((nk, s.M))
    _load().orc_rollout_subset(ctypes.byref(s), _dptr(o), _dptr(a0), _dptr(Va), int(step_idx) & 0xFFFFFFFF,
                               int(k0), int(nk), _dptr(S), _dptr(L))
    return S, L


# ------------------------------------------------------------- gradient ----

def running_cost_grad(p: dict, x) -> np.ndarray:
    s = make_params(p, 0)
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    g = np.zeros(4)
    _load().orc_running_cost_grad(ctypes.byref(s), _dptr(xa), _dptr(g))
    return g


def terminal_cost_grad(p: dict, x) -> np.ndarray:
    s = make_params(p, 0)
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    g = np.zeros(4)
    _load().orc_terminal_cost_grad(ctypes.byref(s), _dptr(xa), _dptr(g))
    return g


def free_energy(p: dict, obs, x0, V, step_idx: int, grad: bool = False):
    """J(V) = -lambda log mean_k exp(-S~_k/lambda) with the noise fixed, and
    optionally dJ/dV (T x 2).  V is taken as float64 as given (not rounded),
    so that finite differences can perturb it."""
    o = _as_f64(obs).reshape(-1, 3)
    s = make_params(p, o.shape[0])
    a0 = _as_f64(x0)
    Va = np.ascontiguousarray(np.asarray(V, dtype=np.float64).reshape(-1))
    g = np.zeros(Va.size) if grad else None
    J = _load().orc_free_energy(ctypes.byref(s), _dptr(o), _dptr(a0), _dptr(Va), int(step_idx) & 0xFFFFFFFF,
                                _dptr(g) if grad else None)
    return (J, g.reshape(-1, 2)) if grad else J
