"""ctypes binding of libramppi.so (declarations and contracts in include/ramppi.h).

Argument marshalling only: every step of the control update runs in the HIP
kernels of the library.  PyTorch provides device memory (the workspace and
the mean sequence are torch tensors) and streams (the current stream of the
tensor's device).  If the library has not been built, every entry point
raises RuntimeError; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libramppi.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "ramppi.h")

MPPI_OK, MPPI_EINVAL, MPPI_ENOMEM, MPPI_EDEVICE, MPPI_EUNSUPPORTED = 0, -1, -2, -3, -4
MPPI_F_DEBUG, MPPI_F_SHIFT, MPPI_F_ALLOW_ZERO_NOISE, MPPI_F_GRAD, MPPI_F_SPLIT_UPDATE = 1, 2, 4, 8, 16
STATUS_NAMES = {0: "MPPI_OK", -1: "MPPI_EINVAL", -2: "MPPI_ENOMEM", -3: "MPPI_EDEVICE", -4: "MPPI_EUNSUPPORTED"}


class MppiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


class Params(ctypes.Structure):
    """Mirror of mppi_params."""
    _fields_ = [
        ("K", ctypes.c_int32), ("T", ctypes.c_int32), ("M", ctypes.c_int32), ("n_obs", ctypes.c_int32),
        ("dt", ctypes.c_float), ("wheelbase", ctypes.c_float),
        ("u_lo", ctypes.c_float * 2), ("u_hi", ctypes.c_float * 2),
        ("sigma_eps", ctypes.c_float * 2), ("sigma_w", ctypes.c_float * 4),
        ("alpha", ctypes.c_float), ("lam", ctypes.c_float), ("gamma", ctypes.c_float), ("eta", ctypes.c_float),
        ("A", ctypes.c_float), ("B", ctypes.c_float), ("C_u", ctypes.c_float),
        ("c_bdry", ctypes.c_float), ("c_obs", ctypes.c_float), ("c_dev", ctypes.c_float), ("c_v", ctypes.c_float),
        ("v_ref", ctypes.c_float), ("c4", ctypes.c_float), ("c5", ctypes.c_float),
        ("track", ctypes.c_float * 5),
        ("seed", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
        ("noise_kind", ctypes.c_uint32),
        ("jump_prob", ctypes.c_float), ("jump_size", ctypes.c_float),
    ]


class DebugPtrs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("u", "S", "L", "cvar", "S_tilde", "w_hat", "u0")]


_lib = None


def lib():
    """The loaded library; RuntimeError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libramppi.so is not built (run: python -m paper_2209_12842_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, V, I32, I64, U32, U64, F = (ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float)
        L.mppi_validate.argtypes = [P(Params)]
        L.mppi_validate.restype = ctypes.c_int
        L.mppi_workspace_bytes.argtypes = [P(Params)]
        L.mppi_workspace_bytes.restype = ctypes.c_size_t
        L.mppi_create.argtypes = [P(Params), P(F), V, ctypes.c_size_t, V, P(V)]
        L.mppi_create.restype = ctypes.c_int
        L.mppi_step.argtypes = [V, P(F), V, U32, P(F), V]
        L.mppi_step.restype = ctypes.c_int
        L.mppi_step_noalloc.argtypes = [P(Params), V, P(F), V, U32, V, V]
        L.mppi_step_noalloc.restype = ctypes.c_int
        L.mppi_grad.argtypes = [V, P(F), V, U32, V, V, V]
        L.mppi_grad.restype = I32
        L.mppi_destroy.argtypes = [V]
        L.mppi_destroy.restype = ctypes.c_int
        L.mppi_serve_start.argtypes = [V, V, U32, V]
        L.mppi_serve_start.restype = I32
        L.mppi_serve_step.argtypes = [V, P(F), U32, P(F)]
        L.mppi_serve_step.restype = I32
        L.mppi_serve_stop.argtypes = [V]
        L.mppi_serve_stop.restype = I32
        L.mppi_last_error.argtypes = []
        L.mppi_last_error.restype = ctypes.c_char_p
        L.mppi_debug_view.argtypes = [V, P(DebugPtrs)]
        L.mppi_debug_view.restype = ctypes.c_int
        L.mppi_timing_enable.argtypes = [V, ctypes.c_int]
        L.mppi_timing_enable.restype = ctypes.c_int
        L.mppi_timing_read.argtypes = [V, P(ctypes.c_double), P(ctypes.c_double), P(I32)]
        L.mppi_timing_read.restype = ctypes.c_int
        L.mppi_philox.argtypes = [U64, V, V, I64, V]
        L.mppi_philox.restype = ctypes.c_int
        L.mppi_normals.argtypes = [U64, V, V, I64, V]
        L.mppi_normals.restype = ctypes.c_int
        L.mppi_cvar.argtypes = [V, I32, I32, F, F, V, V]
        L.mppi_cvar.restype = ctypes.c_int
        L.mppi_batch_workspace_bytes.argtypes = [I32, P(Params)]
        L.mppi_batch_workspace_bytes.restype = ctypes.c_size_t
        L.mppi_batch_create.argtypes = [I32, P(Params), P(P(F)), P(V), V, ctypes.c_size_t, V, P(V)]
        L.mppi_batch_create.restype = ctypes.c_int
        L.mppi_batch_step.argtypes = [V, P(F), P(U32), P(F), V]
        L.mppi_batch_step.restype = ctypes.c_int
        L.mppi_batch_autotune.argtypes = [V, I32, V, P(I32), P(I32)]
        L.mppi_batch_autotune.restype = ctypes.c_int
        L.mppi_batch_set_graph.argtypes = [V, ctypes.c_int]
        L.mppi_batch_set_graph.restype = ctypes.c_int
        L.mppi_batch_debug_view.argtypes = [V, I32, P(DebugPtrs)]
        L.mppi_batch_debug_view.restype = ctypes.c_int
        L.mppi_batch_timing_enable.argtypes = [V, ctypes.c_int]
        L.mppi_batch_timing_enable.restype = I32
        L.mppi_batch_timing_read.argtypes = [V, P(ctypes.c_double), P(ctypes.c_double), P(I32)]
        L.mppi_batch_timing_read.restype = I32
        L.mppi_timing_candidates.argtypes = [V, V, P(U64)]
        L.mppi_timing_candidates.restype = I32
        L.mppi_batch_timing_candidates.argtypes = [V, V, P(U64)]
        L.mppi_batch_timing_candidates.restype = I32
        L.mppi_timing_work.argtypes = [V, V, P(U64), P(U64)]
        L.mppi_timing_work.restype = I32
        L.mppi_batch_timing_work.argtypes = [V, V, P(U64), P(U64)]
        L.mppi_batch_timing_work.restype = I32
        L.mppi_batch_destroy.argtypes = [V]
        L.mppi_batch_destroy.restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions include/ramppi.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mppi_[a-z_0-9]+)\s*\(", text)))


def last_error() -> str:
    return lib().mppi_last_error().decode()


def check(status: int) -> None:
    if status != MPPI_OK:
        raise MppiError(status, last_error())


def make_params(p: dict, n_obs: int, flags: int = 0) -> Params:
    """mppi_params from a workload dict (lambda under the key 'lam')."""
    s = Params()
    s.K, s.T, s.M, s.n_obs = int(p["K"]), int(p["T"]), int(p["M"]), int(n_obs)
    s.dt, s.wheelbase = float(p["dt"]), float(p["wheelbase"])
    for i in range(2):
        s.u_lo[i], s.u_hi[i], s.sigma_eps[i] = float(p["u_lo"][i]), float(p["u_hi"][i]), float(p["sigma_eps"][i])
    for i in range(4):
        s.sigma_w[i] = float(p["sigma_w"][i])
    for name in ("alpha", "lam", "gamma", "eta", "A", "B", "C_u", "c_bdry", "c_obs", "c_dev", "c_v", "v_ref",
                 "c4", "c5"):
        setattr(s, name, float(p[name]))
    for i in range(5):
        s.track[i] = float(p["track"][i])
    s.seed = int(p["seed"]) & 0xFFFFFFFFFFFFFFFF
    s.flags = int(flags) | (MPPI_F_SHIFT if p.get("shift", False) else 0)
    s.noise_kind = int(p.get("noise_kind", 0))
    s.jump_prob = float(p.get("jump_prob", 0.0))
    s.jump_size = float(p.get("jump_size", 0.0))
    return s


def _torch():
    import torch
    return torch


def _stream_ptr(device) -> int:
    """The current torch stream of `device` as a raw hipStream_t."""
    torch = _torch()
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:  # no Stream object per call (about 2 us less per step)
        idx = device.index if isinstance(device, torch.device) else torch.device(device).index
        return raw(torch.cuda.current_device() if idx is None else idx)
    return torch.cuda.current_stream(device).cuda_stream


class Controller:
    """One RA-MPPI controller on one GPU.

    params: workload dict (see workloads.PRESETS), obstacles: n x 3 (cx, cy, r).
    The workspace is a torch uint8 tensor on `device`; steps run on the current
    torch stream of that device."""

    def __init__(self, params: dict, obstacles, device="cuda", debug: bool = False,
                 allow_zero_noise: bool = False, grad: bool = False, split_update: bool = False):
        torch = _torch()
        L = lib()
        obs = np.ascontiguousarray(np.asarray(obstacles, dtype=np.float32).reshape(-1, 3))
        flags = ((MPPI_F_DEBUG if debug else 0) | (MPPI_F_ALLOW_ZERO_NOISE if allow_zero_noise else 0)
                 | (MPPI_F_GRAD if grad else 0) | (MPPI_F_SPLIT_UPDATE if split_update else 0))
        self.params = dict(params)
        self.p = make_params(params, obs.shape[0], flags)
        nbytes = L.mppi_workspace_bytes(ctypes.byref(self.p))
        if nbytes == 0:
            raise MppiError(L.mppi_validate(ctypes.byref(self.p)), last_error())
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._obs = obs
        self._h = ctypes.c_void_p()
        self._u0 = (ctypes.c_float * 2)()
        with torch.cuda.device(self.device):
            check(L.mppi_create(ctypes.byref(self.p), obs.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                ctypes.c_void_p(_stream_ptr(self.device)), ctypes.byref(self._h)))
        self.K, self.T, self.M = self.p.K, self.p.T, self.p.M
        self._x0 = (ctypes.c_float * 4)()
        self._step_fn = L.mppi_step
        self._serve_fn = L.mppi_serve_step
        self._serve_V = None

    def new_V(self, V0=None):
        """A T x 2 float32 mean sequence on the controller's device."""
        torch = _torch()
        if V0 is None:
            return torch.zeros((self.T, 2), dtype=torch.float32, device=self.device)
        return torch.as_tensor(np.asarray(V0, dtype=np.float32).reshape(self.T, 2)).to(self.device)

    def step(self, x0, V, step_idx: int, want_u0: bool = True):
        """Enqueue one step; V (T x 2 float32, contiguous, on the device) is
        updated in place.  Returns the first command (2 floats) when want_u0,
        after waiting for the step; otherwise returns None at once."""
        torch = _torch()
        if not (V.is_cuda and V.dtype == torch.float32 and V.is_contiguous() and V.numel() == 2 * self.T):
            raise ValueError("V must be a contiguous float32 CUDA tensor with T x 2 elements")
        x = self._x0
        x[0], x[1], x[2], x[3] = (float(v) for v in x0)
        u0p = self._u0 if want_u0 else None
        check(self._step_fn(self._h, x, V.data_ptr(), int(step_idx) & 0xFFFFFFFF, u0p, _stream_ptr(V.device)))
        if want_u0:
            return np.array([self._u0[0], self._u0[1]], dtype=np.float32)
        return None

    def free_energy(self, x0, V, step_idx: int):
        """(J, dJ/dV) on the device for the step's samples and draws with the
        noise held fixed; needs grad=True at construction.  V is read only."""
        torch = _torch()
        if not (V.is_cuda and V.dtype == torch.float32 and V.is_contiguous() and V.numel() == 2 * self.T):
            raise ValueError("V must be a contiguous float32 CUDA tensor with T x 2 elements")
        x = self._x0
        x[0], x[1], x[2], x[3] = (float(v) for v in x0)
        J = torch.empty((), dtype=torch.float32, device=V.device)
        g = torch.empty_like(V)
        check(lib().mppi_grad(self._h, x, V.data_ptr(), int(step_idx) & 0xFFFFFFFF, g.data_ptr(), J.data_ptr(),
                              _stream_ptr(V.device)))
        return J, g

    def debug(self) -> dict:
        """Views into the workspace: u (T, K, 2), S, L (K, M), cvar, S_tilde,
        w_hat (K) and u0 (2).  L and w_hat are written only with debug=True."""
        torch = _torch()
        d = DebugPtrs()
        check(lib().mppi_debug_view(self._h, ctypes.byref(d)))
        base = self.workspace.data_ptr()
        f32 = self.workspace.view(torch.uint8)

        def view(ptr, shape):
            n = int(np.prod(shape))
            off = ptr - base
            return f32[off:off + 4 * n].view(torch.float32).view(*shape)

        K, T, M = self.K, self.T, self.M
        return dict(u=view(d.u, (T, K, 2)), S=view(d.S, (K,)), L=view(d.L, (K, M)), cvar=view(d.cvar, (K,)),
                    S_tilde=view(d.S_tilde, (K,)), w_hat=view(d.w_hat, (K,)), u0=view(d.u0, (2,)))

    def timing_enable(self, on: bool = True, resume: bool = False) -> None:
        """Start (clearing earlier records), resume (keeping them) or pause kernel timing."""
        check(lib().mppi_timing_enable(self._h, (2 if resume else 1) if on else 0))

    def timing_read(self) -> tuple[float, float, int]:
        """(summed rollout-kernel ms, summed update-kernels ms, steps) since enable/read."""
        r, u, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        check(lib().mppi_timing_read(self._h, ctypes.byref(r), ctypes.byref(u), ctypes.byref(n)))
        return r.value, u.value, n.value

    def timing_candidates(self) -> int:
        """Exact obstacle tests (wave, state step, obstacle) that passed the broad phase, over the steps
        timed since the last call."""
        n = ctypes.c_uint64()
        check(lib().mppi_timing_candidates(self._h, ctypes.c_void_p(_stream_ptr(self.device)), ctypes.byref(n)))
        return n.value

    def timing_work(self) -> tuple:
        """(exact obstacle tests, broad-phase group tests) over the steps timed since the last call."""
        n, g = ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().mppi_timing_work(self._h, ctypes.c_void_p(_stream_ptr(self.device)), ctypes.byref(n),
                                     ctypes.byref(g)))
        return n.value, g.value

    def serve_start(self, V, idle_ms: int = 2000) -> None:
        """Starts a persistent serving launch (mppi_serve_start) that keeps V
        (T x 2 float32 on the device) for the session and runs one step per
        serve_step call, each bit-identical to step(..., want_u0=True)."""
        torch = _torch()
        if not (V.is_cuda and V.dtype == torch.float32 and V.is_contiguous() and V.numel() == 2 * self.T):
            raise ValueError("V must be a contiguous float32 CUDA tensor with T x 2 elements")
        check(lib().mppi_serve_start(self._h, V.data_ptr(), int(idle_ms), _stream_ptr(V.device)))
        self._serve_V = V  # the session writes it

    def serve_step(self, x0, step_idx: int):
        """Posts the measured state and returns the first command (2 floats)."""
        x = self._x0
        x[0], x[1], x[2], x[3] = (float(v) for v in x0)
        check(self._serve_fn(self._h, x, int(step_idx) & 0xFFFFFFFF, self._u0))
        return np.array([self._u0[0], self._u0[1]], dtype=np.float32)

    def serve_stop(self) -> None:
        """Ends the serving session (nothing to do when none runs)."""
        if self._h:
            check(lib().mppi_serve_stop(self._h))
        self._serve_V = None

    def close(self) -> None:
        if self._h:
            lib().mppi_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def philox(seed: int, ctr):
    """Philox4x32-10 words (n x 4 int32 tensor holding uint32 bits) of n counters."""
    torch = _torch()
    ctr = ctr.contiguous()
    if ctr.dtype != torch.int32 or ctr.dim() != 2 or ctr.shape[1] != 4 or not ctr.is_cuda:
        raise ValueError("ctr must be an (n, 4) int32 CUDA tensor")
    out = torch.empty_like(ctr)
    check(lib().mppi_philox(int(seed) & 0xFFFFFFFFFFFFFFFF, ctypes.c_void_p(ctr.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), ctr.shape[0], ctypes.c_void_p(_stream_ptr(ctr.device))))
    return out


def normals(seed: int, ctr):
    """Four Box-Muller normals (n x 4 float32) per Philox counter."""
    torch = _torch()
    ctr = ctr.contiguous()
    if ctr.dtype != torch.int32 or ctr.dim() != 2 or ctr.shape[1] != 4 or not ctr.is_cuda:
        raise ValueError("ctr must be an (n, 4) int32 CUDA tensor")
    out = torch.empty(ctr.shape, dtype=torch.float32, device=ctr.device)
    check(lib().mppi_normals(int(seed) & 0xFFFFFFFFFFFFFFFF, ctypes.c_void_p(ctr.data_ptr()),
                             ctypes.c_void_p(out.data_ptr()), ctr.shape[0],
                             ctypes.c_void_p(_stream_ptr(ctr.device))))
    return out


def cvar(L, alpha: float, B: float = 1.0):
    """Per-row CVaR of a K x M float32 CUDA tensor."""
    torch = _torch()
    L = L.contiguous()
    if L.dtype != torch.float32 or L.dim() != 2 or not L.is_cuda:
        raise ValueError("L must be a (K, M) float32 CUDA tensor")
    out = torch.empty(L.shape[0], dtype=torch.float32, device=L.device)
    check(lib().mppi_cvar(ctypes.c_void_p(L.data_ptr()), L.shape[0], L.shape[1], float(alpha), float(B),
                          ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream_ptr(L.device))))
    return out


def step_noalloc(params: dict, obstacles, x0, V, step_idx: int, u0=None, allow_zero_noise: bool = False) -> None:
    """One step through mppi_step_noalloc (no handle, no workspace: the
    library's static scratch).  obstacles: n x 3 float32 CUDA tensor (or None
    for none), V: T x 2 float32 CUDA tensor updated in place, u0: None or a
    2-float CUDA tensor receiving the first command.  Enqueues on the current
    stream of V's device and returns."""
    torch = _torch()
    if not (V.is_cuda and V.dtype == torch.float32 and V.is_contiguous()):
        raise ValueError("V must be a contiguous float32 CUDA tensor")
    n_obs = 0
    obs_ptr = None
    if obstacles is not None:
        if not (obstacles.is_cuda and obstacles.dtype == torch.float32 and obstacles.is_contiguous()
                and obstacles.dim() == 2 and obstacles.shape[1] == 3):
            raise ValueError("obstacles must be a contiguous (n, 3) float32 CUDA tensor")
        n_obs = int(obstacles.shape[0])
        obs_ptr = ctypes.c_void_p(obstacles.data_ptr()) if n_obs else None
    if u0 is not None and not (u0.is_cuda and u0.dtype == torch.float32 and u0.numel() == 2 and u0.is_contiguous()):
        raise ValueError("u0 must be a contiguous float32 CUDA tensor of 2 elements")
    pr = make_params(params, n_obs, MPPI_F_ALLOW_ZERO_NOISE if allow_zero_noise else 0)
    if V.numel() != 2 * pr.T:
        raise ValueError("V must hold T x 2 elements")
    x = (ctypes.c_float * 4)(*(float(v) for v in x0))
    with torch.cuda.device(V.device):
        check(lib().mppi_step_noalloc(ctypes.byref(pr), obs_ptr, x, ctypes.c_void_p(V.data_ptr()),
                                      int(step_idx) & 0xFFFFFFFF,
                                      ctypes.c_void_p(u0.data_ptr()) if u0 is not None else None,
                                      ctypes.c_void_p(_stream_ptr(V.device))))


class Batch:
    """Many independent controllers served by one step call (mppi_batch_*).

    params: list of workload dicts, obstacles: list of n_i x 3 arrays.  Each
    controller's mean sequence is a T_i x 2 float32 tensor in `self.V[i]`,
    updated in place by every step."""

    def __init__(self, params: list, obstacles: list, device="cuda", debug: bool = False, V0=None):
        torch = _torch()
        L = lib()
        n = len(params)
        self.n = n
        obs = [np.ascontiguousarray(np.asarray(o, dtype=np.float32).reshape(-1, 3)) for o in obstacles]
        flags = MPPI_F_DEBUG if debug else 0
        self.p = (Params * n)(*[make_params(params[i], obs[i].shape[0], flags) for i in range(n)])
        nbytes = L.mppi_batch_workspace_bytes(n, self.p)
        if nbytes == 0:
            raise MppiError(MPPI_EINVAL, last_error())
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.V = []
        for i in range(n):
            T = self.p[i].T
            v = torch.zeros((T, 2), dtype=torch.float32, device=self.device)
            if V0 is not None and V0[i] is not None:
                v.copy_(torch.as_tensor(np.asarray(V0[i], dtype=np.float32).reshape(T, 2)))
            self.V.append(v)
        self._obs = obs
        optrs = (ctypes.POINTER(ctypes.c_float) * n)(*[o.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) for o in obs])
        vptrs = (ctypes.c_void_p * n)(*[v.data_ptr() for v in self.V])
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.mppi_batch_create(n, self.p, optrs, vptrs, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                      ctypes.c_void_p(_stream_ptr(self.device)), ctypes.byref(self._h)))
        self._x0 = (ctypes.c_float * (4 * n))()
        self._idx = (ctypes.c_uint32 * n)()
        self._u0 = (ctypes.c_float * (2 * n))()

    def step(self, x0, step_idx, want_u0: bool = True):
        """x0: n x 4 states; step_idx: an int (same for all) or n ints."""
        torch = _torch()
        xs = np.asarray(x0, dtype=np.float32).reshape(self.n * 4)
        ctypes.memmove(self._x0, xs.ctypes.data, 16 * self.n)
        idx = np.broadcast_to(np.asarray(step_idx, dtype=np.uint32), (self.n,))
        ctypes.memmove(self._idx, np.ascontiguousarray(idx).ctypes.data, 4 * self.n)
        check(lib().mppi_batch_step(self._h, self._x0, self._idx, self._u0 if want_u0 else None,
                                    _stream_ptr(self.device)))
        if want_u0:
            return np.frombuffer(self._u0, dtype=np.float32).reshape(self.n, 2).copy()
        return None

    def autotune(self, trials: int = 3) -> tuple[int, int]:
        wg, order = ctypes.c_int32(), ctypes.c_int32()
        check(lib().mppi_batch_autotune(self._h, int(trials), ctypes.c_void_p(_stream_ptr(self.device)),
                                        ctypes.byref(wg), ctypes.byref(order)))
        return wg.value, order.value

    def set_graph(self, on: bool) -> None:
        check(lib().mppi_batch_set_graph(self._h, 1 if on else 0))

    def timing_enable(self, on: bool = True) -> None:
        """While on, steps launch directly (no graph) with events around the kernels."""
        check(lib().mppi_batch_timing_enable(self._h, 1 if on else 0))

    def timing_read(self) -> tuple[float, float, int]:
        """(summed rollout-kernel ms, summed update-kernel ms, steps) since enable/read."""
        r, u, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        check(lib().mppi_batch_timing_read(self._h, ctypes.byref(r), ctypes.byref(u), ctypes.byref(n)))
        return r.value, u.value, n.value

    def timing_candidates(self) -> int:
        """Exact obstacle tests (wave, state step, obstacle) that passed the broad phase, over the steps
        timed since the last call."""
        n = ctypes.c_uint64()
        check(lib().mppi_batch_timing_candidates(self._h, ctypes.c_void_p(_stream_ptr(self.device)),
                                                 ctypes.byref(n)))
        return n.value

    def timing_work(self) -> tuple:
        """(exact obstacle tests, broad-phase group tests) over the batch's steps timed since the last call."""
        n, g = ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().mppi_batch_timing_work(self._h, ctypes.c_void_p(_stream_ptr(self.device)), ctypes.byref(n),
                                           ctypes.byref(g)))
        return n.value, g.value

    def debug(self, i: int) -> dict:
        torch = _torch()
        d = DebugPtrs()
        check(lib().mppi_batch_debug_view(self._h, int(i), ctypes.byref(d)))
        base = self.workspace.data_ptr()
        K, T, M = self.p[i].K, self.p[i].T, self.p[i].M

        def view(ptr, shape):
            n = int(np.prod(shape))
            off = ptr - base
            return self.workspace[off:off + 4 * n].view(torch.float32).view(*shape)

        return dict(u=view(d.u, (T, K, 2)), S=view(d.S, (K,)), L=view(d.L, (K, M)), cvar=view(d.cvar, (K,)),
                    S_tilde=view(d.S_tilde, (K,)), w_hat=view(d.w_hat, (K,)), u0=view(d.u0, (2,)))

    def close(self) -> None:
        if self._h:
            lib().mppi_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _free_energy_fn():
    torch = _torch()

    class FreeEnergy(torch.autograd.Function):
        """J(V) of a controller step as a differentiable function of V (the
        sampled controls and disturbances held fixed); forward and backward
        both run in the library's kernels."""

        @staticmethod
        def forward(ctx, V, controller, x0, step_idx):
            J, g = controller.free_energy(x0, V.detach().contiguous(), step_idx)
            ctx.save_for_backward(g)
            return J

        @staticmethod
        def backward(ctx, gJ):
            (g,) = ctx.saved_tensors
            return gJ * g, None, None, None

    return FreeEnergy


_FREE_ENERGY = None


def free_energy(V, controller: "Controller", x0, step_idx: int):
    """Differentiable J(V) (torch autograd) of one controller step."""
    global _FREE_ENERGY
    if _FREE_ENERGY is None:
        _FREE_ENERGY = _free_energy_fn()
    return _FREE_ENERGY.apply(V, controller, x0, step_idx)
