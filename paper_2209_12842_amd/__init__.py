"""MI355X-native Risk-Aware MPPI (arXiv 2209.12842): one control step as HIP
kernels for gfx950 behind a C ABI (include/ramppi.h), with this thin binding.

    from paper_2209_12842_amd import Controller, workloads
    w = workloads.make_world("c2")
    ctl = Controller(w["params"], w["obstacles"])
    V = ctl.new_V()
    u0 = ctl.step(w["x0"], V, step_idx=0)
"""
from ._binding import (MPPI_F_ALLOW_ZERO_NOISE, MPPI_F_DEBUG, MPPI_F_GRAD, MPPI_F_SHIFT, Batch, Controller,
                       MppiError, Params, check, cvar, free_energy, header_functions, last_error, lib, make_params,
                       normals, philox, step_noalloc)

__all__ = ["Batch", "Controller", "MppiError", "Params", "check", "cvar", "header_functions", "last_error", "lib",
           "make_params", "normals", "philox", "free_energy", "step_noalloc", "MPPI_F_DEBUG", "MPPI_F_SHIFT",
           "MPPI_F_ALLOW_ZERO_NOISE", "MPPI_F_GRAD"]
