"""MI355X-native MPPI (arXiv 2409.07563): one MPPI iteration as hand-written
HIP kernels for gfx950 behind the C ABI of include/mppi.h.

    from paper_2409_07563_amd import Controller
    ctl = Controller(problem)        # problem: a workload description
    ctl.iterate(10)
    U = ctl.controls()               # torch tensor [T][m] on the GPU
"""
from ._abi import MPPIError, lib  # noqa: F401
from .controller import Controller, noise, noise_tables  # noqa: F401
from .autograd import MPPISteps, MPPIStep, mppi_step, mppi_steps  # noqa: F401

__all__ = ["Controller", "MPPIError", "lib", "noise", "noise_tables"]
