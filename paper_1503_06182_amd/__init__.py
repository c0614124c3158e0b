"""MI355X (gfx950) VEGAS hot path: counter-keyed events, grid map, phase space,
matrix elements, exact per-iteration combine and grid refinement, behind the C
ABI of include/vegas.h.  ``vegas`` is the ctypes binding."""
from .vegas import (DY_Z, EEMUMU, FP32_ME, FP64, GAUSS, GENZ, W_PLUS, WW_4L, WW_HAD, Integrator,
                    VegasError, load, vegas_sigma, workspace_size)
from .flow import Flow, choose_proposal, train

__all__ = ["Integrator", "VegasError", "Flow", "train", "choose_proposal", "vegas_sigma", "load", "workspace_size", "GAUSS", "GENZ", "EEMUMU",
           "DY_Z", "W_PLUS", "WW_4L", "WW_HAD", "FP64", "FP32_ME"]
