"""Multi-domain retarded Lorenz-gauge potentials on MI355X (gfx950).

The hot path (Green-spectrum generation, source FFTs into a history ring, the
lag-sum multiply-accumulate, inverse FFTs with crop) is hand-written HIP in
librpot.so behind the C-ABI of include/rpot.h; this package is its ctypes
binding.
"""
from .plan import Plan, plan_for_system
from .coupling import Oscillators
from ._lib import RpotError, load, LIB_PATH

__all__ = ["Plan", "plan_for_system", "Oscillators", "RpotError", "load", "LIB_PATH"]
