"""Binding of the oscillator source model (rp_osc_* in include/rpot.h): the
steps either side of the potential evaluation in the propagation loop.  Torch
supplies device memory; projection, update and source synthesis run in
librpot.so kernels on the plan's stream."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib


class Oscillators:
    """Lorentz oscillators with fixed source shapes, driven by the potentials
    of a plan.  bases[n]: CUDA tensor [K_n][4][*dims[n]] (or [K_n][4][N_n]) in the plan's source
    dtype (None where K_n = 0); params[n]: [K_n][4] = omega, gamma, kappa, drive."""

    def __init__(self, plan, bases, params):
        import torch
        self._lib = _lib.load()
        self.plan = plan
        n_osc = [0 if b is None else int(b.shape[0]) for b in bases]
        if len(bases) != plan.n_dom or len(params) != plan.n_dom:
            raise ValueError(f"expected {plan.n_dom} bases and params")
        for b, d in zip(bases, plan.dims):
            if b is not None and (b.device.type != "cuda" or b.dtype != plan.dtype or not b.is_contiguous()
                                  or b.numel() != b.shape[0] * 4 * int(np.prod(d)) or b.shape[1] != 4):
                raise ValueError("each basis must be a contiguous CUDA tensor [K][4][*dims] or [K][4][N] "
                                 "of the plan dtype")
        P = np.ascontiguousarray(np.concatenate([np.asarray(p, np.float64).reshape(-1, 4) for p in params]))
        if P.shape[0] != sum(n_osc):
            raise ValueError("params must hold one row per oscillator")
        self.n_osc = n_osc
        self.total = sum(n_osc)
        self._bases = bases
        h = ctypes.c_void_p()
        k = (ctypes.c_int32 * plan.n_dom)(*n_osc)
        _lib.check_osc(self._lib, None, self._lib.rp_osc_create(
            ctypes.byref(h), plan._h, k, P.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self._h = h
        nb = ctypes.c_size_t()
        self._chk(self._lib.rp_osc_workspace_bytes(h, ctypes.byref(nb)))
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        off = (-self._ws.data_ptr()) % 256
        arr = (ctypes.c_void_p * plan.n_dom)(*[None if b is None else b.data_ptr() for b in bases])
        self._chk(self._lib.rp_osc_bind(h, ctypes.c_void_p(self._ws.data_ptr() + off), nb.value, arr))

    def _chk(self, code):
        _lib.check_osc(self._lib, self._h, code)

    def set_state(self, q, qdot):
        q = np.ascontiguousarray(np.asarray(q, np.float64).reshape(self.total))
        qd = np.ascontiguousarray(np.asarray(qdot, np.float64).reshape(self.total))
        dp = ctypes.POINTER(ctypes.c_double)
        self._chk(self._lib.rp_osc_set_state(self._h, q.ctypes.data_as(dp), qd.ctypes.data_as(dp)))

    def sources(self, src):
        self._chk(self._lib.rp_osc_sources(self._h, self.plan._ptrs(src)))

    def step(self, potentials, e_ext, src_next):
        """Forces from the potentials of step l, update, sources of step l + 1."""
        self._chk(self._lib.rp_osc_step(self._h, self.plan._ptrs(potentials), float(e_ext),
                                        self.plan._ptrs(src_next)))

    def state(self):
        """(q, qdot, phi, psi) host arrays [total]; synchronises the stream."""
        out = [np.zeros(self.total) for _ in range(4)]
        dp = ctypes.POINTER(ctypes.c_double)
        self._chk(self._lib.rp_osc_state(self._h, *[o.ctypes.data_as(dp) for o in out]))
        return tuple(out)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rp_osc_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
