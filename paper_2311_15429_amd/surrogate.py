"""Training workflow of the far-pair surrogate on top of the C-ABI.

The plain method generates the teacher data: a plan configured with audit
sources returns, after every step, the network inputs and the targets (the
least-squares frame coefficients of the plain pair field times the pair
distance) of its audited far pairs (rp_surrogate_teacher).  The scales of the
inputs and targets (rp_surrogate_data_scales), the scaling
(rp_surrogate_scale_data), the network's training (rp_mlp_*) and its relative
RMS (rp_mlp_relative_rms) all run in the library's kernels.  This module only
allocates device memory, draws the initial weights and the random minibatch
indices, and passes pointers.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np

from . import _lib
from .mlp import Mlp

N_FEAT = 22
N_OUT = 80
N_BLOCKS = 6   # input blocks H, g H, f H, g f H, g^2 H, f^2 H


def _ptr(t, row=0):
    """Device address of row `row` of a contiguous 2-D tensor (or None)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr() + row * t.shape[1] * t.element_size())


def _stream():
    import torch
    return ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))


def collect_pair_responses(plan, sources_at, n_steps, start=1, every=1, outputs=None, residual=False):
    """Run `plan` (bound, Green kernels set, surrogate configured with audit
    sources, no network attached) from step 0 to n_steps - 1.  sources_at(l)
    returns the step's source tensors.  From step `start` on, every `every`
    steps, the library writes the inputs and targets of the audited far pairs
    into the next rows of X and T (rp_surrogate_teacher; residual=True: the
    targets minus the multipole terms, for a network that corrects the
    multipole expansion).

    Returns (X [N][n_in], T [N][80]) FP32 device tensors."""
    import torch
    info = plan.surrogate_info()
    n_aud = info["n_audited"]
    if n_aud == 0:
        raise ValueError("the plan has no audited far pairs")
    assert info["n_out"] == N_OUT
    collect = [l for l in range(n_steps) if l >= start and (l - start) % every == 0]
    X = torch.empty((len(collect) * n_aud, info["n_in"]), dtype=torch.float32, device="cuda")
    T = torch.empty((len(collect) * n_aud, N_OUT), dtype=torch.float32, device="cuda")
    outs = outputs or [torch.empty((4,) + d, dtype=plan.dtype, device="cuda") for d in plan.dims]
    lib = _lib.load()
    row = 0
    for l in range(n_steps):
        plan.push_sources(l, sources_at(l))
        plan.retarded_step(l, outs)
        if collect and l == collect[0]:
            collect.pop(0)
            _lib.check(lib, plan._h, lib.rp_surrogate_teacher(plan._h, _ptr(X, row), _ptr(T, row),
                                                               int(bool(residual))))
            row += n_aud
    return X, T


@dataclass
class TrainedSurrogate:
    mlp: Mlp
    in_scale: np.ndarray     # [22]
    out_scale: np.ndarray    # [80]
    n_lags: int
    history: list


def feature_scales(X, T, n_lags):
    """Input scale per moment (1 / RMS of the unmodulated block H over samples
    and lags) and one output scale per potential component (RMS over samples
    and its 20 coefficients), computed by rp_surrogate_data_scales."""
    import torch
    ins = torch.empty(N_FEAT, dtype=torch.float32, device="cuda")
    outs = torch.empty(N_OUT, dtype=torch.float32, device="cuda")
    lib = _lib.load()
    code = lib.rp_surrogate_data_scales(_ptr(X), _ptr(T), int(X.shape[0]), int(n_lags), ctypes.c_void_p(ins.data_ptr()),
                                        ctypes.c_void_p(outs.data_ptr()), _stream())
    if code != _lib.RP_OK:
        raise _lib.RpotError(code, "rp_surrogate_data_scales")
    return ins.cpu().numpy(), outs.cpu().numpy()


def scale_data(X, T, in_scale, out_scale, n_lags):
    """In place: X times the input scales, T over the output scales (either
    may be None), by rp_surrogate_scale_data."""
    import torch
    lib = _lib.load()
    ins = torch.as_tensor(np.asarray(in_scale, dtype=np.float32), device="cuda")
    outs = torch.as_tensor(np.asarray(out_scale, dtype=np.float32), device="cuda")
    n = int((X if X is not None else T).shape[0])
    code = lib.rp_surrogate_scale_data(_ptr(X), _ptr(T), n, int(n_lags), ctypes.c_void_p(ins.data_ptr()),
                                       ctypes.c_void_p(outs.data_ptr()), _stream())
    if code != _lib.RP_OK:
        raise _lib.RpotError(code, "rp_surrogate_scale_data")


def train_surrogate(X, T, n_lags, hidden=256, iters=20000, batch=2048, lr=3e-3, lr_end=1e-5, seed=0,
                    max_batch=None, log_every=0, log=print):
    """Fit the network to (X, T) with Adam on the GPU (cosine learning-rate
    decay from lr to lr_end).  max_batch: the largest inference batch the
    network must serve (the far-pair count of the plans it will attach to).
    X and T are left as they are (the library scales copies)."""
    import torch
    n_in = X.shape[1]
    in_scale, out_scale = feature_scales(X, T, n_lags)
    Xs, Ts = X.clone(), T.clone()
    scale_data(Xs, Ts, in_scale, out_scale, n_lags)
    mlp = Mlp(n_in, hidden, N_OUT, max(batch, max_batch or 0, 1))
    g = torch.Generator(device="cpu").manual_seed(seed)
    parts = []
    for fan_in, fan_out in ((n_in, hidden), (hidden, hidden)):
        parts.append(torch.randn(fan_in * fan_out, generator=g) * math.sqrt(1.0 / fan_in))
        parts.append(torch.zeros(fan_out))
    # the output layer and the linear skip start at zero
    parts += [torch.zeros(hidden * N_OUT), torch.zeros(N_OUT), torch.zeros(n_in * N_OUT)]
    mlp.set_params(torch.cat(parts).float())
    gi = torch.Generator(device="cuda").manual_seed(seed + 1)
    n = Xs.shape[0]
    history = []
    for it in range(iters):
        idx = torch.randint(0, n, (min(batch, n),), generator=gi, device="cuda")
        xb = Xs.index_select(0, idx).contiguous()
        tb = Ts.index_select(0, idx).contiguous()
        lr_t = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * it / max(iters - 1, 1)))
        loss = mlp.train_step(xb, tb, lr_t)
        if log_every and (it % log_every == 0 or it == iters - 1):
            v = float(loss.item())
            history.append((it, v))
            log(f"  iter {it:6d}  loss {v:.3e}  lr {lr_t:.2e}")
    return TrainedSurrogate(mlp, in_scale, out_scale, n_lags, history)


def relative_rms(sur: TrainedSurrogate, X, T):
    """RMS of (prediction - T) over RMS of T (rp_mlp_relative_rms on the
    scaled inputs)."""
    import torch
    Xs = X.clone()
    scale_data(Xs, None, sur.in_scale, sur.out_scale, sur.n_lags)
    osc = torch.as_tensor(np.asarray(sur.out_scale, dtype=np.float32), device="cuda")
    Tc = T.contiguous()
    rel = ctypes.c_double()
    lib = _lib.load()
    _lib.check_mlp(lib, sur.mlp._h, lib.rp_mlp_relative_rms(sur.mlp._h, _ptr(Xs), _ptr(Tc),
                                                             int(X.shape[0]), ctypes.c_void_p(osc.data_ptr()),
                                                             ctypes.byref(rel)))
    return float(rel.value)
