"""Training workflow of the far-pair surrogate on top of the C-ABI.

The plain method generates the teacher data: a plan configured with audit
sources returns, after every step, the network inputs of its far pairs
(rp_surrogate_features) and the least-squares frame coefficients of the plain
pair field of its audited far pairs (rp_surrogate_pair_response).  The network
is trained by the library's own forward/backward/Adam kernels (rp_mlp_*).
Torch supplies device memory, random minibatch indices and the feature
statistics used to scale inputs and outputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .mlp import Mlp

N_FEAT = 22
N_OUT = 80
N_BLOCKS = 6   # input blocks H, g H, f H, g f H, g^2 H, f^2 H


def collect_pair_responses(plan, sources_at, n_steps, start=1, every=1, outputs=None, residual=False):
    """Run `plan` (bound, Green kernels set, surrogate configured with audit
    sources, no network attached) from step 0 to n_steps - 1.  sources_at(l)
    returns the step's source tensors.  From step `start` on, every `every`
    steps, keeps the raw features and the targets (frame coefficients times
    the pair distance) of the audited far pairs.  residual=True: the targets
    are the plain responses minus the multipole terms (for a network that
    corrects the multipole expansion).

    Returns (X [N][n_in], T [N][80]) FP32 device tensors."""
    import torch
    info = plan.surrogate_info()
    pairs = plan.surrogate_pairs()
    aud = np.nonzero(pairs["audited"])[0]
    if len(aud) == 0:
        raise ValueError("the plan has no audited far pairs")
    rows = torch.as_tensor(aud, dtype=torch.long, device="cuda")
    dist = torch.as_tensor(pairs["dist"][aud], dtype=torch.float32, device="cuda")[:, None]
    outs = outputs or [torch.empty((4,) + d, dtype=plan.dtype, device="cuda") for d in plan.dims]
    X, T = [], []
    for l in range(n_steps):
        plan.push_sources(l, sources_at(l))
        plan.retarded_step(l, outs)
        if l >= start and (l - start) % every == 0:
            x = plan.surrogate_features()
            coef, _ = plan.surrogate_pair_response()
            if residual:
                coef = coef - plan.surrogate_multipole_response()
            X.append(x.index_select(0, rows))
            T.append(coef * dist)
    assert info["n_out"] == N_OUT
    return torch.cat(X), torch.cat(T)


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
    and its 20 coefficients), so that the loss weighs coefficient errors by
    their share of the field error; zero columns get scale 1."""
    import torch
    xm = X[:, :n_lags * N_FEAT].reshape(-1, n_lags, N_FEAT)
    rms_in = torch.sqrt(torch.mean(xm.double() ** 2, dim=(0, 1))).cpu().numpy()
    rms_out = torch.sqrt(torch.mean(T.double().reshape(-1, 4, N_OUT // 4) ** 2, dim=(0, 2))).cpu().numpy()
    in_scale = np.where(rms_in > 0, 1.0 / np.maximum(rms_in, 1e-300), 1.0).astype(np.float32)
    out_scale = np.repeat(np.where(rms_out > 0, rms_out, 1.0), N_OUT // 4).astype(np.float32)
    return in_scale, out_scale


def scale_inputs(X, in_scale, n_lags):
    import torch
    s = torch.ones(X.shape[1], dtype=torch.float32, device=X.device)
    s[:N_BLOCKS * n_lags * N_FEAT] = torch.as_tensor(np.tile(in_scale, N_BLOCKS * n_lags), device=X.device)
    return X * s


def train_surrogate(X, T, n_lags, hidden=256, iters=20000, batch=2048, lr=3e-3, lr_end=1e-5, seed=0,
                    max_batch=None, log_every=0, log=print):
    """Fit the network to (X, T) with Adam on the GPU (cosine learning-rate
    decay from lr to lr_end).  max_batch: the largest inference batch the
    network must serve (the far-pair count of the plans it will attach to)."""
    import torch
    n_in = X.shape[1]
    in_scale, out_scale = feature_scales(X, T, n_lags)
    Xs = scale_inputs(X, in_scale, n_lags).contiguous()
    Ts = (T / torch.as_tensor(out_scale, device=T.device)).contiguous()
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


def relative_rms(sur: TrainedSurrogate, X, T, chunk=4096):
    """RMS of (prediction - T) over RMS of T, per sample set."""
    import torch
    Xs = scale_inputs(X, sur.in_scale, sur.n_lags)
    osc = torch.as_tensor(sur.out_scale, device=X.device)
    num = den = 0.0
    chunk = min(chunk, sur.mlp.max_batch)
    for i in range(0, Xs.shape[0], chunk):
        xb = Xs[i:i + chunk].contiguous()
        y = sur.mlp.forward(xb) * osc
        num += float(torch.sum((y - T[i:i + chunk]) ** 2))
        den += float(torch.sum(T[i:i + chunk] ** 2))
    return math.sqrt(num / max(den, 1e-300))
