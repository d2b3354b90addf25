"""Binding of the surrogate network (rp_mlp_* in include/rpot.h): torch tensors
supply device memory; training and inference run in librpot.so kernels."""
from __future__ import annotations

import ctypes

from . import _lib


class Mlp:
    """n_in -> H -> H -> n_out tanh network with a linear skip (n_in -> n_out),
    trained with Adam on the GPU."""

    def __init__(self, n_in, n_hidden, n_out, max_batch, stream=None):
        import torch
        self._lib = _lib.load()
        self.n_in, self.n_hidden, self.n_out, self.max_batch = n_in, n_hidden, n_out, max_batch
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(int(stream.cuda_stream)) if stream is not None else None
        _lib.check_mlp(self._lib, None, self._lib.rp_mlp_create(ctypes.byref(h), n_in, n_hidden, n_out,
                                                                  max_batch, sp))
        self._h = h
        nb = ctypes.c_size_t()
        _lib.check_mlp(self._lib, h, self._lib.rp_mlp_workspace_bytes(h, ctypes.byref(nb)))
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        off = (-self._ws.data_ptr()) % 256
        _lib.check_mlp(self._lib, h, self._lib.rp_mlp_bind(h, ctypes.c_void_p(self._ws.data_ptr() + off),
                                                            nb.value))
        n = ctypes.c_int64()
        _lib.check_mlp(self._lib, h, self._lib.rp_mlp_n_params(h, ctypes.byref(n)))
        self.n_params = int(n.value)
        self._loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def _chk(self, code):
        _lib.check_mlp(self._lib, self._h, code)

    @staticmethod
    def _p(t):
        return ctypes.c_void_p(t.data_ptr())

    def set_params(self, flat):
        import torch
        flat = flat.to("cuda", torch.float32).contiguous()
        assert flat.numel() == self.n_params
        self._chk(self._lib.rp_mlp_set_params(self._h, self._p(flat)))
        torch.cuda.current_stream().synchronize()

    def get_params(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self._chk(self._lib.rp_mlp_get_params(self._h, self._p(out)))
        return out

    def forward(self, x, out=None):
        import torch
        x = x.contiguous()
        assert x.dtype == torch.float32 and x.shape[1] == self.n_in
        y = out if out is not None else torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        self._chk(self._lib.rp_mlp_forward(self._h, self._p(x), int(x.shape[0]), self._p(y)))
        return y

    def loss_grad(self, x, t):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self._chk(self._lib.rp_mlp_loss_grad(self._h, self._p(x.contiguous()), self._p(t.contiguous()),
                                             int(x.shape[0]), self._p(self._loss), self._p(g)))
        return self._loss.clone(), g

    def train_step(self, x, t, lr):
        self._chk(self._lib.rp_mlp_train_step(self._h, self._p(x), self._p(t), int(x.shape[0]), float(lr),
                                              self._p(self._loss)))
        return self._loss

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rp_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def unflatten(flat, n_in, n_hidden, n_out):
    """Split a flat parameter vector into (W1, b1, W2, b2, W3, b3, Ws)."""
    sizes = [n_in * n_hidden, n_hidden, n_hidden * n_hidden, n_hidden, n_hidden * n_out, n_out, n_in * n_out]
    shapes = [(n_in, n_hidden), (n_hidden,), (n_hidden, n_hidden), (n_hidden,), (n_hidden, n_out), (n_out,),
              (n_in, n_out)]
    out, o = [], 0
    for n, sh in zip(sizes, shapes):
        out.append(flat[o:o + n].reshape(sh))
        o += n
    return out
