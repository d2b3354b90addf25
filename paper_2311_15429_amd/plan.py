"""Python face of the retarded-potential library: the same calls as the C-ABI
(include/rpot.h), with torch tensors supplying device memory and the stream.

No arithmetic of the method happens here: every step runs in the HIP kernels
of librpot.so, and a missing library is an error.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib


class Plan:
    """A planned multi-domain evaluation (rp_plan_domains).

    dims [n][3] and origins [n][3] (bohr) describe the sub-domain grids, h/dt/c
    the grid step, time step and speed of light (c may be math.inf).
    precision: "fp64", "fp32", "fp32_ring_fp16", "fp32_ring_bf16" or
    "fp32_ring_i16" (the history ring's storage, rpot.h rp_precision).
    """

    def __init__(self, dims, origins, h, dt, c, precision="fp32", system_id=None, stream=None):
        self._lib = _lib.load()
        dims = np.ascontiguousarray(dims, dtype=np.int32).reshape(-1, 3)
        origins = np.ascontiguousarray(origins, dtype=np.float64).reshape(-1, 3)
        if dims.shape != origins.shape:
            raise ValueError("dims and origins must both be [n][3]")
        self.n_dom = dims.shape[0]
        self.n_systems = 1 if system_id is None else len(set(int(v) for v in system_id))
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.precision = precision
        if precision not in _lib.PRECISION:
            raise ValueError(f"unknown precision {precision!r}")
        sid = None
        if system_id is not None:
            sid = np.ascontiguousarray(system_id, dtype=np.int32)
            if sid.shape != (self.n_dom,):
                raise ValueError("system_id must have one entry per domain")
        self._stream_obj = stream
        stream_ptr = None
        if stream is not None:
            stream_ptr = ctypes.c_void_p(int(stream.cuda_stream))
        handle = ctypes.c_void_p()
        i32p = ctypes.POINTER(ctypes.c_int32)
        code = self._lib.rp_plan_domains(
            ctypes.byref(handle), self.n_dom, dims.ctypes.data_as(i32p),
            origins.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            sid.ctypes.data_as(i32p) if sid is not None else None,
            float(h), float(dt), float(c), _lib.PRECISION[precision], stream_ptr)
        _lib.check(self._lib, None, code)
        self._h = handle
        self.targets = list(range(self.n_dom))
        self._ws = None
        self._host_hist = None

    # -- host-side queries ---------------------------------------------------
    @property
    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        _lib.check(self._lib, self._h, self._lib.rp_workspace_bytes(self._h, ctypes.byref(n)))
        return int(n.value)

    def info(self, s, n):
        lo, hi, depth = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        pad = (ctypes.c_int32 * 3)()
        _lib.check(self._lib, self._h, self._lib.rp_plan_info(
            self._h, int(s), int(n), ctypes.byref(lo), ctypes.byref(hi), pad, ctypes.byref(depth)))
        return int(lo.value), int(hi.value), tuple(int(v) for v in pad), int(depth.value)

    def stats(self) -> dict:
        st = _lib.RpStats()
        _lib.check(self._lib, self._h, self._lib.rp_plan_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in _lib.RpStats._fields_}

    # -- device calls --------------------------------------------------------
    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def bind(self, workspace=None, device="cuda", host_history=None):
        """Bind a workspace (a uint8 CUDA tensor of at least workspace_bytes);
        allocates one with torch when none is given.  With the host tier of a
        split history (history_host), also binds its pinned host buffer
        (host_history, a pinned uint8 CPU tensor of at least host_history_bytes;
        allocated with pin_memory=True when none is given)."""
        import torch
        nbytes = self.workspace_bytes
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        if workspace.device.type != "cuda" or workspace.dtype != torch.uint8:
            raise ValueError("workspace must be a uint8 CUDA tensor")
        ptr = workspace.data_ptr()
        off = (-ptr) % 256
        if workspace.numel() - off < nbytes:
            raise ValueError("workspace too small")
        hb = self.host_history_bytes
        if hb:
            if host_history is None:
                host_history = torch.empty(hb, dtype=torch.uint8, pin_memory=True)
            if host_history.device.type != "cpu" or host_history.dtype != torch.uint8:
                raise ValueError("host_history must be a uint8 CPU tensor")
            if not host_history.is_pinned():
                raise ValueError("host_history must be pinned (pin_memory=True)")
        self._ws = workspace
        _lib.check(self._lib, self._h, self._lib.rp_bind_workspace(
            self._h, ctypes.c_void_p(ptr + off), ctypes.c_size_t(workspace.numel() - off)))
        if hb:
            self._host_hist = host_history
            _lib.check(self._lib, self._h, self._lib.rp_bind_history_host(
                self._h, ctypes.c_void_p(host_history.data_ptr()), ctypes.c_size_t(host_history.numel())))
        return workspace

    def bind_static(self):
        """Bind the plan to the library's fixed device array
        (rp_bind_workspace_static): no device memory is allocated."""
        self._ws = None
        _lib.check(self._lib, self._h, self._lib.rp_bind_workspace_static(self._h))

    def set_green_kernels(self):
        _lib.check(self._lib, self._h, self._lib.rp_set_green_kernels(self._h))

    def _ptrs(self, tensors, allow_none=False):
        """Device pointers of one tensor per domain (allow_none: None for a
        domain that is not a target gives a null pointer)."""
        import torch
        if len(tensors) != self.n_dom:
            raise ValueError(f"expected {self.n_dom} tensors")
        if allow_none and any(t is None for t in tensors):
            for n, t in enumerate(tensors):
                if t is None and n in self.targets:
                    raise ValueError(f"domain {n} is a target and needs an output")
            live = [(t, d) for t, d in zip(tensors, self.dims) if t is not None]
            for t, d in live:
                if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != self.dtype \
                        or tuple(t.shape) != (4, *d) or not t.is_contiguous():
                    raise ValueError(f"output tensors must be contiguous {self.dtype} CUDA tensors [4][Nx][Ny][Nz]")
            return (ctypes.c_void_p * self.n_dom)(*[t.data_ptr() if t is not None else None for t in tensors])
        for t, d in zip(tensors, self.dims):
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
                raise ValueError("tensors must be CUDA tensors")
            if t.dtype != self.dtype:
                raise ValueError(f"tensors must be {self.dtype}")
            if tuple(t.shape) != (4, *d) or not t.is_contiguous():
                raise ValueError(f"tensor must be contiguous with shape {(4, *d)}")
        return (ctypes.c_void_p * self.n_dom)(*[t.data_ptr() for t in tensors])

    def push_sources(self, step, sources):
        arr = self._ptrs(sources)
        _lib.check(self._lib, self._h, self._lib.rp_push_sources(self._h, int(step), arr))

    def retarded_step(self, step, outputs):
        arr = self._ptrs(outputs, allow_none=True)
        _lib.check(self._lib, self._h, self._lib.rp_retarded_step(self._h, int(step), arr))

    def profile_lagsum(self, enable=True):
        _lib.check(self._lib, self._h, self._lib.rp_profile_lagsum(self._h, int(bool(enable))))

    def lagsum_time(self):
        """(summed lag-sum kernel ms, launches) since the last query."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _lib.check(self._lib, self._h, self._lib.rp_lagsum_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def set_tuning(self, knob, value):
        _lib.check(self._lib, self._h, self._lib.rp_set_tuning(self._h, _lib.TUNE[knob], int(value)))

    def get_tuning(self, knob):
        v = ctypes.c_int32()
        _lib.check(self._lib, self._h, self._lib.rp_get_tuning(self._h, _lib.TUNE[knob], ctypes.byref(v)))
        return int(v.value)

    def classes(self):
        """Shape classes: [{"dims", "pad", "n_domains", "fft_lds"}] in class order."""
        n = self.stats()["n_classes"]
        out = []
        for c in range(n):
            dims, pad, nd, v = (ctypes.c_int32 * 3)(), (ctypes.c_int32 * 3)(), ctypes.c_int32(), ctypes.c_int32()
            _lib.check(self._lib, self._h, self._lib.rp_class_info(self._h, c, dims, pad, ctypes.byref(nd)))
            _lib.check(self._lib, self._h, self._lib.rp_get_class_tuning(self._h, c, _lib.TUNE["fft_lds"],
                                                                         ctypes.byref(v)))
            out.append({"dims": tuple(dims), "pad": tuple(pad), "n_domains": int(nd.value), "fft_lds": int(v.value)})
        return out

    def set_class_tuning(self, cls, knob, value):
        """Per-class knob (only "fft_lds"); 0 follows the plan's value."""
        _lib.check(self._lib, self._h, self._lib.rp_set_class_tuning(self._h, int(cls), _lib.TUNE[knob], int(value)))

    def shape_key(self):
        """Autotuner cache key: device, precision and the plan's shape classes
        (grid and FFT pad per domain, with counts) and system count."""
        import torch
        classes = {}
        for n, d in enumerate(self.dims):
            pad = self.info(n, n)[2]
            classes[(d, pad)] = classes.get((d, pad), 0) + 1
        sig = ";".join(f"{d[0]}x{d[1]}x{d[2]}/{p[0]}x{p[1]}x{p[2]}*{c}" for (d, p), c in sorted(classes.items()))
        return (f"{torch.cuda.get_device_name()}|{self.precision}|{sig}|systems={self.n_systems}"
                f"|steps={self.get_tuning('lagsum_steps')}")

    def autotune(self, iters=3, cache=None):
        """Time every lag-sum schedule and, per shape class, every line-pass
        tile on this bound plan and keep the fastest.  With `cache` (a JSON file
        path) a stored choice for the same device and shape classes is applied
        without timing, and a new choice is stored.  Returns {"lagsum_unroll",
        "lagsum_persistent", "fft_lds" (the plan's), "fft_lds_per_class",
        "lagsum_ms", "cached"}."""
        import json
        import os
        key = self.shape_key() if cache else None
        if cache and os.path.exists(cache):
            try:
                rec = json.load(open(cache)).get(key)
            except (OSError, ValueError):
                rec = None
            if rec:
                for k in ("lagsum_unroll", "lagsum_persistent", "fft_lds", "lagsum_cached", "lagsum_tile_major"):
                    if k in rec:
                        self.set_tuning(k, rec[k])
                for c, v in enumerate(rec.get("fft_lds_per_class", [])):
                    self.set_class_tuning(c, "fft_lds", v)
                return dict(rec, cached=True)
        u, pe, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _lib.check(self._lib, self._h, self._lib.rp_autotune(self._h, int(iters), ctypes.byref(u),
                                                             ctypes.byref(pe), ctypes.byref(ms)))
        res = {"lagsum_unroll": int(u.value), "lagsum_persistent": int(pe.value),
               "lagsum_steps": self.get_tuning("lagsum_steps"), "lagsum_cached": self.get_tuning("lagsum_cached"),
               "lagsum_tile_major": self.get_tuning("lagsum_tile_major"),
               "fft_lds": self.get_tuning("fft_lds"),
               "fft_lds_per_class": [c["fft_lds"] for c in self.classes()], "lagsum_ms": float(ms.value)}
        if cache:
            data = {}
            if os.path.exists(cache):
                try:
                    data = json.load(open(cache))
                except (OSError, ValueError):
                    data = {}
            data[key] = res
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(res, cached=False)

    def capture_step(self, sources, outputs):
        """Record one whole step for these fixed buffers as a HIP graph."""
        s_arr = self._ptrs(sources)
        o_arr = self._ptrs(outputs, allow_none=True)
        self._graph_bufs = (list(sources), list(outputs))
        _lib.check(self._lib, self._h, self._lib.rp_capture_step(self._h, s_arr, o_arr))

    def launch_step(self, step):
        """Replay the captured step as step `step`."""
        _lib.check(self._lib, self._h, self._lib.rp_launch_step(self._h, int(step)))

    # -- far-pair surrogate --------------------------------------------------
    def set_targets(self, targets=None):
        """Evaluate only the sub-domains `targets` (indices; every sub-domain
        stays a source).  None or empty: every sub-domain.  Call before bind()."""
        t = np.ascontiguousarray(list(targets or []), dtype=np.int32)
        ptr = t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if t.size else None
        _lib.check(self._lib, self._h, self._lib.rp_plan_targets(self._h, ptr, int(t.size)))
        self.targets = [int(v) for v in t] if t.size else list(range(self.n_dom))

    def history_split(self, min_gap):
        """Split each source's history at lag gaps of at least min_gap lags
        (later windows in spectral rings of their own, fed from a real-space
        ring of the sources).  Call before bind(); min_gap <= 0 switches it off."""
        _lib.check(self._lib, self._h, self._lib.rp_history_split(self._h, int(min_gap)))

    def history_host(self, enable=True):
        """Keep the real-space rings of a split history in pinned host memory
        (streamed back one snapshot per split ring and step on a second
        stream).  Call before bind()."""
        _lib.check(self._lib, self._h, self._lib.rp_history_host(self._h, int(bool(enable))))

    @property
    def host_history_bytes(self):
        """Pinned host bytes the host tier needs (0 when nothing is split)."""
        b = ctypes.c_size_t(0)
        _lib.check(self._lib, self._h, self._lib.rp_history_host_bytes(self._h, ctypes.byref(b)))
        return b.value

    def surrogate_configure(self, far_factor, n_lags=64, audit=()):
        """Far pairs (centre distance > far_factor x the larger box diagonal)
        leave the plain lag sum; `audit` sources keep their plain history.
        Call before bind(); far_factor <= 0 switches the surrogate off."""
        aud = np.ascontiguousarray(list(audit), dtype=np.int32)
        ptr = aud.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if aud.size else None
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_configure(
            self._h, float(far_factor), int(n_lags), ptr, int(aud.size)))

    def surrogate_info(self) -> dict:
        v = [ctypes.c_int32() for _ in range(4)]
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_info(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("n_far", "n_audited", "n_in", "n_out"), (int(x.value) for x in v)))

    def surrogate_pairs(self) -> dict:
        n = self.surrogate_info()["n_far"]
        t, s, a, f = (np.zeros(max(n, 1), np.int32) for _ in range(4))
        d = np.zeros(max(n, 1), np.float64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_pairs(
            self._h, t.ctypes.data_as(i32p), s.ctypes.data_as(i32p),
            d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.ctypes.data_as(i32p), f.ctypes.data_as(i32p)))
        return {"target": t[:n], "source": s[:n], "dist": d[:n], "audited": a[:n].astype(bool),
                "fallen_back": f[:n].astype(bool)}

    def surrogate_attach(self, mlp, in_scale=None, out_scale=None):
        """Use `mlp` (an Mlp, or None to detach) for the far pairs of every later step."""
        fp = ctypes.POINTER(ctypes.c_float)
        if mlp is None:
            _lib.check(self._lib, self._h, self._lib.rp_surrogate_attach(self._h, None, None, None))
            self._mlp = None
            return
        ins = np.ascontiguousarray(in_scale, dtype=np.float32)
        outs = np.ascontiguousarray(out_scale, dtype=np.float32)
        if ins.shape != (22,) or outs.shape != (80,):
            raise ValueError("in_scale must have 22 and out_scale 80 entries")
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_attach(
            self._h, mlp._h, ins.ctypes.data_as(fp), outs.ctypes.data_as(fp)))
        self._mlp = mlp

    def surrogate_multipole(self, enable=True):
        """Analytic multipole terms for the far pairs: True (or 1) instead of a
        network, "hybrid" (or 2) with the attached network's output added as a
        correction, False (or 0) off."""
        mode = 2 if enable == "hybrid" else int(enable)
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_multipole(self._h, mode))
        if mode == 1:
            self._mlp = None

    def surrogate_multipole_response(self):
        """Multipole terms of the audited far pairs at the last completed step
        as frame coefficients [n_aud][80] (device), rows as surrogate_pair_response."""
        import torch
        na = self.surrogate_info()["n_audited"]
        coef = torch.zeros((max(na, 1), 80), dtype=torch.float32, device="cuda")
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_multipole_response(
            self._h, ctypes.c_void_p(coef.data_ptr())))
        return coef[:na]

    def surrogate_features(self, out=None):
        """Network inputs [n_far][n_in] (FP32, device) of the last completed step."""
        import torch
        info = self.surrogate_info()
        x = out if out is not None else torch.empty((info["n_far"], info["n_in"]), dtype=torch.float32,
                                                     device="cuda")
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_features(self._h, ctypes.c_void_p(x.data_ptr())))
        return x

    def surrogate_pair_response(self):
        """Plain pair responses of the audited far pairs at the last completed
        step: (frame coefficients [n_aud][80], residuals [n_aud][8]) on the device."""
        import torch
        na = self.surrogate_info()["n_audited"]
        coef = torch.zeros((max(na, 1), 80), dtype=torch.float32, device="cuda")
        resid = torch.zeros((max(na, 1), 8), dtype=torch.float32, device="cuda")
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_pair_response(
            self._h, ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(resid.data_ptr())))
        return coef[:na], resid[:na]

    def surrogate_judge(self, outputs, tol):
        """Judge the active audited far pairs of the last step against the plain
        sum; returns (pairs that fell back, largest error / budget).  Pairs
        re-admitted by the same call are in self.last_readmitted."""
        arr = self._ptrs(outputs)
        nf, worst, back = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_judge(self._h, arr, float(tol), ctypes.byref(nf),
                                                                    ctypes.byref(worst), ctypes.byref(back)))
        self.last_readmitted = int(back.value)
        return int(nf.value), float(worst.value)

    def surrogate_sample(self, pairs_per_judge=0, fallback_slots=16):
        """Judge the far pairs of non-audit sources too, by the direct sum at 64
        sample points, pairs_per_judge per judge call in turn (0: all; < 0:
        off); a failing pair takes one of fallback_slots slots.  Before bind()."""
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_sample(self._h, int(pairs_per_judge),
                                                                     int(fallback_slots)))

    def surrogate_sample_fields(self, far_pairs, out):
        """Plain pair fields of far pairs `far_pairs` at their 64 sample points
        at the last completed step into the device array out [n][64][4]."""
        import torch
        fp = np.ascontiguousarray(np.asarray(far_pairs, dtype=np.int32).reshape(-1))
        n = int(fp.size)
        if n and (tuple(out.shape) != (n, 64, 4) or not out.is_contiguous() or out.dtype != torch.float32):
            raise ValueError("out must be a contiguous float32 device array [n][64][4]")
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_sample_fields(
            self._h, fp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n, ctypes.c_void_p(out.data_ptr() if n else 0)))
        return out

    def surrogate_judge_stats(self) -> dict:
        """Of the last judge call: far pairs judged by sample and fallbacks
        refused for want of a slot; slots in use; the next pair of the rotation."""
        v = [ctypes.c_int32() for _ in range(4)]
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_judge_stats(self._h, *[ctypes.byref(x) for x in v]))
        return {"sampled": v[0].value, "refused": v[1].value, "slots_used": v[2].value, "next_pair": v[3].value}

    def surrogate_readmit(self, factor):
        """Fallen-back pairs within factor x their budget return to the far-pair
        terms at the next judgement (0: never)."""
        _lib.check(self._lib, self._h, self._lib.rp_surrogate_readmit(self._h, float(factor)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rp_plan_destroy(self._h)
            self._h = None
        self._ws = None
        self._host_hist = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_for_system(system, precision="fp32", stream=None):
    """Plan for a synthetic system description (dims, origins, h, dt, c, ids)."""
    return Plan(system.dims, system.origins, system.h, system.dt,
                system.c if math.isfinite(system.c) else math.inf,
                precision=precision, system_id=system.system_id, stream=stream)
