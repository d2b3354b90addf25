"""Drivers shared by the GPU tests: run the HIP path through the C-ABI binding
on seeded inputs and compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np

from synth.sources import spatial_factors, time_factors


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(system, precision, samples, collect=None, tune=None, split=0, host=False):
    """Push samples[n][l] ([L+1][4][N] FP64) for l = 0..L and step.
    tune: {knob: value} set before binding; split: history split gap (0: off);
    host: real-space rings of the split history in pinned host memory.

    Returns {l: [dom][4][N] FP64 numpy} for l in `collect` (default: all)."""
    import torch
    from paper_2311_15429_amd import plan_for_system
    stream = torch.cuda.current_stream()
    p = plan_for_system(system, precision, stream=stream)
    for k, v in (tune or {}).items():
        p.set_tuning(k, v)
    if split:
        p.history_split(split)
        if host:
            p.history_host(True)
            assert p.host_history_bytes > 0
        assert p.stats()["split_rings"] > 0
    p.bind()
    p.set_green_kernels()
    dt = p.dtype
    outs = [torch.empty((4,) + d, dtype=dt, device="cuda") for d in p.dims]
    L = samples[0].shape[0] - 1
    collect = set(range(L + 1)) if collect is None else set(collect)
    res = {}
    for l in range(L + 1):
        src = [torch.from_numpy(np.ascontiguousarray(samples[n][l]).reshape((4,) + p.dims[n])).to("cuda", dt)
               for n in range(p.n_dom)]
        p.push_sources(l, src)
        p.retarded_step(l, outs)
        if l in collect:
            res[l] = [o.double().cpu().numpy().reshape(4, -1) for o in outs]
    torch.cuda.synchronize()
    p.close()
    return res


def rel_err(got, ref):
    """Per component: max over every point of every domain of |got - ref|
    divided by max |ref| (the error definition used for every parity bar)."""
    g = np.concatenate([np.asarray(x).reshape(4, -1) for x in got], axis=1)
    r = np.concatenate([np.asarray(x).reshape(4, -1) for x in ref], axis=1)
    return np.max(np.abs(g - r), axis=1) / np.maximum(np.max(np.abs(r), axis=1), 1e-300)


class GpuSourceGen:
    """Per-step sources on the GPU from the separable factors (FP64 matmul,
    then cast to the path dtype).  The same factors feed the oracle on the CPU."""

    def __init__(self, system, dtype):
        import torch
        self.system = system
        self.dtype = dtype
        self.B = []
        for d in system.domains:
            b = spatial_factors(d, system.h, system.c)
            self.B.append(torch.from_numpy(b.reshape(b.shape[0], -1)).to("cuda"))

    def step(self, l):
        import torch
        out = []
        for d, B in zip(self.system.domains, self.B):
            A = torch.from_numpy(time_factors(d, self.system.dt, [l])).to("cuda")
            out.append((A @ B).reshape((4,) + tuple(d.dims)).to(self.dtype).contiguous())
        return out


def cpu_sample_fn(system):
    B = [spatial_factors(d, system.h, system.c) for d in system.domains]

    def fn(n, j0, j1):
        A = time_factors(system.domains[n], system.dt, np.arange(j0, j1 + 1))
        nt = B[n].shape[0]
        return (A @ B[n].reshape(nt, -1)).reshape(j1 - j0 + 1, 4, -1)

    return fn


def pick_points(dims, n_pts, rng):
    """Flat indices ([4][Nx][Ny][Nz] layout, z fastest) of n_pts grid points of a
    box: its 8 corners, 6 face centres and 12 edge midpoints, then random
    points on random faces (a quarter of the rest) and random points inside."""
    nx, ny, nz = (int(v) for v in dims)
    hi = (nx - 1, ny - 1, nz - 1)
    mid = (nx // 2, ny // 2, nz // 2)
    pts = set()
    for i in (0, hi[0]):
        for j in (0, hi[1]):
            for k in (0, hi[2]):
                pts.add((i, j, k))
    for a in range(3):
        for side in (0, hi[a]):
            p = list(mid)
            p[a] = side
            pts.add(tuple(p))
    for a in range(3):                      # edges along axis a
        b, c = [x for x in range(3) if x != a]
        for vb in (0, hi[b]):
            for vc in (0, hi[c]):
                p = [0, 0, 0]
                p[a], p[b], p[c] = mid[a], vb, vc
                pts.add(tuple(p))
    n_face = max(0, (n_pts - len(pts)) // 4)
    total = nx * ny * nz
    guard = 0
    while len(pts) < min(n_pts, total) and guard < 100 * n_pts:
        guard += 1
        p = [int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))]
        if n_face > 0:
            a = int(rng.integers(0, 3))
            p[a] = 0 if rng.random() < 0.5 else hi[a]
            n_face -= 1
        pts.add(tuple(p))
    idx = np.array(sorted((i * ny + j) * nz + k for i, j, k in pts), dtype=np.int64)
    return idx[:n_pts] if len(idx) > n_pts else idx
