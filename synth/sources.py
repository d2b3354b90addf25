"""Seeded synthetic sources for the multi-domain retarded-potential workloads.

The paper's sources are Kohn-Sham densities of molecules, which are not
available; seeded analytic Gaussian charges stand in for them.

Charge density of a +/- pair that shares width s and amplitude q(t):
    rho(r, t) = q(t) [g_s(r - c+) - g_s(r - c-)],  g_s(r) = (pi s^2)^(-3/2) exp(-r^2/s^2)
(the potential of g_s per unit charge is erf(r/s)/r).  Its current is the
line-current tube
    J(r, t) = qdot(t) (c+ - c-) int_0^1 g_s(r - c- - u (c+ - c-)) du,
which satisfies d_t rho = -div J exactly in the continuum.  In closed form,
with L = |c+ - c-|, xi = (r - c-).(c+ - c-)/L and rho_perp^2 = |r - c-|^2 - xi^2,
    int_0^1 g_s(...) du = (pi s^2)^(-3/2) exp(-rho_perp^2/s^2)
                          * sqrt(pi) s / (2 L) * [erf(xi/s) - erf((xi - L)/s)].

The 4-vector source given to the library and to the oracle is
S = (rho, Jx/c, Jy/c, Jz/c) with charge +1 (both are component-agnostic).

Every source is separable, S(r, t_j) = sum_terms A[j, term] * B[term](r): this
module returns the spatial factors B ([n_terms][4][Nx*Ny*Nz], z fastest) and
the temporal factors A ([n_steps][n_terms]) per domain, and samples
S_j = A[j] @ B.  It holds none of the retarded-potential arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import erf

C_AU = 137.036


@dataclass
class Charge:
    """One Gaussian charge or +/- pair inside a domain.

    kind: "pair" (centres cp, cm) or "single" (centre cp).
    profile: ("cos", a, w, p) -> q = a cos(w t + p);
             ("const", q);  ("step", q0, q1) -> q0 at sample 0, q1 from sample 1.
    """
    kind: str
    s: float
    cp: np.ndarray
    cm: np.ndarray | None
    profile: tuple


@dataclass
class Domain:
    dims: tuple
    origin: np.ndarray            # position of grid point (0,0,0), bohr
    charges: list = field(default_factory=list)

    @property
    def n_points(self) -> int:
        return int(np.prod(self.dims))


@dataclass
class System:
    h: float
    dt: float
    c: float
    domains: list
    system_id: list | None = None  # per-domain system id (batched plans)
    name: str = ""

    @property
    def dims(self) -> np.ndarray:
        return np.array([d.dims for d in self.domains], dtype=np.int32)

    @property
    def origins(self) -> np.ndarray:
        return np.array([d.origin for d in self.domains], dtype=np.float64)


def grid_points(dom: Domain, h: float) -> np.ndarray:
    """Absolute coordinates of every grid point, [N][3], C order (z fastest)."""
    nx, ny, nz = dom.dims
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    return dom.origin[None, :] + h * pts


def _gauss(pts, centre, s):
    d2 = np.sum((pts - centre[None, :]) ** 2, axis=1)
    return (math.pi * s * s) ** -1.5 * np.exp(-d2 / (s * s))


def _tube(pts, cp, cm, s):
    d = cp - cm
    L = float(np.linalg.norm(d))
    if L == 0.0:
        return np.zeros(len(pts))
    dh = d / L
    rel = pts - cm[None, :]
    xi = rel @ dh
    rp2 = np.maximum(np.sum(rel * rel, axis=1) - xi * xi, 0.0)
    return ((math.pi * s * s) ** -1.5 * np.exp(-rp2 / (s * s))
            * (math.sqrt(math.pi) * s / (2.0 * L)) * (erf(xi / s) - erf((xi - L) / s)))


def spatial_factors(dom: Domain, h: float, c: float) -> np.ndarray:
    """Spatial factors B[term][4][N] (FP64) of one domain's sources."""
    pts = grid_points(dom, h)
    n = len(pts)
    terms = []
    for ch in dom.charges:
        if ch.kind == "pair":
            b = np.zeros((4, n))
            b[0] = _gauss(pts, ch.cp, ch.s) - _gauss(pts, ch.cm, ch.s)
            terms.append(b)
            bj = np.zeros((4, n))
            if math.isfinite(c):
                tube = _tube(pts, ch.cp, ch.cm, ch.s)
                for a in range(3):
                    bj[1 + a] = (ch.cp[a] - ch.cm[a]) * tube / c
            terms.append(bj)
        elif ch.kind == "single":
            b = np.zeros((4, n))
            b[0] = _gauss(pts, ch.cp, ch.s)
            terms.append(b)
        else:
            raise ValueError(ch.kind)
    if not terms:
        return np.zeros((0, 4, n))
    return np.stack(terms)


def _profile(prof, t, j):
    kind = prof[0]
    if kind == "cos":
        a, w, p = prof[1:]
        return a * np.cos(w * t + p), -a * w * np.sin(w * t + p)
    if kind == "const":
        return np.full_like(t, prof[1]), np.zeros_like(t)
    if kind == "step":
        q = np.where(j <= 0, prof[1], prof[2]).astype(np.float64)
        return q, np.zeros_like(t)
    raise ValueError(kind)


def time_factors(dom: Domain, dt: float, steps) -> np.ndarray:
    """Temporal factors A[len(steps)][term] (FP64) at sample indices `steps`."""
    j = np.asarray(steps, dtype=np.int64)
    t = j.astype(np.float64) * dt
    cols = []
    for ch in dom.charges:
        q, qd = _profile(ch.profile, t, j)
        if ch.kind == "pair":
            cols += [q, qd]
        else:
            cols.append(q)
    if not cols:
        return np.zeros((len(j), 0))
    return np.stack(cols, axis=1)


def sample_sources(system: System, steps, factors=None) -> list:
    """Samples S_j for every domain: list over domains of [len(steps)][4][N]."""
    out = []
    for i, dom in enumerate(system.domains):
        B = factors[i] if factors is not None else spatial_factors(dom, system.h, system.c)
        A = time_factors(dom, system.dt, steps)
        nt = B.shape[0]
        if nt == 0:
            out.append(np.zeros((len(steps), 4, dom.n_points)))
            continue
        out.append((A @ B.reshape(nt, -1)).reshape(len(steps), 4, -1))
    return out


# ----------------------------------------------------------------------------
# Workload recipes
# ----------------------------------------------------------------------------

def _random_pairs(rng, dom: Domain, h: float, n_pairs: int):
    lo = dom.origin
    hi = dom.origin + h * (np.array(dom.dims) - 1)
    for _ in range(n_pairs):
        s = rng.uniform(0.8, 1.5)
        cp = rng.uniform(lo, hi)
        cm = rng.uniform(lo, hi)
        a = rng.uniform(0.1, 1.0)
        w = rng.uniform(0.1, 0.5)
        p = rng.uniform(0.0, 2.0 * math.pi)
        dom.charges.append(Charge("pair", s, cp, cm, ("cos", a, w, p)))


def _centred_domain(centre, n, h):
    centre = np.asarray(centre, dtype=np.float64)
    return Domain((n, n, n), centre - 0.5 * (n - 1) * h)


def config1(seed: int = 1) -> System:
    """Two 16^3 domains, h = 0.5, centres 30 bohr apart on x, dt = 0.02, FP64 case."""
    rng = np.random.default_rng(seed)
    h = 0.5
    doms = [_centred_domain((0, 0, 0), 16, h), _centred_domain((30, 0, 0), 16, h)]
    for d in doms:
        _random_pairs(rng, d, h, 2)
    return System(h, 0.02, C_AU, doms, name=f"2x16^3 h=0.5 d=30 seed={seed}")


def _place_centres(rng, n_dom, side_of, box, min_dist, h, max_dist=None, tries=200000):
    centres = []
    sides = [side_of(i) for i in range(n_dom)]
    for i in range(n_dom):
        for _ in range(tries):
            half = 0.5 * sides[i]
            cand = rng.uniform(half, box - half, size=3)
            ok = True
            for j, cj in enumerate(centres):
                dist = float(np.linalg.norm(cand - cj))
                cheb = float(np.max(np.abs(cand - cj)))
                if dist < min_dist or cheb < 0.5 * (sides[i] + sides[j]) + h:
                    ok = False
                    break
                if max_dist is not None and dist > max_dist:
                    ok = False
                    break
            if ok:
                centres.append(cand)
                break
        else:
            raise RuntimeError("placement failed")
    return centres


def config2(seed: int = 0, n_dom: int = 8, n: int = 64, n_pairs: int = 16) -> System:
    """Eight 64^3 domains, h = 0.3, random in a 400-bohr box, dt = 0.01, FP32 case."""
    rng = np.random.default_rng(seed)
    h = 0.3
    side = (n - 1) * h
    centres = _place_centres(rng, n_dom, lambda i: side, 400.0, 20.0, h)
    doms = [_centred_domain(cc, n, h) for cc in centres]
    for d in doms:
        _random_pairs(rng, d, h, n_pairs)
    return System(h, 0.01, C_AU, doms, name=f"{n_dom}x{n}^3 h=0.3 box=400 seed={seed}")


def config3_twin(sys2: System, n: int = 32) -> System:
    """Down-scaled twin: same centres, charges and dt, each domain resampled at n^3
    with the same physical side."""
    n0 = sys2.domains[0].dims[0]
    side = (n0 - 1) * sys2.h
    h = side / (n - 1)
    doms = []
    for d in sys2.domains:
        centre = d.origin + 0.5 * side
        nd = _centred_domain(centre, n, h)
        nd.charges = list(d.charges)
        doms.append(nd)
    return System(h, sys2.dt, sys2.c, doms, name=f"twin {len(doms)}x{n}^3 h={h:.4f}")


def config4(seed: int = 0, n_systems: int = 64, sizes=(32, 48, 64, 96),
            n_dom_range=(2, 16), n_pairs: int = 16) -> System:
    """Batched case: independent systems with uneven domain counts and grid sizes,
    h = 0.3, pair centre distances in [20, 300], dt = 0.01."""
    rng = np.random.default_rng(seed)
    h = 0.3
    doms, sid = [], []
    for s in range(n_systems):
        nd = int(rng.integers(n_dom_range[0], n_dom_range[1] + 1))
        ns = [int(rng.choice(sizes)) for _ in range(nd)]
        sides = [(k - 1) * h for k in ns]
        # centres in a 300-bohr-diameter ball: every pair distance <= 300
        cents = []
        for i in range(nd):
            for _ in range(200000):
                cand = rng.uniform(-150, 150, size=3)
                if np.linalg.norm(cand) > 150.0:
                    continue
                ok = all(np.linalg.norm(cand - cj) >= 20.0 and
                         np.max(np.abs(cand - cj)) >= 0.5 * (sides[i] + sides[j]) + h
                         for j, cj in enumerate(cents))
                if ok:
                    cents.append(cand)
                    break
            else:
                raise RuntimeError("placement failed")
        offset = np.array([1000.0 * s, 0.0, 0.0])
        for i in range(nd):
            d = _centred_domain(cents[i] + offset, ns[i], h)
            _random_pairs(rng, d, h, n_pairs)
            doms.append(d)
            sid.append(s)
    return System(h, 0.01, C_AU, doms, system_id=sid,
                  name=f"{n_systems} systems, sizes {sizes}, seed={seed}")


def config5(seed: int = 0, n_dom: int = 32, n: int = 48, n_pairs: int = 16, box: float = 2000.0) -> System:
    """32 domains of 48^3, h = 0.3, random in a 2000-bohr box, dt = 0.01
    (smaller n_dom, n and box give the same recipe at test size)."""
    rng = np.random.default_rng(seed)
    h = 0.3
    side = (n - 1) * h
    centres = _place_centres(rng, n_dom, lambda i: side, box, 20.0, h)
    doms = [_centred_domain(cc, n, h) for cc in centres]
    for d in doms:
        _random_pairs(rng, d, h, n_pairs)
    return System(h, 0.01, C_AU, doms, name=f"{n_dom}x{n}^3 h=0.3 box={box:g} seed={seed}")


def wire_pair(W: int = 32, L: int = 128, d: int = 128, h: float = 0.3, dt: float = 0.01,
              n_pairs: int = 8, seed: int = 0) -> System:
    """Two elongated W x W x L point domains, long axis z, side by side along y:
    domain 0 occupies y points [0, W), domain 1 [d - W, d), so the box that
    encloses both has W x d x L points (the geometry of the paper's cost
    comparison, Sec. III).  Each domain holds n_pairs seeded charge pairs."""
    if d < 2 * W:
        raise ValueError("the domains would overlap: need d >= 2 W")
    rng = np.random.default_rng(seed)
    doms = [Domain((W, W, L), np.array([0.0, 0.0, 0.0])),
            Domain((W, W, L), np.array([0.0, h * (d - W), 0.0]))]
    for dm in doms:
        _random_pairs(rng, dm, h, n_pairs)
    return System(h, dt, C_AU, doms, name=f"wire pair {W}x{W}x{L} d={d} h={h}")


def enclosing_domain(system: System):
    """One domain whose grid holds every point of every domain of `system`
    (the domains' grids must share the lattice of spacing h).  Returns the
    one-domain System (no charges: its sources are the sub-domains' sources
    placed in it, zero elsewhere) and, per sub-domain, the index slices of
    its block inside the enclosing grid."""
    h = system.h
    lo = np.min(system.origins, axis=0)
    hi = np.max(system.origins + h * (system.dims - 1), axis=0)
    dims = tuple(int(round(v)) + 1 for v in (hi - lo) / h)
    blocks = []
    for dm in system.domains:
        off = (dm.origin - lo) / h
        k = np.rint(off).astype(int)
        if np.max(np.abs(off - k)) > 1e-9:
            raise ValueError("sub-domain grids are not on one lattice")
        blocks.append(tuple(slice(int(k[a]), int(k[a]) + dm.dims[a]) for a in range(3)))
    return System(h, system.dt, system.c, [Domain(dims, lo.copy())], name=f"enclosing {dims}"), blocks


def pair_shapes(dom: Domain, h: float, c: float) -> np.ndarray:
    """Per charge pair of the domain, its fixed source shape [K][4][N]: the
    charge part (component 0) and the current part per unit dq/dt (components
    1-3, divided by c), from the separable factors."""
    B = spatial_factors(dom, h, c)
    if any(ch.kind != "pair" for ch in dom.charges):
        raise ValueError("every charge must be a pair")
    K = len(dom.charges)
    out = np.zeros((K, 4, dom.n_points))
    out[:, 0] = B[0::2, 0]
    out[:, 1:4] = B[1::2, 1:4]
    return out


def paper_pair(d: float, seed: int = 0, n_pairs: int = 8) -> System:
    """The paper's two-molecule geometry (Sec. IV): two 20 x 20 x 50 bohr boxes
    (50 x 50 x 125 points at h = 0.4), long axis z, centres d bohr apart along
    y, dt = 1 as = 0.04134 a.u.; seeded charge pairs stand in for the molecules."""
    rng = np.random.default_rng(seed)
    h, dims = 0.4, (50, 50, 125)
    half = 0.5 * h * (np.array(dims) - 1)
    doms = [Domain(dims, np.array(c, float) - half) for c in ((0.0, 0.0, 0.0), (0.0, d, 0.0))]
    for dm in doms:
        _random_pairs(rng, dm, h, n_pairs)
    return System(h, 0.04134, C_AU, doms, name=f"paper pair d={d:g}")



# ----------------------------------------------------------------------------
# The same sources evaluated with torch (any device), in compact form
# ----------------------------------------------------------------------------

class TorchSources:
    """Sources of the domains of `system` (or of `domains`, a list of indices)
    evaluated with torch on `device` in FP64, from the same seeded charges as
    spatial_factors / time_factors.  Each charge contributes its density
    field to component 0 and, for a pair, its tube field times (c+ - c-)/c to
    components 1-3, so a domain keeps one or two fields per charge instead of
    four components per term.  step(l, dtype) -> list of [4][Nx][Ny][Nz]."""

    def __init__(self, system: System, device, domains=None):
        import torch
        self.torch = torch
        self.system = system
        self.device = torch.device(device)
        self.doms = list(range(len(system.domains))) if domains is None else list(domains)
        self.fields = {}
        for i in self.doms:
            self.fields[i] = self._fields(system.domains[i])

    def _fields(self, dom: Domain):
        torch = self.torch
        h, c = self.system.h, self.system.c
        nx, ny, nz = dom.dims
        f64 = dict(dtype=torch.float64, device=self.device)
        ax = [dom.origin[a] + h * torch.arange(n, **f64) for a, n in enumerate((nx, ny, nz))]
        X, Y, Z = torch.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
        pts = torch.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], dim=1)

        def gauss(centre, s):
            d2 = torch.sum((pts - torch.as_tensor(centre, **f64)[None, :]) ** 2, dim=1)
            return (math.pi * s * s) ** -1.5 * torch.exp(-d2 / (s * s))

        rho, cur, dvec = [], [], []
        for ch in dom.charges:
            if ch.kind == "pair":
                rho.append(gauss(ch.cp, ch.s) - gauss(ch.cm, ch.s))
                d = np.asarray(ch.cp, dtype=np.float64) - np.asarray(ch.cm, dtype=np.float64)
                L = float(np.linalg.norm(d))
                if L == 0.0 or not math.isfinite(c):
                    cur.append(torch.zeros(len(pts), **f64))
                else:
                    dh = torch.as_tensor(d / L, **f64)
                    rel = pts - torch.as_tensor(ch.cm, **f64)[None, :]
                    xi = rel @ dh
                    rp2 = torch.clamp(torch.sum(rel * rel, dim=1) - xi * xi, min=0.0)
                    s = ch.s
                    cur.append((math.pi * s * s) ** -1.5 * torch.exp(-rp2 / (s * s))
                               * (math.sqrt(math.pi) * s / (2.0 * L))
                               * (torch.special.erf(xi / s) - torch.special.erf((xi - L) / s)))
                dvec.append(d / c if math.isfinite(c) else np.zeros(3))
            elif ch.kind == "single":
                rho.append(gauss(ch.cp, ch.s))
                cur.append(None)
                dvec.append(np.zeros(3))
            else:
                raise ValueError(ch.kind)
        n = len(pts)
        R = torch.stack(rho) if rho else torch.zeros((0, n), **f64)
        pairs = [i for i, cf in enumerate(cur) if cf is not None]
        J = torch.stack([cur[i] for i in pairs]) if pairs else torch.zeros((0, n), **f64)
        D = torch.as_tensor(np.array([dvec[i] for i in pairs]).reshape(-1, 3), **f64)
        return R, J, D, pairs

    def step(self, l, dtype=None):
        torch = self.torch
        out = []
        for i in self.doms:
            dom = self.system.domains[i]
            R, J, D, pairs = self.fields[i]
            j = np.array([l], dtype=np.int64)
            t = j.astype(np.float64) * self.system.dt
            q = np.array([_profile(ch.profile, t, j)[0][0] for ch in dom.charges])
            qd = np.array([_profile(ch.profile, t, j)[1][0] for ch in dom.charges])
            S = torch.empty((4, R.shape[1]), dtype=torch.float64, device=self.device)
            S[0] = torch.as_tensor(q, dtype=torch.float64, device=self.device) @ R if len(q) else 0.0
            if pairs:
                w = torch.as_tensor(qd[pairs], dtype=torch.float64, device=self.device)[:, None] * D   # [pairs][3]
                S[1:] = w.T @ J
            else:
                S[1:] = 0.0
            S = S.reshape((4,) + tuple(dom.dims))
            out.append(S if dtype is None else S.to(dtype).contiguous())
        return out
