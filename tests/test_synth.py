"""Checks of the seeded synthetic inputs (not of the method)."""
import math

import numpy as np
import pytest

from synth import sources as sy


def _continuity_residual(h):
    c = sy.C_AU
    n = int(round(8.0 / h)) + 1
    dom = sy.Domain((n, n, n), np.array([-4.0, -4.0, -4.0]))
    dom.charges.append(sy.Charge("pair", 0.9, np.array([0.7, -0.4, 0.9]), np.array([-0.8, 0.5, -0.6]),
                                 ("cos", 0.6, 0.4, 0.7)))
    B = sy.spatial_factors(dom, h, c).reshape(2, 4, n, n, n)
    dt = 0.01
    A = sy.time_factors(dom, dt, [4, 5, 6])
    drho = np.einsum("t,txyz->xyz", (A[2] - A[0]) / (2 * dt), B[:, 0])
    J = np.einsum("t,taxyz->axyz", A[1], B[:, 1:]) * c
    div = sum(np.gradient(J[a], h, axis=a, edge_order=2) for a in range(3))
    k = int(round(1.0 / h))
    inner = (slice(k, -k),) * 3
    return np.max(np.abs(drho[inner] + div[inner])) / np.max(np.abs(drho[inner]))


def test_pair_sources_satisfy_continuity():
    """d_t rho = -div J for the Gaussian pair with the line-current tube: the
    residual of second-order finite differences shrinks ~4x when h halves."""
    e1, e2 = _continuity_residual(0.2), _continuity_residual(0.1)
    assert e1 < 0.06 and e1 / e2 > 3.5


def test_config_geometries():
    s1 = sy.config1(1)
    assert [d.dims for d in s1.domains] == [(16, 16, 16)] * 2
    cen = [d.origin + 0.5 * (np.array(d.dims) - 1) * s1.h for d in s1.domains]
    assert np.allclose(cen[0], 0) and np.allclose(cen[1], [30, 0, 0])
    s2 = sy.config2(0)
    side = 63 * 0.3
    cen = [d.origin + 0.5 * side for d in s2.domains]
    for a in range(8):
        assert np.all(cen[a] >= side / 2 - 1e-9) and np.all(cen[a] <= 400 - side / 2 + 1e-9)
        for b in range(a):
            assert np.linalg.norm(cen[a] - cen[b]) >= 20.0
            assert np.max(np.abs(cen[a] - cen[b])) >= side + 0.3
    assert len(s2.domains[0].charges) == 16


def test_sampling_is_separable_and_seeded():
    s1 = sy.config1(2)
    a = sy.sample_sources(s1, [0, 3])
    b = sy.sample_sources(sy.config1(2), [0, 3])
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert a[0].shape == (2, 4, 16 ** 3)
    assert not np.array_equal(a[0][0], a[0][1])
    # J/c components are small compared with rho (v/c)
    assert np.max(np.abs(a[0][:, 1:])) < 0.05 * np.max(np.abs(a[0][:, 0]))
    assert math.isfinite(float(np.sum(a[1])))


def test_wire_pair_and_enclosing_domain():
    s = sy.wire_pair(W=8, L=24, d=40, h=0.5, dt=0.02, n_pairs=1)
    encl, blocks = sy.enclosing_domain(s)
    assert tuple(encl.domains[0].dims) == (8, 40, 24)
    pts = sy.grid_points(encl.domains[0], s.h).reshape(8, 40, 24, 3)
    for dm, b in zip(s.domains, blocks):
        assert np.allclose(pts[b].reshape(-1, 3), sy.grid_points(dm, s.h))
    with pytest.raises(ValueError):
        sy.wire_pair(W=8, L=24, d=15)


def test_torch_sources_equal_the_separable_samples():
    """The torch evaluation of the sources (compact fields) gives the samples
    A[l] @ B of spatial_factors / time_factors."""
    torch = pytest.importorskip("torch")
    s = sy.config5(3, n_dom=3, n=9, box=300.0)
    gen = sy.TorchSources(s, "cpu")
    S = sy.sample_sources(s, [0, 7, 40])
    for k, l in enumerate([0, 7, 40]):
        got = gen.step(l)
        for n in range(3):
            ref = S[n][k]
            g = got[n].numpy().reshape(4, -1)
            for c in range(4):             # each component against its own scale
                assert np.max(np.abs(g[c] - ref[c])) <= 1e-13 * np.max(np.abs(ref[c])), (l, n, c)
