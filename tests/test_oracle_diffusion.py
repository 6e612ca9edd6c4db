"""Pins of the oracle's extracellular substances (paper Sec. 2.1: substance diffusion as a
standalone operation, secretion and chemotaxis as agent behaviours) and of the soma-clustering
step built from them (the Sec. 3.4 benchmark).

* The diffusion step is checked against scipy's n-dimensional convolution with the 7-point
  kernel ('nearest' edges = a closed boundary), against the exact one-step image of a unit
  impulse (dyadic coefficients), against the discrete Neumann eigenmodes (cosines at voxel
  centres, whose one-step factor is known in closed form), and for mass conservation.
* Secretion against a histogram of voxel indices built with numpy; agents on voxel faces and
  outside the grid fix the voxel rule.
* Chemotaxis on linear fields, whose central differences are exact, and on uniform fields.
* The soma step with no secretion and no chemotaxis is the mechanical step, bit for bit.
"""
import math

import numpy as np
import pytest

ndimage = pytest.importorskip("scipy.ndimage")


def kernel7(lam, kdec):
    k = np.zeros((3, 3, 3))
    k[1, 1, 1] = 1.0 - 6.0 * lam - kdec
    for a in range(3):
        for s in (0, 2):
            idx = [1, 1, 1]
            idx[a] = s
            k[tuple(idx)] = lam
    return k


def as_zyx(c, f):
    return c.reshape(f.nz, f.ny, f.nx)


def test_diffuse_matches_convolution(orc):
    rng = np.random.default_rng(3)
    for nx, ny, nz in ((7, 5, 9), (1, 6, 4), (13, 1, 1), (2, 2, 2)):
        f = orc.field(nx, ny, nz, 2.5)
        c = rng.uniform(0.0, 10.0, nx * ny * nz)
        lam, kdec = 0.15, 0.004
        got = as_zyx(orc.diffuse(f, c, lam, kdec), f)
        ref = ndimage.convolve(as_zyx(c, f), kernel7(lam, kdec), mode="nearest")
        assert np.allclose(got, ref, rtol=0, atol=1e-13 * 10.0), (nx, ny, nz)


def test_unit_impulse_one_step(orc):
    f = orc.field(6, 5, 4, 1.0)
    lam = 0.125  # dyadic: every value below is exact
    for (i, j, k), faces in (((2, 2, 1), 0), ((0, 2, 1), 1), ((0, 0, 0), 3), ((5, 4, 3), 3)):
        c = np.zeros(6 * 5 * 4)
        c[i + 6 * (j + 5 * k)] = 1.0
        out = as_zyx(orc.diffuse(f, c, lam, 0.0), f)
        # each missing neighbour (closed face) keeps its share in the voxel
        assert out[k, j, i] == 1.0 - (6 - faces) * lam
        nb = [(i + 1, j, k), (i - 1, j, k), (i, j + 1, k), (i, j - 1, k), (i, j, k + 1), (i, j, k - 1)]
        inside = [(a, b, e) for a, b, e in nb if 0 <= a < 6 and 0 <= b < 5 and 0 <= e < 4]
        assert len(inside) == 6 - faces
        for a, b, e in inside:
            assert out[e, b, a] == lam
        assert out.sum() == 1.0
        assert np.count_nonzero(out) == 1 + len(inside)


def test_neumann_eigenmodes(orc):
    """cos(pi a (i + 1/2) / n) per axis is an eigenvector of the closed-boundary difference
    operator with eigenvalue -2 (1 - cos(pi a / n)); one step multiplies it by
    1 - lam * sum_axes 2 (1 - cos(pi a / n)) - kdec."""
    nx, ny, nz = 11, 8, 6
    f = orc.field(nx, ny, nz, 3.0)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="xy")
    lam, kdec = 0.1, 0.002
    for a, b, e in ((1, 0, 0), (0, 3, 0), (2, 1, 5), (10, 7, 5)):
        mode = (np.cos(math.pi * a * (i + 0.5) / nx) * np.cos(math.pi * b * (j + 0.5) / ny)
                * np.cos(math.pi * e * (k + 0.5) / nz))
        c = np.transpose(mode, (2, 0, 1)).ravel()  # (z, y, x) order, x fastest
        factor = 1.0 - lam * sum(2.0 * (1.0 - math.cos(math.pi * m / n))
                                 for m, n in ((a, nx), (b, ny), (e, nz))) - kdec
        out = orc.diffuse(f, c, lam, kdec)
        assert np.allclose(out, factor * c, rtol=0, atol=1e-14), (a, b, e)


def test_mass_conservation_and_uniform_field(orc):
    rng = np.random.default_rng(5)
    f = orc.field(9, 10, 11, 1.0)
    c = rng.uniform(0.0, 1.0, 990)
    out = orc.diffuse(f, c, 1.0 / 6.0, 0.0)
    assert abs(out.sum() - c.sum()) <= 990 * 4 * np.finfo(float).eps * c.sum()
    assert out.min() >= 0.0  # stable at lam = 1/6: a convex combination of neighbours
    u = np.full(990, 3.7)
    out = orc.diffuse(f, u, 0.16, 0.01)
    assert np.all(out == out[0])  # every difference is exactly zero
    assert out[0] == pytest.approx(3.7 * 0.99, rel=1e-15)


def test_coefficients(orc):
    lam, kdec = orc.diffusion_coefficients(250.0, 0.1, 0.01, 5.0)
    assert lam == pytest.approx(0.1, rel=1e-15) and kdec == pytest.approx(0.001, rel=1e-15)


def agents(xyz, types):
    xyz = np.asarray(xyz, dtype=float)
    return dict(x=xyz[:, 0].copy(), y=xyz[:, 1].copy(), z=xyz[:, 2].copy(),
                state=np.asarray(types, dtype=np.uint8))


def test_secretion_histogram(orc):
    f = orc.field(8, 6, 5, 4.0, x0=-10.0, y0=2.0, z0=0.0)
    V = 8 * 6 * 5
    rng = np.random.default_rng(9)
    n = 3000
    pos = np.stack([rng.uniform(-14.0, 26.0, n), rng.uniform(-2.0, 30.0, n), rng.uniform(-4.0, 24.0, n)], 1)
    pos[:50, 0] = -10.0 + 4.0 * rng.integers(0, 9, 50)  # on voxel faces (and the far face 22)
    types = rng.integers(0, 3, n)  # type 2 is inert
    s = agents(pos, types)
    c = np.full(2 * V, 0.5)
    orc.secrete(f, s, 0.25, c)
    ix = np.clip(np.floor((pos[:, 0] + 10.0) / 4.0), 0, 7).astype(int)
    iy = np.clip(np.floor((pos[:, 1] - 2.0) / 4.0), 0, 5).astype(int)
    iz = np.clip(np.floor(pos[:, 2] / 4.0), 0, 4).astype(int)
    m = np.zeros(2 * V, dtype=np.int64)
    live = types < 2
    np.add.at(m, types[live] * V + ix[live] + 8 * (iy[live] + 6 * iz[live]), 1)
    assert np.array_equal(c, 0.5 + 0.25 * m)
    assert m.sum() == live.sum()


def test_chemotaxis_linear_and_uniform_fields(orc):
    nx, ny, nz, h = 10, 9, 8, 2.0
    f = orc.field(nx, ny, nz, h)
    V = nx * ny * nz
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    lin = np.zeros((nz, ny, nx))
    lin[k.T, j.T, i.T] = 3.0 * i.T - 2.0 * j.T + 0.5 * k.T  # exact in binary64
    c = np.concatenate([lin.ravel(), np.full(V, 1.0)])  # substance 1 uniform
    rng = np.random.default_rng(2)
    n = 400
    pos = rng.uniform(2.0 + 1e-9, 2.0 * (np.array([nx, ny, nz]) - 1) - 1e-9, (n, 3))  # interior voxels
    types = np.where(np.arange(n) % 2 == 0, 0, 1)
    s = agents(pos, types)
    orc.chemotaxis(f, s, c, 0.7)
    disp = np.stack([s["x"], s["y"], s["z"]], 1) - pos
    g = np.array([3.0, -2.0, 0.5]) * 2.0  # central differences over two voxels
    u = g / np.linalg.norm(g)
    assert np.allclose(disp[0::2], 0.7 * u, rtol=0, atol=1e-14)
    assert np.all(disp[1::2] == 0.0)  # a uniform field has no gradient


def test_chemotaxis_boundary_one_sided(orc):
    f = orc.field(4, 1, 1, 1.0)
    c = np.concatenate([np.array([0.0, 1.0, 4.0, 9.0]), np.zeros(4)])
    s = agents([[0.5, 0.5, 0.5], [3.5, 0.5, 0.5], [9.0, 0.0, 0.0]], [0, 0, 0])
    orc.chemotaxis(f, s, c, 1.0)
    # voxel 0: neighbour below is itself -> g = c1 - c0 > 0; voxel 3 (also agents beyond the
    # grid): g = c3 - c2 > 0
    assert list(s["x"]) == [1.5, 4.5, 10.0]
    assert list(s["y"]) == [0.5, 0.5, 0.0]


def test_soma_step_without_substance_effects_is_mechanics(orc):
    n = 1500
    s = orc.generate_soma(n, 4, 120.0, 10.0, 15.0, 0.4)
    ref = {k: v.copy() for k, v in s.items()}
    f = orc.field(24, 24, 24, 5.0)
    c = np.random.default_rng(1).uniform(0, 1, 2 * 24 ** 3)
    p = orc.soma_params(250.0, 0.1, 0.0, 0.0)
    c_next, fx, fy, fz = orc.soma_step(s, f, c.copy(), p)
    rfx, rfy, rfz, _, _ = orc.mech_step(ref)
    for k in "xyz":
        assert np.array_equal(s[k], ref[k])
    assert np.array_equal(fx, rfx) and np.array_equal(fz, rfz)
    lam, kdec = orc.diffusion_coefficients(250.0, 0.1, 0.01, 5.0)
    for sub in range(2):
        part = slice(sub * 24 ** 3, (sub + 1) * 24 ** 3)
        assert np.array_equal(c_next[part], orc.diffuse(f, c[part], lam, kdec))


def test_soma_step_order_secrete_diffuse_move(orc):
    """Three cells on a coarse grid: each secretes into its voxel, the fields diffuse, then each
    climbs its own substance's gradient.  A type-1 cell alone sits on a symmetric maximum and
    stays; two type-0 cells in neighbouring voxels each see the other's source and move toward
    each other, by exactly `speed`."""
    f = orc.field(9, 9, 9, 10.0)
    V = 9 ** 3
    s = dict(x=np.array([45.0, 55.0, 45.0]), y=np.array([45.0, 45.0, 75.0]), z=np.array([45.0, 45.0, 45.0]),
             d=np.array([1.0, 1.0, 1.0]), adh=np.array([1e30, 1e30, 1e30]),
             state=np.array([0, 0, 1], dtype=np.uint8))
    c = np.zeros(2 * V)
    p = orc.soma_params(1000.0, 0.0, 1.0, 0.5, dt=0.01)  # lam = 0.1
    c_next, *_ = orc.soma_step(s, f, c, p)
    v0 = 4 + 9 * (4 + 9 * 4)
    assert c[v0] == 1.0 and c[v0 + 1] == 1.0 and c[V + v0 + 27] == 1.0  # secreted before diffusing
    assert c_next[v0] == 0.5  # 1 + lam * (5 * (0 - 1) + (1 - 1)), exact
    assert s["x"][0] == 45.5 and s["x"][1] == 54.5  # toward each other
    assert s["y"][0] == 45.0 and s["z"][1] == 45.0
    assert (s["x"][2], s["y"][2], s["z"][2]) == (45.0, 75.0, 45.0)  # alone: g = 0


def test_soma_parameter_checks(orc):
    s = orc.generate_soma(10, 0, 50.0, 10.0, 15.0, 0.4)
    f = orc.field(5, 5, 5, 10.0)
    c = np.zeros(250)
    for bad in (dict(D=1e6), dict(D=-1.0), dict(decay=-0.5), dict(speed=-1.0), dict(secrete=math.nan)):
        kw = dict(D=100.0, decay=0.0, secrete=1.0, speed=1.0)
        kw.update(bad)
        with pytest.raises(orc.OracleError):
            orc.soma_step(s, f, c, orc.soma_params(**kw))
