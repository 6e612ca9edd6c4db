"""Pins of the oracle's tumour-spheroid behaviour beyond growth and division (paper Sec. 3.2:
apoptosis, Brownian migration, and the spheroid diameter taken from the convex hull of the
cells).

* Apoptosis and migration are rebuilt from numpy's own Philox (purposes 6 and 7 of the draw
  layout), so the counter layout, the Bernoulli threshold and the survivors' renumbering are
  checked against something other than the oracle's generator.
* Mechanics never changes counts, diameters or the id order, so an independent diameter-only
  model (a list in id order: survivors kept in order, grown, split, daughters appended) fixes the
  population size and the multiset of diameters of a full run exactly.
* With no apoptosis and no migration the step is the plain spheroid step, bit for bit.
* The hull diameter is checked on solids whose volume is known in closed form.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from test_oracle_rng import numpy_draw, _u
from test_oracle_spheroid import G, H

RNG_APO, RNG_MIG = 6, 7


def threshold(p):
    """floor(p * 2^64) of the double p, exactly."""
    return int(Fraction(p) * (1 << 64))


def dies(seed, i, step, p, salt=0):
    return int(numpy_draw(seed, salt, RNG_APO, 0, i, step)[0]) < threshold(p)


def onc_params(orc, seed=0, p_apo=0.0, migrate=0.0, **mech):
    mp = dict(k=2.0, gamma=1.0, dt=0.01, max_disp=3.0)
    mp.update(mech)
    return orc.oncology_params(G, 14.0, H, seed, p_apo, migrate, **mp)


def state_of(orc, init, capacity):
    return orc.SpheroidState(init, capacity=capacity)


def test_apoptosis_extremes(orc):
    init = orc.generate_ball(300, 3, 20.0, 9.0, 14.0, 0.4)
    st = state_of(orc, init, 400)
    st.apoptosis(0.0, 3, 0)
    assert int(st.n[0]) == 300
    for k in ("x", "y", "z", "d", "adh"):
        assert np.array_equal(st.view(k), init[k])
    st.apoptosis(1.0, 3, 1)
    assert int(st.n[0]) == 0
    st.apoptosis(0.5, 3, 2)  # an empty population stays empty
    assert int(st.n[0]) == 0


def test_apoptosis_matches_numpy_draws_and_renumbers(orc):
    n, seed, step, p = 2000, 11, 7, 0.3
    init = orc.generate_ball(n, seed, 30.0, 9.0, 14.0, 0.4)
    init["adh"] = np.arange(n) * 0.001  # tells the survivors apart
    st = state_of(orc, init, n)
    st.apoptosis(p, seed, step)
    alive = np.array([not dies(seed, i, step, p) for i in range(n)])
    assert 0.25 * n < n - alive.sum() < 0.35 * n
    assert int(st.n[0]) == alive.sum()
    for k in ("x", "y", "z", "d", "adh"):
        # survivors in their old id order, renumbered 0 .. n'-1
        assert np.array_equal(st.view(k), init[k][alive])


def test_migration_matches_numpy_draws(orc):
    n, seed, step, s = 3000, 5, 12, 1.5
    init = orc.generate_cube(n, seed, 100.0, 10.0, 15.0, 0.4)
    st = state_of(orc, init, n)
    st.migrate(s, seed, step)
    w = np.stack([numpy_draw(seed, 0, RNG_MIG, 0, i, step)[:3] for i in range(n)])
    u = _u(w)
    disp = np.stack([st.view(k) - init[k] for k in "xyz"], axis=1)
    # every axis moves by at most s, with zero mean and variance s^2 / 3 (uniform on [-s, s])
    assert np.all(np.abs(disp) <= s * (1 + 1e-12))
    assert np.all(np.abs(disp.mean(axis=0)) < 4 * s / math.sqrt(3 * n))
    assert np.allclose(disp.var(axis=0), s * s / 3, rtol=0.08)
    # and the draws are those of purpose 7 at (id, step)
    for a, k in enumerate("xyz"):
        assert np.array_equal(st.view(k), init[k] + s * (2.0 * u[:, a] - 1.0))
    before = {k: st.view(k).copy() for k in "xyz"}
    st.migrate(0.0, seed, step + 1)
    for k in "xyz":
        assert np.array_equal(st.view(k), before[k])


def test_without_apoptosis_and_migration_it_is_the_spheroid_step(orc):
    init = orc.generate_ball(600, 2, 22.0, 14.0 * H, 14.0, 0.4)
    a = state_of(orc, init, 5000)
    b = state_of(orc, init, 5000)
    sp = orc.spheroid_params(G, 14.0, H, 2, k=2.0, gamma=1.0, dt=0.01, max_disp=3.0)
    op = onc_params(orc, seed=2)
    for t in range(8):
        a.step(sp, t)
        b.oncology_step(op, t)
        assert int(a.n[0]) == int(b.n[0])
        for k in ("x", "y", "z", "d", "adh"):
            assert np.array_equal(a.view(k), b.view(k))


def onc_count_model(d0, steps, seed, p_apo):
    """Diameters in id order through apoptosis (numpy draws), growth and division."""
    d = list(d0)
    counts = []
    for t in range(steps):
        d = [v for i, v in enumerate(d) if not dies(seed, i, t, p_apo)]
        d = [v * G for v in d]
        n0 = len(d)
        for i in range(n0):
            if d[i] >= 14.0:
                d[i] = d[i] * H
                d.append(d[i])
        counts.append(len(d))
    return counts, d


def test_counts_and_diameters_match_model(orc):
    seed, p_apo, steps = 4, 0.03, 20
    init = orc.generate_ball(300, seed, 22.0, 14.0 * H, 14.0, 0.4)
    st = state_of(orc, init, 20000)
    p = onc_params(orc, seed=seed, p_apo=p_apo, migrate=1.0)
    counts = []
    for t in range(steps):
        st.oncology_step(p, t)
        counts.append(int(st.n[0]))
    ref_counts, ref_d = onc_count_model(init["d"], steps, seed, p_apo)
    assert counts == ref_counts
    assert np.array_equal(st.view("d"), np.array(ref_d))  # same order too: ids are positions


def test_one_division_then_migration_closed_form(orc):
    """One cell divides; mother and daughter then migrate with their own (post-division) ids.
    A huge adherence gates the mechanics, so the positions are the closed form."""
    seed, step, s = 8, 3, 0.75
    init = dict(x=np.array([10.0]), y=np.array([-4.0]), z=np.array([2.5]), d=np.array([13.99]),
                adh=np.array([1e30]))
    st = state_of(orc, init, 4)
    st.oncology_step(onc_params(orc, seed=seed, migrate=s), step)
    assert int(st.n[0]) == 2
    u = orc.division_axis(seed, 0, step)
    dp = 13.99 * G * H
    q = 0.25 * dp
    for i, sign in ((0, -1.0), (1, 1.0)):
        w = _u(numpy_draw(seed, 0, RNG_MIG, 0, i, step)[:3])
        for a, k in enumerate("xyz"):
            want = (init[k][0] + sign * (q * u[a])) + s * (2.0 * w[a] - 1.0)
            assert st.arr[k][i] == want
        assert st.arr["d"][i] == dp


def test_parameter_checks(orc):
    init = orc.generate_ball(10, 0, 10.0, 9.0, 14.0, 0.4)
    st = state_of(orc, init, 20)
    for bad in (dict(p_apo=-0.1), dict(p_apo=1.5), dict(migrate=-1.0), dict(migrate=math.inf)):
        with pytest.raises(orc.OracleError):
            st.oncology_step(onc_params(orc, **bad), 0)


# ---- hull diameter --------------------------------------------------------------------------
def sphere_d(volume):
    return (6.0 * volume / math.pi) ** (1.0 / 3.0)


def test_hull_diameter_of_a_cube_with_interior_points(orc):
    a = 7.0
    corners = np.array([[i, j, k] for i in (0, a) for j in (0, a) for k in (0, a)], dtype=float)
    inner = np.random.default_rng(1).uniform(0.5, a - 0.5, size=(500, 3))
    pts = np.concatenate([inner, corners]) + np.array([100.0, -30.0, 5.0])
    assert orc.hull_diameter(pts[:, 0], pts[:, 1], pts[:, 2]) == pytest.approx(sphere_d(a ** 3), rel=1e-13)


def test_hull_diameter_of_a_tetrahedron(orc):
    p = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0], [0.0, 4.0, 0.0], [0.0, 0.0, 5.0]])
    # V = |det(b - a, c - a, d - a)| / 6 = 60 / 6
    assert orc.hull_diameter(p[:, 0], p[:, 1], p[:, 2]) == pytest.approx(sphere_d(10.0), rel=1e-13)


def test_hull_diameter_of_points_on_a_sphere(orc):
    """Fibonacci points on a sphere of radius R: the hull is an inscribed polytope whose volume
    lies between that of the sphere of radius R cos(theta) and of radius R, theta the largest
    angular gap (below 4 / sqrt(m) for m points), so the diameter lies in [2R cos(theta), 2R)."""
    R, m = 50.0, 4000
    k = np.arange(m) + 0.5
    phi = np.arccos(1 - 2 * k / m)
    th = math.pi * (1 + 5 ** 0.5) * k
    x, y, z = R * np.cos(th) * np.sin(phi), R * np.sin(th) * np.sin(phi), R * np.cos(phi)
    d = orc.hull_diameter(x, y, z)
    assert 2 * R * math.cos(4 / math.sqrt(m)) < d < 2 * R


def test_hull_diameter_degenerate(orc):
    assert orc.hull_diameter(np.zeros(3), np.zeros(3), np.zeros(3)) == 0.0
    x = np.random.default_rng(2).uniform(0, 1, 50)
    assert orc.hull_diameter(x, 2 * x, np.zeros(50)) == 0.0  # all in one plane
