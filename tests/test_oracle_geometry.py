"""Pins of the oracle's cylinder geometry (paper Sec. 2.2: neurite elements are cylinders with a
point mass at the distal end; spheres and cylinders interact mechanically on the same grid).

* Closest-point routines against brute-force minimisation over dense parameter grids, and
  against closed forms (perpendicular, parallel, collinear and degenerate segments).
* Pair forces against the sphere-sphere closed form (d = 12, separation 10: F = 4 - sqrt 6) for
  a sphere at a cylinder's side and for crossed cylinders, with the point-mass share.
* Metamorphic: a population of spheres gives the sphere step bit for bit; cylinders of length 0
  give the sphere step with their diameters bit for bit.
* Contact counts against an O(n^2) loop over all pairs (the grid diameter makes the 27-box
  walk complete).
"""
import math

import numpy as np
import pytest

from paper_2006_06775_amd import synth

F10 = 4.0 - math.sqrt(6.0)  # d = 12 and 12 at separation 10, k = 2, gamma = 1


def seg_dist(p, q, c, t):
    return np.linalg.norm(np.asarray(p) + t * (np.asarray(q) - np.asarray(p)) - np.asarray(c))


def test_segment_point_param(orc):
    rng = np.random.default_rng(1)
    ts = np.linspace(0.0, 1.0, 20001)
    for _ in range(200):
        p, q, c = rng.normal(size=3) * 5, rng.normal(size=3) * 5, rng.normal(size=3) * 8
        t = orc.segment_point_param(p, q, c)
        assert 0.0 <= t <= 1.0
        brute = min(np.linalg.norm(p[None, :] + ts[:, None] * (q - p)[None, :] - c[None, :], axis=1))
        assert seg_dist(p, q, c, t) <= brute + 1e-12
    assert orc.segment_point_param([0, 0, 0], [2, 0, 0], [5, 1, 0]) == 1.0
    assert orc.segment_point_param([0, 0, 0], [2, 0, 0], [-5, 1, 0]) == 0.0
    assert orc.segment_point_param([0, 0, 0], [2, 0, 0], [0.5, 3, 0]) == 0.25
    assert orc.segment_point_param([1, 1, 1], [1, 1, 1], [9, 9, 9]) == 1.0  # a point: its distal end


def brute_seg_seg(p1, q1, p2, q2, m=401):
    s = np.linspace(0, 1, m)
    a = p1[None, :] + s[:, None] * (q1 - p1)[None, :]
    b = p2[None, :] + s[:, None] * (q2 - p2)[None, :]
    d = np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2)
    i, j = np.unravel_index(np.argmin(d), d.shape)
    # refine around the grid minimum
    s2 = np.clip(s[i] + np.linspace(-2, 2, 401) / (m - 1), 0, 1)
    t2 = np.clip(s[j] + np.linspace(-2, 2, 401) / (m - 1), 0, 1)
    a = p1[None, :] + s2[:, None] * (q1 - p1)[None, :]
    b = p2[None, :] + t2[:, None] * (q2 - p2)[None, :]
    return np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2).min()


def test_segment_segment_params(orc):
    rng = np.random.default_rng(2)
    for k in range(150):
        p1, q1, p2, q2 = (rng.normal(size=3) * 4 for _ in range(4))
        if k % 5 == 0:  # parallel pairs
            q2 = p2 + (q1 - p1) * rng.uniform(0.2, 2.0)
        s, t = orc.segment_segment_params(p1, q1, p2, q2)
        assert 0.0 <= s <= 1.0 and 0.0 <= t <= 1.0
        got = np.linalg.norm(p1 + s * (q1 - p1) - (p2 + t * (q2 - p2)))
        assert got <= brute_seg_seg(p1, q1, p2, q2) + 1e-9, k


def test_segment_segment_closed_forms(orc):
    # crossed at right angles, one above the other by 1: midpoints
    assert orc.segment_segment_params([0, 0, 0], [2, 0, 0], [1, -1, 1], [1, 1, 1]) == (0.5, 0.5)
    # closest points at ends: the first segment's end faces the second's start
    assert orc.segment_segment_params([0, 0, 0], [1, 0, 0], [3, 0, 0], [5, 0, 0]) == (1.0, 0.0)
    # parallel, overlapping in x: any pair at distance 2 (s starts from 0)
    s, t = orc.segment_segment_params([0, 0, 0], [4, 0, 0], [1, 2, 0], [3, 2, 0])
    assert s == 0.25 and t == 0.0
    # degenerate: a point against a segment, two points
    assert orc.segment_segment_params([1, 1, 1], [1, 1, 1], [0, 0, 0], [4, 0, 0]) == (1.0, 0.25)
    assert orc.segment_segment_params([0, 0, 0], [4, 0, 0], [3, 5, 0], [3, 5, 0]) == (0.75, 1.0)
    assert orc.segment_segment_params([0, 0, 0], [0, 0, 0], [3, 5, 0], [3, 5, 0]) == (1.0, 1.0)


def test_reach(orc):
    assert orc.cylinder_reach([0, 0, 0], [3, 4, 0], 1.5) == 11.5


def test_sphere_at_a_cylinder_side(orc):
    C, S = orc.GEOM_CYLINDER, orc.GEOM_SPHERE
    p, q = np.array([-10.0, 0.0, 0.0]), np.array([10.0, 0.0, 0.0])
    c = np.array([3.0, 10.0, 0.0])
    hit, f_s = orc.geom_pair(S, c, 12.0, c, 0.0, C, q, 0.0, p, 12.0)
    assert hit and f_s[0] == 0.0 and f_s[2] == 0.0 and f_s[1] == pytest.approx(F10, rel=1e-15)
    hit, f_c = orc.geom_pair(C, q, 0.0, p, 12.0, S, c, 12.0, c, 0.0)
    share = 13.0 / 20.0  # closest point (3, 0, 0) along p -> q
    assert hit and f_c[1] == pytest.approx(-share * F10, rel=1e-15)
    assert f_c[1] == share * (-f_s[1])  # the same pair term, scaled by the point-mass share
    # beyond the distal end the closest point is the end itself: a sphere-sphere pair there
    c2 = np.array([20.0, 0.0, 0.0])
    hit, f_c2 = orc.geom_pair(C, q, 0.0, p, 12.0, S, c2, 12.0, c2, 0.0)
    assert hit and f_c2[0] == pytest.approx(-F10, rel=1e-15)
    hit, _ = orc.geom_pair(S, np.array([3.0, 12.0, 0.0]), 12.0, c, 0.0, C, q, 0.0, p, 12.0)
    assert not hit  # separation 12 = (12 + 12) / 2: no overlap


def test_crossed_cylinders(orc):
    C = orc.GEOM_CYLINDER
    p1, q1 = np.array([0.0, 0.0, 0.0]), np.array([20.0, 0.0, 0.0])
    p2, q2 = np.array([5.0, -10.0, 10.0]), np.array([5.0, 30.0, 10.0])
    hit, f1 = orc.geom_pair(C, q1, 0.0, p1, 12.0, C, q2, 0.0, p2, 12.0)
    # closest points (5, 0, 0) at s = 1/4 and (5, 0, 10) at t = 1/4: separation 10 along -z
    assert hit and f1[0] == 0.0 and f1[1] == 0.0
    assert f1[2] == pytest.approx(-0.25 * F10, rel=1e-15)
    hit, f2 = orc.geom_pair(C, q2, 0.0, p2, 12.0, C, q1, 0.0, p1, 12.0)
    assert f2[2] == pytest.approx(0.25 * F10, rel=1e-15)


def sphere_state(s):
    return dict(x=s["x"].copy(), y=s["y"].copy(), z=s["z"].copy(), d=s["d"].copy(), adh=s["adh"].copy())


def test_only_spheres_is_the_sphere_step(orc):
    s = synth.neurite_mix(3000, 110.0, sphere_frac=1.0, seed=3)
    ref = sphere_state(s)
    fx, fy, fz, nc = orc.geom_step(s)
    rfx, rfy, rfz, rnc, _ = orc.mech_step(ref)
    for k in "xyz":
        assert np.array_equal(s[k], ref[k])
    assert np.array_equal(fx, rfx) and np.array_equal(fy, rfy) and np.array_equal(fz, rfz)
    assert np.array_equal(nc, rnc) and nc.sum() > 3000


def test_zero_length_cylinders_are_spheres_of_their_diameter(orc):
    s = synth.neurite_mix(2500, 100.0, sphere_frac=0.3, dc=(6.0, 12.0), seed=4)
    cyl = s["state"] == 1
    for a, b in (("px", "x"), ("py", "y"), ("pz", "z")):
        s[a] = s[b].copy()  # length 0
    ref = sphere_state(s)
    ref["d"] = np.where(cyl, s["dc"], s["d"])
    fx, fy, fz, nc = orc.geom_step(s)
    rfx, rfy, rfz, rnc, _ = orc.mech_step(ref)
    assert np.array_equal(s["d"], ref["d"])  # the grid diameter of a point cylinder is dc
    for k in "xyz":
        assert np.array_equal(s[k], ref[k])
    assert np.array_equal(fx, rfx) and np.array_equal(fz, rfz) and np.array_equal(nc, rnc)


def test_contact_counts_match_all_pairs(orc):
    s = synth.neurite_mix(400, 45.0, sphere_frac=0.25, length=(4.0, 14.0), dc=(1.0, 4.0), seed=5)
    n = 400
    pre = {k: v.copy() for k, v in s.items()}
    _, _, _, nc = orc.geom_step(s)
    body = []
    for i in range(n):
        q = np.array([pre["x"][i], pre["y"][i], pre["z"][i]])
        p = np.array([pre["px"][i], pre["py"][i], pre["pz"][i]])
        body.append((int(pre["state"][i]), q, pre["d"][i], p, pre["dc"][i]))
    brute = np.zeros(n, dtype=np.uint32)
    for i in range(n):
        for j in range(n):
            if i != j:
                hit, _ = orc.geom_pair(*body[i], *body[j])
                brute[i] += hit
    assert np.array_equal(nc, brute)
    assert nc.sum() > 100
    # contacts are mutual
    assert all(orc.geom_pair(*body[i], *body[j])[0] == orc.geom_pair(*body[j], *body[i])[0]
               for i in range(0, n, 7) for j in range(0, n, 5) if i != j)
