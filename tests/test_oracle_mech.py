"""Pins of the oracle's sphere-sphere force and displacement.

The force law F(delta) = k*delta - gamma*sqrt(rhat*delta), rhat = ri*rj/(ri+rj), is pinned by
closed forms that follow from it by calculus, not by retyping it: the value at one overlap,
its zero crossing delta* = gamma^2*rhat/k^2, its minimum -gamma^2*rhat/(4k) at delta*/4, the
repulsive sign, exact antisymmetry, and the summed force against an O(N^2) brute-force sum in a
different order.  The displacement is pinned by the two-sphere trajectory, the gate edge at
|F| = adh and the clamp length.
"""
import math

import numpy as np
import pytest

import inputs


def test_two_sphere_force_value(orc):
    # d1 = d2 = 12 (rhat = 3), k = 2, gamma = 1, separation 10 -> delta = 2, F = 4 - sqrt(6)
    hit, f = orc.pair_force((0, 0, 0), 12.0, (10.0, 0, 0), 12.0)
    assert hit
    assert f[0] == pytest.approx(-(4.0 - math.sqrt(6.0)), rel=1e-15)  # pushed away from +x
    assert f[1] == 0.0 and f[2] == 0.0


@pytest.mark.parametrize("d1,d2", [(12.0, 12.0), (10.0, 15.0)])  # both give rhat = 3
def test_zero_crossing_and_minimum(orc, d1, d2):
    k, g = 2.0, 1.0
    rhat = (d1 / 2) * (d2 / 2) / (d1 / 2 + d2 / 2)
    assert rhat == 3.0
    s = (d1 + d2) / 2
    dstar = g * g * rhat / (k * k)  # 0.75
    hit, f = orc.pair_force((0, 0, 0), d1, (s - dstar, 0, 0), d2, k, g)
    assert hit and f[0] == 0.0  # exactly: 1.5 - sqrt(2.25)
    hit, f = orc.pair_force((0, 0, 0), d1, (0, 0, s - dstar / 4), d2, k, g)
    assert hit and f[2] == 0.375  # attraction -0.375 pulls i toward j at +z
    # the minimum: neighbouring overlaps are less attractive
    for dd in (dstar / 4 * 0.9, dstar / 4 * 1.1):
        _, f2 = orc.pair_force((0, 0, 0), d1, (0, 0, s - dd), d2, k, g)
        assert f2[2] < 0.375


def test_no_contact_and_touching(orc):
    hit, f = orc.pair_force((0, 0, 0), 10.0, (10.0, 0, 0), 10.0)  # delta == 0
    assert not hit and not f.any()
    hit, f = orc.pair_force((0, 0, 0), 10.0, (10.5, 0, 0), 10.0)
    assert not hit
    hit, f = orc.pair_force((1, 2, 3), 10.0, (1, 2, 3), 10.0)  # coincident centres
    assert hit and not f.any()


def test_repulsive_at_large_overlap(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        pi = rng.uniform(-5, 5, 3)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        pj = pi + u * rng.uniform(0.5, 6.0)  # deep overlap of two 12-um spheres
        hit, f = orc.pair_force(pi, 12.0, pj, 12.0)
        assert hit and np.dot(f, pi - pj) > 0


@pytest.mark.parametrize("bits", [64, 32])
def test_antisymmetry_bit_exact(orc, bits):
    rng = np.random.default_rng(2)
    for _ in range(300):
        pi = rng.uniform(0, 20, 3)
        pj = rng.uniform(0, 20, 3)
        di, dj = rng.uniform(8, 15, 2)
        h1, f1 = orc.pair_force(pi, di, pj, dj, bits=bits)
        h2, f2 = orc.pair_force(pj, dj, pi, di, bits=bits)
        assert h1 == h2
        assert np.array_equal(f1, -f2)


def test_f32_close_to_f64(orc):
    rng = np.random.default_rng(3)
    for _ in range(300):
        pi = rng.uniform(0, 10, 3)
        pj = rng.uniform(0, 10, 3)
        h1, f1 = orc.pair_force(pi, 12.0, pj, 12.0, bits=64)
        h2, f2 = orc.pair_force(pi, 12.0, pj, 12.0, bits=32)
        if h1 and h2:
            assert np.allclose(f1, f2, rtol=1e-4, atol=1e-5)


def test_displacement_gate_edge(orc):
    a = 0.4
    flag, disp = orc.displacement((a, 0.0, 0.0), a, 0.01, 3.0)  # |F| == adh moves
    assert flag == 0 and disp[0] == 0.01 * a
    flag, disp = orc.displacement((a, 0.0, 0.0), np.nextafter(a, 1.0), 0.01, 3.0)
    assert flag == 1 and not disp.any()
    flag, disp = orc.displacement((np.nextafter(a, 0.0), 0.0, 0.0), a, 0.01, 3.0)
    assert flag == 1


def test_displacement_clamp(orc):
    f = np.array([10.0, -12.0, 6.0])  # |F| = 16.7332
    flag, disp = orc.displacement(f, 0.4, 1.0, 3.0)
    assert flag == 2
    assert np.linalg.norm(disp) == pytest.approx(3.0, rel=1e-15)
    assert np.allclose(disp / np.linalg.norm(disp), f / np.linalg.norm(f), rtol=1e-15)
    flag, disp = orc.displacement(f, 0.4, 0.1, 3.0)  # 1.67 < 3: not clamped
    assert flag == 0 and np.array_equal(disp, 0.1 * f)


def test_two_sphere_step(orc):
    s = dict(x=np.array([0.0, 10.0]), y=np.zeros(2), z=np.zeros(2), d=np.full(2, 12.0),
             adh=np.full(2, 0.4))
    fx, fy, fz, nc, fl = orc.mech_step(s, k=2.0, gamma=1.0, dt=0.01)
    F = 4.0 - math.sqrt(6.0)
    assert fx[0] == pytest.approx(-F, rel=1e-15) and fx[1] == -fx[0]
    assert nc.tolist() == [1, 1] and fl.tolist() == [0, 0]
    assert s["x"][0] == pytest.approx(-0.01 * F, rel=1e-14)
    assert s["x"][1] - s["x"][0] == pytest.approx(10.0 + 0.02 * F, rel=1e-15)


def test_two_sphere_gated(orc):
    s = dict(x=np.array([0.0, 11.25]), y=np.zeros(2), z=np.zeros(2), d=np.full(2, 12.0),
             adh=np.full(2, 0.4))
    x0 = s["x"].copy()
    fx, *_rest, fl = orc.mech_step(s)
    assert np.all(fx == 0.0) and fl.tolist() == [1, 1] and np.array_equal(s["x"], x0)


def brute_force_sum(s, bits=64, k=2.0, gamma=1.0):
    """Summed forces by visiting all j for each i (no grid, ascending j order)."""
    n = len(s["x"])
    out = np.zeros((n, 3))
    x, y, z, d = s["x"], s["y"], s["z"], s["d"]
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    dz = z[:, None] - z[None, :]
    dist = np.sqrt((dx * dx + dy * dy) + dz * dz)
    ri = 0.5 * d
    delta = (ri[:, None] + ri[None, :]) - dist
    np.fill_diagonal(delta, -1.0)
    mask = delta > 0
    contrib_abs = np.zeros(n)
    for i in range(n):
        js = np.nonzero(mask[i])[0]
        for j in js:
            hit, f = orc_pair(s, i, j, bits, k, gamma)
            out[i] += f
            contrib_abs[i] += np.linalg.norm(f)
    return out, contrib_abs, mask.sum(axis=1)


def orc_pair(s, i, j, bits, k, gamma):
    from oracle import oracle as o
    return o.pair_force((s["x"][i], s["y"][i], s["z"][i]), s["d"][i],
                        (s["x"][j], s["y"][j], s["z"][j]), s["d"][j], k, gamma, bits)


@pytest.mark.parametrize("bits", [64, 32])
def test_summed_force_vs_brute_force(orc, bits):
    s = inputs.uniform_cube(500, 80.0, seed=4)
    ref, absum, nref = brute_force_sum(s, bits)
    s2 = {k: v.copy() for k, v in s.items()}
    fx, fy, fz, nc, fl = orc.mech_step(s2, force_bits=bits)
    got = np.stack([fx, fy, fz], axis=1)
    assert np.array_equal(nc, nref)
    err = np.linalg.norm(got - ref, axis=1)
    assert np.all(err <= 1e-13 * np.maximum(absum, 1e-300) + 1e-300)


@pytest.mark.parametrize("bits", [64, 32])
def test_reach_adversarial_pairs(orc, bits):
    """Pairs at the edge of the 27-box reach (across corners, edges and faces, the partner of
    the largest diameter): the grid finds exactly the brute-force contacts, and in binary64 the
    even-numbered pairs touch and the odd-numbered ones miss, as built."""
    s = inputs.reach_adversarial(96, 12.0, seed=7)
    n = len(s["x"])
    pos = np.stack([s["x"], s["y"], s["z"]], axis=1)
    near = np.linalg.norm(pos[:, None, :] - pos[None, :, :], axis=2) < 24.0
    nref = np.zeros(n, dtype=np.int64)
    for i in range(n):
        for j in np.nonzero(near[i])[0]:
            if j != i:
                nref[i] += bool(orc_pair(s, i, j, bits, 2.0, 1.0)[0])
    s2 = {k: v.copy() for k, v in s.items()}
    fx, fy, fz, nc, fl = orc.mech_step(s2, force_bits=bits)
    assert np.array_equal(nc, nref)
    if bits == 64:
        assert np.array_equal(nref.reshape(-1, 2)[:, 0], np.tile([1, 0], 48))


def test_net_force_vanishes(orc):
    s = inputs.uniform_cube(4096, 200.0, seed=0)
    s2 = {k: v.copy() for k, v in s.items()}
    fx, fy, fz, nc, fl = orc.mech_step(s2)
    # |sum_i F_i| <= c * eps * sum_i sum_j |F_ij|; sum |F_i| bounds from below the pair sum
    total_abs = np.abs(fx).sum() + np.abs(fy).sum() + np.abs(fz).sum()
    net = np.array([fx.sum(), fy.sum(), fz.sum()])
    assert np.linalg.norm(net) <= 64 * np.finfo(float).eps * total_abs * 4.3
    assert nc.mean() > 3.0  # about 4.3 contacts per agent at this packing


def test_synchronous_update(orc):
    """Positions after the step depend only on positions before it: re-ordering agent ids
    (a permutation) permutes the results exactly when the canonical sum order is kept."""
    s = inputs.uniform_cube(800, 100.0, seed=12)
    a = {k: v.copy() for k, v in s.items()}
    fa = orc.mech_step(a)
    b = {k: v.copy() for k, v in s.items()}
    fb = orc.mech_step(b)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(fa[0], fb[0])  # deterministic
    # a translation by an exact multiple of the box edge leaves every force bit-identical
    b2 = {k: v.copy() for k, v in s.items()}
    shift = 16.0 * 2 ** 0  # exact in binary; keeps dx bits if |x| ranges stay in one binade
    for key in ("x", "y", "z"):
        b2[key] = b2[key] + shift
    fb2 = orc.mech_step(b2)
    rel = np.abs(fb2[0] - fa[0]).max() / np.abs(fa[0]).max()
    assert rel < 1e-12


def test_mech_validation(orc):
    s = inputs.uniform_cube(10, 100.0, seed=1)
    for kw in [dict(dt=0.0), dict(dt=-1.0), dict(max_disp=0.0), dict(force_bits=16)]:
        with pytest.raises(orc.OracleError) as e:
            orc.mech_step({k: v.copy() for k, v in s.items()}, **kw)
        assert e.value.rc == orc.EINVAL


def test_empty_and_single(orc):
    s = dict(x=np.zeros(0), y=np.zeros(0), z=np.zeros(0), d=np.zeros(0), adh=np.zeros(0))
    orc.mech_step(s)
    s = dict(x=np.array([1.0]), y=np.array([2.0]), z=np.array([3.0]), d=np.array([10.0]),
             adh=np.array([0.4]))
    fx, fy, fz, nc, fl = orc.mech_step(s)
    assert fx[0] == 0.0 and nc[0] == 0 and fl[0] == 1 and s["x"][0] == 1.0


def test_mech_sample_matches_full_step(orc):
    """The sampled-agent entry used at full size computes each agent's force exactly as the
    full step does (same grid, same candidate order)."""
    st = orc.generate_cube(3000, 7, 180.0, 10.0, 15.0, 0.4)
    ids = np.array([0, 1, 17, 1500, 2999])
    for bits in (64, 32):
        s2 = {k: v.copy() for k, v in st.items()}
        fx, fy, fz, nc, _ = orc.mech_step(s2, force_bits=bits)
        sx, sy, sz, snc = orc.mech_sample(st, ids, force_bits=bits)
        assert np.array_equal(sx, fx[ids]) and np.array_equal(sy, fy[ids]) and np.array_equal(sz, fz[ids])
        assert np.array_equal(snc, nc[ids])
