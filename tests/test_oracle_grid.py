"""Pins of the oracle's uniform grid (paper Sec. 2.1: equal boxes, an agent belongs to the box of
its centre, neighbours = own box + 26 around it, box edge from the largest agent).

Keys, sorted order and start offsets are checked against a direct numpy recomputation of the
definition; contact sets found through the 27-box search are checked against brute force over
all O(N^2) pairs, which needs no grid at all.
"""
import numpy as np
import pytest

import inputs


def recompute_grid(x, y, z, d, box=0.0):
    b = box if box > 0 else d.max()
    c = np.stack([np.floor(x / b), np.floor(y / b), np.floor(z / b)]).astype(np.int64)
    cmin = c.min(axis=1)
    dims = c.max(axis=1) - cmin + 1
    rel = c - cmin[:, None]
    key = rel[0] + dims[0] * (rel[1] + dims[1] * rel[2])
    order = np.lexsort((np.arange(len(x)), key))  # primary key, then id
    nb = int(np.prod(dims))
    start = np.searchsorted(key[order], np.arange(nb + 1), side="left")
    return b, cmin, dims, key, order, start


@pytest.mark.parametrize("case", ["uniform", "faces", "clustered", "lattice"])
def test_keys_order_start(orc, case):
    if case == "uniform":
        s = inputs.uniform_cube(3000, 200.0, seed=1)
    elif case == "faces":
        s = inputs.box_face_adversarial(2000, 12.0, seed=2)
    elif case == "clustered":
        s = inputs.clustered(2500, 300.0, seed=3)
    else:
        s = inputs.lattice(9, 11.0, 12.0, origin=-40.0)
    info, key, order, start = orc.grid(s["x"], s["y"], s["z"], s["d"])
    b, cmin, dims, k2, o2, s2 = recompute_grid(s["x"], s["y"], s["z"], s["d"])
    assert info["b"] == b
    assert tuple(info["cmin"]) == tuple(cmin) and tuple(info["dims"]) == tuple(dims)
    assert np.array_equal(key, k2)
    assert np.array_equal(order, o2)
    assert np.array_equal(start, s2)


def brute_force_contacts(x, y, z, d, key):
    """All pairs with (ri + rj) - dist > 0, listed per agent in ascending (key, id)."""
    n = len(x)
    out = []
    for i in range(n):
        dx = x[i] - x
        dy = y[i] - y
        dz = z[i] - z
        dist = np.sqrt((dx * dx + dy * dy) + dz * dz)
        hit = ((0.5 * d[i] + 0.5 * d) - dist) > 0
        hit[i] = False
        j = np.nonzero(hit)[0]
        j = j[np.lexsort((j, key[j]))]
        out.append(j)
    return out


@pytest.mark.parametrize("case", ["uniform", "faces", "clustered", "dense"])
def test_contacts_equal_brute_force(orc, case):
    if case == "uniform":
        s = inputs.uniform_cube(1500, 150.0, seed=5)
    elif case == "faces":
        s = inputs.box_face_adversarial(1200, 10.0, cells=5, d=None, seed=6)
        s["d"][:] = np.random.default_rng(0).uniform(5.0, 10.0, len(s["d"]))
        s["d"][0] = 10.0
    elif case == "clustered":
        s = inputs.clustered(1200, 200.0, clusters=4, seed=7)
    else:
        s = inputs.uniform_cube(2000, 60.0, seed=8)  # heavy overlap, many per box
    counts, offsets, ids = orc.contacts(s["x"], s["y"], s["z"], s["d"])
    _, key, _, _ = orc.grid(s["x"], s["y"], s["z"], s["d"])
    bf = brute_force_contacts(s["x"], s["y"], s["z"], s["d"], key.astype(np.int64))
    assert counts.sum() > 0
    for i in range(len(s["x"])):
        got = ids[offsets[i]: offsets[i] + counts[i]]
        assert np.array_equal(got, bf[i]), i


def test_contacts_independent_of_box_size(orc):
    """Any box edge at least the largest diameter finds the same contact sets (metamorphic)."""
    s = inputs.uniform_cube(1500, 150.0, seed=9)
    c0, o0, i0 = orc.contacts(s["x"], s["y"], s["z"], s["d"])
    for box in [s["d"].max() * 1.37, 31.0]:
        c1, o1, i1 = orc.contacts(s["x"], s["y"], s["z"], s["d"], box=box)
        assert np.array_equal(c0, c1)
        for i in range(0, len(c0), 13):
            assert set(i0[o0[i]:o0[i] + c0[i]]) == set(i1[o1[i]:o1[i] + c1[i]])


def test_periodic_min_image_contacts(orc):
    L, R = 100.0, 2.0
    s = inputs.sir_uniform(3000, L, seed=10)
    counts, offsets, ids = orc.contacts(s["x"], s["y"], s["z"], None, box=8.0, periodic=True,
                                        L=L, radius=R)
    x, y, z = s["x"], s["y"], s["z"]
    for i in range(0, 3000, 3):
        dd = []
        for a in (x, y, z):
            v = a[i] - a
            v = np.where(v > L / 2, v - L, np.where(v < -L / 2, v + L, v))
            dd.append(v)
        d2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]
        hit = d2 <= R * R
        hit[i] = False
        assert set(ids[offsets[i]:offsets[i] + counts[i]].tolist()) == set(np.nonzero(hit)[0].tolist())
    assert counts.sum() > 0


def test_periodic_grid_shape(orc):
    info, key, order, start = orc.grid([1.0, 4999.0], [0.0, 2500.0], [10.0, 4999.999], None,
                                       box=20.0, periodic=True, L=5000.0)
    assert info["b"] == 20.0 and info["dims"] == (250, 250, 250)
    assert key[0] == 0
    assert key[1] == 249 + 250 * (125 + 250 * 249)


def test_grid_validation(orc):
    s = inputs.uniform_cube(50, 100.0, seed=1)
    with pytest.raises(orc.OracleError) as e:
        orc.grid(s["x"], s["y"], s["z"], s["d"], box=s["d"].max() * 0.99)
    assert e.value.rc == orc.EINVAL
    with pytest.raises(orc.OracleError) as e:
        orc.grid(s["x"], s["y"], s["z"], None, box=40.0, periodic=True, L=100.0)
    assert e.value.rc == orc.EINVAL  # fewer than 3 boxes per axis
    x = s["x"].copy()
    x[3] = np.nan
    with pytest.raises(orc.OracleError) as e:
        orc.grid(x, s["y"], s["z"], s["d"])
    assert e.value.rc == orc.ENONFINITE
    with pytest.raises(orc.OracleError) as e:
        orc.grid(s["x"], s["y"], s["z"], s["d"], max_boxes=10)
    assert e.value.rc == orc.ETOOMANYBOXES


def test_grid_single_agent(orc):
    info, key, order, start = orc.grid([5.0], [-3.0], [1e6], [10.0])
    assert info["nboxes"] == 1 and key.tolist() == [0] and start.tolist() == [0, 1]


def test_lattice_span_beyond_max_boxes_is_refused(orc):
    """Two agents 2^31 boxes apart (lattice coordinates -2^30 and 2^30 - 1 at b = 10): the
    lattice has 2^31 boxes along x, more than max_boxes, and the grid is refused."""
    b = 10.0
    x = np.array([-(2.0 ** 30) * b + 5.0, (2.0 ** 30 - 1.0) * b + 5.0])
    yz = np.array([5.0, 5.0])
    assert np.floor(x / b).tolist() == [-(2.0 ** 30), 2.0 ** 30 - 1.0]
    with pytest.raises(orc.OracleError) as e:
        orc.grid(x, yz, yz, np.array([b, b]), max_boxes=1 << 16)
    assert e.value.rc == orc.ETOOMANYBOXES
    # the same pair 2^16 - 1 boxes apart still fits exactly
    x2 = np.array([5.0, (2.0 ** 16 - 1.0) * b + 5.0])
    info, key, order, start = orc.grid(x2, yz, yz, np.array([b, b]), max_boxes=1 << 16)
    assert info["dims"] == (1 << 16, 1, 1) and key.tolist() == [0, (1 << 16) - 1]
