"""Pins of the oracle's tumour-spheroid growth and division (paper Sec. 3.2: cell growth and
duplication; the growth/division benchmark of Sec. 3.4).

Mechanics never changes counts or diameters, so an independent diameter-only model (a list of
diameters, grown and split each step) fixes the population size and the multiset of diameters
exactly.  Each division is checked for centre-of-mass and volume conservation and for its
random axis against numpy's Philox.
"""
import numpy as np
import pytest

from test_oracle_rng import numpy_draw, _u

G = 1.05 ** (1.0 / 3.0)
H = 0.5 ** (1.0 / 3.0)


def diameter_model(d0, steps, grow=G, div_d=14.0, h=H, capacity=None):
    d = list(d0)
    counts = []
    for _ in range(steps):
        d = [v * grow for v in d]
        n0 = len(d)
        for i in range(n0):
            if d[i] >= div_d and (capacity is None or len(d) < capacity):
                d[i] = d[i] * h
                d.append(d[i])
        counts.append(len(d))
    return counts, d


def params(orc, seed=0, **mech):
    mp = dict(k=2.0, gamma=1.0, dt=0.01, max_disp=3.0)
    mp.update(mech)
    return orc.spheroid_params(G, 14.0, H, seed, **mp)


def test_counts_and_diameters_match_model(orc):
    init = orc.generate_ball(400, 1, 25.0, 14.0 * H, 14.0, 0.4)
    st = orc.SpheroidState(init, capacity=20000)
    p = params(orc, seed=1)
    counts = []
    for t in range(30):
        st.step(p, t)
        counts.append(int(st.n[0]))
    ref_counts, ref_d = diameter_model(init["d"], 30)
    assert counts == ref_counts
    assert np.array_equal(np.sort(st.view("d")), np.sort(np.array(ref_d)))


def test_division_geometry(orc):
    init = dict(x=np.array([1.0, 50.0]), y=np.array([2.0, 50.0]), z=np.array([3.0, 50.0]),
                d=np.array([13.9, 10.0]), adh=np.array([0.4, 0.7]))
    st = orc.SpheroidState(init, capacity=10)
    p = params(orc, seed=9)
    st.grow_divide(p, 5)
    assert int(st.n[0]) == 3
    d_grown = 13.9 * G
    dp = d_grown * H
    assert st.arr["d"][0] == dp and st.arr["d"][2] == dp and st.arr["d"][1] == 10.0 * G
    assert st.arr["adh"][2] == 0.4
    m = np.array([st.arr[k][0] for k in "xyz"])
    c = np.array([st.arr[k][2] for k in "xyz"])
    assert np.allclose((m + c) / 2, [1.0, 2.0, 3.0], rtol=0, atol=4e-16 * 4)
    assert np.linalg.norm(c - m) == pytest.approx(dp / 2, rel=1e-15)
    # volume conservation: two daughters of diameter d*h hold the mother's volume
    assert 2 * dp ** 3 == pytest.approx(d_grown ** 3, rel=1e-14)
    # axis from the DIV draws of mother id 0 at step 5
    for attempt in range(64):
        v = 2.0 * _u(numpy_draw(9, 0, 5, attempt, 0, 5)[:3]) - 1.0
        s = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]
        if 0.0 < s <= 1.0:
            break
    u = v / np.sqrt(s)
    assert np.array_equal(orc.division_axis(9, 0, 5), u)
    assert np.allclose((c - m) / np.linalg.norm(c - m), u, rtol=1e-14)


def test_daughter_ids_follow_mother_id_order(orc):
    n = 50
    init = dict(x=np.arange(n) * 30.0, y=np.zeros(n), z=np.zeros(n),
                d=np.where(np.arange(n) % 3 == 0, 13.95, 9.0), adh=np.full(n, 0.4))
    st = orc.SpheroidState(init, capacity=1000)
    st.grow_divide(params(orc), 0)
    mothers = np.nonzero(init["d"] * G >= 14.0)[0]
    assert int(st.n[0]) == n + len(mothers)
    for r, i in enumerate(mothers):
        # the daughter sits opposite its mother about the mother's old centre
        assert (st.arr["x"][n + r] + st.arr["x"][i]) / 2 == pytest.approx(i * 30.0, abs=1e-12)


def test_capacity_overflow(orc):
    n = 20
    init = dict(x=np.arange(n) * 30.0, y=np.zeros(n), z=np.zeros(n), d=np.full(n, 13.99),
                adh=np.full(n, 0.4))
    st = orc.SpheroidState(init, capacity=25)
    ov = st.grow_divide(params(orc), 0)
    assert ov and int(st.n[0]) == 25
    assert np.all(st.arr["d"][:5] == 13.99 * G * H)  # first five mothers (by id) divided
    assert np.all(st.arr["d"][5:20] == 13.99 * G)    # the rest only grew
    counts, _ = diameter_model(init["d"], 1, capacity=25)
    assert counts == [25]


@pytest.mark.slow
def test_literal_growth_config_counts(orc):
    """10,000 cells in a ball of radius 60 um, 60 steps: count sequence of the diameter model."""
    init = orc.generate_ball(10000, 0, 60.0, 14.0 * H, 14.0, 0.4)
    counts, _ = diameter_model(init["d"], 60)
    assert 1.5e5 < counts[-1] < 2.5e5
