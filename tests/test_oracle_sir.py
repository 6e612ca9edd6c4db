"""Pins of the oracle's SIR step (paper Sec. 3.3: infection with a probability when an infected
agent is within the infection radius, recovery with a probability every step, bounded random
movement; agents counted per group).

Deterministic cases (probabilities 0 or 1, no movement) are counted by hand.  Probabilistic
cases are recomputed independently with brute-force minimum-image distances and numpy's Philox.
"""
import numpy as np
import pytest

from test_oracle_rng import numpy_draw, _u

S, I, R = 0, 1, 2


def sir_p(orc, L=100.0, box=10.0, r=2.0, p_inf=1.0, p_rec=0.0, walk=0.0, seed=0):
    return orc.sir_params(L, box, r, p_inf, p_rec, walk, seed)


def hand_lattice():
    pts = [
        ((50.0, 50.0, 50.0), I),     # 0 infected source
        ((52.0, 50.0, 50.0), S),     # 1 exactly at the radius: infected (inclusive)
        ((50.0, np.nextafter(52.0, 60.0), 50.0), S),  # 2 one ulp beyond: stays S
        ((50.0, 50.0, 48.0), S),     # 3 at the radius along -z: infected
        ((0.5, 10.0, 10.0), I),      # 4 infected source near the x = 0 face
        ((99.0, 10.0, 10.0), S),     # 5 minimum-image distance 1.5 through the wrap: infected
        ((50.0, 51.0, 50.0), R),     # 6 recovered stays recovered
        ((51.0, 50.0, 50.0), S),     # 7 inside the radius: infected
        ((20.0, 80.0, 20.0), S),     # 8 isolated
        ((50.0, 50.0, 50.0), S),     # 9 coincident with the source: infected
        ((54.0, 50.0, 50.0), S),     # 10 within 2 of agent 1 only, which is S at t: stays S
    ]
    x = np.array([p[0][0] for p in pts])
    y = np.array([p[0][1] for p in pts])
    z = np.array([p[0][2] for p in pts])
    st = np.array([p[1] for p in pts], dtype=np.uint8)
    return dict(x=x, y=y, z=z, state=st)


def test_hand_counted_infection(orc):
    s = hand_lattice()
    x0 = s["x"].copy()
    counts = orc.sir_step(s, sir_p(orc), 0)
    assert s["state"].tolist() == [1, 1, 0, 1, 1, 1, 2, 1, 0, 1, 0]
    assert counts.tolist() == [3, 7, 1]
    assert np.array_equal(s["x"], x0)  # no movement


def test_recovering_agent_still_infects(orc):
    s = hand_lattice()
    orc.sir_step(s, sir_p(orc, p_rec=1.0), 0)
    assert s["state"].tolist() == [2, 1, 0, 1, 2, 1, 2, 1, 0, 1, 0]


def test_no_infection_probability(orc):
    s = hand_lattice()
    counts = orc.sir_step(s, sir_p(orc, p_inf=0.0), 0)
    assert s["state"].tolist() == [1, 0, 0, 0, 1, 0, 2, 0, 0, 0, 0]
    assert counts.tolist() == [8, 2, 1]


def test_pure_recovery_matches_draws(orc):
    n = 500
    rng = np.random.default_rng(3)
    s = dict(x=rng.uniform(0, 100, n), y=rng.uniform(0, 100, n), z=rng.uniform(0, 100, n),
             state=np.ones(n, dtype=np.uint8))
    orc.sir_step(s, sir_p(orc, p_inf=0.0, p_rec=0.25, seed=5), 17)
    T = int(0.25 * 2 ** 64)
    exp = [R if int(numpy_draw(5, 0, 3, 0, i, 17)[0]) < T else I for i in range(n)]
    assert s["state"].tolist() == exp


def reference_sir_step(s, L, r, p_inf, p_rec, walk, seed, step):
    """Brute force: every pair's minimum-image distance, numpy Philox draws."""
    n = len(s["x"])
    x, y, z, st = s["x"], s["y"], s["z"], s["state"]
    T_inf = int(np.floor(np.float64(p_inf) * 2.0 ** 64)) if p_inf < 1 else None
    T_rec = int(np.floor(np.float64(p_rec) * 2.0 ** 64)) if p_rec < 1 else None
    nxt = st.copy()
    infected = st == I
    for i in range(n):
        if st[i] == S:
            dd = []
            for a in (x, y, z):
                v = a[i] - a
                v = np.where(v > L / 2, v - L, np.where(v < -L / 2, v + L, v))
                dd.append(v)
            d2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]
            hit = (d2 <= r * r) & infected
            hit[i] = False
            m = int(hit.sum())
            for c in range(m):
                if int(numpy_draw(seed, 0, 4, c, i, step)[0]) < T_inf:
                    nxt[i] = I
                    break
        elif st[i] == I:
            if int(numpy_draw(seed, 0, 3, 0, i, step)[0]) < T_rec:
                nxt[i] = R
    pos = []
    for a_idx, a in enumerate((x, y, z)):
        w = np.array([numpy_draw(seed, 0, 2, 0, i, step)[a_idx] for i in range(n)], dtype=np.uint64)
        v = a + walk * (2.0 * _u(w) - 1.0)
        v = np.where(v < 0.0, v + L, v)
        v = np.where(v >= L, v - L, v)
        v = np.where(v == L, 0.0, v)
        pos.append(v)
    return dict(x=pos[0], y=pos[1], z=pos[2], state=nxt)


def test_probabilistic_step_matches_brute_force(orc):
    n, L = 2000, 100.0  # the paper's epidemiology setting: 2000 agents in a cube of length 100
    rng = np.random.default_rng(11)
    s = dict(x=rng.uniform(0, L, n), y=rng.uniform(0, L, n), z=rng.uniform(0, L, n),
             state=rng.choice(np.array([0, 1, 2], dtype=np.uint8), n, p=[0.7, 0.25, 0.05]))
    for step in range(3):
        ref = reference_sir_step(s, L, 4.0, 0.3, 0.1, 1.0, 21, step)
        orc.sir_step(s, orc.sir_params(L, 5.0, 4.0, 0.3, 0.1, 1.0, 21), step)
        for key in ("x", "y", "z", "state"):
            assert np.array_equal(s[key], ref[key]), (key, step)


def test_invariants_over_many_steps(orc):
    n, L = 3000, 100.0
    g = orc.generate_sir(n, 2, L, 30)
    prev = None
    for step in range(40):
        x0 = g["x"].copy()
        counts = orc.sir_step(g, orc.sir_params(L, 4.0, 3.0, 0.3, 0.05, 1.0, 2), step)
        assert counts.sum() == n
        assert np.all((g["x"] >= 0) & (g["x"] < L))
        dx = np.abs(g["x"] - x0)
        dx = np.minimum(dx, L - dx)
        assert dx.max() <= 1.0 + 1e-12
        if prev is not None:
            assert counts[0] <= prev[0] and counts[2] >= prev[2]
        prev = counts
    assert prev[2] > 0


def test_wrap_corner(orc):
    # an agent just below 0 after the walk wraps to a value in [0, L)
    s = dict(x=np.array([1e-17, 50.0]), y=np.array([5.0, 5.0]), z=np.array([5.0, 5.0]),
             state=np.zeros(2, dtype=np.uint8))
    for step in range(20):
        orc.sir_step(s, orc.sir_params(100.0, 10.0, 2.0, 0.0, 0.0, 1.0, 3), step)
        assert np.all((s["x"] >= 0) & (s["x"] < 100.0))


def test_sir_validation(orc):
    s = hand_lattice()
    with pytest.raises(orc.OracleError):
        orc.sir_step(s, orc.sir_params(100.0, 1.0, 2.0, 0.3, 0.1, 1.0, 0), 0)  # box < radius
    with pytest.raises(orc.OracleError):
        orc.sir_step(s, orc.sir_params(100.0, 40.0, 2.0, 0.3, 0.1, 1.0, 0), 0)  # < 3 boxes
