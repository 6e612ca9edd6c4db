"""Pins of the oracle's counter-based generator and seeded initial states.

Philox4x64-10 is pinned to two independent things: the published known-answer vectors
(tests/golden/philox4x64_10_kat.json) and numpy's own Philox bit generator, which implements the
same algorithm and pre-increments counter word 0 before each block.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers(orc):
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        ctr = [int(c, 16) for c in v["ctr"]]
        key = [int(k, 16) for k in v["key"]]
        out = [int(o, 16) for o in v["out"]]
        assert [int(w) for w in orc.philox(ctr, key)] == out


def test_philox_matches_numpy(orc):
    rng = np.random.default_rng(7)
    for _ in range(300):
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64)
        ctr[0] |= np.uint64(1)  # numpy adds one to word 0 first; keep word 0 >= 1 (no borrow)
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64)
        c = ctr.copy()
        c[0] -= np.uint64(1)
        ref = np.random.Philox(key=key, counter=c).random_raw(4)
        assert np.array_equal(orc.philox(ctr, key), ref)


def numpy_draw(seed, salt, purpose, attempt, agent_id, step):
    """One block of the method's draw layout, built from numpy's Philox."""
    ctr = np.array([purpose + (attempt << 8) - 1, agent_id, step, 0], dtype=np.uint64)
    return np.random.Philox(key=np.array([seed, salt], dtype=np.uint64), counter=ctr).random_raw(4)


def test_draw_layout(orc):
    for seed, salt, purpose, attempt, i, step in [(0, 0, 1, 0, 0, 0), (5, 9, 4, 17, 123456, 199),
                                                  (2 ** 40, 3, 5, 63, 2 ** 31, 7)]:
        assert np.array_equal(orc.draw(seed, salt, purpose, attempt, i, step),
                              numpy_draw(seed, salt, purpose, attempt, i, step))


def test_u01_exact(orc):
    for w in [0, 1, 2 ** 11 - 1, 2 ** 11, 2 ** 63, 2 ** 64 - 1, 0x123456789ABCDEF0]:
        u = orc.u01(w)
        assert Fraction(u) == Fraction(w >> 11, 2 ** 53)
        assert 0.0 <= u < 1.0


def test_bernoulli_threshold(orc):
    for p in [0.3, 0.01, 0.5, 1e-300, 0.9999999999999999]:
        T = int(Fraction(p) * 2 ** 64)  # floor of the exact product
        if T == 0:
            assert not orc.bernoulli(0, p)
            continue
        assert orc.bernoulli(T - 1, p) and not orc.bernoulli(T, p)
    assert not orc.bernoulli(0, 0.0) and not orc.bernoulli(0, -1.0)
    assert orc.bernoulli(2 ** 64 - 1, 1.0) and orc.bernoulli(2 ** 64 - 1, 2.0)


def _u(w):
    return (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def test_generate_cube_matches_numpy_construction(orc):
    n, seed, L = 300, 11, 200.0
    got = orc.generate_cube(n, seed, L, 10.0, 15.0, 0.4, salt=3)
    w = np.stack([numpy_draw(seed, 3, 1, 0, i, 0) for i in range(n)])
    assert np.array_equal(got["x"], L * _u(w[:, 0]))
    assert np.array_equal(got["y"], L * _u(w[:, 1]))
    assert np.array_equal(got["z"], L * _u(w[:, 2]))
    assert np.array_equal(got["d"], 10.0 + (15.0 - 10.0) * _u(w[:, 3]))
    assert np.all(got["adh"] == 0.4)
    assert got["x"].min() >= 0 and got["x"].max() < L


def test_generate_ball_rejection(orc):
    n, seed, R = 400, 2, 60.0
    dlo, dhi = 14.0 * 0.5 ** (1 / 3), 14.0
    got = orc.generate_ball(n, seed, R, dlo, dhi, 0.4)
    for i in range(0, n, 7):
        for attempt in range(64):
            w = numpy_draw(seed, 0, 1, attempt, i, 0)
            v = 2.0 * _u(w[:3]) - 1.0
            if (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2] <= 1.0:
                break
        assert got["x"][i] == R * v[0] and got["y"][i] == R * v[1] and got["z"][i] == R * v[2]
        assert got["d"][i] == dlo + (dhi - dlo) * _u(w[3:4])[0]
    r2 = got["x"] ** 2 + got["y"] ** 2 + got["z"] ** 2
    assert np.all(r2 <= R * R * (1 + 1e-12))


def test_generate_sir(orc):
    got = orc.generate_sir(1000, 4, 5000.0, 7)
    assert got["state"][:7].tolist() == [1] * 7 and np.all(got["state"][7:] == 0)
    w = np.stack([numpy_draw(4, 0, 1, 0, i, 0) for i in range(1000)])
    assert np.array_equal(got["x"], 5000.0 * _u(w[:, 0]))


@pytest.mark.parametrize("n", [0, 1])
def test_generate_degenerate(orc, n):
    g = orc.generate_cube(n, 0, 200.0, 10.0, 15.0, 0.4)
    assert len(g["x"]) == n
