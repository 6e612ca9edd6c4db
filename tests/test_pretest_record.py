"""The mechanics pre-test on 8-byte records, modelled in numpy from its definition and checked
against the oracle's contact decision: every pair that either pair law (binary64 or binary32,
reading R21) counts as a contact must pass the record test, so the filter in front of the exact
law drops no contact.

The record, per axis: the box index c (floor of the coordinate over the box edge b, as the key
rounds it) mod 4 in the top 2 of 16 bits, above the offset within the box in units of b / 2^14,
floor((v * fl(1/b) - c) * 2^14) clamped to [0, 2^14 - 1]; the radius in the same units, rounded
up plus one.  The test reads each axis difference modulo 2^16 as a signed 16-bit value and
compares the exact integer squared distance with (R_i + R_j)^2.  This is a model of the
definition, not the kernel's code; the GPU parity tests check the kernel bit for bit.

Pairs sit at the edge of contact (distance (r_i + r_j)(1 + e), |e| <= 1e-6 and a few at 0),
in boxes at lattice coordinates up to 2^30, with box edges from the largest diameter to five
times it.  A control set of pairs b / 100 beyond contact (164 units) must fail the test, so
it is not vacuous.
"""
import numpy as np

from oracle import oracle as orc


def encode_axis(v, c, inv_b):
    u = (v * inv_b - c) * 16384.0
    q = np.clip(np.floor(np.maximum(u, 0.0)), 0, 16383).astype(np.int64)
    return ((c & 3) << 14) | q


def encode_radius(r, inv_b):
    return np.minimum(np.ceil(r * inv_b * 16384.0) + 1.0, 65535.0).astype(np.int64)


def signed16(d):
    d = d & 0xFFFF
    return np.where(d >= 32768, d - 65536, d)


def record_test(vi, vj, ri, rj, b):
    """Pass/fail of the record test for pairs (arrays of shape (n, 3) and (n,))."""
    inv_b = 1.0 / b
    ci = np.floor(vi / b[:, None]).astype(np.int64)
    cj = np.floor(vj / b[:, None]).astype(np.int64)
    assert np.all(np.abs(cj - ci) <= 1), "a candidate's box is within one of the agent's"
    ai = encode_axis(vi, ci, inv_b[:, None])
    aj = encode_axis(vj, cj, inv_b[:, None])
    d = signed16(aj - ai)
    # every field difference is below 2^15 in magnitude, so the kernel's packed 16-bit
    # arithmetic (x, y as a signed dot product below 2^31, z added as an unsigned word) is exact
    assert np.all(np.abs(d) < (1 << 15))
    d2 = (d * d).sum(axis=1)
    assert np.all(d2 < (3 << 30))
    sr = encode_radius(ri, inv_b) + encode_radius(rj, inv_b)
    return d2 < sr * sr


def edge_pairs(n, rng, rel, gap=0.0):
    b = rng.uniform(4.0, 40.0, n)
    scale = rng.uniform(1.0, 5.0, n)  # box edge over the largest diameter
    ri = rng.uniform(0.04, 1.0, n) * b / (2.0 * scale)
    rj = rng.uniform(0.04, 1.0, n) * b / (2.0 * scale)
    c = rng.integers(-(1 << 30), 1 << 30, size=(n, 3)).astype(np.float64)
    vi = (c + rng.uniform(0.0, 1.0, (n, 3))) * b[:, None]
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    vj = vi + ((ri + rj) * (1.0 + rel) + gap * b)[:, None] * u
    return vi, vj, ri, rj, b


def test_record_test_keeps_every_contact():
    rng = np.random.default_rng(20060677)
    n = 6000
    rel = np.concatenate([rng.uniform(-1e-6, 1e-6, n - 200), np.zeros(200)])
    vi, vj, ri, rj, b = edge_pairs(n, rng, rel)
    passed = record_test(vi, vj, ri, rj, b)
    contacts = 0
    for k in range(n):
        hit = any(orc.pair_force(vi[k], 2.0 * ri[k], vj[k], 2.0 * rj[k], 2.0, 1.0, bits)[0] for bits in (64, 32))
        contacts += hit
        assert not hit or passed[k], (k, vi[k], vj[k], ri[k], rj[k], b[k])
    assert contacts > n // 4  # the set does straddle the contact distance


def test_record_test_rejects_pairs_a_hundredth_of_a_box_apart():
    rng = np.random.default_rng(7)
    n = 4000
    vi, vj, ri, rj, b = edge_pairs(n, rng, np.zeros(n), gap=0.01)
    assert not record_test(vi, vj, ri, rj, b).any()
