"""Pins of the oracle's binary32 pair law (the FP32-force path).

The reading of that path: the separation x_i - x_j is formed in binary64 and then rounded to
binary32; the distance, overlap, rhat, F, F/dist and the three products are binary32 operations,
each correctly rounded; the per-agent sum of the widened terms stays in binary64.  Each case
below has a result that IEEE rounding fixes by hand, chosen so that a plausible misreading fails
one of them:

* positions rounded to binary32 before the subtraction breaks translation invariance (the
  binary64 difference of two positions on a fine dyadic grid is exact at any offset, a binary32
  rounding of the positions is not);
* the law evaluated in binary64 and rounded at the end gives other closed-form values and
  another contact decision at the edge of contact;
* a binary32 accumulation of the terms gives another sum.
"""
import math

import numpy as np
import pytest

# correctly rounded binary32 square roots (IEEE 754: the representable value nearest the real
# root), as bit patterns
SQRT12_F32 = np.uint32(0x405DB3D7).view(np.float32)  # 3.464101552963257
SQRT6_F32 = np.uint32(0x401CC471).view(np.float32)   # 2.4494898319244385


def test_sqrt_constants_are_the_nearest_binary32():
    for v, c in ((12.0, SQRT12_F32), (6.0, SQRT6_F32)):
        lo, hi = np.nextafter(c, np.float32(0)), np.nextafter(c, np.float32(np.inf))
        err = abs(float(c) - math.sqrt(v))
        assert err < abs(float(lo) - math.sqrt(v)) and err < abs(float(hi) - math.sqrt(v))


def test_f32_closed_form_power_of_two_separation(orc):
    # d = 12, 12 (r = 6, 6: rhat = 36/12 = 3 exactly), separation 8 along x, k = gamma = 1:
    # dist = 8, delta = 4, rhat*delta = 12, F = 4 - fl32(sqrt 12), exact by Sterbenz's lemma
    # (fl32(sqrt 12) lies in [2, 8]); F/8 and (F/8)*8 are exact, so the term is -F exactly.
    F = np.float32(4.0) - SQRT12_F32
    assert float(F) == 0.5358984470367432
    hit, f = orc.pair_force((0.0, 0.0, 0.0), 12.0, (8.0, 0.0, 0.0), 12.0, k=1.0, gamma=1.0, bits=32)
    assert hit
    assert f[0] == -float(F) and f[1] == 0.0 and f[2] == 0.0
    # the law evaluated in binary64 and rounded afterwards would give 0.5358983874320984
    assert float(np.float32(4.0 - math.sqrt(12.0))) != float(F)


def test_f32_closed_form_along_each_axis(orc):
    # the same pair along y and z, and with j on the negative side (the term flips sign)
    F = float(np.float32(4.0) - SQRT12_F32)
    for axis in range(3):
        for sign in (1.0, -1.0):
            pj = [0.0, 0.0, 0.0]
            pj[axis] = 8.0 * sign
            hit, f = orc.pair_force((0.0, 0.0, 0.0), 12.0, pj, 12.0, k=1.0, gamma=1.0, bits=32)
            assert hit
            want = np.zeros(3)
            want[axis] = -sign * F
            assert np.array_equal(f, want)


def test_f32_force_at_separation_ten(orc):
    # d = 12, 12, separation 10, k = 2, gamma = 1: F = 4 - fl32(sqrt 6) exactly (Sterbenz).
    # The term along x is fl32(fl32(F / 10) * 10), which rounds back to F here.  The law
    # evaluated wholly in binary64 and rounded at the end gives fl32(4 - sqrt 6) =
    # 1.5505102872848511 instead.
    F = float(np.float32(4.0) - SQRT6_F32)
    assert F == 1.5505101680755615
    assert float(np.float32(np.float32(F) / np.float32(10.0)) * np.float32(10.0)) == F
    hit, f = orc.pair_force((10.0, 0.0, 0.0), 12.0, (0.0, 0.0, 0.0), 12.0, k=2.0, gamma=1.0, bits=32)
    assert hit
    assert f[0] == F and f[1] == 0.0 and f[2] == 0.0
    assert float(np.float32(4.0 - math.sqrt(6.0))) == 1.5505102872848511


def test_f32_equilibrium_and_minimum_exact(orc):
    # rhat = 3, k = 2, gamma = 1: every operation below is exact in binary32
    #   separation 11.25: delta = 0.75, F = 1.5 - sqrt(2.25) = 0
    #   separation 8 + 3.8125 = 11.8125: delta = 0.1875, F = 0.375 - sqrt(0.5625) = -0.375
    hit, f = orc.pair_force((0.0, 0.0, 0.0), 12.0, (11.25, 0.0, 0.0), 12.0, bits=32)
    assert hit and not f.any()
    hit, f = orc.pair_force((0.0, 0.0, 0.0), 12.0, (0.0, 0.0, 11.8125), 12.0, bits=32)
    assert hit
    s = np.float32(-0.375) / np.float32(11.8125)
    assert f[2] == float(s * np.float32(-11.8125)) and f[0] == 0.0 and f[1] == 0.0
    assert f[2] > 0.0  # attraction pulls i (at the origin) toward j at +z


def test_f32_contact_decided_in_binary32(orc):
    # separation 12 - 2^-30: binary64 sees an overlap of 2^-30, but the separation rounded to
    # binary32 is 12 exactly (binary32 spacing at 12 is 2^-20), so delta = 0: no contact
    sep = 12.0 - 2.0 ** -30
    assert orc.pair_force((0.0, 0.0, 0.0), 12.0, (sep, 0.0, 0.0), 12.0, bits=64)[0]
    hit, f = orc.pair_force((0.0, 0.0, 0.0), 12.0, (sep, 0.0, 0.0), 12.0, bits=32)
    assert not hit and not f.any()
    # one binary32 step closer is a contact with delta = 2^-20 in both laws
    sep = 12.0 - 2.0 ** -20
    assert orc.pair_force((0.0, 0.0, 0.0), 12.0, (sep, 0.0, 0.0), 12.0, bits=32)[0]


def test_f32_separation_formed_in_binary64(orc):
    # Positions on the 2^-20 grid within 2^8 of the origin: adding T = 2^20 keeps them exact in
    # binary64 and their difference exact, so the law's input -- and its result -- must not
    # change.  Rounding the positions to binary32 first (spacing 2^-3 at 2^20) would.
    rng = np.random.default_rng(7)
    T = 2.0 ** 20
    changed_if_rounded_first = 0
    for _ in range(300):
        pi = np.round(rng.uniform(0, 20, 3) * 2 ** 20) / 2 ** 20
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        pj = np.round((pi + u * rng.uniform(2.0, 11.0)) * 2 ** 20) / 2 ** 20
        di, dj = rng.uniform(8, 12, 2)
        h0, f0 = orc.pair_force(pi, di, pj, dj, bits=32)
        h1, f1 = orc.pair_force(pi + T, di, pj + T, dj, bits=32)
        assert h0 == h1 and np.array_equal(f0, f1)
        a = (pi + T).astype(np.float32) - (pj + T).astype(np.float32)
        changed_if_rounded_first += bool(np.any(a != (pi - pj).astype(np.float32)))
    assert changed_if_rounded_first > 250  # the misreading would differ on nearly every pair


def test_f32_terms_accumulate_in_binary64(orc):
    # agent 0 at the origin between agent 1 at x = +8 and agent 2 at x = -11.99 (all d = 12,
    # k = gamma = 1): its force is the binary64 sum of the two widened binary32 terms, and the
    # binary32 sum of the same terms is a different number
    s = dict(x=np.array([0.0, 8.0, -11.99]), y=np.zeros(3), z=np.zeros(3), d=np.full(3, 12.0),
             adh=np.full(3, 100.0))
    _, t1 = orc.pair_force((0.0, 0.0, 0.0), 12.0, (8.0, 0.0, 0.0), 12.0, k=1.0, gamma=1.0, bits=32)
    _, t2 = orc.pair_force((0.0, 0.0, 0.0), 12.0, (-11.99, 0.0, 0.0), 12.0, k=1.0, gamma=1.0, bits=32)
    fx, fy, fz, nc, fl = orc.mech_step(s, k=1.0, gamma=1.0, dt=0.01, force_bits=32)
    assert nc[0] == 2
    assert fx[0] == t1[0] + t2[0]
    assert fx[0] != float(np.float32(t1[0]) + np.float32(t2[0]))
    assert fy[0] == 0.0 and fz[0] == 0.0
    assert fl.tolist() == [1, 1, 1]  # adh 100 gates every agent: positions unchanged
    assert s["x"].tolist() == [0.0, 8.0, -11.99]


@pytest.mark.parametrize("sep", [8.0, 10.0, 11.0, 11.9])
def test_f32_and_f64_laws_agree_to_binary32_rounding(orc, sep):
    # the two laws are the same function; they differ by the rounding of about ten binary32
    # operations (each within 2^-24 relative), amplified at most by the cancellation in F
    _, f64 = orc.pair_force((0.0, 0.0, 0.0), 12.0, (sep, 0.0, 0.0), 12.0, bits=64)
    _, f32 = orc.pair_force((0.0, 0.0, 0.0), 12.0, (sep, 0.0, 0.0), 12.0, bits=32)
    delta = 12.0 - sep
    cancel = (2.0 * delta + math.sqrt(3.0 * delta)) / abs(2.0 * delta - math.sqrt(3.0 * delta))
    assert abs(f32[0] - f64[0]) <= 16 * 2.0 ** -24 * cancel * abs(f64[0])
