"""The cylinder walk's filter, modelled in numpy from its definition and checked against the
oracle's contact decision: every pair of bodies (sphere or cylinder) that the oracle's pair law
counts as a contact must pass the midpoint-sphere test, so the filter in front of the
closest-point law drops no contact.

The filter record of a body: the sphere about its midpoint that holds it (a cylinder's midpoint
(p + q) / 2 and radius |q - p| / 2 + d_c / 2; a sphere's centre and radius), in binary32 relative
to the lattice origin o = cmin * b, the radius scaled by 1.0006; the test compares the binary32
squared distance with (R_i + R_j)^2 + slack, the slack of the binary32 pre-test for a lattice of
edge b and its largest dims.  This is a model of the definition, not the kernel's code; the GPU
parity tests check the kernel bit for bit.

Pairs are moved to the edge of contact by bisection on the oracle's own decision (the last
position where it still reports a contact), with the bodies up to 2^20 um from the origin.  A
control set moved 1 % past the midpoint spheres' reach must fail the test.
"""
import math

import numpy as np

from oracle import oracle as orc

F32 = np.float32


def pretest_slack(b, dims, cmin):
    dm = max(dims)
    omax = max(abs(c * b) for c in cmin)
    M = (dm + 1.0) * b + 2.0 ** -48 * omax
    e = 2.0 ** -22 * (M + b)
    return float(F32(4.0 * (b + e) * e) * F32(1.001))


def body_sphere(kind, x, d, p, dc):
    """Midpoint and radius of the sphere holding the body (binary64)."""
    if kind == 1:
        m = 0.5 * (np.asarray(p) + np.asarray(x))
        return m, 0.5 * math.sqrt(float(np.dot(np.asarray(x) - p, np.asarray(x) - p))) + 0.5 * dc
    return np.asarray(x, dtype=np.float64), 0.5 * d


def record(m, rad, origin):
    return np.array([F32(m[0] - origin[0]), F32(m[1] - origin[1]), F32(m[2] - origin[2]),
                     F32(rad * 1.0006)], dtype=F32)


def fma32(a, b, c):
    # a * b is exact in binary64 for binary32 a, b; one rounding of the sum to binary32
    return F32(np.float64(a) * np.float64(b) + np.float64(c))


def passes(ri, rj, slack):
    dx, dy, dz = F32(ri[0] - rj[0]), F32(ri[1] - rj[1]), F32(ri[2] - rj[2])
    d2 = fma32(dz, dz, fma32(dy, dy, F32(dx * dx)))
    s = F32(ri[3] + rj[3])
    return bool(d2 < fma32(s, s, F32(slack)))


def random_body(rng, base):
    if rng.random() < 0.3:
        return dict(kind=0, x=base + rng.uniform(-1, 1, 3), d=float(rng.uniform(2.0, 15.0)), p=np.zeros(3), dc=0.0)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    length = float(rng.choice([0.0, rng.uniform(0.5, 25.0)]))
    q = base + rng.uniform(-1, 1, 3)
    dc = float(rng.uniform(0.5, 3.0))
    return dict(kind=1, x=q, d=2.0 * length + dc, p=q - length * u, dc=dc)


def shifted(b, v):
    out = dict(b)
    out["x"] = b["x"] + v
    out["p"] = b["p"] + v
    return out


def hit(bi, bj):
    return orc.geom_pair(bi["kind"], bi["x"], bi["d"], bi["p"], bi["dc"],
                         bj["kind"], bj["x"], bj["d"], bj["p"], bj["dc"])[0]


def test_midpoint_filter_keeps_every_contact():
    rng = np.random.default_rng(11)
    kept = fails = 0
    for trial in range(300):
        base = np.full(3, float(rng.choice([0.0, 1000.0, 2.0 ** 20])))
        bi = random_body(rng, base)
        bj = random_body(rng, base)
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        if not hit(bi, bj):  # start from a contact: move j onto i's midpoint
            mi, _ = body_sphere(bi["kind"], bi["x"], bi["d"], bi["p"], bi["dc"])
            mj, _ = body_sphere(bj["kind"], bj["x"], bj["d"], bj["p"], bj["dc"])
            bj = shifted(bj, mi - mj)
            if not hit(bi, bj):
                continue
        # bisection on the oracle's decision along v: lo keeps a contact, hi does not
        lo, hi = 0.0, 100.0
        assert not hit(bi, shifted(bj, hi * v))
        for _ in range(70):
            mid = 0.5 * (lo + hi)
            if hit(bi, shifted(bj, mid * v)):
                lo = mid
            else:
                hi = mid
        edge = shifted(bj, lo * v)
        assert hit(bi, edge)
        mi, ri = body_sphere(bi["kind"], bi["x"], bi["d"], bi["p"], bi["dc"])
        mj, rj = body_sphere(edge["kind"], edge["x"], edge["d"], edge["p"], edge["dc"])
        # the lattice of the pair: box edge the larger grid diameter (the kernel's is the largest)
        b = max(bi["d"], edge["d"])
        pts = np.array([bi["x"], edge["x"]])
        cmin = [int(math.floor(c / b)) for c in pts.min(axis=0)]
        cmax = [int(math.floor(c / b)) for c in pts.max(axis=0)]
        dims = [hi_ - lo_ + 1 for lo_, hi_ in zip(cmin, cmax)]
        origin = [c * b for c in cmin]
        slack = pretest_slack(b, dims, cmin)
        assert ri + rj <= b * (1.0 + 1e-12)  # the slack assumes it
        if not passes(record(mi, ri, origin), record(mj, rj, origin), slack):
            fails += 1
        kept += 1
        # control: 1 % past the midpoint spheres' reach fails
        far = mj + (mj - mi) / max(np.linalg.norm(mj - mi), 1e-30) * (1.01 * (ri + rj) - np.linalg.norm(mj - mi))
        assert not passes(record(mi, ri, origin), record(far, rj, origin), slack)
    assert kept >= 250
    assert fails == 0
