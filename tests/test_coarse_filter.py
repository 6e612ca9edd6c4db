"""The crowded kernel's coarse pre-test on the matrix cores, modelled in numpy from its
definition: for every pair that the binary32 pre-test (maybe_touch) keeps, the coarse value
must be negative, so the coarse filter in front of it drops nothing.

The model: coordinates relative to the wavefront's first agent o, a' = a - o and c' = c - o in
binary32; the agent vector (a'x, a'y, a'z, a.w, 1, A) and the candidate vector
(-2c'x, -2c'y, -2c'z, -2c.w, C, 1) with A = |a'|^2 - a.w^2 - slack - k (|a'|^2 + a.w^2 + slack)
and C = |c'|^2 - c.w^2 - k (|c'|^2 + c.w^2), k = 2^-14, each formed in binary32 as the kernel
forms it; the dot product is summed in binary32 two products at a time (each step one fused
multiply-add of the pair's second product onto the first product plus the running sum, the
rounding the device probe measured for one step), in the kernel's K order.  This is a model of
the definition, not the kernel's code; the GPU parity tests (among them a lattice whose axis
pairs sit within 1e-8 um of contact) check the kernel bit for bit.

Pairs sit at the edge of maybe_touch's own decision (found by bisection in binary32), at
lattice coordinates up to 600 um, in wavefronts spread over up to three boxes.  Without the
margin k the model drops some of them, so the test is not vacuous.
"""
import numpy as np

F = np.float32
K_MARGIN = F(2.0 ** -14)


def f32(x):
    return F(x)


def fma(a, b, c):
    # a * b is exact in binary64 for binary32 a, b; one rounding of the sum to binary32
    return F(np.float64(a) * np.float64(b) + np.float64(c))


def maybe_touch(a, c, slack):
    dx, dy, dz = f32(a[0] - c[0]), f32(a[1] - c[1]), f32(a[2] - c[2])
    d2 = fma(dz, dz, fma(dy, dy, f32(dx * dx)))
    s = f32(a[3] + c[3])
    return bool(d2 < fma(s, s, slack))


def agent_vec(a, o, slack, k):
    ax, ay, az, aw = f32(a[0] - o[0]), f32(a[1] - o[1]), f32(a[2] - o[2]), a[3]
    a2 = fma(az, az, fma(ay, ay, f32(ax * ax)))
    w2 = f32(aw * aw)
    A = f32(f32(f32(a2 - w2) - slack) - f32(k * f32(f32(a2 + w2) + slack)))
    return [ax, ay, az, aw, F(1.0), A]


def cand_vec(c, o, k):
    cx, cy, cz, cw = f32(c[0] - o[0]), f32(c[1] - o[1]), f32(c[2] - o[2]), c[3]
    c2 = fma(cz, cz, fma(cy, cy, f32(cx * cx)))
    w2 = f32(cw * cw)
    C = f32(f32(c2 - w2) - f32(k * f32(c2 + w2)))
    return [f32(-2.0 * cx), f32(-2.0 * cy), f32(-2.0 * cz), f32(-2.0 * cw), C, F(1.0)]


def coarse_value(av, cv):
    acc = F(0.0)
    for s in range(3):  # one instruction: the pair (2s, 2s + 1) added to the running sum
        acc = fma(cv[2 * s + 1], av[2 * s + 1], f32(f32(cv[2 * s] * av[2 * s]) + acc))
    return acc


def edge_pairs(rng, n, spread):
    """(agent, candidate, origin) triples at the edge of maybe_touch's decision."""
    out = []
    slack = F(1e-4)
    while len(out) < n:
        o = rng.uniform(0.0, 600.0, 3).astype(np.float64)
        a = np.array([*(o + rng.uniform(0.0, spread, 3)), rng.uniform(3.0, 7.0)], dtype=F)
        rc = F(rng.uniform(3.0, 7.0))
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        lo, hi = 0.0, 40.0  # bisection on the distance along v: lo touches, hi does not
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            c = np.array([*(a[:3].astype(np.float64) + mid * v), rc], dtype=F)
            if maybe_touch(a, c, slack):
                lo = mid
            else:
                hi = mid
        c = np.array([*(a[:3].astype(np.float64) + lo * v), rc], dtype=F)
        if maybe_touch(a, c, slack):
            out.append((a, c, np.array([F(o[0]), F(o[1]), F(o[2])]), slack))
    return out


def dropped(pairs, k):
    n = 0
    for a, c, o, slack in pairs:
        if coarse_value(agent_vec(a, o, slack, k), cand_vec(c, o, k)) >= 0.0:
            n += 1
    return n


def test_coarse_filter_keeps_every_maybe_touch_pair():
    rng = np.random.default_rng(3)
    pairs = edge_pairs(rng, 3000, 42.0)
    assert dropped(pairs, K_MARGIN) == 0
    # the margin is what keeps them: without it the binary32 roundings drop some
    assert dropped(pairs, F(0.0)) > 0
