"""GPU parity: the gfx950 path through the C ABI against the CPU oracle, on the same seeded
inputs.  Integer work (keys, order, start offsets, contact sets, SIR states, division ids and
counts) must be bit-exact.  Binary64 forces and positions must agree within
1e-9 * max(|x_ref|, L) (positions) and 1e-9 * sum_j |F_ij| (forces); the design aims at bit
equality, and the tests report how many agents are bit-equal.
"""
import math
import sys

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - the gpu marker deselects these on CPU
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2006_06775_amd import bdm  # noqa: E402
from oracle import oracle as orc  # noqa: E402

TOL = 1e-9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def population(arrays, capacity=None, max_boxes=1 << 22, spheres=True, state=False):
    n = len(arrays["x"])
    pop = bdm.Population(capacity or max(n, 1), max_boxes, spheres=spheres, with_state=state)
    pop.load(arrays)
    return pop


def mech_p(**kw):
    base = dict(k=2.0, gamma=1.0, dt=0.01, max_disp=3.0, box=0.0, force_bits=64)
    base.update(kw)
    return bdm.params(**base)


# ---------------------------------------------------------------------------------------------
def test_ieee_sqrt_div_bitwise():
    say("case: fp_probe")
    r = np.random.default_rng(0)
    a = np.concatenate([r.uniform(0, 1e3, 200000), r.uniform(0, 1e-3, 50000),
                        np.exp(r.uniform(-700, 700, 50000)), [0.0, 1.0, 2.0, 4.0, 1e-310, 5e-324]])
    b = np.concatenate([r.uniform(1e-3, 1e3, len(a) - 6), [1.0, 3.0, 7.0, 1e-300, 3.0, 2.0]])
    ta = torch.tensor(a, device="cuda")
    tb = torch.tensor(b, device="cuda")
    s, d, sf, df = (o.cpu().numpy() for o in bdm.fp_probe(ta, tb))
    assert np.array_equal(s.view(np.uint64), np.sqrt(a).view(np.uint64))
    assert np.array_equal(d.view(np.uint64), (a / b).view(np.uint64))
    with np.errstate(over="ignore"):
        fa, fb = a.astype(np.float32), b.astype(np.float32)
    ok = np.isfinite(fa) & np.isfinite(fb) & (fb != 0)
    assert np.array_equal(sf[ok].view(np.uint32), np.sqrt(fa[ok]).view(np.uint32))
    assert np.array_equal(df[ok].view(np.uint32), (fa[ok] / fb[ok]).view(np.uint32))


# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("kind,n", [("cube", 4096), ("cube", 4097), ("ball", 10000), ("sir", 5003),
                                    ("cube", 0), ("cube", 1)])
def test_generator_bit_exact(kind, n):
    say(f"case: generate {kind} n={n}")
    cap = max(n, 1)
    if kind == "cube":
        ref = orc.generate_cube(n, 7, 200.0, 10.0, 15.0, 0.4, salt=3)
        g = bdm.gen(bdm.GEN_CUBE, n, 200.0, 10.0, 15.0, 0.4, seed=7, salt=3)
        pop = bdm.Population(cap, 1 << 14)
    elif kind == "ball":
        h = 0.5 ** (1 / 3)
        ref = orc.generate_ball(n, 1, 60.0, 14.0 * h, 14.0, 0.4)
        g = bdm.gen(bdm.GEN_BALL, n, 60.0, 14.0 * h, 14.0, 0.4, seed=1)
        pop = bdm.Population(cap, 1 << 14)
    else:
        ref = orc.generate_sir(n, 5, 5000.0, 5)
        g = bdm.gen(bdm.GEN_SIR, n, 5000.0, 0.0, 0.0, 0.0, n_infected=5, seed=5)
        pop = bdm.Population(cap, 1 << 14, spheres=False, with_state=True)
    bdm.generate(pop.soa, g)
    assert pop.n == n
    got = pop.read()
    for k in ("x", "y", "z"):
        assert np.array_equal(got[k].view(np.uint64), ref[k].view(np.uint64)), k
    if kind != "sir":
        assert np.array_equal(got["diam"].view(np.uint64), ref["d"].view(np.uint64))
    else:
        assert np.array_equal(got["state"], ref["state"])


# ---------------------------------------------------------------------------------------------
def grid_cases():
    return {
        "c0": orc.generate_cube(4096, 0, 200.0, 10.0, 15.0, 0.4),
        "ragged": inputs.uniform_cube(5001, 230.0, seed=4),
        "faces": inputs.box_face_adversarial(3000, 12.0, seed=2),
        "clustered": inputs.clustered(4000, 300.0, seed=3),
        "negative": {k: (v - 500.0 if k in "xyz" else v) for k, v in inputs.uniform_cube(2000, 150.0, seed=5).items()},
        # far from the origin: lattice coordinates near 10^8 (the pre-test records keep the box
        # index mod 4 and the offset within the box)
        "far": {k: (v + 1.0e9 if k in "xyz" else v) for k, v in inputs.uniform_cube(2000, 150.0, seed=6).items()},
        "single": dict(x=np.array([3.0]), y=np.array([4.0]), z=np.array([5.0]), d=np.array([10.0]), adh=np.array([0.4])),
        "empty": dict(x=np.zeros(0), y=np.zeros(0), z=np.zeros(0), d=np.zeros(0), adh=np.zeros(0)),
        "reach": inputs.reach_adversarial(192, 12.0, seed=7),
        "crowded": inputs.uniform_cube(3000, 10.0, dmin=10.0, dmax=10.0, seed=11),
        "onebox": dict(x=np.full(300, 1.0) + np.arange(300) * 1e-3, y=np.ones(300), z=np.ones(300), d=np.full(300, 10.0), adh=np.full(300, 0.4)),
    }


@pytest.mark.parametrize("case", list(grid_cases().keys()))
def test_grid_lockstep_bit_exact(case):
    say(f"case: grid {case}")
    s = grid_cases()[case]
    n = len(s["x"])
    pop = population(s, capacity=max(n, 1))
    bdm.grid_build(pop.soa, mech_p(), pop.ws)
    info, key, order, start = bdm.grid_export(pop.ws)
    assert info["valid"] == 1 and info["flags"] == 0
    ref_info, rk, ro, rs = orc.grid(s["x"], s["y"], s["z"], s["d"])
    if n == 0:
        assert info["nboxes"] == 0 and start.tolist() == [0]
        return
    assert info["b"] == ref_info["b"]
    assert info["cmin"] == tuple(ref_info["cmin"]) and info["dims"] == tuple(ref_info["dims"])
    assert np.array_equal(key, rk)
    assert np.array_equal(order, ro)
    assert np.array_equal(start, rs)


def test_grid_rebuilds_on_the_last_lattice():
    """A plain build keys the agents on the last build's lattice while it reduces their bounds,
    and keys them again only when the bounds give another lattice (after clearing what it
    counted).  Every rebuild below must equal the oracle's grid of the same positions: the same
    lattice with agents moved between boxes, the extremes moved (a new origin and dims), a
    failed build in between (a non-finite coordinate), a changed box edge, and the periodic
    lattice twice."""
    say("case: grid rebuilds on the last lattice")
    s = inputs.uniform_cube(5001, 230.0, seed=21)
    n = len(s["x"])
    pop = population(s, capacity=n, max_boxes=1 << 16)

    def check(arr, p, **kw):
        for k in "xyz":
            pop.t[k][:n].copy_(torch.as_tensor(arr[k]))
        bdm.grid_build(pop.soa, p, pop.ws)
        info, key, order, start = bdm.grid_export(pop.ws)
        assert info["valid"] == 1 and info["flags"] == 0
        ref_info, rk, ro, rs = orc.grid(arr["x"], arr["y"], arr["z"], arr["d"], **kw)
        assert info["b"] == ref_info["b"]
        assert info["cmin"] == tuple(ref_info["cmin"]) and info["dims"] == tuple(ref_info["dims"])
        assert np.array_equal(key, rk) and np.array_equal(order, ro) and np.array_equal(start, rs)
        return info

    pop.t["n"].fill_(0)                             # a last lattice without boxes
    bdm.grid_build(pop.soa, mech_p(), pop.ws)
    assert bdm.grid_info(pop.ws)["valid"] == 1 and bdm.grid_info(pop.ws)["nboxes"] == 0
    pop.t["n"].fill_(n)
    first = check(s, mech_p())                      # nothing counted: keyed once, after the bounds
    again = check(s, mech_p())                      # the same positions on the last lattice
    assert again["cmin"] == first["cmin"] and again["dims"] == first["dims"]
    # agents exchange places (the bounds and so the lattice stay): keys on the last lattice stand
    rng = np.random.default_rng(5)
    perm = rng.permutation(n)
    moved = {k: (v[perm] if k in "xyz" else v) for k, v in s.items()}
    assert check(moved, mech_p())["dims"] == first["dims"]
    # one agent leaves the lattice by five boxes: new dims, the counted histogram is cleared
    far = {k: v.copy() for k, v in moved.items()}
    far["x"][17] = far["x"].max() + 5.0 * first["b"]
    assert check(far, mech_p())["dims"] != first["dims"]
    # the lowest agent moves up into the lattice: a new origin
    up = {k: v.copy() for k, v in far.items()}
    low = int(np.argmin(up["z"]))
    up["z"][low] = up["z"].max()
    check(up, mech_p())
    # a build that fails after counting on the last lattice, then a good one
    bad = {k: v.copy() for k, v in up.items()}
    bad["y"][300] = np.nan
    for k in "xyz":
        pop.t[k][:n].copy_(torch.as_tensor(bad[k]))
    bdm.grid_build(pop.soa, mech_p(), pop.ws)
    assert bdm.status(pop.ws, clear=True) & bdm.FLAG_NONFINITE
    assert bdm.grid_info(pop.ws)["valid"] == 0
    check(up, mech_p())
    check(up, mech_p())
    # an explicit box edge (another lattice), then the largest diameter again
    check(up, mech_p(box=20.0), box=20.0)
    check(up, mech_p(box=20.0), box=20.0)
    check(up, mech_p())
    # the periodic lattice, built twice
    sp = inputs.sir_uniform(20000, 100.0, seed=2)
    per = population(sp, spheres=False, state=True, max_boxes=30 ** 3)
    p = bdm.params(box=4.0, periodic=1, L=100.0)
    ref_info, rk, ro, rs = orc.grid(sp["x"], sp["y"], sp["z"], None, box=4.0, periodic=True, L=100.0)
    for _ in range(2):
        bdm.grid_build(per.soa, p, per.ws)
        info, key, order, start = bdm.grid_export(per.ws)
        assert info["valid"] == 1 and info["dims"] == (25, 25, 25)
        assert np.array_equal(key, rk) and np.array_equal(order, ro) and np.array_equal(start, rs)


def test_grid_periodic_bit_exact():
    say("case: grid periodic")
    s = inputs.sir_uniform(20000, 100.0, seed=1)
    pop = population(s, spheres=False, state=True, max_boxes=30 ** 3)
    p = bdm.params(box=4.0, periodic=1, L=100.0)
    bdm.grid_build(pop.soa, p, pop.ws)
    info, key, order, start = bdm.grid_export(pop.ws)
    ref_info, rk, ro, rs = orc.grid(s["x"], s["y"], s["z"], None, box=4.0, periodic=True, L=100.0)
    assert info["dims"] == (25, 25, 25)
    assert np.array_equal(key, rk) and np.array_equal(order, ro) and np.array_equal(start, rs)


def test_grid_explicit_box_and_flags():
    say("case: grid flags")
    s = inputs.uniform_cube(1000, 100.0, seed=9)
    pop = population(s, max_boxes=1 << 16)
    bdm.grid_build(pop.soa, mech_p(box=20.0), pop.ws)
    info, key, order, start = bdm.grid_export(pop.ws)
    _, rk, ro, rs = orc.grid(s["x"], s["y"], s["z"], s["d"], box=20.0)
    assert np.array_equal(key, rk) and np.array_equal(order, ro) and np.array_equal(start, rs)
    # box below the largest diameter: flagged, grid invalid, a following step moves nothing
    bdm.grid_build(pop.soa, mech_p(box=5.0), pop.ws)
    assert bdm.status(pop.ws, clear=True) & bdm.FLAG_BOXSMALL
    assert bdm.grid_info(pop.ws)["valid"] == 0
    x0 = pop.t["x"][:1000].clone()
    bdm.mech_step(pop.soa, mech_p(box=5.0), pop.ws)
    assert torch.equal(pop.t["x"][:1000], x0)
    assert bdm.status(pop.ws, clear=True) == bdm.FLAG_NOGRID  # the step reports the missing grid
    # a mechanical step on a workspace that never held a grid moves nothing and says so
    fresh = population(s, max_boxes=1 << 16)
    bdm.mech_step(fresh.soa, mech_p(), fresh.ws)
    assert torch.equal(fresh.t["x"][:1000], torch.as_tensor(s["x"], device="cuda"))
    assert bdm.status(fresh.ws) == bdm.FLAG_NOGRID
    # too many boxes for the workspace
    small = population(s, max_boxes=10)
    bdm.grid_build(small.soa, mech_p(), small.ws)
    assert bdm.status(small.ws) & bdm.FLAG_BOXES
    # non-finite input
    s2 = {k: v.copy() for k, v in s.items()}
    s2["y"][17] = np.inf
    bad = population(s2)
    bdm.grid_build(bad.soa, mech_p(), bad.ws)
    assert bdm.status(bad.ws) & bdm.FLAG_NONFINITE


def test_grid_lattice_span_beyond_int32():
    """Two agents 2^31 boxes apart along x (lattice coordinates -2^30 and 2^30 - 1, both inside
    the device's coordinate range): the span does not fit int32 and far exceeds max_boxes, so
    the build must fail with BDM_FLAG_BOXES and leave no valid grid, as the oracle refuses it."""
    say("case: grid lattice span 2^31")
    b = 10.0
    s = dict(x=np.array([-(2.0 ** 30) * b + 5.0, (2.0 ** 30 - 1.0) * b + 5.0]), y=np.array([5.0, 5.0]),
             z=np.array([5.0, 5.0]), d=np.array([b, b]), adh=np.array([0.4, 0.4]))
    with pytest.raises(orc.OracleError) as e:
        orc.grid(s["x"], s["y"], s["z"], s["d"], max_boxes=1 << 16)
    assert e.value.rc == orc.ETOOMANYBOXES
    pop = population(s, max_boxes=1 << 16)
    bdm.grid_build(pop.soa, mech_p(), pop.ws)
    assert bdm.status(pop.ws) & bdm.FLAG_BOXES
    info = bdm.grid_info(pop.ws)
    assert info["valid"] == 0 and info["n"] == 0


def test_mech_step_refuses_a_foreign_or_used_grid():
    """A mechanical step needs an open-space build of the same agents that no step has used:
    after a periodic (SIR) build, or a second time after one build, it moves nothing and sets
    BDM_FLAG_NOGRID."""
    say("case: mech step after a periodic build / twice on one build")
    s = inputs.uniform_cube(1000, 100.0, seed=9)
    pop = population(s, state=True, max_boxes=1 << 16)
    bdm.grid_build(pop.soa, bdm.params(box=20.0, periodic=1, L=100.0), pop.ws)
    x0 = pop.t["x"][:1000].clone()
    bdm.mech_step(pop.soa, mech_p(), pop.ws)
    assert torch.equal(pop.t["x"][:1000], x0)
    assert bdm.status(pop.ws, clear=True) == bdm.FLAG_NOGRID
    bdm.grid_build(pop.soa, mech_p(), pop.ws)
    bdm.mech_step(pop.soa, mech_p(), pop.ws)
    assert bdm.status(pop.ws, clear=True) == 0
    x1 = pop.t["x"][:1000].clone()
    bdm.mech_step(pop.soa, mech_p(), pop.ws)
    assert torch.equal(pop.t["x"][:1000], x1)
    assert bdm.status(pop.ws, clear=True) == bdm.FLAG_NOGRID
    bdm.sim_step(pop.soa, bdm.MODEL_MECH, mech_p(), 0, pop.ws)  # a build and a step: fine again
    assert bdm.status(pop.ws) == 0


def test_argument_validation():
    say("case: validation")
    pop = population(inputs.uniform_cube(100, 50.0, seed=1))
    for kw in (dict(dt=0.0), dict(max_disp=-1.0), dict(force_bits=16), dict(periodic=1)):
        with pytest.raises(bdm.BdmError) as e:
            bdm.mech_step(pop.soa, mech_p(**kw), pop.ws)
        assert e.value.rc == bdm.EINVAL
    ws = bdm.Workspace(pop.ws.ptr, 100, pop.ws.capacity, pop.ws.max_boxes)
    with pytest.raises(bdm.BdmError) as e:
        bdm.grid_build(pop.soa, mech_p(), ws)
    assert e.value.rc == bdm.ENOWS


# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("case,bits", [("c0", 64), ("c0", 32), ("faces", 64), ("clustered", 64),
                                       ("clustered", 32), ("reach", 64), ("reach", 32)])
def test_contacts_bit_exact(case, bits):
    say(f"case: contacts {case} bits={bits}")
    s = grid_cases()[case]
    n = len(s["x"])
    pop = population(s)
    bdm.grid_build(pop.soa, mech_p(), pop.ws)
    counts, offsets, ids = bdm.contacts(pop.ws, mech_p(force_bits=bits), n)
    _, _, order, _ = bdm.grid_export(pop.ws)
    rc, ro, ri = orc.contacts(s["x"], s["y"], s["z"], s["d"], force_bits=bits)
    for slot in range(n):
        a = order[slot]
        got = ids[offsets[slot]: offsets[slot] + counts[slot]]
        exp = ri[ro[a]: ro[a] + rc[a]]
        assert np.array_equal(got, exp), (slot, a)


def test_sir_contacts_bit_exact():
    say("case: sir contacts")
    s = inputs.sir_uniform(20000, 100.0, seed=2)
    pop = population(s, spheres=False, state=True, max_boxes=40 ** 3)
    p = bdm.params(box=4.0, periodic=1, L=100.0, r_inf=3.0)
    bdm.grid_build(pop.soa, p, pop.ws)
    counts, offsets, ids = bdm.contacts(pop.ws, p, 20000)
    _, _, order, _ = bdm.grid_export(pop.ws)
    rc, ro, ri = orc.contacts(s["x"], s["y"], s["z"], None, box=4.0, periodic=True, L=100.0,
                              radius=3.0)
    for slot in range(20000):
        a = order[slot]
        assert sorted(ids[offsets[slot]: offsets[slot] + counts[slot]].tolist()) == \
            sorted(ri[ro[a]: ro[a] + rc[a]].tolist())


# ---------------------------------------------------------------------------------------------
def pair_abs_sum(s, force_bits=64):
    """sum_j |F_ij| per agent over the oracle's contact lists, for the force tolerance.  Only a
    scale: the magnitudes are evaluated in numpy (binary64, k = 2, gamma = 1), all pairs at once,
    since a population of a few thousand agents in one box has millions of contacts."""
    counts, offsets, ids = orc.contacts(s["x"], s["y"], s["z"], s["d"], force_bits=force_bits)
    n = len(s["x"])
    counts = np.asarray(counts, dtype=np.int64)
    total = int(counts.sum())
    if total == 0:
        return np.zeros(n)
    owner = np.repeat(np.arange(n), counts)
    first = np.repeat(np.asarray(offsets, dtype=np.int64), counts)
    within = np.arange(total) - np.repeat(np.cumsum(counts) - counts, counts)
    j = np.asarray(ids, dtype=np.int64)[first + within]
    x, y, z, r = (np.asarray(s[k], dtype=np.float64) for k in ("x", "y", "z", "d"))
    r = 0.5 * r
    dist = np.sqrt((x[owner] - x[j]) ** 2 + (y[owner] - y[j]) ** 2 + (z[owner] - z[j]) ** 2)
    delta = np.maximum(r[owner] + r[j] - dist, 0.0)
    rhat = r[owner] * r[j] / (r[owner] + r[j])
    f = np.abs(2.0 * delta - np.sqrt(rhat * delta))
    return np.bincount(owner, weights=f, minlength=n)


def compare_state(got, ref, L, what, fabs=None, fref=None):
    n = len(ref["x"])
    scale = L
    if n:
        scale = max(L, float(np.max(np.abs(np.concatenate([ref["x"], ref["y"], ref["z"]])))))
    bit = np.ones(n, dtype=bool)
    for k in ("x", "y", "z"):
        err = np.abs(got[k] - ref[k])
        assert np.all(err <= TOL * scale), (what, k, float(err.max()))
        bit &= got[k].view(np.uint64) == ref[k].view(np.uint64)
    if fref is not None:
        for k, rk in zip(("fx", "fy", "fz"), fref):
            err = np.abs(got[k] - rk)
            assert np.all(err <= TOL * np.maximum(fabs, 1e-300)), (what, k, float(err.max()))
            bit &= got[k].view(np.uint64) == rk.view(np.uint64)
    say(f"{what}: {int(bit.sum())}/{n} agents bit-equal")
    return bit


@pytest.mark.parametrize("case,bits", [("c0", 64), ("ragged", 64), ("clustered", 64), ("faces", 64),
                                       ("reach", 64), ("c0", 32), ("clustered", 32), ("reach", 32),
                                       ("crowded", 64), ("single", 64), ("empty", 64), ("far", 64),
                                       ("far", 32), ("negative", 64)])
def test_mech_step_lockstep(case, bits):
    say(f"case: mech lockstep {case} bits={bits}")
    s = grid_cases()[case]
    n = len(s["x"])
    pop = population(s)
    p = mech_p(force_bits=bits)
    bdm.grid_build(pop.soa, p, pop.ws)
    bdm.mech_step(pop.soa, p, pop.ws)
    assert bdm.status(pop.ws) == 0
    got = pop.read()
    ref = {k: v.copy() for k, v in s.items()}
    fx, fy, fz, nc, fl = orc.mech_step(ref, force_bits=bits)
    fabs = pair_abs_sum(s, bits) if n else np.zeros(0)
    bit = compare_state(got, ref, 200.0, f"mech {case}/{bits}", fabs, (fx, fy, fz))
    assert bit.all(), "expected bit equality with the oracle (same operations, same order)"


@pytest.mark.parametrize("case,bits", [("c0", 64), ("clustered", 64), ("crowded", 64), ("onebox", 64),
                                       ("crowded8", 64), ("crowded8", 32), ("crowded", 32), ("ragged", 32)])
def test_crowded_kernel_lockstep(case, bits):
    """The spheroid model's mechanics kernel (longer queue; wavefronts whose lanes share their
    boxes walk the union of their runs together) with growth 1 and no division is one plain
    mechanical step, so it must equal the oracle's bit for bit.  `crowded8`: about 150 agents
    in each of 8 boxes, so wavefronts straddle boxes and rows end in ragged chunks."""
    say(f"case: crowded-kernel lockstep {case} bits={bits}")
    if case == "crowded8":
        s = inputs.uniform_cube(1237, 20.0, dmin=10.0, dmax=10.0, seed=12)
    else:
        s = grid_cases()[case]
    pop = population(s)
    p = mech_p(force_bits=bits, grow=1.0, div_d=1e300, half_cbrt=0.5 ** (1 / 3), seed=3)
    bdm.sim_step(pop.soa, bdm.MODEL_SPHEROID, p, 0, pop.ws)
    assert bdm.status(pop.ws) == 0
    assert pop.n == len(s["x"])
    got = pop.read()
    ref = {k: v.copy() for k, v in s.items()}
    fx, fy, fz, nc, fl = orc.mech_step(ref, force_bits=bits)
    bit = compare_state(got, ref, 200.0, f"crowded kernel {case}/{bits}", pair_abs_sum(s, bits), (fx, fy, fz))
    assert bit.all(), "expected bit equality with the oracle (same operations, same order)"


@pytest.mark.parametrize("bits", [64, 32])
def test_mech_step_past_4gib_records(bits):
    """A workspace whose packed records pass 4 GiB (capacity above 2^27) switches the mechanics
    kernel from range-checked 32-bit buffer offsets to plain global loads; a small population in
    it must still step bit for bit like the oracle."""
    say(f"case: mech lockstep, capacity 2^27 + 256, bits={bits}")
    s = grid_cases()["ragged"]
    pop = population(s, capacity=(1 << 27) + 256, max_boxes=1 << 16)
    p = mech_p(force_bits=bits)
    bdm.grid_build(pop.soa, p, pop.ws)
    bdm.mech_step(pop.soa, p, pop.ws)
    assert bdm.status(pop.ws) == 0
    got = pop.read()
    ref = {k: v.copy() for k, v in s.items()}
    fx, fy, fz, nc, fl = orc.mech_step(ref, force_bits=bits)
    bit = compare_state(got, ref, 230.0, f"mech 2^27 capacity/{bits}", pair_abs_sum(s, bits), (fx, fy, fz))
    assert bit.all()
    del pop
    torch.cuda.empty_cache()


@pytest.mark.parametrize("bits", [64, 32])
def test_mech_step_explicit_box(bits):
    """An explicit box edge of three times the largest diameter: spheres are small against the
    box, so the pre-test records hold radii of a few hundred units and many boxes per reach."""
    say(f"case: mech lockstep, explicit box 45, bits={bits}")
    s = grid_cases()["c0"]
    pop = population(s)
    p = mech_p(force_bits=bits, box=45.0)
    bdm.grid_build(pop.soa, p, pop.ws)
    bdm.mech_step(pop.soa, p, pop.ws)
    assert bdm.status(pop.ws) == 0
    got = pop.read()
    ref = {k: v.copy() for k, v in s.items()}
    fx, fy, fz, nc, fl = orc.mech_step(ref, box=45.0, force_bits=bits)
    bit = compare_state(got, ref, 200.0, f"mech box 45/{bits}", pair_abs_sum(s, bits), (fx, fy, fz))
    assert bit.all()


def test_mech_clamp_and_gate_regimes():
    say("case: mech clamp/gate")
    s = inputs.uniform_cube(3000, 200.0, seed=21)  # with dt 0.5 all three regimes occur
    pop = population(s)
    p = mech_p(dt=0.5, max_disp=0.7)
    bdm.grid_build(pop.soa, p, pop.ws)
    bdm.mech_step(pop.soa, p, pop.ws)
    got = pop.read()
    ref = {k: v.copy() for k, v in s.items()}
    fx, fy, fz, nc, fl = orc.mech_step(ref, dt=0.5, max_disp=0.7)
    assert (fl == 2).sum() > 100 and (fl == 1).sum() > 100 and (fl == 0).sum() > 100
    bit = compare_state(got, ref, 200.0, "clamp/gate", pair_abs_sum(s), (fx, fy, fz))
    assert bit.all()


def test_c0_ten_steps_fp64():
    """4096 agents in a 200 um cube, d in [10, 15), adh 0.4, k 2, gamma 1, dt 0.01, 10 steps."""
    say("case: C0 trajectory")
    n = 4096
    pop = bdm.Population(n, 1 << 14)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, 200.0, 10.0, 15.0, 0.4, seed=0))
    ref = orc.generate_cube(n, 0, 200.0, 10.0, 15.0, 0.4)
    p = mech_p()
    for step in range(10):
        bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
        fx, fy, fz, nc, fl = orc.mech_step(ref)
    assert bdm.status(pop.ws) == 0
    got = pop.read()
    bit = compare_state(got, ref, 200.0, "C0 10 steps")
    assert bit.all()


def test_fp32_force_error_report():
    say("case: FP32 vs FP64 oracle")
    n = 4096
    pop = bdm.Population(n, 1 << 14)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, 200.0, 10.0, 15.0, 0.4, seed=0))
    ref64 = orc.generate_cube(n, 0, 200.0, 10.0, 15.0, 0.4)
    ref32 = {k: v.copy() for k, v in ref64.items()}
    p = mech_p(force_bits=32)
    for step in range(10):
        bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
        orc.mech_step(ref64)
        orc.mech_step(ref32, force_bits=32)
    got = pop.read()
    compare_state(got, ref32, 200.0, "FP32 path vs FP32 oracle")
    err = max(float(np.abs(got[k] - ref64[k]).max()) for k in ("x", "y", "z"))
    say(f"FP32-force max position error vs FP64 oracle after 10 steps: {err:.3e} um "
        f"({err / 200.0:.3e} of L)")
    assert err < 1e-3


# ---------------------------------------------------------------------------------------------
def test_sir_states_bit_exact():
    say("case: SIR dense")
    n, L = 200000, 200.0  # about 4 contacts per agent at radius 2
    pop = bdm.Population(n, 110 ** 3, spheres=False, with_state=True)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_SIR, n, L, n_infected=n // 100, seed=3))
    ref = orc.generate_sir(n, 3, L, n // 100)
    p = bdm.params(box=2.0, periodic=1, L=L, r_inf=2.0, p_inf=0.3, p_rec=0.01, walk=1.0, seed=3)
    op = orc.sir_params(L, 2.0, 2.0, 0.3, 0.01, 1.0, 3)
    for step in range(12):
        bdm.sim_step(pop.soa, bdm.MODEL_SIR, p, step, pop.ws)
        rc = orc.sir_step(ref, op, step)
        assert bdm.sir_counts(pop.ws) == rc.tolist(), step
    got = pop.read()
    assert np.array_equal(got["state"], ref["state"])
    for k in ("x", "y", "z"):
        assert np.array_equal(got[k].view(np.uint64), ref[k].view(np.uint64))
    assert bdm.status(pop.ws) == 0


def test_spheroid_growth_division():
    say("case: spheroid")
    n0, cap = 1000, 40000
    h = 0.5 ** (1 / 3)
    g = 1.05 ** (1 / 3)
    pop = bdm.Population(cap, 1 << 18)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_BALL, n0, 28.0, 14.0 * h, 14.0, 0.4, seed=2))
    st = orc.SpheroidState(orc.generate_ball(n0, 2, 28.0, 14.0 * h, 14.0, 0.4), cap)
    p = bdm.params(grow=g, div_d=14.0, half_cbrt=h, seed=2)
    op = orc.spheroid_params(g, 14.0, h, 2)
    for step in range(25):
        bdm.sim_step(pop.soa, bdm.MODEL_SPHEROID, p, step, pop.ws)
        st.step(op, step)
        assert pop.n == int(st.n[0]), step
    got = pop.read()
    ref = {k: st.view(k) for k in ("x", "y", "z", "d")}
    assert np.array_equal(got["diam"].view(np.uint64), ref["d"].view(np.uint64))
    bit = compare_state(got, ref, 100.0, "spheroid 25 steps")
    assert bit.all()
    assert bdm.status(pop.ws) == 0


def test_spheroid_capacity_overflow():
    say("case: spheroid overflow")
    n = 64
    s = dict(x=np.arange(n) * 30.0, y=np.zeros(n), z=np.zeros(n), d=np.full(n, 13.99),
             adh=np.full(n, 0.4))
    pop = population(s, capacity=80)
    p = bdm.params(grow=1.05 ** (1 / 3), div_d=14.0, half_cbrt=0.5 ** (1 / 3), seed=1)
    bdm.sim_step(pop.soa, bdm.MODEL_SPHEROID, p, 0, pop.ws)
    assert pop.n == 80
    assert bdm.status(pop.ws) & bdm.FLAG_CAPACITY
    st = orc.SpheroidState(s, 80)
    st.step(orc.spheroid_params(1.05 ** (1 / 3), 14.0, 0.5 ** (1 / 3), 1), 0)
    got = pop.read()
    assert np.array_equal(got["diam"], st.view("d"))
