"""GPU: the contact decisions of the mechanics kernels themselves, checked against the oracle.

The traced entry points run the same kernels as the step (separate instantiations of the same
code: box culling, the 8-byte or binary32 pre-test, the cooperative walk, the queued and packed
exact passes) and record, per agent, how many contacts the step added and an order-sensitive
hash of their box-sorted positions.  The oracle's contact lists (candidates of the 27 boxes in
ascending (key, id), contact iff delta > 0 under the same pair law) give the expected values.
This catches a dropped or extra contact whose term is exactly zero (pairs at the equilibrium
overlap delta = gamma^2 rhat / k^2, coincident centres), which force sums cannot show.
"""
import sys

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2006_06775_amd import bdm  # noqa: E402
from oracle import oracle as orc  # noqa: E402

MUL = 0x9E3779B1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def expected(s, order, bits, box=0.0):
    """(counts, hashes) per box-sorted slot from the oracle's contact lists."""
    n = len(order)
    rc, ro, ri = orc.contacts(s["x"], s["y"], s["z"], s["d"], box=box, force_bits=bits)
    pos = np.empty(n, dtype=np.uint64)
    pos[order] = np.arange(n, dtype=np.uint64)
    cnt = np.asarray(rc, dtype=np.int64)[order]
    off = np.asarray(ro, dtype=np.int64)[order]
    ids = np.asarray(ri, dtype=np.int64)
    h = np.zeros(n, dtype=np.uint64)
    for k in range(int(cnt.max()) if n else 0):
        m = cnt > k
        h[m] = (h[m] * np.uint64(MUL) + pos[ids[off[m] + k]] + np.uint64(1)) & np.uint64(0xFFFFFFFF)
    return cnt.astype(np.uint32), h.astype(np.uint32)


def u32(t, n):
    return t[:n].cpu().numpy().view(np.uint32)


def equilibrium_case(seed=0):
    # d = 12 (rhat = 3), k = 2, gamma = 1: F = 0 exactly at delta* = gamma^2 rhat / k^2 = 0.75
    # (separation 11.25), so a dropped contact there leaves every force unchanged
    rhat, k, gamma = 3.0, 2.0, 1.0
    sep = 12.0 - gamma * gamma * rhat / (k * k)
    assert sep == 11.25
    s = inputs.separated_pairs(400, 12.0, sep, coincident=40, seed=seed)
    for bits in (64, 32):
        hit, f = orc.pair_force((0.0, 0.0, 0.0), 12.0, (sep, 0.0, 0.0), 12.0, k=k, gamma=gamma, bits=bits)
        assert hit and f[0] == 0.0 and f[1] == 0.0 and f[2] == 0.0
    return s


def cases():
    c = {
        "c0": orc.generate_cube(4096, 0, 200.0, 10.0, 15.0, 0.4),
        "ragged": inputs.uniform_cube(5001, 230.0, seed=4),
        "faces": inputs.box_face_adversarial(3000, 12.0, seed=2),
        "clustered": inputs.clustered(4000, 300.0, seed=3),
        "reach": inputs.reach_adversarial(192, 12.0, seed=7),
        "far": {k: (v + 1.0e9 if k in "xyz" else v) for k, v in inputs.uniform_cube(2000, 150.0, seed=6).items()},
        "crowded8": inputs.uniform_cube(1237, 20.0, dmin=10.0, dmax=10.0, seed=12),
        "equilibrium": equilibrium_case(),
        "touching": inputs.touching_lattice(seed=5),
    }
    return c


def traced_step(s, bits, model):
    n = len(s["x"])
    pop = bdm.Population(max(n, 1), 1 << 22)
    pop.load(s)
    counts = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    hashes = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    p = bdm.params(force_bits=bits, grow=1.0, div_d=1e300, seed=3)
    bdm.sim_step_traced(pop.soa, model, p, 0, pop.ws, counts, hashes)
    assert bdm.status(pop.ws) == 0
    _, _, order, _ = bdm.grid_export(pop.ws)
    return u32(counts, n), u32(hashes, n), order


@pytest.mark.parametrize("case,bits,model", [
    ("c0", 64, "mech"), ("c0", 32, "mech"), ("ragged", 64, "mech"), ("faces", 64, "mech"),
    ("clustered", 64, "mech"), ("clustered", 32, "mech"), ("reach", 64, "mech"), ("reach", 32, "mech"),
    ("far", 64, "mech"), ("equilibrium", 64, "mech"), ("equilibrium", 32, "mech"),
    ("c0", 64, "crowded"), ("clustered", 32, "crowded"), ("crowded8", 64, "crowded"),
    ("crowded8", 32, "crowded"), ("equilibrium", 64, "crowded"), ("touching", 64, "crowded"),
    ("touching", 32, "crowded"), ("touching", 64, "mech")])
def test_traced_contacts_match_oracle(case, bits, model):
    """Every contact the kernel adds, in its order, is the oracle's, for the plain kernel and
    for the spheroid model's crowded kernel (growth 1, no division: one mechanical step)."""
    say(f"case: traced contacts {case} bits={bits} kernel={model}")
    s = cases()[case]
    m = bdm.MODEL_MECH if model == "mech" else bdm.MODEL_SPHEROID
    counts, hashes, order = traced_step(s, bits, m)
    ec, eh = expected(s, order, bits)
    bad = np.nonzero((counts != ec) | (hashes != eh))[0]
    say(f"{len(order)} agents, {int(ec.sum())} contacts, {len(bad)} differ")
    assert len(bad) == 0, (bad[:10], counts[bad[:10]], ec[bad[:10]])
    if case == "equilibrium":
        assert ec.sum() >= 2 * 400 + 2 * 40  # every pair (both sides) is a contact
    if case == "touching":  # pairs within 1e-6 of touching, on both sides of it
        dd = np.sqrt(sum((s[k][:, None] - s[k][None, :]) ** 2 for k in "xyz"))
        assert ((dd < 10.0) & (dd > 10.0 - 1e-6)).sum() >= 100 and ((dd >= 10.0) & (dd < 10.0 + 1e-6)).sum() >= 100


def test_traced_step_results_equal_untraced():
    """The traced kernel is the same step: its positions and forces equal the plain step's."""
    say("case: traced vs untraced step")
    s = cases()["c0"]
    n = len(s["x"])
    outs = []
    for traced in (False, True):
        pop = bdm.Population(n, 1 << 22)
        pop.load(s)
        p = bdm.params()
        if traced:
            c = torch.zeros(n, dtype=torch.int32, device="cuda")
            bdm.sim_step_traced(pop.soa, bdm.MODEL_MECH, p, 0, pop.ws, c, c.clone())
        else:
            bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, 0, pop.ws)
        outs.append(pop.read(("x", "y", "z", "fx", "fy", "fz")))
    for k in outs[0]:
        assert np.array_equal(outs[0][k].view(np.uint64), outs[1][k].view(np.uint64)), k


def test_traced_batch_contacts_match_oracle():
    """The batch kernel's contact decisions, per slot of a mix of sizes and precisions."""
    say("case: traced batch contacts")
    mix = [(inputs.uniform_cube(3000, 160.0, seed=31), 64), (equilibrium_case(seed=5), 32),
           (inputs.clustered(2500, 250.0, seed=32), 64), (inputs.uniform_cube(700, 90.0, seed=33), 32)]
    offs, off, boff, lay = [], 0, 0, []
    nbox = 1 << 16
    for s, bits in mix:
        n = len(s["x"])
        lay.append((off, n, boff, nbox))
        off += (n + bdm.SLOT_ALIGN - 1) // bdm.SLOT_ALIGN * bdm.SLOT_ALIGN
        boff += nbox
    b = bdm.Batch(off, boff, len(mix))
    for i, ((s, bits), (o, n, bo, nb)) in enumerate(zip(mix, lay)):
        for k, key in (("x", "x"), ("y", "y"), ("z", "z"), ("d", "diam"), ("adh", "adh")):
            b.t[key][o:o + n].copy_(torch.as_tensor(s[k]))
        b.t["id"][o:o + n].copy_(torch.arange(n, dtype=torch.int32))
        b.n[i] = n
        b.set_slot(i, o, n, bo, nb, 1, bdm.params(force_bits=bits))
    counts = torch.zeros(off, dtype=torch.int32, device="cuda")
    hashes = torch.zeros(off, dtype=torch.int32, device="cuda")
    b.step_traced(counts, hashes)
    torch.cuda.synchronize()
    for i, ((s, bits), (o, n, bo, nb)) in enumerate(zip(mix, lay)):
        flags, left = b.slot_status(i)
        assert flags == 0 and left == 0
        order = b.t["id"][o:o + n].cpu().numpy().view(np.uint32)  # box-sorted after the step
        ec, eh = expected(s, order, bits)
        got_c = counts[o:o + n].cpu().numpy().view(np.uint32)
        got_h = hashes[o:o + n].cpu().numpy().view(np.uint32)
        assert np.array_equal(got_c, ec) and np.array_equal(got_h, eh), i
