"""GPU: the batched form.  Many independent mechanical simulations of uneven sizes packed into
one population and stepped together must give, for every simulation, exactly the result of the
same simulation run alone through the plain entry points (and, for one of them, the oracle's)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2006_06775_amd import bdm  # noqa: E402
from oracle import oracle as orc  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edge(n):
    return 200.0 * (n / 4096.0) ** (1.0 / 3.0)


# (agents, steps, force_bits, explicit box or 0, seed)
MIX = [(1000, 3, 64, 0.0, 1), (5000, 5, 32, 0.0, 2), (20000, 4, 64, 15.0, 3), (3000, 6, 32, 18.0, 4),
       (50000, 2, 64, 0.0, 5), (1500, 7, 64, 0.0, 6)]


def alone(n, steps, bits, box, seed):
    pop = bdm.Population(n, bdm.box_count_hint(edge(n), 10.0, 4))
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, edge(n), 10.0, 15.0, 0.4, seed=seed))
    p = bdm.params(force_bits=bits, box=box)
    for step in range(steps):
        bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
    assert bdm.status(pop.ws) == 0
    return pop.read(("x", "y", "z", "fx", "fy", "fz"))


def layout(mix):
    """Aligned agent ranges and box ranges for the mix."""
    off, boff, out = 0, 0, []
    for n, steps, bits, box, seed in mix:
        nb = bdm.box_count_hint(edge(n), 10.0, 4)
        out.append((off, n, boff, nb))
        off += (n + bdm.SLOT_ALIGN - 1) // bdm.SLOT_ALIGN * bdm.SLOT_ALIGN
        boff += (nb + bdm.BOX_ALIGN - 1) // bdm.BOX_ALIGN * bdm.BOX_ALIGN
    return out, off, boff


def run_batch(mix, slots=8, late=(), grid_cap=0):
    lay, cap, boxes = layout(mix)
    b = bdm.Batch(cap, boxes, slots, grid_cap=grid_cap)
    started = set()

    def start(i):
        n, steps, bits, box, seed = mix[i]
        off, cap_i, boff, nb = lay[i]
        bdm.generate(b.view(i, off, cap_i), bdm.gen(bdm.GEN_CUBE, n, edge(n), 10.0, 15.0, 0.4, seed=seed))
        b.set_slot(i, off, cap_i, boff, nb, steps, bdm.params(force_bits=bits, box=box))
        started.add(i)

    for i in range(len(mix)):
        if i not in late:
            start(i)
    for it in range(max(m[1] for m in mix) + 3):
        if it == 2:
            for i in late:
                start(i)  # admitted while the others are mid-run
        b.step()
    torch.cuda.synchronize()
    out = []
    for i in range(len(mix)):
        flags, left = b.slot_status(i)
        assert flags == 0 and left == 0, (i, flags, left)
        off, cap_i, _, _ = lay[i]
        out.append(b.read_slot(i, off, cap_i))
    return out


@pytest.mark.parametrize("grid_cap", [0, -1, 64])
def test_batch_equals_alone_bitwise(grid_cap):
    """Every slot equals its plain run bit for bit, whatever the work split: the default striding
    grid, one workgroup per tile (its own mechanics kernel), and a tiny striding grid."""
    say(f"case: batch mix vs alone, grid_cap {grid_cap}")
    got = run_batch(MIX, late=(1, 4), grid_cap=grid_cap)
    for i, m in enumerate(MIX):
        ref = alone(*m)
        for k in ("x", "y", "z", "fx", "fy", "fz"):
            assert np.array_equal(got[i][k].view(np.uint64), ref[k].view(np.uint64)), (i, k)
    say("all slots bit-identical to their plain runs")


def test_batch_slot_against_oracle():
    say("case: batch slot vs oracle")
    mix = [(2000, 4, 64, 0.0, 11), (4096, 3, 64, 0.0, 0)]
    got = run_batch(mix, slots=2)
    ref = orc.generate_cube(4096, 0, 200.0, 10.0, 15.0, 0.4)
    for _ in range(3):
        orc.mech_step(ref)
    for k in ("x", "y", "z"):
        assert np.array_equal(got[1][k].view(np.uint64), ref[k].view(np.uint64))


def test_batch_slot_reuse_and_idle():
    say("case: batch reuse")
    mix = [(3000, 2, 64, 0.0, 21), (6000, 3, 32, 0.0, 22)]
    lay, cap, boxes = layout(mix)
    b = bdm.Batch(cap, boxes, 4)
    # first occupant of slot 0, then reuse its range for a different simulation
    off, cap0, boff, nb = lay[0]
    bdm.generate(b.view(0, off, cap0), bdm.gen(bdm.GEN_CUBE, 3000, edge(3000), 10.0, 15.0, 0.4, seed=99))
    b.set_slot(0, off, cap0, boff, nb, 1, bdm.params())
    b.step()
    b.clear_slot(0, off, cap0)
    for i, (n, steps, bits, box, seed) in enumerate(mix):
        o, c, bo, nbx = lay[i]
        bdm.generate(b.view(i, o, c), bdm.gen(bdm.GEN_CUBE, n, edge(n), 10.0, 15.0, 0.4, seed=seed))
        b.set_slot(i, o, c, bo, nbx, steps, bdm.params(force_bits=bits, box=box))
    for _ in range(5):
        b.step()  # slots idle once their steps are done; idle slots 2, 3 never ran
    for i, m in enumerate(mix):
        o, c, _, _ = lay[i]
        got = b.read_slot(i, o, c)
        ref = alone(*m)
        for k in ("x", "y", "z"):
            assert np.array_equal(got[k].view(np.uint64), ref[k].view(np.uint64)), (i, k)


def test_batch_graph_replay():
    say("case: batch graph replay")
    mix = [(4000, 6, 64, 0.0, 31), (9000, 6, 32, 0.0, 32)]
    lay, cap, boxes = layout(mix)
    b = bdm.Batch(cap, boxes, 2)
    for i, (n, steps, bits, box, seed) in enumerate(mix):
        o, c, bo, nbx = lay[i]
        bdm.generate(b.view(i, o, c), bdm.gen(bdm.GEN_CUBE, n, edge(n), 10.0, 15.0, 0.4, seed=seed))
        b.set_slot(i, o, c, bo, nbx, steps, bdm.params(force_bits=bits, box=box))
    b.step()  # warm (first launches), eager
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.step(stream=s)
    for _ in range(5):
        g.replay()
        torch.cuda.synchronize()
        _ = b.n.cpu()  # eager work and a synchronisation between replays
    for i, m in enumerate(mix):
        o, c, _, _ = lay[i]
        got = b.read_slot(i, o, c)
        ref = alone(*m)
        for k in ("x", "y", "z"):
            assert np.array_equal(got[k].view(np.uint64), ref[k].view(np.uint64)), (i, k)


def test_batch_validation():
    say("case: batch validation")
    for bad in (-2, 1, 63, 65537):
        with pytest.raises(bdm.BdmError):
            bdm.Batch(4096, 10000, 2, grid_cap=bad)
    b = bdm.Batch(4096, 10000, 2)
    with pytest.raises(bdm.BdmError):
        b.set_slot(0, 100, 1000, 0, 1000, 1, bdm.params())  # misaligned
    with pytest.raises(bdm.BdmError):
        b.set_slot(2, 0, 1000, 0, 1000, 1, bdm.params())  # slot out of range
    with pytest.raises(bdm.BdmError):
        b.set_slot(0, 0, 5000, 0, 1000, 1, bdm.params())  # range beyond capacity
    with pytest.raises(bdm.BdmError):
        b.set_slot(0, 0, 1000, 0, 1000, 1, bdm.params(dt=0.0))
