"""GPU: bdm_sim_step_noalloc -- the step with the library's static device scratch as its
workspace -- against bdm_sim_step with a caller workspace, through the C ABI.  Two calls in a
row, the second on a smaller population (the array keeps the first call's contents, which the
second must not see), for the mechanics and the spheroid model; then an SIR step.  Every result
must be bit-identical to the workspace step's, and the status word must read zero."""
import sys

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2006_06775_amd import bdm  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edge(n):
    return 200.0 * (n / 4096.0) ** (1.0 / 3.0)


def pair(s, max_boxes, state=False):
    """Two populations holding the same agents: one stepped with a workspace, one without."""
    n = len(s["x"])
    spheres = "d" in s
    a = bdm.Population(n, max_boxes, spheres=spheres, with_state=state)
    b = bdm.Population(n, max_boxes, spheres=spheres, with_state=state)
    a.load(s)
    b.load(s)
    return a, b


def same(a, b, keys):
    ra, rb = a.read(keys), b.read(keys)
    for k in ra:
        assert np.array_equal(ra[k].view(np.uint8), rb[k].view(np.uint8)), k


@pytest.mark.parametrize("model", ["mech", "spheroid"])
def test_noalloc_step_equals_workspace_step(model):
    m = bdm.MODEL_MECH if model == "mech" else bdm.MODEL_SPHEROID
    p = bdm.params(force_bits=64, grow=1.05 ** (1 / 3), div_d=14.0, seed=5)
    for call, n in enumerate((9000, 2500)):  # the second call is smaller
        say(f"case: noalloc {model} call {call} n={n}")
        s = inputs.uniform_cube(n, edge(n), seed=60 + call)
        max_boxes = bdm.box_count_hint(edge(n), 10.0, 4)
        assert bdm.workspace_bytes(n, max_boxes) <= bdm.NOALLOC_SCRATCH_BYTES
        a, b = pair(s, max_boxes)
        if m == bdm.MODEL_SPHEROID:  # room for the daughters
            a = bdm.Population(2 * n, max_boxes)
            b = bdm.Population(2 * n, max_boxes)
            a.load(s)
            b.load(s)
        flags = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        bdm.sim_step(a.soa, m, p, call, a.ws)
        bdm.sim_step_noalloc(b.soa, m, p, call, max_boxes, flags)
        torch.cuda.synchronize()
        assert bdm.status(a.ws) == 0
        assert int(flags.item()) == 0
        assert a.n == b.n
        same(a, b, ("x", "y", "z", "diam", "fx", "fy", "fz"))


def test_noalloc_sir_step_equals_workspace_step():
    say("case: noalloc SIR")
    n, L = 40000, 60.0
    s = inputs.sir_uniform(n, L, seed=9)
    p = bdm.params(box=2.0, periodic=1, L=L, r_inf=2.0, p_inf=0.3, p_rec=0.01, walk=1.0, seed=9)
    a, b = pair(s, 30 ** 3, state=True)
    flags = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    for step in range(2):
        bdm.sim_step(a.soa, bdm.MODEL_SIR, p, step, a.ws)
        bdm.sim_step_noalloc(b.soa, bdm.MODEL_SIR, p, step, 30 ** 3, flags)
    torch.cuda.synchronize()
    assert int(flags.item()) == 0 and bdm.status(a.ws) == 0
    same(a, b, ("x", "y", "z", "state"))


def test_noalloc_rejects_a_population_beyond_the_scratch():
    say("case: noalloc size limit")
    n = 1 << 20
    pop = bdm.Population(16, 64)
    big = bdm.Soa(n, pop.soa.n, pop.soa.x, pop.soa.y, pop.soa.z, pop.soa.diam, pop.soa.adh,
                  pop.soa.fx, pop.soa.fy, pop.soa.fz, pop.soa.id, None)
    with pytest.raises(bdm.BdmError) as e:
        bdm.sim_step_noalloc(big, bdm.MODEL_MECH, bdm.params(), 0, 1 << 20)
    assert e.value.rc == bdm.ENOWS
    assert "static scratch" in str(e.value)
