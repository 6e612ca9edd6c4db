"""GPU: the stationary-region skip (paper Sec. 2.3 (iv)) changes no result.

With skip_static = 1 a mechanical step skips the neighbour walk of agents whose neighbourhood
did not change in the last step and keeps their last force and position.  The trajectory must
equal the oracle's (which never skips) bit for bit at every step, and equal the same run without
the skip.  The runs relax (dt 0.3), so that most agents become stationary and are skipped."""
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

DT = 0.3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bits(a):
    return a.view(np.uint64)


def test_skip_trajectory_equals_oracle():
    """4096 agents in a 200 um cube, d in [10, 15), 30 relaxing steps, lockstep with the oracle."""
    n = 4096
    pop = bdm.Population(n, 1 << 14)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, 200.0, 10.0, 15.0, 0.4, seed=0))
    ref = orc.generate_cube(n, 0, 200.0, 10.0, 15.0, 0.4)
    p = bdm.params(dt=DT, skip_static=1)
    skipped = []
    for step in range(30):
        say(f"case: skip lockstep step {step}")
        bdm.grid_build(pop.soa, p, pop.ws)
        bdm.mech_step(pop.soa, p, pop.ws)
        fx, fy, fz, nc, fl = orc.mech_step(ref, dt=DT)
        got = pop.read(("x", "y", "z", "fx", "fy", "fz"))
        for k, r in (("x", ref["x"]), ("y", ref["y"]), ("z", ref["z"]), ("fx", fx), ("fy", fy), ("fz", fz)):
            assert np.array_equal(bits(got[k]), bits(r)), (step, k)
        info = bdm.grid_info(pop.ws)
        skipped.append(info["skipped"])
        assert info["flags"] == 0
        assert info["skipped"] <= int((fl == 1).sum())  # only gated agents are skipped
    say(f"agents skipped per step: {skipped}")
    assert skipped[0] == 0 and max(skipped) > n // 2


@pytest.mark.parametrize("case", ["ragged", "clustered", "faces"])
def test_skip_equals_plain_steps(case):
    """The same run through bdm_sim_step with and without the skip, including populations whose
    lattice changes between steps (the skip then waits for an unchanged one)."""
    s = {"ragged": inputs.uniform_cube(5001, 230.0, seed=4),
         "clustered": inputs.clustered(4000, 300.0, seed=3),
         "faces": inputs.box_face_adversarial(3000, 12.0, seed=2)}[case]
    n = len(s["x"])
    pops = []
    for skip in (0, 1):
        pop = bdm.Population(n, 1 << 20)
        pop.load(s)
        p = bdm.params(dt=DT, skip_static=skip)
        total = 0
        for step in range(25):
            bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
            total += bdm.grid_info(pop.ws)["skipped"]
        assert bdm.status(pop.ws) == 0
        pops.append((pop.read(("x", "y", "z", "fx", "fy", "fz")), total))
    (a, _), (b, total) = pops
    say(f"{case}: {total} agent-steps skipped")
    for k in a:
        assert np.array_equal(bits(a[k]), bits(b[k])), k
    if case == "ragged":  # (clumps and face-packed agents spread: their lattice grows every step)
        assert total > 0


def test_skip_needs_matching_build():
    """A build for the skipping step and a step that does not skip (or the reverse) do not mix:
    the step reports BDM_FLAG_NOGRID and moves nothing."""
    s = inputs.uniform_cube(2000, 150.0, seed=8)
    pop = bdm.Population(2000, 1 << 16)
    pop.load(s)
    for build_skip, step_skip in ((1, 0), (0, 1)):
        bdm.grid_build(pop.soa, bdm.params(skip_static=build_skip), pop.ws)
        x0 = pop.t["x"][:2000].clone()
        bdm.mech_step(pop.soa, bdm.params(skip_static=step_skip), pop.ws)
        assert torch.equal(pop.t["x"][:2000], x0)
        assert bdm.status(pop.ws, clear=True) == bdm.FLAG_NOGRID


def test_skip_full_size_sampled():
    """2^24 agents at the mechanics workload's density, 24 relaxing steps with the skip, then one
    more: sampled forces and positions against the oracle's step on the GPU's positions, and the
    whole state against the same run without the skip."""
    n, L = 1 << 24, 3200.0
    say(f"case: skip n={n}")
    out = []
    for skip in (1, 0):
        pop = bdm.Population(n, bdm.box_count_hint(L, 11.9, 3))
        bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, L, 8.0, 12.0, 0.4, seed=0))
        p = bdm.params(dt=DT, skip_static=skip)
        for step in range(24):
            bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
        st = pop.read(("x", "y", "z", "diam"))
        bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, 24, pop.ws)
        info = bdm.grid_info(pop.ws)
        assert info["flags"] == 0
        res = pop.read(("x", "y", "z", "fx", "fy", "fz"))
        out.append((st, res, info["skipped"]))
        del pop
        torch.cuda.empty_cache()
    (st, res, skipped), (st0, res0, _) = out
    say(f"last step skipped {skipped} of {n} agents")
    assert skipped > n // 4
    for k in res:
        assert np.array_equal(bits(res[k]), bits(res0[k])), k
    x_t = dict(x=st["x"], y=st["y"], z=st["z"], d=st["diam"], adh=np.full(n, 0.4))
    ids = np.unique(np.random.default_rng(5).integers(0, n, 20000))
    fx, fy, fz, nc = orc.mech_sample(x_t, ids, dt=DT)
    for k, r in (("fx", fx), ("fy", fy), ("fz", fz)):
        assert np.array_equal(bits(res[k][ids]), bits(r)), k
    for j, i in enumerate(ids):
        flag, disp = orc.displacement((fx[j], fy[j], fz[j]), 0.4, DT, 3.0)
        exp = [x_t[a][i] if flag == 1 else x_t[a][i] + disp[c] for c, a in enumerate("xyz")]
        assert [res["x"][i], res["y"][i], res["z"][i]] == exp, i


def relaxed_population(skip, n=1 << 14, steps=40, seed=0):
    """2^14 agents at the 2^24 workload's density (d in [8, 12)), `steps` relaxing steps; every
    agent is gated after about 20 of them, so the later steps change nothing."""
    L = 3200.0 / 1024 ** (1.0 / 3.0)
    pop = bdm.Population(n, 1 << 18)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, L, 8.0, 12.0, 0.4, seed=seed))
    p = bdm.params(dt=DT, skip_static=skip)
    skipped = []
    for step in range(steps):
        bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
        skipped.append(bdm.grid_info(pop.ws)["skipped"])
    return pop, skipped


def test_relaxed_steps_change_nothing_and_a_new_law_recomputes():
    """Once a step skipped every agent, the next steps skip their build and walk whole; they
    must still equal the run without the skip, and a change of the force law must bring the
    full step back (no agent skipped) with the same results as without the skip."""
    say("case: frozen relaxed steps")
    out = []
    for skip in (0, 1):
        pop, skipped = relaxed_population(skip)
        p2 = bdm.params(k=2.5, gamma=1.25, dt=DT, skip_static=skip)
        for step in range(40, 48):
            bdm.sim_step(pop.soa, bdm.MODEL_MECH, p2, step, pop.ws)
            skipped.append(bdm.grid_info(pop.ws)["skipped"])
        assert bdm.status(pop.ws) == 0
        out.append((pop.read(("x", "y", "z", "fx", "fy", "fz")), skipped, pop.n))
    (a, _, _), (b, skipped, n) = out
    say(f"skipped per step: {skipped}")
    for k in a:
        assert np.array_equal(bits(a[k]), bits(b[k])), k
    assert skipped[38] == n and skipped[39] == n  # relaxed: whole steps skipped
    assert skipped[40] == 0  # another force law: every agent walks again
    assert max(skipped[41:]) > n // 2  # and the skip resumes under the new law


def test_relaxed_build_then_step_with_another_law_is_refused():
    """A build that found nothing to do belongs to its force law: a mechanical step asking for
    another law reports BDM_FLAG_NOGRID and moves nothing."""
    say("case: frozen build, other law")
    pop, skipped = relaxed_population(1)
    assert skipped[-1] == pop.n
    p = bdm.params(dt=DT, skip_static=1)
    bdm.grid_build(pop.soa, p, pop.ws)
    x0 = pop.t["x"][:pop.n].clone()
    bdm.mech_step(pop.soa, bdm.params(k=3.0, dt=DT, skip_static=1), pop.ws)
    assert torch.equal(pop.t["x"][:pop.n], x0)
    assert bdm.status(pop.ws, clear=True) == bdm.FLAG_NOGRID
