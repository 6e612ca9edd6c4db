"""GPU parity at the workloads' own configurations, through the C ABI.

* Mechanics at 2^24 spheres (3200 um cube, d in [8, 12)), 20 steps.  At steps 1, 10 and 19 --
  where the agents arrive already box-sorted from the previous step, the path bench.py times --
  the GPU's positions x_t are read back, and that step's keys, sorted order and box starts are
  compared in full with the oracle's grid of x_t; forces and new positions of sampled agents
  with the oracle's step on x_t (orc_mech_sample, exactly as its full step computes them); and
  the contact counts of the same agents, recorded by the traced kernels on x_t.
* The binary32 pair law: 20 steps of 2^18 agents at the same density against the binary64
  oracle's trajectory, whose largest position difference is reported.
* SIR at 10^7 agents in the periodic 5000^3 cube (box 20, radius 2, p_inf 0.3, p_rec 0.01,
  walk 1, 0.1 % infected), 200 steps: at steps 0, 100 and 199 the oracle takes one step from
  the GPU's state and states, positions and S/I/R counts must agree bit for bit.
* The tumour spheroid from 10^4 cells in a 60 um ball, the literal 60 steps, against the
  oracle's own 60-step trajectory: counts every step, then ids, diameters and positions.  The
  run is split into consecutive tests (module state) so that none runs long without output.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2006_06775_amd import bdm  # noqa: E402
from oracle import oracle as orc  # noqa: E402

K, GAMMA, DT, MAX_DISP = 2.0, 1.0, 0.01, 3.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edge(n):
    return 200.0 * (n / 4096.0) ** (1.0 / 3.0)


# ---------------------------------------------------------------------------------------------
def sample_ids(n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.integers(0, n, 20000), np.arange(0, 256),
                                     np.arange(n - 300, n)]))


def mech_checkpoint(pop, p, step, bits, n, seed):
    """Step `step` of the population with the comparisons described above."""
    st = pop.read(("x", "y", "z", "diam"))
    x_t = dict(x=st["x"], y=st["y"], z=st["z"], d=st["diam"], adh=np.full(n, 0.4))
    ids_in = pop.t["id"][:n].cpu().numpy().view(np.uint32).copy()  # input order of this build
    bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
    info, key, order, start = bdm.grid_export(pop.ws)
    rinfo, rkey, rorder, rstart = orc.grid(x_t["x"], x_t["y"], x_t["z"], x_t["d"])
    assert info["b"] == rinfo["b"] and info["dims"] == tuple(rinfo["dims"])
    key_by_id = np.empty(n, dtype=np.uint32)
    key_by_id[ids_in] = key
    assert np.array_equal(key_by_id, rkey), "keys"
    assert np.array_equal(order, rorder), "order"
    assert np.array_equal(start, rstart), "starts"
    out = pop.read(("x", "y", "z", "fx", "fy", "fz"))
    ids = sample_ids(n, seed + step)
    fx, fy, fz, nc = orc.mech_sample(x_t, ids, k=K, gamma=GAMMA, dt=DT, max_disp=MAX_DISP, force_bits=bits)
    for name, r in (("fx", fx), ("fy", fy), ("fz", fz)):
        assert np.array_equal(out[name][ids].view(np.uint64), r.view(np.uint64)), name
    moved = 0
    for j, i in enumerate(ids):
        flag, disp = orc.displacement((fx[j], fy[j], fz[j]), 0.4, DT, MAX_DISP)
        exp = [x_t[a][i] if flag == 1 else x_t[a][i] + disp[c] for c, a in enumerate("xyz")]
        moved += flag != 1
        assert [out["x"][i], out["y"][i], out["z"][i]] == exp, (step, i)
    # the traced kernels on x_t: contact counts of the sampled agents
    tr = bdm.Population(n, pop.max_boxes)
    tr.load(x_t)
    counts = torch.zeros(n, dtype=torch.int32, device="cuda")
    hashes = torch.zeros(n, dtype=torch.int32, device="cuda")
    bdm.sim_step_traced(tr.soa, bdm.MODEL_MECH, p, step, tr.ws, counts, hashes)
    _, _, torder, _ = bdm.grid_export(tr.ws)
    slot_of = np.empty(n, dtype=np.int64)
    slot_of[torder] = np.arange(n)
    got_nc = counts.cpu().numpy().view(np.uint32)[slot_of[ids]]
    assert np.array_equal(got_nc, nc), "contact counts"
    del tr, counts, hashes
    say(f"step {step}: keys, order, starts of {n} agents equal; {len(ids)} sampled agents bit-equal "
        f"({int(nc.sum())} contacts, {moved} moved)")


@pytest.mark.parametrize("bits,checks", [(64, (1, 10, 19)), (32, (1, 19))])
def test_mechanics_full_size_twenty_steps(bits, checks):
    n, L = 1 << 24, 3200.0
    say(f"case: mechanics n={n} 20 steps force_bits={bits}")
    pop = bdm.Population(n, bdm.box_count_hint(L, 11.9, 3))
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, L, 8.0, 12.0, 0.4, seed=0))
    p = bdm.params(k=K, gamma=GAMMA, dt=DT, max_disp=MAX_DISP, force_bits=bits)
    for step in range(20):
        if step in checks:
            mech_checkpoint(pop, p, step, bits, n, seed=bits)
        else:
            bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
    assert bdm.status(pop.ws) == 0
    del pop
    torch.cuda.empty_cache()


def test_fp32_error_against_fp64_oracle_twenty_steps():
    """Largest position difference of the binary32 pair law after 20 steps against the binary64
    oracle, at the mechanics workload's density (2^18 agents)."""
    n = 1 << 18
    L = edge(n)
    say(f"case: binary32 law vs binary64 oracle, n={n}, 20 steps")
    pop = bdm.Population(n, bdm.box_count_hint(L, 11.9, 3))
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, L, 8.0, 12.0, 0.4, seed=0))
    ref = orc.generate_cube(n, 0, L, 8.0, 12.0, 0.4)
    p = bdm.params(k=K, gamma=GAMMA, dt=DT, max_disp=MAX_DISP, force_bits=32)
    for step in range(20):
        bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
        orc.mech_step(ref, k=K, gamma=GAMMA, dt=DT, max_disp=MAX_DISP)
    got = pop.read(("x", "y", "z"))
    err = max(float(np.abs(got[a] - ref[a]).max()) for a in "xyz")
    say(f"binary32 pair law: max |x_gpu - x_oracle64| after 20 steps of {n} agents = {err:.3e} um "
        f"({err / L:.3e} of the cube edge)")
    assert 0.0 < err < 0.05


# ---------------------------------------------------------------------------------------------
SIR_N, SIR_L, SIR_STEPS = 10_000_000, 5000.0, 200
_sir = {}


def sir_to(step):
    """Advance the module's SIR run (GPU only) until `step` is the next step to take."""
    if not _sir:
        pop = bdm.Population(SIR_N, 250 ** 3, spheres=False, with_state=True)
        bdm.generate(pop.soa, bdm.gen(bdm.GEN_SIR, SIR_N, SIR_L, n_infected=SIR_N // 1000, seed=0))
        _sir.update(pop=pop, next=0,
                    p=bdm.params(box=20.0, periodic=1, L=SIR_L, r_inf=2.0, p_inf=0.3, p_rec=0.01, walk=1.0, seed=0),
                    op=orc.sir_params(SIR_L, 20.0, 2.0, 0.3, 0.01, 1.0, 0))
    pop = _sir["pop"]
    while _sir["next"] < step:
        bdm.sim_step(pop.soa, bdm.MODEL_SIR, _sir["p"], _sir["next"], pop.ws)
        _sir["next"] += 1
    return pop


@pytest.mark.parametrize("step", [0, 100, 199])
def test_sir_full_size_step(step):
    say(f"case: SIR n={SIR_N} step {step}")
    pop = sir_to(step)
    st = pop.read(("x", "y", "z", "state"))
    if step == 0:
        g = orc.generate_sir(SIR_N, 0, SIR_L, SIR_N // 1000)
        for a in ("x", "y", "z", "state"):
            assert np.array_equal(st[a], g[a]), a
    ref = {a: st[a].copy() for a in ("x", "y", "z", "state")}
    rc = orc.sir_step(ref, _sir["op"], step)
    bdm.sim_step(pop.soa, bdm.MODEL_SIR, _sir["p"], step, pop.ws)
    _sir["next"] = step + 1
    got = pop.read(("x", "y", "z", "state"))
    assert bdm.sir_counts(pop.ws) == rc.tolist()
    assert np.array_equal(got["state"], ref["state"])
    for a in "xyz":
        assert np.array_equal(got[a].view(np.uint64), ref[a].view(np.uint64)), a
    assert bdm.status(pop.ws) == 0
    say(f"step {step}: S/I/R {rc.tolist()} equal, states and positions bit-equal")
    if step == SIR_STEPS - 1:
        _sir.clear()
        torch.cuda.empty_cache()


# ---------------------------------------------------------------------------------------------
H, G = 0.5 ** (1 / 3), 1.05 ** (1 / 3)
_sph = {}


@pytest.mark.parametrize("first,last", [(0, 40), (40, 50), (50, 55), (55, 60)])
def test_spheroid_literal_sixty_steps(first, last):
    say(f"case: spheroid 10^4 cells, steps {first}..{last - 1}")
    if first == 0:
        cap = 300_000
        pop = bdm.Population(cap, 1 << 22)
        bdm.generate(pop.soa, bdm.gen(bdm.GEN_BALL, 10_000, 60.0, 14.0 * H, 14.0, 0.4, seed=0))
        st = orc.SpheroidState(orc.generate_ball(10_000, 0, 60.0, 14.0 * H, 14.0, 0.4), cap)
        _sph.update(pop=pop, st=st, p=bdm.params(grow=G, div_d=14.0, half_cbrt=H, seed=0),
                    op=orc.spheroid_params(G, 14.0, H, 0), next=0)
    assert _sph["next"] == first, "runs in order after the previous part"
    pop, st = _sph["pop"], _sph["st"]
    for step in range(first, last):
        bdm.sim_step(pop.soa, bdm.MODEL_SPHEROID, _sph["p"], step, pop.ws)
        st.step(_sph["op"], step)
        assert pop.n == int(st.n[0]), step
    _sph["next"] = last
    assert bdm.status(pop.ws) == 0
    got = pop.read(("x", "y", "z", "diam"))
    ref = {a: st.view(a) for a in ("x", "y", "z", "d")}
    assert np.array_equal(got["diam"].view(np.uint64), ref["d"].view(np.uint64))
    for a in "xyz":
        assert np.array_equal(got[a].view(np.uint64), ref[a].view(np.uint64)), (last, a)
    say(f"after step {last - 1}: {pop.n} cells, ids, diameters and positions bit-equal")
    if last == 60:
        assert pop.n == 198928
        _sph.clear()
        torch.cuda.empty_cache()
