"""GPU parity at the full benchmark size: 2^24 spheres in a 3200 um cube, d in [8, 12), one grid
build and one mechanical step through the C ABI, in the launch configuration bench.py times.

The oracle generates the same 2^24 agents and builds the same grid on the CPU (cheap: linear
time), so the generator output, box edge, lattice, every key, the whole sorted order and every
box start are compared in full, bit for bit.  Stepping all 2^24 agents on one core would take
minutes, so forces and new positions are compared on a sample of agents (random, plus the
first and last agents and whole wavefronts at tile boundaries), each computed by the oracle
exactly as its full step would (orc_mech_sample: same grid, same candidate order).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - the gpu marker deselects these on CPU
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2006_06775_amd import bdm  # noqa: E402
from oracle import oracle as orc  # noqa: E402

N, L = 1 << 24, 3200.0
K, GAMMA, DT, MAX_DISP = 2.0, 1.0, 0.01, 3.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ref():
    say(f"case: oracle generate_cube n={N}")
    return orc.generate_cube(N, 0, L, 8.0, 12.0, 0.4)


def sample_ids(n, seed):
    rng = np.random.default_rng(seed)
    picks = [rng.integers(0, n, 20000), np.arange(0, 256), np.arange(n - 300, n),
             np.arange(1 << 23, (1 << 23) + 64)]
    return np.unique(np.concatenate(picks))


@pytest.mark.parametrize("bits", [64, 32])
def test_full_size_grid_and_sampled_step(ref, bits):
    say(f"case: full size n={N} force_bits={bits}")
    pop = bdm.Population(N, bdm.box_count_hint(L, 11.9, 3))
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, N, L, 8.0, 12.0, 0.4, seed=0))
    got = pop.read(("x", "y", "z", "diam"))
    for a, b in (("x", "x"), ("y", "y"), ("z", "z"), ("diam", "d")):
        assert np.array_equal(got[a], ref[b]), a
    del got

    p = bdm.params(k=K, gamma=GAMMA, dt=DT, max_disp=MAX_DISP, force_bits=bits)
    bdm.grid_build(pop.soa, p, pop.ws)
    info, key, order, start = bdm.grid_export(pop.ws)
    rinfo, rkey, rorder, rstart = orc.grid(ref["x"], ref["y"], ref["z"], ref["d"])
    assert info["valid"] == 1 and info["flags"] == 0
    assert info["b"] == rinfo["b"]
    assert info["cmin"] == tuple(rinfo["cmin"]) and info["dims"] == tuple(rinfo["dims"])
    assert np.array_equal(key, rkey)
    assert np.array_equal(order, rorder)
    assert np.array_equal(start, rstart)
    del key, order, start, rkey, rorder, rstart

    bdm.mech_step(pop.soa, p, pop.ws)
    assert bdm.status(pop.ws) == 0
    out = pop.read(("x", "y", "z", "fx", "fy", "fz"))
    ids = sample_ids(N, seed=bits)
    fx, fy, fz, nc = orc.mech_sample(ref, ids, k=K, gamma=GAMMA, dt=DT, max_disp=MAX_DISP, force_bits=bits)
    assert nc.sum() > len(ids)  # the sample has contacts (about 2.2 per agent)
    for name, r in (("fx", fx), ("fy", fy), ("fz", fz)):
        assert np.array_equal(out[name][ids], r), name
    moved = 0
    for n_, i in enumerate(ids):
        flag, disp = orc.displacement((fx[n_], fy[n_], fz[n_]), ref["adh"][i], DT, MAX_DISP)
        exp = [ref[a][i] if flag == 1 else ref[a][i] + disp[c] for c, a in enumerate("xyz")]
        moved += flag != 1
        assert [out["x"][i], out["y"][i], out["z"][i]] == exp, i
    say(f"sampled {len(ids)} agents, {int(nc.sum())} contacts, {moved} moved: bit-equal")
    assert moved > 0
