"""Box-edge autotuner for the served simulations.

The box edge is a per-simulation parameter: any edge at least the largest diameter gives the
same contact sets, but it changes the work.  A larger box means fewer boxes (a cheaper grid
build) and more candidates per agent (a dearer mechanics step).  The best edge depends on the
simulation's size.  For small simulations the fixed costs of a step dominate, for large ones
the candidate walk does.

`plan()` measures this on the device.  For each size class it runs a few plain steps of a
population shaped like the served requests, at each candidate factor of the largest diameter,
and keeps the fastest factor per class.  `BoxPlan.box_for(n)` then gives each request the edge
of its size class (the nearest class on a log scale).  Each slot of the batch carries its own
edge, so the plan costs the batch nothing.  The summation order follows the edge, so a served
result still equals the same request served alone with the same edge.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

SIZE_CLASSES = (1_000, 10_000, 100_000, 1_000_000)
FACTORS = (1.0, 1.2, 1.4)


def pick(table: dict) -> dict:
    """{n: {factor: seconds per agent-update}} -> {n: fastest factor} (ties: the smaller one)."""
    return {n: min(row, key=lambda f: (row[f], f)) for n, row in table.items()}


@dataclass
class BoxPlan:
    d_hi: float                       # largest diameter of the requests
    best: dict                        # size class -> factor
    table: dict = field(default_factory=dict)
    seconds: float = 0.0              # time spent measuring

    def factor_for(self, n: int) -> float:
        classes = sorted(self.best)
        c = min(classes, key=lambda s: abs(math.log(max(n, 1)) - math.log(s)))
        return self.best[c]

    def box_for(self, n: int) -> float:
        return self.d_hi * self.factor_for(n)

    def summary(self) -> dict:
        return dict(factors={str(k): v for k, v in sorted(self.best.items())},
                    ns_per_agent_update={str(n): {str(f): round(t * 1e9, 3) for f, t in row.items()}
                                         for n, row in sorted(self.table.items())},
                    seconds=round(self.seconds, 3))


def measure(n: int, factor: float, steps: int = 3, seed: int = 12345) -> float:
    """Seconds per agent-update of plain binary32-force steps of n agents shaped like a served
    request (C0 density, d in [10, 15)) with box edge factor * 15 um."""
    import torch

    from . import bdm, serve
    box = serve.D_HI * factor
    edge = serve.cube_edge(n)
    pop = bdm.Population(n, serve.box_reserve(n, box))
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, edge, serve.D_LO, serve.D_HI, 0.4, seed=seed))
    p = bdm.params(k=2.0, gamma=1.0, dt=0.01, max_disp=3.0, box=box, force_bits=32)
    bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, 0, pop.ws)  # warm-up (and box-sorted order)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for step in range(steps):
        bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step + 1, pop.ws)
    e.record()
    torch.cuda.synchronize()
    flags = bdm.status(pop.ws)
    if flags:
        raise RuntimeError(f"tune: device flags {flags:#x} at n={n}, factor {factor}")
    return s.elapsed_time(e) * 1e-3 / (steps * n)


def plan(classes=SIZE_CLASSES, factors=FACTORS, steps: int = 3) -> BoxPlan:
    import time

    from . import serve
    t0 = time.perf_counter()
    table = {n: {f: measure(n, f, steps) for f in factors} for n in classes}
    return BoxPlan(serve.D_HI, pick(table), table, time.perf_counter() - t0)


def fixed(factor: float = 1.0) -> BoxPlan:
    """A plan that gives every request the same edge (no measurement)."""
    from . import serve
    return BoxPlan(serve.D_HI, {SIZE_CLASSES[0]: factor})
