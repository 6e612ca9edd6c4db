"""Autotuner of the batched step: the box edge per simulation size and the work split.

Two knobs change the work of a batched step without changing any result:

* The box edge, a per-simulation parameter.  Any edge at least the largest diameter gives the
  same contact sets, but a larger box means fewer boxes (a cheaper grid build) and more
  candidates per agent (a dearer mechanics step), and the balance depends on the simulation's
  size: for small simulations the fixed costs of a step dominate, for large ones the walk does.
  The summation order follows the edge, so a served result still equals the same request
  served alone with the same edge.
* The work split, a per-batch launch parameter: how many workgroups the per-tile launches of a
  batched step deal the packed tiles to (they stride over them, neighbouring tiles of a round on
  one XCD).  Fewer workgroups run longer strides; more pay more workgroup launches and idle
  tails.  The tile itself (256 agents, four wavefronts) is fixed by the kernels' register and
  LDS budget.

`plan()` times the batched step itself on the device.  For each size class it runs a batch of
simulations of that size (C0's density, d in [10, 15), binary32 pair law, as served) at each
candidate factor of the largest diameter and keeps the fastest factor per class.  It then runs
a batch that mixes sizes like the served stream, each simulation at its class's edge, at each
candidate work split, and keeps the fastest split (the default unless another is at least 2 %
faster).  `BoxPlan.box_for(n)` gives each request the edge of its size class (the nearest class
on a log scale) and `BoxPlan.grid_cap` the split.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

SIZE_CLASSES = (1_000, 10_000, 100_000, 1_000_000)
FACTORS = (1.0, 1.2, 1.4)
GRID_CAPS = (2048, 4096, 8192, 16384, 32768, -1)  # -1: one workgroup per tile
DEFAULT_CAP = 8192
CLASS_AGENTS = 2_000_000  # agents per size-class batch (at least one simulation)


def pick(table: dict) -> dict:
    """{n: {factor: seconds per agent-update}} -> {n: fastest factor} (ties: the smaller one)."""
    return {n: min(row, key=lambda f: (row[f], f)) for n, row in table.items()}


def pick_cap(row: dict, default: int = DEFAULT_CAP, margin: float = 0.02) -> int:
    """Fastest work split, or the default unless another is faster by more than `margin`.  Among
    splits within `margin` of the fastest, one workgroup per tile (-1) is taken: it has no
    striding loop and fills the device for any mix of slots, which a served stream varies more
    than the measured batch does (the two best splits timing within 0.3 % of each other, a
    32768-workgroup cap served the stream at 1.28x against 1.37-1.46x for one per tile)."""
    best = min(row, key=lambda c: (row[c], c))
    if default in row and row[best] > (1.0 - margin) * row[default]:
        return default
    if -1 in row and row[-1] <= (1.0 + margin) * row[best]:
        return -1
    return best


@dataclass
class BoxPlan:
    d_hi: float                       # largest diameter of the requests
    best: dict                        # size class -> factor
    table: dict = field(default_factory=dict)
    seconds: float = 0.0              # time spent measuring
    grid_cap: int = 0                 # work split of the batched step (0: the library default)
    split_table: dict = field(default_factory=dict)  # grid cap -> seconds per agent-update

    def factor_for(self, n: int) -> float:
        classes = sorted(self.best)
        c = min(classes, key=lambda s: abs(math.log(max(n, 1)) - math.log(s)))
        return self.best[c]

    def box_for(self, n: int) -> float:
        return self.d_hi * self.factor_for(n)

    def summary(self) -> dict:
        return dict(factors={str(k): v for k, v in sorted(self.best.items())},
                    ns_per_agent_update={str(n): {str(f): round(t * 1e9, 4) for f, t in row.items()}
                                         for n, row in sorted(self.table.items())},
                    grid_cap=self.grid_cap or DEFAULT_CAP,
                    split_ns_per_agent_update={str(c): round(t * 1e9, 4) for c, t in sorted(self.split_table.items())},
                    measured="batched step", seconds=round(self.seconds, 3))


def measure_batch(sizes, boxes, grid_cap: int = 0, steps: int = 3, seed: int = 12345) -> float:
    """Seconds per agent-update of batched binary32-force steps of simulations of `sizes` agents
    shaped like served requests (C0 density, d in [10, 15)), simulation i with box edge boxes[i]."""
    import torch

    from . import bdm, serve
    align = bdm.SLOT_ALIGN
    lay, off, boff = [], 0, 0
    for n, box in zip(sizes, boxes):
        nb = serve.box_reserve(n, box)
        lay.append((off, boff, nb))
        off += (n + align - 1) // align * align
        boff += (nb + bdm.BOX_ALIGN - 1) // bdm.BOX_ALIGN * bdm.BOX_ALIGN
    b = bdm.Batch(off, boff, len(sizes), grid_cap=grid_cap)
    for i, (n, box) in enumerate(zip(sizes, boxes)):
        o, bo, nb = lay[i]
        bdm.generate(b.view(i, o, n), bdm.gen(bdm.GEN_CUBE, n, serve.cube_edge(n), serve.D_LO, serve.D_HI, 0.4,
                                              seed=seed + i))
        b.set_slot(i, o, n, bo, nb, steps + 1, serve.mech_params(box))
    b.step()  # warm-up (and box-sorted order)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(steps):
        b.step()
    e.record()
    torch.cuda.synchronize()
    for i in range(len(sizes)):
        flags, _ = b.slot_status(i)
        if flags:
            raise RuntimeError(f"tune: slot {i} ({sizes[i]} agents) status {flags:#x}")
    return s.elapsed_time(e) * 1e-3 / (steps * sum(sizes))


def mixed_sizes(count: int = 24, seed: int = 7, n_min: int = 1_000, n_max: int = 2_000_000):
    """Sizes drawn like the served stream's (log-uniform)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return [int(v) for v in np.exp(rng.uniform(math.log(n_min), math.log(n_max), count))]


def plan(classes=SIZE_CLASSES, factors=FACTORS, caps=GRID_CAPS, steps: int = 3) -> BoxPlan:
    import time

    from . import serve
    t0 = time.perf_counter()
    table = {}
    for n in classes:
        copies = max(1, min(64, CLASS_AGENTS // n))
        table[n] = {f: measure_batch([n] * copies, [serve.D_HI * f] * copies, steps=steps) for f in factors}
    best = pick(table)
    p = BoxPlan(serve.D_HI, best, table)
    sizes = mixed_sizes()
    boxes = [p.box_for(n) for n in sizes]
    p.split_table = {c: measure_batch(sizes, boxes, grid_cap=c, steps=steps) for c in caps}
    p.grid_cap = pick_cap(p.split_table)
    p.seconds = time.perf_counter() - t0
    return p


def fixed(factor: float = 1.0, grid_cap: int = 0) -> BoxPlan:
    """A plan that gives every request the same edge and the default split (no measurement)."""
    from . import serve
    return BoxPlan(serve.D_HI, {SIZE_CLASSES[0]: factor}, grid_cap=grid_cap)
