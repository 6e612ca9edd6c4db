"""Continuous-batching server for independent mechanical simulations on one GPU.

Requests arrive over time (a seeded Poisson trace).  Each is one simulation: `n` spheres at the
density of 4096 agents in a 200 um cube, diameters in [10, 15) um, run for `steps` mechanical
steps with binary32 pair forces and binary64 positions.  The server keeps one packed population
(`bdm.Batch`): a request is admitted as soon as a slot and a contiguous agent range and box
range are free (admission by HBM footprint), its agents are generated in place, and from then
on it advances with every batched step together with whatever else is running.  Finished
requests are read back to the host and their ranges freed.  Latency is arrival -> results on
the host.  `run_plain` serves the same trace one request at a time with plain launches, for
comparison.

Host-side logic only (allocation, admission, bookkeeping); every step of every simulation runs
in libbdm.so's kernels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

ALIGN = 1024            # agent-range alignment of a batch slot
DENSITY_N, DENSITY_L = 4096, 200.0
D_LO, D_HI = 10.0, 15.0


def cube_edge(n: int) -> float:
    return DENSITY_L * (n / DENSITY_N) ** (1.0 / 3.0)


def box_reserve(n: int, box: float) -> int:
    """Histogram entries reserved for a simulation of n agents with box edge `box` (the cube
    grows by a few boxes per side as the agents relax outward)."""
    per = int(math.floor(cube_edge(n) / box)) + 1 + 4
    return per ** 3


def box_edge(box, n: int) -> float:
    """The box edge of a request of n agents: a fixed edge, or a tune.BoxPlan's choice."""
    return float(box.box_for(n)) if hasattr(box, "box_for") else float(box)


def mech_params(box: float):
    """The served simulations' parameters (C0's mechanics, binary32 pair law) with box edge `box`."""
    from . import bdm
    return bdm.params(k=2.0, gamma=1.0, dt=0.01, max_disp=3.0, box=box, force_bits=32)


@dataclass
class Request:
    rid: int
    arrival: float   # seconds after the start of the trace
    n: int
    steps: int
    seed: int


def make_trace(count=512, seed=0, rate=100.0, n_min=1_000, n_max=2_000_000, s_min=10, s_max=100):
    """Seeded Poisson arrivals (rate per second); n log-uniform in [n_min, n_max], steps uniform
    in {s_min..s_max}."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = np.exp(rng.uniform(math.log(n_min), math.log(n_max), count)).astype(np.int64)
    steps = rng.integers(s_min, s_max + 1, count)
    return [Request(i, float(arrivals[i]), int(ns[i]), int(steps[i]), int(seed * 1_000_003 + i))
            for i in range(count)]


class RangeAllocator:
    """First-fit allocator of aligned half-open ranges in [0, size)."""

    def __init__(self, size: int, align: int = 1):
        self.size, self.align = int(size), int(align)
        self.free = [(0, self.size)]  # sorted, disjoint, coalesced

    def alloc(self, length: int):
        need = (int(length) + self.align - 1) // self.align * self.align
        for k, (a, b) in enumerate(self.free):
            start = (a + self.align - 1) // self.align * self.align
            if start + need <= b:
                pieces = []
                if a < start:
                    pieces.append((a, start))
                if start + need < b:
                    pieces.append((start + need, b))
                self.free[k:k + 1] = pieces
                return start, need
        return None

    def release(self, start: int, length: int):
        self.free.append((start, start + length))
        self.free.sort()
        merged = []
        for a, b in self.free:
            if merged and merged[-1][1] >= a:
                merged[-1] = (merged[-1][0], max(merged[-1][1], b))
            else:
                merged.append((a, b))
        self.free = merged

    def free_total(self) -> int:
        return sum(b - a for a, b in self.free)


@dataclass
class Running:
    req: Request
    slot: int
    agent_off: int
    agent_len: int
    box_off: int
    box_len: int
    left: int


@dataclass
class ServeStats:
    latencies: list = field(default_factory=list)
    agent_updates: int = 0
    wall: float = 0.0
    batch_steps: int = 0
    max_concurrent: int = 0
    failed: list = field(default_factory=list)  # (request id, status bits) of failed requests

    def summary(self):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return dict(requests=len(self.latencies), failed=len(self.failed), agent_updates=self.agent_updates,
                    wall_s=self.wall, agent_updates_per_s=self.agent_updates / max(self.wall, 1e-12),
                    p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
                    batch_steps=self.batch_steps, max_concurrent=self.max_concurrent)


class Server:
    """Packed population of `slots` simulation slots with `capacity` agents in total."""

    def __init__(self, capacity: int, max_boxes: int, slots: int = 64, box=D_HI,
                 use_graph: bool = True, keep_results=False):
        import torch

        from . import bdm
        self.torch, self.bdm = torch, bdm
        self.capacity = (int(capacity) + ALIGN - 1) // ALIGN * ALIGN
        self.max_boxes, self.slots = int(max_boxes), int(slots)
        self.box = box  # one edge for every request, or a tune.BoxPlan (edge per request size)
        self.batch = bdm.Batch(self.capacity, self.max_boxes, self.slots, grid_cap=int(getattr(box, "grid_cap", 0)))
        self.agents = RangeAllocator(self.capacity, ALIGN)
        self.boxes = RangeAllocator(self.max_boxes, bdm.BOX_ALIGN)
        self.free_slots = list(range(self.slots))[::-1]
        self.running: dict[int, Running] = {}
        self.stream = torch.cuda.Stream()
        self.graph = None
        self.use_graph = use_graph
        # True keeps every result on the host; a set of request ids keeps only those
        self.keep_results = keep_results
        self.results: dict[int, dict] = {}

    @staticmethod
    def footprint_bytes(n: int, box: float = D_HI) -> int:
        """HBM a request occupies: packed SoA (68 B/agent) + workspace (118 B/agent) + 4 B/agent
        of margin (bounds partials, alignment) + per reserved box 4 B of box start, 1 B of
        stationary mark and 12 B per bucket of 64 boxes."""
        return int(n * (68 + 118 + 4) + (5 + 12 / 64) * box_reserve(n, box))

    def box_of(self, req: Request) -> float:
        return box_edge(self.box, req.n)

    def fits(self, req: Request) -> bool:
        return req.n <= self.capacity and box_reserve(req.n, self.box_of(req)) <= self.max_boxes

    def try_admit(self, req: Request) -> bool:
        if not self.free_slots:
            return False
        a = self.agents.alloc(req.n)
        if a is None:
            return False
        box = self.box_of(req)
        nb = box_reserve(req.n, box)
        bx = self.boxes.alloc(nb)
        if bx is None:
            self.agents.release(*a)
            return False
        slot = self.free_slots.pop()
        bdm = self.bdm
        with self.torch.cuda.stream(self.stream):
            view = self.batch.view(slot, a[0], req.n)
            bdm.generate(view, bdm.gen(bdm.GEN_CUBE, req.n, cube_edge(req.n), D_LO, D_HI, 0.4, seed=req.seed),
                         stream=self.stream)
            self.batch.set_slot(slot, a[0], req.n, bx[0], bx[1], req.steps, mech_params(box), stream=self.stream)
        self.running[slot] = Running(req, slot, a[0], a[1], bx[0], bx[1], req.steps)
        return True

    def step(self):
        if self.use_graph:
            if self.graph is None:
                self.batch.step(stream=self.stream)  # first launches outside the capture
                self.torch.cuda.current_stream().wait_stream(self.stream)
                self.graph = self.torch.cuda.CUDAGraph()
                with self.torch.cuda.graph(self.graph, stream=self.stream):
                    self.batch.step(stream=self.stream)
                # the capture did not execute: the eager step above was this step's work
                return
            with self.torch.cuda.stream(self.stream):
                self.graph.replay()
        else:
            self.batch.step(stream=self.stream)

    def retire(self, slot: int):
        """Read a finished request back and free its slot.  Returns (request, status bits): a
        slot whose grid build or step met a device condition (bits != 0) did not do its work,
        and its result must not count."""
        r = self.running.pop(slot)
        with self.torch.cuda.stream(self.stream):
            out = self.batch.read_slot(slot, r.agent_off, r.req.n, keys=("x", "y", "z"))
            flags, _ = self.batch.slot_status(slot, stream=self.stream)
            self.batch.clear_slot(slot, r.agent_off, r.req.n, stream=self.stream)
        self.agents.release(r.agent_off, r.agent_len)
        self.boxes.release(r.box_off, r.box_len)
        self.free_slots.append(slot)
        keep = self.keep_results
        if keep is True or (keep and r.req.rid in keep):
            self.results[r.req.rid] = out
        return r, flags

    def run(self, trace, time_scale: float = 1.0) -> ServeStats:
        """Serve `trace` in real time (arrival times multiplied by time_scale)."""
        stats = ServeStats()
        pending = sorted(trace, key=lambda r: r.arrival)
        for r in pending:
            if not self.fits(r):
                raise ValueError(f"request {r.rid} ({r.n} agents) can never fit this server")
        queue: list[Request] = []
        k = 0
        t0 = time.perf_counter()
        while k < len(pending) or queue or self.running:
            now = time.perf_counter() - t0
            while k < len(pending) and pending[k].arrival * time_scale <= now:
                queue.append(pending[k])
                k += 1
            while queue and self.try_admit(queue[0]):  # FIFO admission
                queue.pop(0)
            if not self.running:
                if k < len(pending):
                    wait = pending[k].arrival * time_scale - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(wait)
                continue
            stats.max_concurrent = max(stats.max_concurrent, len(self.running))
            self.step()
            stats.batch_steps += 1
            done = []
            for slot, r in self.running.items():
                r.left -= 1
                if r.left == 0:
                    done.append(slot)
            for slot in done:
                r, flags = self.retire(slot)  # reads results back: synchronises the stream
                if flags:
                    stats.failed.append((r.req.rid, flags))
                    continue
                stats.latencies.append(time.perf_counter() - t0 - r.req.arrival * time_scale)
                stats.agent_updates += r.req.n * r.req.steps
        self.stream.synchronize()
        stats.wall = time.perf_counter() - t0
        return stats


def run_plain(trace, time_scale: float = 1.0, box=D_HI, keep_results=False):
    """Serve the trace one request at a time with plain launches (FIFO, no batching); `box` and
    `keep_results` as for Server."""
    import torch

    from . import bdm
    stats = ServeStats()
    results = {}
    pending = sorted(trace, key=lambda r: r.arrival)
    cap = max(r.n for r in pending)
    pop = bdm.Population(cap, max(box_reserve(r.n, box_edge(box, r.n)) for r in pending))
    t0 = time.perf_counter()
    for r in pending:
        wait = r.arrival * time_scale - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        view = bdm.Soa(r.n, pop.soa.n, pop.soa.x, pop.soa.y, pop.soa.z, pop.soa.diam, pop.soa.adh,
                       pop.soa.fx, pop.soa.fy, pop.soa.fz, pop.soa.id, None)
        bdm.generate(view, bdm.gen(bdm.GEN_CUBE, r.n, cube_edge(r.n), D_LO, D_HI, 0.4, seed=r.seed))
        p = mech_params(box_edge(box, r.n))
        for step in range(r.steps):
            bdm.sim_step(view, bdm.MODEL_MECH, p, step, pop.ws)
        out = {}
        dev = {k: torch.empty(r.n, dtype=torch.float64, device="cuda") for k in ("x", "y", "z")}
        bdm.read_agents(view, dev["x"], dev["y"], dev["z"])
        out = {k: v.cpu().numpy() for k, v in dev.items()}
        flags = bdm.status(pop.ws, clear=True)
        if flags:
            stats.failed.append((r.rid, flags))
            continue
        if keep_results is True or (keep_results and r.rid in keep_results):
            results[r.rid] = out
        stats.latencies.append(time.perf_counter() - t0 - r.arrival * time_scale)
        stats.agent_updates += r.n * r.steps
        stats.batch_steps += r.steps
        stats.max_concurrent = 1
    torch.cuda.synchronize()
    stats.wall = time.perf_counter() - t0
    return stats, results
