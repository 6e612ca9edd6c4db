#!/usr/bin/env python3
"""Throughput of the mechanical hot path on one MI355X.

Workload: 2^24 spheres uniform in a 3200 um cube (the density of 4096 agents in a 200 um cube),
diameters uniform in [8, 12) um, adherence 0.4, k = 2, gamma = 1, dt = 0.01, clamp 3 um, box
edge = largest diameter, grid rebuilt every step.  One timed step = one full pass of the hot
path over all agents: grid build (bounds, key/histogram, scan, scatter, canonical order) then
the mechanical step (27-box gather, pair force, gate, clamp, integrate), in binary64.

Prints ONE JSON line: agent-updates/s of the whole step (value), per-phase times, the
dominant kernel's roofline (algorithmic bytes / measured kernel time against 8 TB/s), the same
run with binary32 pair forces and its position difference, and the single-thread CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
N_DEFAULT = 1 << 24


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N_DEFAULT, help="agents (default 2^24)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the binary32-force run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 22,
                    help="agents in the oracle's bounded sample (same density)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_mech_fp64_n16m.json"),
                    help="HBM bytes per mech_step launch from rocprofv3 counters (optional)")
    ap.add_argument("--no-serve", action="store_true", help="skip the batched/served stream")
    ap.add_argument("--no-skip", action="store_true", help="skip the stationary-skip comparison")
    ap.add_argument("--no-workloads", action="store_true", help="skip the other workloads (spheroid, oncology, soma clustering, SIR)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-budget-gib", type=float, default=4.0,
                    help="HBM the server may hold for resident simulations")
    return ap.parse_args()


def cube_edge(n):
    return 200.0 * (n / 4096.0) ** (1.0 / 3.0)


def run_variant(bdm, torch, n, L, steps, warmup, force_bits):
    """Generate, warm up, then time `steps` full steps.  Returns timings and the population."""
    b_guess = 11.9
    max_boxes = bdm.box_count_hint(L, b_guess, margin=3)
    pop = bdm.Population(n, max_boxes)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, L, 8.0, 12.0, 0.4, seed=0))
    p = bdm.params(k=2.0, gamma=1.0, dt=0.01, max_disp=3.0, box=0.0, force_bits=force_bits)
    stream = torch.cuda.current_stream()
    for step in range(warmup):
        bdm.grid_build(pop.soa, p, pop.ws)
        bdm.mech_step(pop.soa, p, pop.ws)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(steps):
        e0, e1, e2 = ev[step]
        e0.record(stream)
        bdm.grid_build(pop.soa, p, pop.ws)
        e1.record(stream)
        bdm.mech_step(pop.soa, p, pop.ws)
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    grid_ms = sum(a.elapsed_time(b) for a, b, _ in ev) / steps
    mech_ms = sum(b.elapsed_time(c) for _, b, c in ev) / steps
    flags = bdm.status(pop.ws)
    info = bdm.grid_info(pop.ws)
    return dict(wall=wall, grid_ms=grid_ms, mech_ms=mech_ms, flags=flags, info=info, pop=pop)


def stationary_skip(bdm, torch, n, L, relax=24, steps=20, dt=0.3):
    """The stationary-region skip (paper Sec. 2.3 (iv)) on the mechanics workload as it relaxes:
    dt 0.3 (30 times the benchmark's), `relax` timed steps while agents come to rest (each
    followed by a read of the skipped count), then `steps` timed steps, then `steps` more timed one
    by one, once without and once with the skip, from the same seed; the two end states must be
    bit-identical."""
    out, ends = {}, {}
    for skip in (0, 1):
        pop = bdm.Population(n, bdm.box_count_hint(L, 11.9, 3))
        bdm.generate(pop.soa, bdm.gen(bdm.GEN_CUBE, n, L, 8.0, 12.0, 0.4, seed=0))
        p = bdm.params(k=2.0, gamma=1.0, dt=dt, max_disp=3.0, box=0.0, force_bits=64, skip_static=skip)
        skipped = []

        def relaxing(step):
            bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, step, pop.ws)
            skipped.append(bdm.grid_info(pop.ws)["skipped"])  # (synchronises: a few us per step)
        t_relax = timed_steps(torch, relaxing, relax)

        def one(step):
            bdm.sim_step(pop.soa, bdm.MODEL_MECH, p, relax + step, pop.ws)
        t = timed_steps(torch, one, steps)
        per_step = timed_each(torch, lambda step: one(steps + step), steps)
        info = bdm.grid_info(pop.ws)
        out["skip" if skip else "plain"] = dict(ms_per_step=round(t * 1e3 / steps, 4),
                                                agent_updates_per_s=n * steps / t,
                                                relaxing_ms_per_step=round(t_relax * 1e3 / relax, 4),
                                                skipped_per_relaxing_step=skipped,
                                                ms_each_of_next_steps=per_step,
                                                skipped_last_step=info["skipped"], flags=info["flags"])
        ends[skip] = pop.read(("x", "y", "z", "fx", "fy", "fz"))  # after relax + 2 * steps steps
        del pop
        torch.cuda.empty_cache()
    same = all(np.array_equal(ends[0][k].view(np.uint64), ends[1][k].view(np.uint64)) for k in ends[0])
    out.update(dt=dt, relax_steps=relax, timed_steps=steps, bit_identical=same,
               speedup=out["plain"]["ms_per_step"] / out["skip"]["ms_per_step"],
               relaxing_speedup=out["plain"]["relaxing_ms_per_step"] / out["skip"]["relaxing_ms_per_step"],
               skipped_fraction_last_step=out["skip"]["skipped_last_step"] / n)
    return out


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def measured_traffic(path, n):
    """HBM bytes per mech_step launch from the rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None
    when there is none for this size or the kernel source changed since it was taken."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    from paper_2006_06775_amd.rocprof_summary import source_digest
    if t.get("n") != n or t.get("source_digest") != source_digest():
        return None
    return t.get("bytes_per_launch")


def serving(args):
    """Stream of independent simulations (n log-uniform in [1e3, 2e6], 10-100 steps, binary32
    pair forces): continuous batching vs one-at-a-time plain launches, as a closed system
    (every request present at t = 0: capacity) and as a Poisson stream at 0.8 x the batched
    capacity (latency at the same offered load)."""
    import torch

    from paper_2006_06775_amd import serve, tune
    plan = tune.plan()  # box edge per request size, measured on this device
    per_agent = 68 + 118 + 4
    cap = int(args.serve_budget_gib * (1 << 30) / (per_agent + (5 + 12 / 64) * 1.6))
    boxes = int(cap * 1.6)
    slots = 64
    # closed-system calibration: every request present at t = 0
    calib = serve.make_trace(args.serve_requests, seed=0, rate=1e9)
    srv = serve.Server(cap, boxes, slots, box=plan)
    c = srv.run(calib).summary()
    del srv
    torch.cuda.empty_cache()
    rate = 0.8 * c["requests"] / c["wall_s"]
    trace = serve.make_trace(args.serve_requests, seed=0, rate=rate)
    # a seeded sample of the requests is kept from both forms and compared bit for bit
    sample = set(int(i) for i in np.random.default_rng(7).choice(len(trace), 16, replace=False))
    srv = serve.Server(cap, boxes, slots, box=plan, keep_results=sample)
    b = srv.run(trace).summary()
    served = srv.results
    del srv
    torch.cuda.empty_cache()
    p_stats, alone = serve.run_plain(trace, box=plan, keep_results=sample)
    p = p_stats.summary()
    pc_stats, _ = serve.run_plain(calib, box=plan)  # plain capacity: the same closed system
    pc = pc_stats.summary()
    failed = {"batched_stream": b["failed"], "plain_stream": p["failed"], "batched_closed": c["failed"],
              "plain_closed": pc["failed"]}
    if any(failed.values()):
        raise SystemExit(f"served requests failed on the device: {failed}")
    equal = sum(all(np.array_equal(served[r][k].view(np.uint64), alone[r][k].view(np.uint64)) for k in "xyz")
                for r in sample)
    if equal != len(sample):
        raise SystemExit(f"served results differ from plain launches: {equal}/{len(sample)} bit-equal")
    return {
        "requests": args.serve_requests, "arrival_rate_per_s": rate, "slots": slots,
        "box_plan": plan.summary(),
        "hbm_budget_gib": args.serve_budget_gib, "force_precision": "fp32 pair law, fp64 positions",
        "batched": {k: b[k] for k in ("agent_updates_per_s", "p50_latency_s", "p99_latency_s", "wall_s",
                                      "batch_steps", "max_concurrent")},
        "plain": {k: p[k] for k in ("agent_updates_per_s", "p50_latency_s", "p99_latency_s", "wall_s")},
        "batched_over_plain": b["agent_updates_per_s"] / p["agent_updates_per_s"],
        "closed_system": {
            "batched": {k: c[k] for k in ("agent_updates_per_s", "wall_s", "p50_latency_s", "p99_latency_s")},
            "plain": {k: pc[k] for k in ("agent_updates_per_s", "wall_s", "p50_latency_s", "p99_latency_s")},
            "batched_over_plain": c["agent_updates_per_s"] / pc["agent_updates_per_s"],
        },
        "agent_updates": b["agent_updates"],
        "failed_requests": failed,
        "served_equal_to_plain": {"sampled_requests": len(sample), "bit_equal": equal},
    }


def timed_steps(torch, fn, steps):
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for step in range(steps):
        fn(step)
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) * 1e-3


def timed_each(torch, fn, steps):
    """Milliseconds of each of `steps` calls, from HIP events around each (one sync at the end)."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for step in range(steps):
        ev[step][0].record()
        fn(step)
        ev[step][1].record()
    torch.cuda.synchronize()
    return [round(a.elapsed_time(b), 4) for a, b in ev]


def workloads():
    """The other workloads on the same grid, at their full sizes: the tumour spheroid (60
    steps, and on to about 4e6 cells) and the SIR epidemic."""
    import torch

    from paper_2006_06775_amd import bdm
    out = {}
    # tumour spheroid: 10^4 cells in a 60 um ball, +5 % volume per step, division at 14 um,
    # 60 steps (about 2e5 cells at the end), binary64
    h, g = 0.5 ** (1 / 3), 1.05 ** (1 / 3)
    steps = 60
    pop = bdm.Population(300_000, 1 << 22)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_BALL, 10_000, 60.0, 14.0 * h, 14.0, 0.4, seed=0))
    p = bdm.params(grow=g, div_d=14.0, half_cbrt=h, seed=0)

    def sph(step):
        bdm.sim_step(pop.soa, bdm.MODEL_SPHEROID, p, step, pop.ws)
    t = timed_steps(torch, sph, steps)
    n_end = pop.n
    flags = bdm.status(pop.ws)
    del pop
    out["spheroid"] = dict(cells_start=10_000, cells_end=n_end, steps=steps, seconds=t,
                           steps_per_s=steps / t, flags=flags, precision="fp64")
    torch.cuda.empty_cache()
    # the same growth run on to about 4e6 cells (122 steps); the live count of every step is
    # copied on the device, so the run never waits for the host
    steps = 122
    pop = bdm.Population(5_000_000, 1 << 24)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_BALL, 10_000, 60.0, 14.0 * h, 14.0, 0.4, seed=0))
    counts = torch.zeros(steps, dtype=torch.int64, device="cuda")

    def sph4m(step):
        bdm.sim_step(pop.soa, bdm.MODEL_SPHEROID, p, step, pop.ws)
        counts[step:step + 1].copy_(pop.t["n"])
    t = timed_steps(torch, sph4m, steps)
    updates = int(counts.sum().item())
    out["spheroid_4m"] = dict(cells_start=10_000, cells_end=pop.n, steps=steps, seconds=t,
                              steps_per_s=steps / t, agent_updates_per_s=updates / t,
                              flags=bdm.status(pop.ws), precision="fp64")
    del pop, counts
    torch.cuda.empty_cache()
    # tumour spheroid with apoptosis and Brownian migration: the same 10^4 cells, 1 % death
    # chance per step, migration up to 1 um per axis and step, 60 steps; the spheroid diameter
    # (equal-volume sphere of the hull of the centres) before and after
    from paper_2006_06775_amd import observe
    steps = 60
    pop = bdm.Population(300_000, 1 << 22)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_BALL, 10_000, 60.0, 14.0 * h, 14.0, 0.4, seed=0))
    p_onc = bdm.params(grow=g, div_d=14.0, half_cbrt=h, seed=0, p_apo=0.01, migrate=1.0)
    d_start = observe.spheroid_diameter(pop)
    counts = torch.zeros(steps, dtype=torch.int64, device="cuda")

    def onc(step):
        bdm.sim_step(pop.soa, bdm.MODEL_ONCOLOGY, p_onc, step, pop.ws)
        counts[step:step + 1].copy_(pop.t["n"])
    t = timed_steps(torch, onc, steps)
    updates = int(counts.sum().item())
    stats = {}
    t0 = time.perf_counter()
    d_end = observe.spheroid_diameter(pop, stats=stats)
    t_obs = time.perf_counter() - t0
    out["oncology"] = dict(cells_start=10_000, cells_end=pop.n, steps=steps, seconds=t, steps_per_s=steps / t,
                           agent_updates_per_s=updates / t, p_apo=0.01, migrate_um=1.0,
                           diameter_um_start=round(d_start, 3), diameter_um_end=round(d_end, 3),
                           diameter_seconds=round(t_obs, 4), hull_candidates=stats.get("candidates"),
                           flags=bdm.status(pop.ws), precision="fp64")
    del pop, counts
    torch.cuda.empty_cache()
    # soma clustering: 2^21 cells of two types in a 1600 um cube (C0's density, d in [10, 15)),
    # each type secreting its own substance on 320^3 voxels of 5 um; per step secretion (1 per
    # cell), diffusion (D 250 um^2 per unit time, decay 0.1, dt 0.01: lam 0.1), chemotaxis
    # (0.1 um per step), grid and binary64 mechanics
    n, L = 1 << 21, 1600.0
    steps = 20
    pop = bdm.Population(n, bdm.box_count_hint(L, 14.9, 3), with_state=True)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_SOMA, n, L, 10.0, 15.0, 0.4, seed=0))
    fld = bdm.Field(320, 320, 320, 5.0)
    p_soma = bdm.params(diff_D=250.0, diff_decay=0.1, secrete=1.0, chemo_speed=0.1)
    fld.step(pop.soa, p_soma, pop.ws)  # warm-up (and box-sorted order)

    def soma(step):
        fld.step(pop.soa, p_soma, pop.ws)
    t = timed_steps(torch, soma, steps)
    flags = bdm.status(pop.ws)

    def diff_only(step):
        fld.diffuse(p_soma)
    t_diff = timed_steps(torch, diff_only, steps) / steps
    voxels = 2 * fld.V
    diff_gbps = voxels * 16 / t_diff / 1e9  # one binary64 read and one write per voxel
    out["soma_clustering"] = dict(
        cells=n, voxels=voxels, steps=steps, seconds=t, steps_per_s=steps / t, agent_updates_per_s=n * steps / t,
        flags=flags, precision="fp64",
        diffusion=dict(ms_per_launch=round(t_diff * 1e3, 4), voxel_updates_per_s=voxels / t_diff,
                       roofline=dict(bound="hbm", achieved=round(diff_gbps, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                                     frac=round(diff_gbps / HBM_PEAK_GBPS, 4), bytes_per_voxel=16,
                                     scope="k_diffuse, both substances, one launch")))
    del pop, fld
    torch.cuda.empty_cache()
    # spheres and cylinders (neurite elements): 2^20 agents, 20 % spheres d in [10, 15), 80 %
    # cylinders of length [4, 8) and diameter [1, 2), in an 800 um cube; binary64 law
    from paper_2006_06775_amd import synth
    n = 1 << 20
    s = synth.neurite_mix(n, 800.0, seed=0)
    pop = bdm.Population(n, 1 << 22, with_state=True)
    pop.load({k: s[k] for k in ("x", "y", "z", "d", "adh", "state")})
    cyl = bdm.Cylinders(n)
    cyl.load(s)
    del s
    crec, p_geom = cyl.rec(), bdm.params()
    counts = torch.zeros(n, dtype=torch.int32, device="cuda")
    bdm.geom_step(pop.soa, crec, p_geom, pop.ws, counts)  # warm-up (and box-sorted order)
    contacts = int(counts.sum().item())

    def geom(step):
        bdm.geom_step(pop.soa, crec, p_geom, pop.ws)
    steps = 20
    t = timed_steps(torch, geom, steps)
    out["neurites"] = dict(agents=n, cylinders_fraction=0.8, steps=steps, seconds=t, steps_per_s=steps / t,
                           agent_updates_per_s=n * steps / t, contacts_per_agent=round(contacts / n, 3),
                           flags=bdm.status(pop.ws), precision="fp64")
    del pop, cyl, counts
    torch.cuda.empty_cache()
    # SIR: 10^7 points in a periodic 5000^3 cube, box 20 (250^3 boxes), radius 2, p_inf 0.3,
    # p_rec 0.01, walk 1, 0.1 % infected, 200 steps
    n, L, steps = 10_000_000, 5000.0, 200
    pop = bdm.Population(n, 250 ** 3, spheres=False, with_state=True)
    bdm.generate(pop.soa, bdm.gen(bdm.GEN_SIR, n, L, n_infected=n // 1000, seed=0))
    p = bdm.params(box=20.0, periodic=1, L=L, r_inf=2.0, p_inf=0.3, p_rec=0.01, walk=1.0, seed=0)

    def sir(step):
        bdm.sim_step(pop.soa, bdm.MODEL_SIR, p, step, pop.ws)
    t = timed_steps(torch, sir, steps)
    nboxes = bdm.grid_info(pop.ws)["nboxes"]
    # algorithmic bytes of one SIR step per agent: keys (read x, y, z 24, write key 4), sort
    # (read key, x, y, z, state, id 33; write the sorted record x, y, z, state, id 29), the
    # step (read the record 29, write x, y, z, state, id 29) and the box starts 4 (B + 1) / N
    sir_bytes = n * (24 + 4 + 33 + 29 + 29 + 29) + 4.0 * (nboxes + 1)
    gbps = sir_bytes * steps / t / 1e9
    out["sir"] = dict(agents=n, steps=steps, seconds=t, agent_updates_per_s=n * steps / t,
                      final_SIR=bdm.sir_counts(pop.ws), flags=bdm.status(pop.ws),
                      roofline=dict(bound="hbm", achieved=round(gbps, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                                    frac=round(gbps / HBM_PEAK_GBPS, 4),
                                    algorithmic_bytes_per_step=int(sir_bytes),
                                    scope="whole step: periodic grid build + SIR kernels"))
    del pop
    torch.cuda.empty_cache()
    return out


def host_cpu():
    """Model, clock and core counts of the host this runs on (from /proc/cpuinfo)."""
    model, mhz = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("cpu MHz") and mhz is None:
                    mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(model=model, mhz=mhz, nproc=usable, logical_cpus=os.cpu_count())


def cpu_baseline(n_sample):
    """Single-thread oracle: one mechanical step (grid + forces + move) of n_sample agents at
    the workload's density."""
    from oracle import oracle as orc
    L = cube_edge(n_sample)
    s = orc.generate_cube(n_sample, 0, L, 8.0, 12.0, 0.4)
    t0 = time.perf_counter()
    orc.mech_step(s, k=2.0, gamma=1.0, dt=0.01, max_disp=3.0)
    dt = time.perf_counter() - t0
    return dict(value=n_sample / dt, unit="agent-updates/s", cores=1, kind="oracle",
                host=host_cpu(),
                sample=f"one mechanical step (grid build + forces + move, binary64) of "
                       f"{n_sample} agents at the benchmark's density (cube edge {L:.1f} um), "
                       f"single thread, {dt:.1f} s")


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2006_06775_amd import bdm

    torch.cuda.set_device(0)
    n, L = args.n, cube_edge(args.n)
    r64 = run_variant(bdm, torch, n, L, args.steps, args.warmup, 64)
    if r64["flags"]:
        print(f"device status flags {r64['flags']:#x}", file=sys.stderr)
        sys.exit(1)
    ms_step = r64["wall"] * 1e3 / args.steps
    value = n * args.steps / r64["wall"]
    nboxes = r64["info"]["nboxes"]

    # dominant-kernel roofline: the mechanical step's algorithmic traffic per agent-update is
    # read x, y, z, d, adh (40 B) + box starts (4 (B + 1) / N) + write forces (24) and
    # positions (24)
    mech_bytes = n * (40.0 + 24.0 + 24.0) + 4.0 * (nboxes + 1)
    mech_gbps = mech_bytes / (r64["mech_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(args.traffic_json, n)
    roofline = dict(bound="hbm", kernel="k_mech<binary64>", achieved=round(mech_gbps, 1),
                    peak=HBM_PEAK_GBPS, unit="GB/s", frac=round(mech_gbps / HBM_PEAK_GBPS, 4),
                    traffic=traffic, algorithmic_bytes_per_launch=int(mech_bytes),
                    launch_ms=round(r64["mech_ms"], 4))
    fp32 = None
    if not args.no_fp32:
        r32 = run_variant(bdm, torch, n, L, args.steps, args.warmup, 32)
        # position difference vs the binary64 path after the same steps (the binary64 path is
        # bit-identical to the oracle in the parity tests)
        a, b = r32["pop"].read(("x", "y", "z")), r64["pop"].read(("x", "y", "z"))
        err = max(float(abs(a[k] - b[k]).max()) for k in ("x", "y", "z"))
        fp32 = dict(value=n * args.steps / r32["wall"], ms_per_step=r32["wall"] * 1e3 / args.steps,
                    grid_ms=round(r32["grid_ms"], 4), mech_ms=round(r32["mech_ms"], 4),
                    max_pos_diff_vs_fp64_um=err, max_pos_diff_rel_L=err / L,
                    steps_compared=args.warmup + args.steps, flags=r32["flags"])
        del r32, a, b
    del r64["pop"]
    torch.cuda.empty_cache()

    skip = None if args.no_skip else stationary_skip(bdm, torch, n, L)
    served = None if args.no_serve else serving(args)
    other = None if args.no_workloads else workloads()
    copy_gbps = copy_bandwidth(torch)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_sample)
    out = {
        "metric": "agent-updates/sec in mech_step",
        "value": value,
        "unit": "agent-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"mechanics, {n} spheres in a {L:.0f} um cube, d in [8,12) um, "
                               f"grid rebuilt every step", "n_agents": n, "cube_edge_um": L,
                   "boxes": nboxes, "box_edge_um": r64["info"]["b"], "force_precision": "fp64",
                   "step": "grid_build + mech_step"},
        "phases_ms": {"grid_build": round(r64["grid_ms"], 4), "mech_step": round(r64["mech_ms"], 4)},
        "mech_step_only_agent_updates_per_s": n / (r64["mech_ms"] * 1e-3),
        "roofline": roofline,
        "fp32_forces": fp32,
        "stationary_skip": skip,
        "served_stream": served,
        "other_workloads": other,
        "copy_kernel_GBps": round(copy_gbps, 1),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
