"""Spheroid diameter of a cell population (paper Sec. 3.2: the diameter follows from the volume of
the convex hull that encloses all cells; the equal-volume sphere's diameter, (6 V / pi)^(1/3)).

An observable read between steps, not part of a step.  The O(n) work runs on the device in the
library's two hull calls:

1. `bdm_extreme_points`: for `ndir` directions spread over the sphere, the agent with the largest
   support in each direction.  These agents span a polytope P inside the hull.
2. The host builds P's faces from those few points (Qhull, through scipy).
3. `bdm_hull_candidates`: every agent not strictly inside P by a margin.  Agents strictly inside P
   are not vertices of the hull, so the hull of the candidates is the hull of all agents.
4. The host builds the hull of the candidates (a few percent of the agents for a ball-shaped
   spheroid) and returns the equal-volume diameter.

Only the extreme points and the candidates leave the device.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import bdm


def directions(m: int) -> np.ndarray:
    """m unit vectors on a Fibonacci spiral (row k = (ux, uy, uz))."""
    k = np.arange(m) + 0.5
    polar = np.arccos(1.0 - 2.0 * k / m)
    turn = math.pi * (1.0 + math.sqrt(5.0)) * k
    return np.stack([np.cos(turn) * np.sin(polar), np.sin(turn) * np.sin(polar), np.cos(polar)], axis=1)


def _gather(pop: bdm.Population, slots: torch.Tensor) -> np.ndarray:
    idx = slots.to(torch.int64)
    return torch.stack([pop.t[k].index_select(0, idx) for k in ("x", "y", "z")], dim=1).cpu().numpy()


def _hull_volume(pts: np.ndarray) -> float:
    from scipy.spatial import ConvexHull, QhullError
    if len(pts) < 4:
        return 0.0
    try:
        return float(ConvexHull(pts).volume)
    except QhullError:  # all points in one plane (or fewer than four distinct ones)
        return 0.0


def spheroid_diameter(pop: bdm.Population, ndir: int = 128, tol_rel: float = 1e-9, stats: dict | None = None,
                      stream=None) -> float:
    """Equal-volume diameter of the convex hull of the live agents' centres (0 for fewer than four
    agents or agents in one plane).  `stats`, if given, receives the candidate count."""
    from scipy.spatial import ConvexHull, QhullError
    n = pop.n
    if n < 4:
        return 0.0
    dev = pop.t["x"].device
    dirs = torch.tensor(directions(ndir), dtype=torch.float64, device=dev)
    work = torch.empty(ndir, dtype=torch.int64, device=dev)
    ext = torch.empty(ndir, dtype=torch.int32, device=dev)
    bdm.extreme_points(pop.soa, dirs, work, ext, stream)
    ext = torch.unique(ext)
    pts = _gather(pop, ext)
    try:
        inner = ConvexHull(pts)
        planes = inner.equations  # outward unit normal and offset: n . x + c <= 0 inside
    except QhullError:
        planes = None
    if planes is None or len(planes) > bdm.HULL_MAX_PLANES:
        cand = torch.arange(n, dtype=torch.int32, device=dev)  # flat set: every agent is a candidate
    else:
        # the plane test's rounding is a few ulps of the largest |coordinate| and |offset|
        scale = float(np.abs(pts).max() + np.abs(planes[:, 3]).max()) + 1.0
        pl = torch.tensor(planes, dtype=torch.float64, device=dev)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        cap = min(n, max(4096, n // 8))
        cand = torch.empty(cap, dtype=torch.int32, device=dev)
        bdm.hull_candidates(pop.soa, pl, tol_rel * scale, cand, count, stream)
        m = int(count.item())
        if m > cap:
            cand = torch.empty(m, dtype=torch.int32, device=dev)
            bdm.hull_candidates(pop.soa, pl, tol_rel * scale, cand, count, stream)
        cand = torch.sort(cand[:m]).values
    if stats is not None:
        stats["candidates"] = int(cand.numel())
        stats["extreme"] = int(ext.numel())
    vol = _hull_volume(_gather(pop, cand))
    return (6.0 * vol / math.pi) ** (1.0 / 3.0)
