"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module only places agents (numpy's own seeded generator, fixed lattices, hand-made edge
cases); it holds none of the method's arithmetic.  The method's own seeded generator (Philox
keyed by seed and agent id) is implemented separately by the oracle and by the GPU library.
"""
from __future__ import annotations

import numpy as np


def uniform_cube(n, L, dmin=10.0, dmax=15.0, adh=0.4, seed=0):
    """n spheres uniform in [0, L)^3, diameters uniform in [dmin, dmax)."""
    r = np.random.default_rng(seed)
    return dict(x=r.uniform(0, L, n), y=r.uniform(0, L, n), z=r.uniform(0, L, n),
                d=r.uniform(dmin, dmax, n), adh=np.full(n, adh))


def cube_side_for(n, density_n=4096, density_L=200.0):
    """Edge of the cube holding n agents at the density of density_n agents in density_L^3."""
    return density_L * (n / density_n) ** (1.0 / 3.0)


def box_face_adversarial(n, b, cells=6, d=None, seed=0):
    """Agents whose coordinates sit exactly on box faces x = m*b (and a few just below/above),
    diameter b (so b is the box edge)."""
    r = np.random.default_rng(seed)
    m = r.integers(0, cells, size=(n, 3)).astype(np.float64)
    pos = m * b
    jitter_kind = r.integers(0, 3, size=(n, 3))
    pos = np.where(jitter_kind == 1, np.nextafter(pos, -np.inf), pos)
    pos = np.where(jitter_kind == 2, np.nextafter(pos, np.inf), pos)
    dd = np.full(n, b if d is None else d)
    dd[0] = b  # the largest diameter fixes the box edge
    return dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), d=dd,
                adh=np.full(n, 0.4))


def lattice(k, spacing, d, origin=0.0, adh=0.4):
    """k^3 spheres on a cubic lattice, x fastest."""
    g = origin + spacing * np.arange(k, dtype=np.float64)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    n = k ** 3
    return dict(x=x.ravel().copy(), y=y.ravel().copy(), z=z.ravel().copy(), d=np.full(n, float(d)),
                adh=np.full(n, adh))


def clustered(n, L, clusters=8, spread=6.0, dmin=8.0, dmax=12.0, seed=0):
    """Strongly non-uniform placement: Gaussian clumps (many agents per box)."""
    r = np.random.default_rng(seed)
    centres = r.uniform(0.2 * L, 0.8 * L, size=(clusters, 3))
    which = r.integers(0, clusters, n)
    pos = centres[which] + r.normal(0.0, spread, size=(n, 3))
    return dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(),
                d=r.uniform(dmin, dmax, n), adh=np.full(n, 0.4))


def sir_uniform(n, L, infected_fraction=0.01, seed=0):
    r = np.random.default_rng(seed)
    st = (r.random(n) < infected_fraction).astype(np.uint8)
    return dict(x=r.uniform(0, L, n), y=r.uniform(0, L, n), z=r.uniform(0, L, n), state=st)


def reach_adversarial(pairs, b=12.0, seed=0):
    """Pairs of spheres across box corners, edges and faces at the edge of the 27-box reach.

    Sphere c has the largest diameter b (it fixes the box edge) and sits just inside the
    neighbour box along a corner, edge or face direction u; sphere a (radius in [b/4, b/2])
    sits at c - dist * u, with dist = (r_a + r_c) (1 -+ 1e-12): even-numbered pairs touch,
    odd-numbered ones miss.  Along u the nearest point of c's box is then almost as far from a
    as the whole reach r_a + b/2.  Pairs are 4 boxes apart, so no two pairs interact."""
    r = np.random.default_rng(seed)
    dirs = (np.array([1.0, 1.0, 1.0]), np.array([1.0, 1.0, 0.0]), np.array([1.0, 0.0, 0.0]))
    xs, ds = [], []
    for k in range(pairs):
        m = np.array([k % 8, (k // 8) % 8, k // 64], dtype=np.float64) * 4.0 + 2.0
        d = dirs[k % 3] * r.choice([-1.0, 1.0], 3)
        perm = r.permutation(3)
        d = d[perm]
        u = d / np.linalg.norm(d)
        # the corner, edge or face point of the lattice, mid-box along the unused axes
        point = np.where(d != 0.0, m * b, (m + 0.5) * b)
        c = point + np.sign(d) * (1e-9 * b)
        ra = r.uniform(0.25 * b, 0.5 * b)
        dist = (ra + 0.5 * b) * (1.0 - 1e-12 if k % 2 == 0 else 1.0 + 1e-12)
        a = c - dist * u
        xs += [a, c]
        ds += [2.0 * ra, b]
    pos = np.array(xs)
    return dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), d=np.array(ds),
                adh=np.full(len(ds), 0.4))


def separated_pairs(npairs, d, separation, spacing=40.0, coincident=0, seed=0):
    """Pairs of equal spheres (diameter d) whose centres lie exactly `separation` apart along x,
    y or z (axis-aligned, so the separation is exact in binary64), the pairs `spacing` apart on a
    jittered lattice; then `coincident` pairs of spheres at one and the same centre."""
    r = np.random.default_rng(seed)
    k = int(np.ceil((npairs + coincident) ** (1.0 / 3.0)))
    cells = np.stack(np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij"), -1)
    cells = cells.reshape(-1, 3)[: npairs + coincident].astype(np.float64)
    base = cells * spacing + np.round(r.uniform(0.0, 4.0, cells.shape) * 64.0) / 64.0
    axis = r.integers(0, 3, npairs + coincident)
    off = np.zeros_like(base)
    off[np.arange(npairs), axis[:npairs]] = separation
    a, b = base, base + off
    pos = np.concatenate([a, b])
    n = len(pos)
    return dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), d=np.full(n, float(d)),
                adh=np.full(n, 0.4))


def touching_lattice(m=8, spacing=2.5, d=10.0, jitter=1e-8, seed=0):
    """A crowded block (m^3 spheres of diameter d on a cubic lattice of `spacing`, d / spacing an
    integer, so every box holds many agents) in which every axis-aligned pair d apart touches
    exactly, up to an x jitter of +-`jitter` per sphere: about half of those pairs overlap by
    about `jitter` and the others miss by as much.  Far below the binary32 copies' rounding, it
    puts many pairs on the contact boundary of every pre-test."""
    r = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    pos = g.astype(np.float64) * spacing + 5.0
    pos[:, 0] += r.choice([-jitter, jitter], len(pos))
    n = len(pos)
    return dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), d=np.full(n, float(d)),
                adh=np.full(n, 0.4))
