"""Seeded synthetic populations that the device generator does not produce (numpy, host side).

Input construction only: positions, shapes and kinds drawn from numpy's Philox stream; the
library computes everything else (grid diameters included).
"""
from __future__ import annotations

import numpy as np

SPHERE, CYLINDER = 0, 1


def neurite_mix(n: int, L: float, sphere_frac: float = 0.2, d=(10.0, 15.0), length=(4.0, 8.0),
                dc=(1.0, 2.0), adh: float = 0.4, seed: int = 0) -> dict:
    """Somata (spheres) and neurite elements (cylinders) in the cube [0, L)^3.

    Each agent's position (a sphere's centre, a cylinder's distal end) is uniform in the cube; a
    fraction `sphere_frac` are spheres of diameter uniform in d, the rest cylinders of length
    uniform in `length`, diameter uniform in `dc` and a direction uniform on the sphere (from
    normal deviates), the proximal end at position - length * direction.  Keys: x, y, z, d (0 for
    a cylinder: the step sets its grid diameter), adh, state (kind: 0 sphere, 1 cylinder), px, py,
    pz (a sphere's own centre), dc (0 for a sphere)."""
    rng = np.random.Generator(np.random.Philox(seed))
    pos = rng.uniform(0.0, L, (n, 3))
    kind = np.where(rng.uniform(0.0, 1.0, n) < sphere_frac, SPHERE, CYLINDER).astype(np.uint8)
    dsph = rng.uniform(d[0], d[1], n)
    ln = rng.uniform(length[0], length[1], n)
    dcyl = rng.uniform(dc[0], dc[1], n)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    prox = pos - ln[:, None] * u
    sph = kind == SPHERE
    prox[sph] = pos[sph]
    return dict(x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy(), d=np.where(sph, dsph, 0.0),
                adh=np.full(n, adh), state=kind, px=prox[:, 0].copy(), py=prox[:, 1].copy(), pz=prox[:, 2].copy(),
                dc=np.where(sph, 0.0, dcyl))
