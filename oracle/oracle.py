"""ctypes wrapper of the CPU oracle (bdm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline leg
of the benchmark, never by the GPU library or its Python binding.  Arrays are numpy, in agent-id
order (index == id).  Every function mirrors one C entry point; see bdm_oracle.c for the
definitions and the paper passages they follow.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BDM_ORACLE_LIB selects another build of the same source (the sanitizer run of the pins)
LIB_PATH = os.environ.get("BDM_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

OK, EINVAL, ENOMEM, ENONFINITE, ETOOMANYBOXES = 0, -1, -2, -3, -4
RNG_INIT, RNG_MOVE, RNG_REC, RNG_INF, RNG_DIV, RNG_APO, RNG_MIG = 1, 2, 3, 4, 5, 6, 7
SIR_S, SIR_I, SIR_R = 0, 1, 2


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"oracle {what} failed with code {rc}")
        self.rc = rc


class _Grid(C.Structure):
    _fields_ = [("b", C.c_double), ("periodic", C.c_int32), ("L", C.c_double),
                ("cmin", C.c_int64 * 3), ("dims", C.c_int64 * 3), ("nboxes", C.c_int64)]


class _MechParams(C.Structure):
    _fields_ = [("k", C.c_double), ("gamma", C.c_double), ("dt", C.c_double),
                ("max_disp", C.c_double), ("box", C.c_double), ("force_bits", C.c_int32),
                ("max_boxes", C.c_int64)]


class _SpheroidParams(C.Structure):
    _fields_ = [("mech", _MechParams), ("grow", C.c_double), ("div_d", C.c_double),
                ("half_cbrt", C.c_double), ("seed", C.c_uint64), ("salt", C.c_uint64)]


class _OncologyParams(C.Structure):
    _fields_ = [("sph", _SpheroidParams), ("p_apo", C.c_double), ("migrate", C.c_double)]


class _Field(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64), ("x0", C.c_double),
                ("y0", C.c_double), ("z0", C.c_double), ("h", C.c_double)]


class _SomaParams(C.Structure):
    _fields_ = [("mech", _MechParams), ("D", C.c_double), ("decay", C.c_double),
                ("secrete", C.c_double), ("speed", C.c_double)]


class _SirParams(C.Structure):
    _fields_ = [("L", C.c_double), ("box", C.c_double), ("r_inf", C.c_double),
                ("p_inf", C.c_double), ("p_rec", C.c_double), ("walk", C.c_double),
                ("max_boxes", C.c_int64), ("seed", C.c_uint64), ("salt", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build  # noqa: WPS433 (local build step)
            _build.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


_D = C.POINTER(C.c_double)
_U8 = C.POINTER(C.c_uint8)
_U32 = C.POINTER(C.c_uint32)
_U64 = C.POINTER(C.c_uint64)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)


def _declare(L):
    L.orc_philox4x64_10.argtypes = [_U64, _U64, _U64]
    L.orc_philox4x64_10.restype = None
    L.orc_draw.argtypes = [C.c_uint64] * 6 + [_U64]
    L.orc_draw.restype = None
    L.orc_u01.argtypes = [C.c_uint64]
    L.orc_u01.restype = C.c_double
    L.orc_bernoulli.argtypes = [C.c_uint64, C.c_double]
    L.orc_bernoulli.restype = C.c_int
    L.orc_generate_cube.argtypes = [C.c_int64, C.c_uint64, C.c_uint64, C.c_double, C.c_double,
                                    C.c_double, C.c_double, _D, _D, _D, _D, _D]
    L.orc_generate_ball.argtypes = L.orc_generate_cube.argtypes
    L.orc_generate_sir.argtypes = [C.c_int64, C.c_uint64, C.c_uint64, C.c_double, C.c_int64,
                                   _D, _D, _D, _U8]
    L.orc_grid_setup.argtypes = [C.c_int64, _D, _D, _D, _D, C.c_double, C.c_int32, C.c_double,
                                 C.c_int64, C.POINTER(_Grid)]
    L.orc_grid_sort.argtypes = [C.c_int64, _D, _D, _D, C.POINTER(_Grid), _U32, _U32, _U32]
    L.orc_pair_force_f64.argtypes = [C.c_double] * 10 + [_D]
    L.orc_pair_force_f32.argtypes = [C.c_double] * 10 + [_D]
    L.orc_displacement.argtypes = [C.c_double] * 6 + [_D]
    L.orc_mech_step.argtypes = [C.c_int64, _D, _D, _D, _D, _D, C.POINTER(_MechParams), _D, _D,
                                _D, _U32, _U8]
    L.orc_mech_sample.argtypes = [C.c_int64, _D, _D, _D, _D, C.POINTER(_MechParams), C.c_int64, _I64,
                                  _D, _D, _D, _U32]
    L.orc_contacts.argtypes = [C.c_int64, _D, _D, _D, _D, C.c_double, C.c_int32, C.c_double,
                               C.c_double, C.c_int32, C.c_int64, _U32, _I64, _U32]
    L.orc_division_axis.argtypes = [C.c_uint64] * 4 + [_D]
    L.orc_division_axis.restype = None
    L.orc_grow_divide.argtypes = [_I64, C.c_int64, _D, _D, _D, _D, _D,
                                  C.POINTER(_SpheroidParams), C.c_int64, _I32]
    L.orc_spheroid_step.argtypes = [_I64, C.c_int64, _D, _D, _D, _D, _D,
                                    C.POINTER(_SpheroidParams), C.c_int64, _D, _D, _D, _I32]
    L.orc_apoptosis.argtypes = [_I64, _D, _D, _D, _D, _D, C.c_double, C.c_uint64, C.c_uint64,
                                C.c_int64]
    L.orc_migrate.argtypes = [C.c_int64, _D, _D, _D, C.c_double, C.c_uint64, C.c_uint64, C.c_int64]
    L.orc_oncology_step.argtypes = [_I64, C.c_int64, _D, _D, _D, _D, _D,
                                    C.POINTER(_OncologyParams), C.c_int64, _D, _D, _D, _I32]
    _F = C.POINTER(_Field)
    L.orc_diffuse.argtypes = [_F, _D, _D, C.c_double, C.c_double]
    L.orc_diffusion_coefficients.argtypes = [C.c_double] * 4 + [_D]
    L.orc_diffusion_coefficients.restype = None
    L.orc_secrete.argtypes = [_F, C.c_int64, _D, _D, _D, _U8, C.c_double, _D]
    L.orc_chemotaxis.argtypes = [_F, C.c_int64, _D, _D, _D, _U8, _D, C.c_double]
    L.orc_soma_step.argtypes = [C.c_int64, _D, _D, _D, _D, _D, _U8, _F, _D, _D,
                                C.POINTER(_SomaParams), _D, _D, _D]
    _V3 = C.POINTER(C.c_double)
    L.orc_segment_point_param.argtypes = [_V3, _V3, _V3]
    L.orc_segment_point_param.restype = C.c_double
    L.orc_segment_segment_params.argtypes = [_V3, _V3, _V3, _V3, _D, _D]
    L.orc_segment_segment_params.restype = None
    L.orc_cylinder_reach.argtypes = [_V3, _V3, C.c_double]
    L.orc_cylinder_reach.restype = C.c_double
    L.orc_geom_pair.argtypes = [C.c_int, _V3, C.c_double, _V3, C.c_double, C.c_int, _V3, C.c_double, _V3,
                                C.c_double, C.c_double, C.c_double, _D]
    L.orc_geom_step.argtypes = [C.c_int64, _D, _D, _D, _D, _D, _U8, _D, _D, _D, _D, C.POINTER(_MechParams),
                                _D, _D, _D, _U32]
    L.orc_sir_step.argtypes = [C.c_int64, _D, _D, _D, _U8, C.POINTER(_SirParams), C.c_int64, _I64]
    for name in ("orc_generate_cube", "orc_generate_ball", "orc_generate_sir", "orc_grid_setup",
                 "orc_grid_sort", "orc_pair_force_f64", "orc_pair_force_f32", "orc_displacement",
                 "orc_mech_step", "orc_mech_sample", "orc_contacts", "orc_grow_divide", "orc_spheroid_step",
                 "orc_apoptosis", "orc_migrate", "orc_oncology_step", "orc_sir_step", "orc_diffuse",
                 "orc_secrete", "orc_chemotaxis", "orc_soma_step", "orc_geom_pair", "orc_geom_step"):
        getattr(L, name).restype = C.c_int


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


# ---------------------------------------------------------------------------------------------
# RNG
# ---------------------------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c, C.c_uint64), _p(k, C.c_uint64), _p(out, C.c_uint64))
    return out


def draw(seed, salt, purpose, attempt, agent_id, step) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_draw(seed, salt, purpose, attempt, agent_id, step, _p(out, C.c_uint64))
    return out


def u01(w: int) -> float:
    return lib().orc_u01(int(w))


def bernoulli(w: int, p: float) -> bool:
    return bool(lib().orc_bernoulli(int(w), float(p)))


# ---------------------------------------------------------------------------------------------
# Generators
# ---------------------------------------------------------------------------------------------
def _zeros(n, dt=np.float64):
    return np.zeros(max(int(n), 0), dtype=dt)


def generate_cube(n, seed, L, dmin, dmax, adh, salt=0):
    x, y, z, d, a = (_zeros(n) for _ in range(5))
    _check(lib().orc_generate_cube(n, seed, salt, L, dmin, dmax, adh, _p(x, C.c_double),
                                   _p(y, C.c_double), _p(z, C.c_double), _p(d, C.c_double),
                                   _p(a, C.c_double)), "generate_cube")
    return dict(x=x, y=y, z=z, d=d, adh=a)


def generate_ball(n, seed, R, dlo, dhi, adh, salt=0):
    x, y, z, d, a = (_zeros(n) for _ in range(5))
    _check(lib().orc_generate_ball(n, seed, salt, R, dlo, dhi, adh, _p(x, C.c_double),
                                   _p(y, C.c_double), _p(z, C.c_double), _p(d, C.c_double),
                                   _p(a, C.c_double)), "generate_ball")
    return dict(x=x, y=y, z=z, d=d, adh=a)


def generate_sir(n, seed, L, n_infected, salt=0):
    x, y, z = (_zeros(n) for _ in range(3))
    s = _zeros(n, np.uint8)
    _check(lib().orc_generate_sir(n, seed, salt, L, n_infected, _p(x, C.c_double),
                                  _p(y, C.c_double), _p(z, C.c_double), _p(s, C.c_uint8)),
           "generate_sir")
    return dict(x=x, y=y, z=z, state=s)


# ---------------------------------------------------------------------------------------------
# Grid
# ---------------------------------------------------------------------------------------------
def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def grid(x, y, z, d=None, box=0.0, periodic=False, L=0.0, max_boxes=1 << 31):
    """Grid parameters plus keys[n] (id order), order[n] (ids sorted by (key, id)) and
    start[nboxes + 1]."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    d = None if d is None else _f64(d)
    n = len(x)
    g = _Grid()
    _check(lib().orc_grid_setup(n, _p(x, C.c_double), _p(y, C.c_double), _p(z, C.c_double),
                                _p(d, C.c_double), box, int(periodic), L, max_boxes, C.byref(g)),
           "grid_setup")
    key = _zeros(n, np.uint32)
    order = _zeros(n, np.uint32)
    start = np.zeros(g.nboxes + 1, dtype=np.uint32)
    if n:
        _check(lib().orc_grid_sort(n, _p(x, C.c_double), _p(y, C.c_double), _p(z, C.c_double),
                                   C.byref(g), _p(key, C.c_uint32), _p(order, C.c_uint32),
                                   _p(start, C.c_uint32)), "grid_sort")
    info = dict(b=g.b, cmin=tuple(g.cmin), dims=tuple(g.dims), nboxes=g.nboxes)
    return info, key, order, start


# ---------------------------------------------------------------------------------------------
# Mechanics
# ---------------------------------------------------------------------------------------------
def pair_force(pi, di, pj, dj, k=2.0, gamma=1.0, bits=64):
    out = np.zeros(3)
    fn = lib().orc_pair_force_f64 if bits == 64 else lib().orc_pair_force_f32
    hit = fn(*map(float, pi), float(di), *map(float, pj), float(dj), k, gamma, _p(out, C.c_double))
    return bool(hit), out


def displacement(f, adh, dt, max_disp):
    out = np.zeros(3)
    flag = lib().orc_displacement(*map(float, f), adh, dt, max_disp, _p(out, C.c_double))
    return flag, out


def mech_params(k=2.0, gamma=1.0, dt=0.01, max_disp=3.0, box=0.0, force_bits=64,
                max_boxes=1 << 31):
    return _MechParams(k, gamma, dt, max_disp, box, force_bits, max_boxes)


def mech_step(state, k=2.0, gamma=1.0, dt=0.01, max_disp=3.0, box=0.0, force_bits=64,
              max_boxes=1 << 31, with_contacts=False):
    """One mechanical step, in place on state['x'|'y'|'z'].  Returns (fx, fy, fz, ncontact, flags)."""
    for key in ("x", "y", "z", "d", "adh"):
        state[key] = _f64(state[key])
    n = len(state["x"])
    p = mech_params(k, gamma, dt, max_disp, box, force_bits, max_boxes)
    fx, fy, fz = _zeros(n), _zeros(n), _zeros(n)
    nc = _zeros(n, np.uint32)
    fl = _zeros(n, np.uint8)
    _check(lib().orc_mech_step(n, _p(state["x"], C.c_double), _p(state["y"], C.c_double),
                               _p(state["z"], C.c_double), _p(state["d"], C.c_double),
                               _p(state["adh"], C.c_double), C.byref(p), _p(fx, C.c_double),
                               _p(fy, C.c_double), _p(fz, C.c_double), _p(nc, C.c_uint32),
                               _p(fl, C.c_uint8)), "mech_step")
    return fx, fy, fz, nc, fl


def mech_sample(state, ids, k=2.0, gamma=1.0, dt=0.01, max_disp=3.0, box=0.0, force_bits=64,
                max_boxes=1 << 31):
    """Summed (pre-gate) forces and contact counts of the agents `ids` in one mechanical step on
    `state` (not modified), each computed exactly as mech_step does."""
    x, y, z, d = (_f64(state[k_]) for k_ in ("x", "y", "z", "d"))
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    m = len(ids)
    p = mech_params(k, gamma, dt, max_disp, box, force_bits, max_boxes)
    fx, fy, fz = _zeros(m), _zeros(m), _zeros(m)
    nc = _zeros(m, np.uint32)
    _check(lib().orc_mech_sample(len(x), _p(x, C.c_double), _p(y, C.c_double), _p(z, C.c_double),
                                 _p(d, C.c_double), C.byref(p), m, _p(ids, C.c_int64),
                                 _p(fx, C.c_double), _p(fy, C.c_double), _p(fz, C.c_double),
                                 _p(nc, C.c_uint32)), "mech_sample")
    return fx, fy, fz, nc


def contacts(x, y, z, d=None, box=0.0, periodic=False, L=0.0, radius=0.0, force_bits=64,
             max_boxes=1 << 31):
    """Contact lists in canonical order as (counts[n], offsets[n], ids[sum])."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    d = None if d is None else _f64(d)
    n = len(x)
    counts = _zeros(n, np.uint32)
    args = (n, _p(x, C.c_double), _p(y, C.c_double), _p(z, C.c_double), _p(d, C.c_double), box,
            int(periodic), L, radius, force_bits, max_boxes)
    _check(lib().orc_contacts(*args, _p(counts, C.c_uint32), None, None), "contacts")
    offsets = np.zeros(n, dtype=np.int64)
    if n:
        offsets[1:] = np.cumsum(counts.astype(np.int64))[:-1]
    ids = np.zeros(int(counts.sum()), dtype=np.uint32)
    _check(lib().orc_contacts(*args, _p(counts, C.c_uint32), _p(offsets, C.c_int64),
                              _p(ids, C.c_uint32)), "contacts")
    return counts, offsets, ids


# ---------------------------------------------------------------------------------------------
# Spheroid
# ---------------------------------------------------------------------------------------------
def spheroid_params(grow, div_d, half_cbrt, seed, salt=0, **mech):
    return _SpheroidParams(mech_params(**mech), grow, div_d, half_cbrt, seed, salt)


def division_axis(seed, agent_id, step, salt=0):
    out = np.zeros(3)
    lib().orc_division_axis(seed, salt, agent_id, step, _p(out, C.c_double))
    return out


def oncology_params(grow, div_d, half_cbrt, seed, p_apo, migrate, salt=0, **mech):
    return _OncologyParams(spheroid_params(grow, div_d, half_cbrt, seed, salt, **mech), p_apo, migrate)


def hull_diameter(x, y, z) -> float:
    """Spheroid diameter [Sec. 3.2]: the diameter of the sphere whose volume equals that of the
    convex hull of the cell centres, (6 V / pi)^(1/3).  The hull volume is Qhull's (through
    scipy).  Fewer than four points, or points in one plane, give 0."""
    from scipy.spatial import ConvexHull, QhullError
    pts = np.stack([_f64(x), _f64(y), _f64(z)], axis=1)
    if len(pts) < 4:
        return 0.0
    try:
        vol = ConvexHull(pts).volume
    except QhullError:
        return 0.0
    return float((6.0 * vol / np.pi) ** (1.0 / 3.0))


class SpheroidState:
    """Spheroid population with room for `capacity` agents (arrays sized to capacity)."""

    def __init__(self, init: dict, capacity: int):
        n = len(init["x"])
        self.capacity = int(capacity)
        self.n = np.array([n], dtype=np.int64)
        self.arr = {}
        for key in ("x", "y", "z", "d", "adh"):
            a = np.zeros(self.capacity, dtype=np.float64)
            a[:n] = init[key]
            self.arr[key] = a
        self.f = [np.zeros(self.capacity) for _ in range(3)]

    def view(self, key):
        return self.arr[key][: int(self.n[0])]

    def step(self, params: _SpheroidParams, step: int):
        ov = np.zeros(1, dtype=np.int32)
        a = self.arr
        _check(lib().orc_spheroid_step(_p(self.n, C.c_int64), self.capacity,
                                       _p(a["x"], C.c_double), _p(a["y"], C.c_double),
                                       _p(a["z"], C.c_double), _p(a["d"], C.c_double),
                                       _p(a["adh"], C.c_double), C.byref(params), step,
                                       _p(self.f[0], C.c_double), _p(self.f[1], C.c_double),
                                       _p(self.f[2], C.c_double), _p(ov, C.c_int32)),
               "spheroid_step")
        return bool(ov[0])

    def grow_divide(self, params: _SpheroidParams, step: int):
        ov = np.zeros(1, dtype=np.int32)
        a = self.arr
        _check(lib().orc_grow_divide(_p(self.n, C.c_int64), self.capacity,
                                     _p(a["x"], C.c_double), _p(a["y"], C.c_double),
                                     _p(a["z"], C.c_double), _p(a["d"], C.c_double),
                                     _p(a["adh"], C.c_double), C.byref(params), step,
                                     _p(ov, C.c_int32)), "grow_divide")
        return bool(ov[0])


    def oncology_step(self, params: _OncologyParams, step: int):
        ov = np.zeros(1, dtype=np.int32)
        a = self.arr
        _check(lib().orc_oncology_step(_p(self.n, C.c_int64), self.capacity,
                                       _p(a["x"], C.c_double), _p(a["y"], C.c_double),
                                       _p(a["z"], C.c_double), _p(a["d"], C.c_double),
                                       _p(a["adh"], C.c_double), C.byref(params), step,
                                       _p(self.f[0], C.c_double), _p(self.f[1], C.c_double),
                                       _p(self.f[2], C.c_double), _p(ov, C.c_int32)),
               "oncology_step")
        return bool(ov[0])

    def apoptosis(self, p_apo: float, seed: int, step: int, salt: int = 0):
        a = self.arr
        _check(lib().orc_apoptosis(_p(self.n, C.c_int64), _p(a["x"], C.c_double),
                                   _p(a["y"], C.c_double), _p(a["z"], C.c_double),
                                   _p(a["d"], C.c_double), _p(a["adh"], C.c_double), p_apo, seed,
                                   salt, step), "apoptosis")

    def migrate(self, migrate: float, seed: int, step: int, salt: int = 0):
        a = self.arr
        _check(lib().orc_migrate(int(self.n[0]), _p(a["x"], C.c_double), _p(a["y"], C.c_double),
                                 _p(a["z"], C.c_double), migrate, seed, salt, step), "migrate")


# ---------------------------------------------------------------------------------------------
# SIR
# ---------------------------------------------------------------------------------------------
def sir_params(L, box, r_inf, p_inf, p_rec, walk, seed, salt=0, max_boxes=1 << 31):
    return _SirParams(L, box, r_inf, p_inf, p_rec, walk, max_boxes, seed, salt)


def sir_step(state, params: _SirParams, step: int):
    """One SIR step in place on state['x'|'y'|'z'|'state']; returns the S, I, R counts."""
    for key in ("x", "y", "z"):
        state[key] = _f64(state[key])
    state["state"] = np.ascontiguousarray(state["state"], dtype=np.uint8)
    counts = np.zeros(3, dtype=np.int64)
    n = len(state["x"])
    _check(lib().orc_sir_step(n, _p(state["x"], C.c_double), _p(state["y"], C.c_double),
                              _p(state["z"], C.c_double), _p(state["state"], C.c_uint8),
                              C.byref(params), step, _p(counts, C.c_int64)), "sir_step")
    return counts


# ---------------------------------------------------------------------------------------------
# Extracellular substances and soma clustering
# ---------------------------------------------------------------------------------------------
def field(nx, ny, nz, h, x0=0.0, y0=0.0, z0=0.0):
    return _Field(nx, ny, nz, x0, y0, z0, h)


def field_size(f: _Field) -> int:
    return int(f.nx * f.ny * f.nz)


def diffusion_coefficients(D, decay, dt, h):
    out = np.zeros(2)
    lib().orc_diffusion_coefficients(D, decay, dt, h, _p(out, C.c_double))
    return float(out[0]), float(out[1])


def diffuse(f: _Field, c, lam, kdec):
    """One diffusion step of one substance (array of nx*ny*nz, x fastest); returns the new array."""
    c = _f64(c)
    out = np.empty_like(c)
    _check(lib().orc_diffuse(C.byref(f), _p(c, C.c_double), _p(out, C.c_double), lam, kdec), "diffuse")
    return out


def _agents(state):
    for key in ("x", "y", "z"):
        state[key] = _f64(state[key])
    state["state"] = np.ascontiguousarray(state["state"], dtype=np.uint8)
    return len(state["x"])


def secrete(f: _Field, state, q, c):
    """Secretion in place on c (both substances, 2*nx*ny*nz)."""
    n = _agents(state)
    _check(lib().orc_secrete(C.byref(f), n, _p(state["x"], C.c_double), _p(state["y"], C.c_double),
                             _p(state["z"], C.c_double), _p(state["state"], C.c_uint8), q,
                             _p(c, C.c_double)), "secrete")


def chemotaxis(f: _Field, state, c, speed):
    """Chemotaxis in place on state['x'|'y'|'z'] along the substances c."""
    n = _agents(state)
    c = _f64(c)
    _check(lib().orc_chemotaxis(C.byref(f), n, _p(state["x"], C.c_double), _p(state["y"], C.c_double),
                                _p(state["z"], C.c_double), _p(state["state"], C.c_uint8),
                                _p(c, C.c_double), speed), "chemotaxis")


def soma_params(D, decay, secrete, speed, **mech):
    return _SomaParams(mech_params(**mech), D, decay, secrete, speed)


def generate_soma(n, seed, L, dmin, dmax, adh, salt=0):
    """Cells uniform in [0, L)^3 (as generate_cube) with cell type id mod 2 in 'state'."""
    s = generate_cube(n, seed, L, dmin, dmax, adh, salt)
    s["state"] = (np.arange(n) & 1).astype(np.uint8)
    return s


def soma_step(state, f: _Field, c, params: _SomaParams):
    """One soma-clustering step in place on state (x, y, z) and on c (secretion); returns
    (c_next, fx, fy, fz)."""
    n = _agents(state)
    for key in ("d", "adh"):
        state[key] = _f64(state[key])
    c_next = np.empty_like(c)
    fx, fy, fz = _zeros(n), _zeros(n), _zeros(n)
    _check(lib().orc_soma_step(n, _p(state["x"], C.c_double), _p(state["y"], C.c_double),
                               _p(state["z"], C.c_double), _p(state["d"], C.c_double),
                               _p(state["adh"], C.c_double), _p(state["state"], C.c_uint8), C.byref(f),
                               _p(c, C.c_double), _p(c_next, C.c_double), C.byref(params),
                               _p(fx, C.c_double), _p(fy, C.c_double), _p(fz, C.c_double)), "soma_step")
    return c_next, fx, fy, fz


# ---------------------------------------------------------------------------------------------
# Cylinder geometry (neurite elements)
# ---------------------------------------------------------------------------------------------
GEOM_SPHERE, GEOM_CYLINDER = 0, 1


def segment_point_param(p, q, c) -> float:
    p, q, c = (_f64(v) for v in (p, q, c))
    return float(lib().orc_segment_point_param(_p(p, C.c_double), _p(q, C.c_double), _p(c, C.c_double)))


def segment_segment_params(p1, q1, p2, q2):
    a = [_f64(v) for v in (p1, q1, p2, q2)]
    s, t = np.zeros(1), np.zeros(1)
    lib().orc_segment_segment_params(*(_p(v, C.c_double) for v in a), _p(s, C.c_double), _p(t, C.c_double))
    return float(s[0]), float(t[0])


def cylinder_reach(p, q, dc) -> float:
    p, q = _f64(p), _f64(q)
    return float(lib().orc_cylinder_reach(_p(p, C.c_double), _p(q, C.c_double), dc))


def geom_pair(kind_i, xi, di, pi, dci, kind_j, xj, dj, pj, dcj, k=2.0, gamma=1.0):
    """(hit, force on i) between body i and body j."""
    xi, pi, xj, pj = (_f64(v) for v in (xi, pi, xj, pj))
    out = np.zeros(3)
    hit = lib().orc_geom_pair(kind_i, _p(xi, C.c_double), di, _p(pi, C.c_double), dci, kind_j,
                              _p(xj, C.c_double), dj, _p(pj, C.c_double), dcj, k, gamma, _p(out, C.c_double))
    return bool(hit), out


def geom_step(state, k=2.0, gamma=1.0, dt=0.01, max_disp=3.0, box=0.0, max_boxes=1 << 31):
    """One mechanical step of spheres and cylinders, in place on state['x'|'y'|'z'|'d'] (keys
    also 'adh', 'state' = kind, 'px', 'py', 'pz', 'dc').  Returns (fx, fy, fz, ncontact)."""
    for key in ("x", "y", "z", "d", "adh", "px", "py", "pz", "dc"):
        state[key] = _f64(state[key])
    state["state"] = np.ascontiguousarray(state["state"], dtype=np.uint8)
    n = len(state["x"])
    p = mech_params(k, gamma, dt, max_disp, box, 64, max_boxes)
    fx, fy, fz = _zeros(n), _zeros(n), _zeros(n)
    nc = _zeros(n, np.uint32)
    _check(lib().orc_geom_step(n, *(_p(state[k_], C.c_double) for k_ in ("x", "y", "z", "d", "adh")),
                               _p(state["state"], C.c_uint8),
                               *(_p(state[k_], C.c_double) for k_ in ("px", "py", "pz", "dc")), C.byref(p),
                               _p(fx, C.c_double), _p(fy, C.c_double), _p(fz, C.c_double), _p(nc, C.c_uint32)),
           "geom_step")
    return fx, fy, fz, nc
