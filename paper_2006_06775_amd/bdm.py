"""Python binding of libbdm.so (C ABI in include/bdm.h): argument marshalling only.

Every step of the hot path runs in the library's gfx950 kernels; this module only builds the
C structs from torch tensors (device memory) and passes torch's current HIP stream.  There is
no fallback: if libbdm.so is missing or cannot load, importing this module raises.

Function names follow the C entry points without the ``bdm_`` prefix.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field

import torch  # loads the HIP runtime that libbdm.so then binds to (same soname)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbdm.so")

OK, EINVAL, ENOWS, EHIP, ENODEV = 0, -1, -2, -3, -4
(FLAG_CAPACITY, FLAG_BOXES, FLAG_NONFINITE, FLAG_BOXSMALL, FLAG_NOGRID, FLAG_SCAN,
 FLAG_BADCOUNT, FLAG_BADID) = (0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40, 0x80)
MODEL_MECH, MODEL_SPHEROID, MODEL_SIR, MODEL_ONCOLOGY = 0, 1, 2, 3
GEN_CUBE, GEN_BALL, GEN_SIR, GEN_SOMA = 0, 1, 2, 3

# Exported C symbols, in declaration order of include/bdm.h.
SYMBOLS = (
    "bdm_workspace_bytes", "bdm_workspace_init", "bdm_generate", "bdm_grid_build",
    "bdm_mech_step", "bdm_sim_step", "bdm_read_agents", "bdm_status", "bdm_sir_counts",
    "bdm_grid_info", "bdm_grid_export", "bdm_contacts", "bdm_sim_step_traced", "bdm_sim_step_noalloc",
    "bdm_batch_workspace_bytes", "bdm_batch_init", "bdm_batch_set_slot", "bdm_batch_clear_slot",
    "bdm_batch_step", "bdm_batch_step_traced", "bdm_batch_slot_status", "bdm_fp_probe",
    "bdm_extreme_points", "bdm_hull_candidates", "bdm_field_init", "bdm_diffuse", "bdm_soma_step",
    "bdm_geom_step",
    "bdm_strerror", "bdm_last_error",
)
MAX_SLOTS, SLOT_ALIGN, BOX_ALIGN = 4096, 1024, 64


class BdmError(RuntimeError):
    def __init__(self, rc: int, what: str, detail: str = ""):
        super().__init__(f"{what}: {STRERROR.get(rc, rc)} ({rc}) {detail}".strip())
        self.rc = rc


STRERROR = {OK: "ok", EINVAL: "invalid argument", ENOWS: "workspace missing or too small",
            EHIP: "HIP runtime error", ENODEV: "no usable gfx950 device"}


class Soa(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("n", C.c_void_p), ("x", C.c_void_p),
                ("y", C.c_void_p), ("z", C.c_void_p), ("diam", C.c_void_p),
                ("adh", C.c_void_p), ("fx", C.c_void_p), ("fy", C.c_void_p),
                ("fz", C.c_void_p), ("id", C.c_void_p), ("state", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("k", C.c_double), ("gamma", C.c_double), ("dt", C.c_double),
                ("max_disp", C.c_double), ("box", C.c_double), ("force_bits", C.c_int32),
                ("periodic", C.c_int32), ("L", C.c_double), ("r_inf", C.c_double),
                ("p_inf", C.c_double), ("p_rec", C.c_double), ("walk", C.c_double),
                ("grow", C.c_double), ("div_d", C.c_double), ("half_cbrt", C.c_double),
                ("seed", C.c_uint64), ("salt", C.c_uint64), ("skip_static", C.c_int32),
                ("p_apo", C.c_double), ("migrate", C.c_double), ("diff_D", C.c_double),
                ("diff_decay", C.c_double), ("secrete", C.c_double), ("chemo_speed", C.c_double)]


class Gen(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int64), ("L", C.c_double), ("dlo", C.c_double),
                ("dhi", C.c_double), ("adh", C.c_double), ("n_infected", C.c_int64),
                ("seed", C.c_uint64), ("salt", C.c_uint64)]


class Workspace(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("bytes", C.c_size_t), ("capacity", C.c_int64),
                ("max_boxes", C.c_int64)]


class BatchRec(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("bytes", C.c_size_t), ("capacity", C.c_int64),
                ("max_boxes", C.c_int64), ("slots", C.c_int32), ("grid_cap", C.c_int32)]


class FieldRec(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("x0", C.c_double),
                ("y0", C.c_double), ("z0", C.c_double), ("h", C.c_double), ("c", C.c_void_p),
                ("c_next", C.c_void_p), ("count", C.c_void_p)]


class CylRec(C.Structure):
    _fields_ = [("px", C.c_void_p), ("py", C.c_void_p), ("pz", C.c_void_p), ("dc", C.c_void_p)]


class GridDesc(C.Structure):
    _fields_ = [("b", C.c_double), ("cmin", C.c_int32 * 3), ("dims", C.c_int32 * 3),
                ("nboxes", C.c_int64), ("n", C.c_int64), ("valid", C.c_int32),
                ("flags", C.c_uint32), ("skipped", C.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2006_06775_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "bdm_workspace_bytes": ([C.c_int64, C.c_int64], C.c_size_t),
        "bdm_workspace_init": ([P, P], C.c_int),
        "bdm_generate": ([P, P, P], C.c_int),
        "bdm_grid_build": ([P, P, P, P], C.c_int),
        "bdm_mech_step": ([P, P, P, P], C.c_int),
        "bdm_sim_step": ([P, C.c_int32, P, C.c_int64, P, P], C.c_int),
        "bdm_read_agents": ([P] * 10, C.c_int),
        "bdm_status": ([P, P, C.c_int32, P], C.c_int),
        "bdm_sir_counts": ([P, P, P], C.c_int),
        "bdm_grid_info": ([P, P, P], C.c_int),
        "bdm_grid_export": ([P, P, P, P, P], C.c_int),
        "bdm_contacts": ([P, P, P, P, P, P], C.c_int),
        "bdm_sim_step_traced": ([P, C.c_int32, P, C.c_int64, P, P, P, P], C.c_int),
        "bdm_sim_step_noalloc": ([P, C.c_int32, P, C.c_int64, C.c_int64, P, P], C.c_int),
        "bdm_batch_step_traced": ([P, P, P, P, P], C.c_int),
        "bdm_fp_probe": ([P, P, C.c_int64, P, P, P, P, P], C.c_int),
        "bdm_batch_workspace_bytes": ([C.c_int64, C.c_int64, C.c_int32], C.c_size_t),
        "bdm_batch_init": ([P, P], C.c_int),
        "bdm_batch_set_slot": ([P, C.c_int32, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                C.c_int64, P, P], C.c_int),
        "bdm_batch_clear_slot": ([P, C.c_int32, C.c_int64, C.c_int64, P], C.c_int),
        "bdm_batch_step": ([P, P, P], C.c_int),
        "bdm_batch_slot_status": ([P, C.c_int32, P, P, P], C.c_int),
        "bdm_extreme_points": ([P, P, C.c_int32, P, P, P], C.c_int),
        "bdm_hull_candidates": ([P, P, C.c_int32, C.c_double, P, C.c_int64, P, P], C.c_int),
        "bdm_field_init": ([P, P], C.c_int),
        "bdm_diffuse": ([P, P, P], C.c_int),
        "bdm_soma_step": ([P, P, P, P, P], C.c_int),
        "bdm_geom_step": ([P, P, P, P, P, P], C.c_int),
        "bdm_strerror": ([C.c_int], C.c_char_p),
        "bdm_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc: int, what: str):
    if rc != OK:
        raise BdmError(rc, what, _lib.bdm_last_error().decode())


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ref(s):
    return C.byref(s)


# ---------------------------------------------------------------------------------------------
# Parameter records
# ---------------------------------------------------------------------------------------------
def params(k=2.0, gamma=1.0, dt=0.01, max_disp=3.0, box=0.0, force_bits=64, periodic=0, L=0.0,
           r_inf=0.0, p_inf=0.0, p_rec=0.0, walk=0.0, grow=1.05 ** (1.0 / 3.0), div_d=14.0,
           half_cbrt=0.5 ** (1.0 / 3.0), seed=0, salt=0, skip_static=0, p_apo=0.0,
           migrate=0.0, diff_D=0.0, diff_decay=0.0, secrete=0.0, chemo_speed=0.0) -> Params:
    return Params(k, gamma, dt, max_disp, box, force_bits, periodic, L, r_inf, p_inf, p_rec,
                  walk, grow, div_d, half_cbrt, seed, salt, skip_static, p_apo, migrate, diff_D,
                  diff_decay, secrete, chemo_speed)


def gen(kind=GEN_CUBE, n=0, L=200.0, dlo=10.0, dhi=15.0, adh=0.4, n_infected=0, seed=0,
        salt=0) -> Gen:
    return Gen(kind, n, L, dlo, dhi, adh, n_infected, seed, salt)


# ---------------------------------------------------------------------------------------------
# Population: caller-owned device arrays + workspace, allocated with torch
# ---------------------------------------------------------------------------------------------
@dataclass
class Population:
    capacity: int
    max_boxes: int
    spheres: bool = True
    with_state: bool = False
    device: str = "cuda"
    t: dict = field(default_factory=dict)

    def __post_init__(self):
        cap, dev = int(self.capacity), self.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.t["n"] = torch.zeros(1, dtype=torch.int64, device=dev)
        for k in ("x", "y", "z"):
            self.t[k] = torch.zeros(cap, **f64)
        if self.spheres:
            for k in ("diam", "adh", "fx", "fy", "fz"):
                self.t[k] = torch.zeros(cap, **f64)
        self.t["id"] = torch.zeros(cap, dtype=torch.int32, device=dev)
        if self.with_state:
            self.t["state"] = torch.zeros(cap, dtype=torch.uint8, device=dev)
        nbytes = _lib.bdm_workspace_bytes(cap, int(self.max_boxes))
        if nbytes == 0:
            raise BdmError(ENOWS, "workspace_bytes", f"capacity={cap} max_boxes={self.max_boxes}")
        # torch's caching allocator returns 256-byte-aligned (in fact 512) blocks
        self.ws_tensor = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.ws = Workspace(self.ws_tensor.data_ptr(), nbytes, cap, int(self.max_boxes))
        self.soa = Soa(cap, _ptr(self.t["n"]), *(_ptr(self.t.get(k)) for k in
                       ("x", "y", "z", "diam", "adh", "fx", "fy", "fz", "id", "state")))
        workspace_init(self.ws)

    @property
    def n(self) -> int:
        return int(self.t["n"].item())

    def load(self, arrays: dict, ids=None):
        """Copy host/device arrays (id order) into the population; ids default to 0..n-1."""
        n = len(arrays["x"])
        if n > self.capacity:
            raise BdmError(EINVAL, "load", f"{n} agents > capacity {self.capacity}")
        for k, v in arrays.items():
            key = "diam" if k == "d" else k
            if key not in self.t:
                continue
            self.t[key][:n].copy_(torch.as_tensor(v).to(self.t[key].dtype))
        idv = torch.arange(n, dtype=torch.int32) if ids is None else torch.as_tensor(ids)
        self.t["id"][:n].copy_(idv.to(torch.int32))
        self.t["n"].fill_(n)

    def read(self, keys=("x", "y", "z", "diam", "fx", "fy", "fz", "state")) -> dict:
        """Agents in id order, as host numpy arrays."""
        n = self.n
        out = {}
        dev = {}
        for k in keys:
            if k in self.t:
                dev[k] = torch.empty(n, dtype=self.t[k].dtype, device=self.device)
        read_agents(self.soa, dev.get("x"), dev.get("y"), dev.get("z"), dev.get("diam"),
                    dev.get("fx"), dev.get("fy"), dev.get("fz"), dev.get("state"))
        for k, v in dev.items():
            out[k] = v.cpu().numpy()
        return out


# ---------------------------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------------------------
def workspace_bytes(capacity: int, max_boxes: int) -> int:
    return int(_lib.bdm_workspace_bytes(capacity, max_boxes))


def workspace_init(ws: Workspace, stream=None):
    _check(_lib.bdm_workspace_init(_ref(ws), _stream(stream)), "workspace_init")


def generate(soa: Soa, g: Gen, stream=None):
    _check(_lib.bdm_generate(_ref(soa), _ref(g), _stream(stream)), "generate")


def grid_build(soa: Soa, p: Params, ws: Workspace, stream=None):
    _check(_lib.bdm_grid_build(_ref(soa), _ref(p), _ref(ws), _stream(stream)), "grid_build")


def mech_step(soa: Soa, p: Params, ws: Workspace, stream=None):
    _check(_lib.bdm_mech_step(_ref(soa), _ref(p), _ref(ws), _stream(stream)), "mech_step")


def sim_step(soa: Soa, model: int, p: Params, step: int, ws: Workspace, stream=None):
    _check(_lib.bdm_sim_step(_ref(soa), model, _ref(p), step, _ref(ws), _stream(stream)),
           "sim_step")


def read_agents(soa: Soa, x=None, y=None, z=None, diam=None, fx=None, fy=None, fz=None,
                state=None, stream=None):
    _check(_lib.bdm_read_agents(_ref(soa), *(_ptr(t) for t in (x, y, z, diam, fx, fy, fz, state)),
                                _stream(stream)), "read_agents")


def status(ws: Workspace, clear: bool = False, stream=None) -> int:
    f = C.c_uint32(0)
    _check(_lib.bdm_status(_ref(ws), C.byref(f), int(clear), _stream(stream)), "status")
    return int(f.value)


def sir_counts(ws: Workspace, stream=None):
    c = (C.c_int64 * 3)()
    _check(_lib.bdm_sir_counts(_ref(ws), c, _stream(stream)), "sir_counts")
    return [int(v) for v in c]


def grid_info(ws: Workspace, stream=None) -> dict:
    d = GridDesc()
    _check(_lib.bdm_grid_info(_ref(ws), C.byref(d), _stream(stream)), "grid_info")
    return dict(b=d.b, cmin=tuple(d.cmin), dims=tuple(d.dims), nboxes=d.nboxes, n=d.n,
                valid=d.valid, flags=d.flags, skipped=d.skipped)


def grid_export(ws: Workspace, stream=None):
    """(key[n] in input order, order[n] sorted ids, start[nboxes + 1]) as host numpy arrays."""
    info = grid_info(ws, stream)
    n, nb = info["n"], info["nboxes"]
    key = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    order = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    start = torch.empty(nb + 1, dtype=torch.int32, device="cuda")
    _check(_lib.bdm_grid_export(_ref(ws), _ptr(key), _ptr(order), _ptr(start), _stream(stream)),
           "grid_export")
    u32 = lambda t: t.cpu().numpy().view("uint32")  # noqa: E731
    return info, u32(key)[:n], u32(order)[:n], u32(start)


def contacts(ws: Workspace, p: Params, n: int = None, stream=None):
    """Per sorted slot: counts[n], offsets[n], ids[sum] (host numpy); n is the binned count."""
    n = grid_info(ws, stream)["n"]
    counts = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
    _check(_lib.bdm_contacts(_ref(ws), _ref(p), _ptr(counts), None, None, _stream(stream)),
           "contacts")
    c64 = counts[:n].to(torch.int64)
    offsets = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
    if n > 1:
        offsets[1:n] = torch.cumsum(c64, 0)[:-1]
    total = int(c64.sum().item()) if n else 0
    ids = torch.zeros(max(total, 1), dtype=torch.int32, device="cuda")
    _check(_lib.bdm_contacts(_ref(ws), _ref(p), _ptr(counts), _ptr(offsets), _ptr(ids),
                             _stream(stream)), "contacts")
    u32 = lambda t: t.cpu().numpy().view("uint32")  # noqa: E731
    return u32(counts)[:n], offsets[:n].cpu().numpy(), u32(ids)[:total]


def sim_step_traced(soa: Soa, model: int, p: Params, step: int, ws: Workspace, counts, hashes,
                    stream=None):
    """sim_step through the traced kernels; counts/hashes: device int32 tensors of capacity."""
    _check(_lib.bdm_sim_step_traced(_ref(soa), model, _ref(p), step, _ref(ws), _ptr(counts),
                                    _ptr(hashes), _stream(stream)), "sim_step_traced")


NOALLOC_SCRATCH_BYTES = 64 << 20


def sim_step_noalloc(soa: Soa, model: int, p: Params, step: int, max_boxes: int, flags=None,
                     stream=None):
    """sim_step with the library's static device scratch as the workspace; flags: optional device
    int32 tensor of one element that receives the status bits."""
    _check(_lib.bdm_sim_step_noalloc(_ref(soa), model, _ref(p), step, max_boxes, _ptr(flags),
                                     _stream(stream)), "sim_step_noalloc")


HULL_MAX_DIRS, HULL_MAX_PLANES = 256, 1024


def extreme_points(soa: Soa, dirs: torch.Tensor, work: torch.Tensor, out_slot: torch.Tensor, stream=None):
    """dirs: device float64 (ndir, 3); work: device 8-byte tensor of ndir; out_slot: device int32
    of ndir (the smallest slot maximising each direction's support)."""
    dirs = dirs.contiguous()
    ndir = dirs.shape[0]
    if work.numel() < ndir or out_slot.numel() < ndir or work.element_size() != 8:
        raise BdmError(EINVAL, "extreme_points", "work and out_slot need ndir entries")
    _check(_lib.bdm_extreme_points(_ref(soa), _ptr(dirs), ndir, _ptr(work), _ptr(out_slot),
                                   _stream(stream)), "extreme_points")


def hull_candidates(soa: Soa, planes: torch.Tensor, tol: float, out_slot: torch.Tensor,
                    out_count: torch.Tensor, stream=None):
    """planes: device float64 (nplane, 4) rows (nx, ny, nz, c); out_slot: device int32 (its length
    is max_out); out_count: device int64 of one element (the number of candidates)."""
    planes = planes.contiguous()
    _check(_lib.bdm_hull_candidates(_ref(soa), _ptr(planes), planes.shape[0], tol,
                                    _ptr(out_slot), out_slot.numel(), _ptr(out_count), _stream(stream)),
           "hull_candidates")


class Field:
    """Two substances on an nx*ny*nz voxel grid (device tensors c, c_next, count; see bdm_field).
    `step` runs bdm_soma_step and swaps c and c_next; `diffuse` runs bdm_diffuse and swaps."""

    def __init__(self, nx: int, ny: int, nz: int, h: float, origin=(0.0, 0.0, 0.0), device="cuda"):
        V = int(nx) * int(ny) * int(nz)
        self.dims, self.h, self.origin, self.V = (int(nx), int(ny), int(nz)), float(h), tuple(origin), V
        self.c = torch.zeros(2 * V, dtype=torch.float64, device=device)
        self.c_next = torch.zeros(2 * V, dtype=torch.float64, device=device)
        self.count = torch.zeros(2 * V, dtype=torch.int32, device=device)
        field_init(self.rec())

    def rec(self) -> FieldRec:
        return FieldRec(*self.dims, *self.origin, self.h, _ptr(self.c), _ptr(self.c_next), _ptr(self.count))

    def swap(self):
        self.c, self.c_next = self.c_next, self.c

    def load(self, values):
        self.c.copy_(torch.as_tensor(values, dtype=torch.float64))

    def diffuse(self, p: Params, stream=None):
        diffuse(self.rec(), p, stream)
        self.swap()

    def step(self, soa: Soa, p: Params, ws: Workspace, stream=None):
        soma_step(soa, p, self.rec(), ws, stream)
        self.swap()


def field_init(f: FieldRec, stream=None):
    _check(_lib.bdm_field_init(_ref(f), _stream(stream)), "field_init")


def diffuse(f: FieldRec, p: Params, stream=None):
    _check(_lib.bdm_diffuse(_ref(f), _ref(p), _stream(stream)), "diffuse")


def soma_step(soa: Soa, p: Params, f: FieldRec, ws: Workspace, stream=None):
    _check(_lib.bdm_soma_step(_ref(soa), _ref(p), _ref(f), _ref(ws), _stream(stream)), "soma_step")


class Cylinders:
    """Proximal ends and diameters of cylinder agents, by agent id (device tensors of capacity)."""

    def __init__(self, capacity: int, device="cuda"):
        f64 = dict(dtype=torch.float64, device=device)
        self.t = {k: torch.zeros(max(int(capacity), 1), **f64) for k in ("px", "py", "pz", "dc")}

    def load(self, arrays: dict):
        for k, v in self.t.items():
            src = torch.as_tensor(arrays[k], dtype=torch.float64)
            v[:len(src)].copy_(src)

    def rec(self) -> CylRec:
        return CylRec(*(_ptr(self.t[k]) for k in ("px", "py", "pz", "dc")))


def geom_step(soa: Soa, cyl: CylRec, p: Params, ws: Workspace, counts=None, stream=None):
    _check(_lib.bdm_geom_step(_ref(soa), _ref(cyl), _ref(p), _ref(ws), _ptr(counts), _stream(stream)), "geom_step")


def fp_probe(a: torch.Tensor, b: torch.Tensor, stream=None):
    n = a.numel()
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(2)] + \
           [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(2)]
    _check(_lib.bdm_fp_probe(_ptr(a), _ptr(b), n, *(_ptr(o) for o in outs), _stream(stream)),
           "fp_probe")
    return outs


# ---------------------------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------------------------
def batch_workspace_bytes(capacity: int, max_boxes: int, slots: int) -> int:
    return int(_lib.bdm_batch_workspace_bytes(capacity, max_boxes, slots))


def batch_init(b: BatchRec, stream=None):
    _check(_lib.bdm_batch_init(_ref(b), _stream(stream)), "batch_init")


def batch_set_slot(b: BatchRec, slot: int, agent_off: int, capacity: int, box_off: int,
                   max_boxes: int, steps: int, p: Params, stream=None):
    _check(_lib.bdm_batch_set_slot(_ref(b), slot, agent_off, capacity, box_off, max_boxes, steps,
                                   _ref(p), _stream(stream)), "batch_set_slot")


def batch_clear_slot(b: BatchRec, slot: int, agent_off: int, capacity: int, stream=None):
    _check(_lib.bdm_batch_clear_slot(_ref(b), slot, agent_off, capacity, _stream(stream)),
           "batch_clear_slot")


def batch_step(soa: Soa, b: BatchRec, stream=None):
    _check(_lib.bdm_batch_step(_ref(soa), _ref(b), _stream(stream)), "batch_step")


def batch_step_traced(soa: Soa, b: BatchRec, counts, hashes, stream=None):
    _check(_lib.bdm_batch_step_traced(_ref(soa), _ref(b), _ptr(counts), _ptr(hashes),
                                      _stream(stream)), "batch_step_traced")


def batch_slot_status(b: BatchRec, slot: int, stream=None):
    f = C.c_uint32(0)
    left = C.c_int64(0)
    _check(_lib.bdm_batch_slot_status(_ref(b), slot, C.byref(f), C.byref(left), _stream(stream)),
           "batch_slot_status")
    return int(f.value), int(left.value)


class Batch:
    """Packed population of `slots` independent mechanical simulations: caller-owned arrays of
    `capacity` agents, per-slot live counts, and the batch workspace (torch allocations)."""

    FIELDS = ("x", "y", "z", "diam", "adh", "fx", "fy", "fz")

    def __init__(self, capacity: int, max_boxes: int, slots: int, device: str = "cuda", grid_cap: int = 0):
        self.capacity, self.max_boxes, self.slots = int(capacity), int(max_boxes), int(slots)
        self.t = {k: torch.zeros(self.capacity, dtype=torch.float64, device=device)
                  for k in self.FIELDS}
        self.t["id"] = torch.zeros(self.capacity, dtype=torch.int32, device=device)
        self.n = torch.zeros(self.slots, dtype=torch.int64, device=device)
        nbytes = batch_workspace_bytes(self.capacity, self.max_boxes, self.slots)
        if nbytes == 0:
            raise BdmError(ENOWS, "batch_workspace_bytes",
                           f"capacity={capacity} max_boxes={max_boxes} slots={slots}")
        self.ws_tensor = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.rec = BatchRec(self.ws_tensor.data_ptr(), nbytes, self.capacity, self.max_boxes,
                            self.slots, int(grid_cap))
        self.soa = Soa(self.capacity, _ptr(self.n), *(_ptr(self.t[k]) for k in self.FIELDS),
                       _ptr(self.t["id"]), None)
        batch_init(self.rec)

    def view(self, slot: int, agent_off: int, capacity: int) -> Soa:
        """The slot's agent range as a plain population (n points at the slot's count)."""
        def at(k, size):
            return self.t[k].data_ptr() + agent_off * size
        return Soa(capacity, self.n.data_ptr() + 8 * slot, *(at(k, 8) for k in self.FIELDS),
                   at("id", 4), None)

    def set_slot(self, slot, agent_off, capacity, box_off, max_boxes, steps, p: Params, stream=None):
        batch_set_slot(self.rec, slot, agent_off, capacity, box_off, max_boxes, steps, p, stream)

    def clear_slot(self, slot, agent_off, capacity, stream=None):
        batch_clear_slot(self.rec, slot, agent_off, capacity, stream)

    def step(self, stream=None):
        batch_step(self.soa, self.rec, stream)

    def step_traced(self, counts, hashes, stream=None):
        batch_step_traced(self.soa, self.rec, counts, hashes, stream)

    def slot_status(self, slot, stream=None):
        return batch_slot_status(self.rec, slot, stream)

    def read_slot(self, slot: int, agent_off: int, capacity: int, keys=("x", "y", "z", "fx", "fy", "fz")):
        """The slot's agents in id order, as host numpy arrays."""
        v = self.view(slot, agent_off, capacity)
        n = int(self.n[slot].item())
        dev = {k: torch.empty(n, dtype=torch.float64, device=self.n.device) for k in keys}
        read_agents(v, dev.get("x"), dev.get("y"), dev.get("z"), dev.get("diam"), dev.get("fx"),
                    dev.get("fy"), dev.get("fz"), None)
        return {k: t.cpu().numpy() for k, t in dev.items()}


def box_count_hint(L: float, b: float, margin: int = 2) -> int:
    """Boxes of a cubic domain of edge L at box edge b, with `margin` spare layers per axis."""
    per = int(math.floor(L / b)) + 1 + margin
    return per ** 3
