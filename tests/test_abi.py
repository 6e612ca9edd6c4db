"""The C-ABI library loads and exports every entry point include/bdm.h declares; host-side
argument validation returns its documented codes without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bdm.h")
LIB = os.path.join(ROOT, "paper_2006_06775_amd", "libbdm.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bdm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for need in ("bdm_generate", "bdm_grid_build", "bdm_mech_step", "bdm_sim_step",
                 "bdm_workspace_bytes", "bdm_status"):
        assert need in syms


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build libbdm.so first (paper_2006_06775_amd/build.py)"
    lib = C.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_symbol_list_matches_header():
    from paper_2006_06775_amd import bdm
    assert sorted(bdm.SYMBOLS) == declared_symbols()


def test_workspace_bytes_host_only():
    from paper_2006_06775_amd import bdm
    assert bdm.workspace_bytes(-1, 10) == 0
    assert bdm.workspace_bytes(10, -1) == 0
    assert bdm.workspace_bytes(1 << 33, 10) == 0
    a = bdm.workspace_bytes(4096, 3000)
    b = bdm.workspace_bytes(8192, 3000)
    assert 0 < a < b and a % 256 == 0
    # per agent: packed double4 record 32 B, its binary32 copy 16 and 8-byte pre-test record,
    # adherence 8, id 4, key 4, rank 4, bucket item 4, scratch id 4, state 1, division flag and
    # rank 4 + 4 = 93 B; for the stationary skip the moved flag 1 and the last force 24 = 118 B
    # plus one 64-byte bounds partial per 1024 agents and 16 B of skip counts per 256
    assert b - a == 4096 * 118 + 4 * 64 + 16 * 16
    # per box: start 4 B and the stationary-skip mark 1 B, plus bucket count, bucket start and
    # crowded-bucket entry 4 + 4 + 4 per 64 boxes
    c = bdm.workspace_bytes(4096, 3000 + 64 * 1000)
    assert abs((c - a) - 64 * 1000 * (5 + 12 / 64)) <= 4 * 256


def test_validation_without_gpu():
    from paper_2006_06775_amd import bdm
    lib = bdm.lib()
    assert lib.bdm_grid_build(None, None, None, None) == bdm.ENOWS
    ws = bdm.Workspace(256, 10, 100, 100)  # too small
    assert lib.bdm_grid_build(None, None, C.byref(ws), None) == bdm.ENOWS
    assert b"needs" in lib.bdm_last_error()
    assert lib.bdm_generate(None, None, None) == bdm.EINVAL
    soa = bdm.Soa(10, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 0)
    g = bdm.gen(n=11)
    assert lib.bdm_generate(C.byref(soa), C.byref(g), None) == bdm.EINVAL  # n > capacity
    g = bdm.gen(kind=7, n=1)
    assert lib.bdm_generate(C.byref(soa), C.byref(g), None) == bdm.EINVAL
    assert lib.bdm_strerror(bdm.ENOWS) == b"workspace missing or too small"
    assert lib.bdm_fp_probe(None, None, -1, None, None, None, None, None) == bdm.EINVAL
    # the static-scratch step refuses a population beyond its array before touching a device
    big = bdm.Soa(1 << 22, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 0)
    p = bdm.params()
    assert lib.bdm_sim_step_noalloc(C.byref(big), 0, C.byref(p), 0, 1 << 20, None, None) == bdm.ENOWS
    assert b"static scratch" in lib.bdm_last_error()
    assert bdm.workspace_bytes(1 << 22, 1 << 20) > bdm.NOALLOC_SCRATCH_BYTES


def test_batch_work_split_validation_without_gpu():
    """The batch's work split is checked on the host before anything else: 0 (the default
    stride), -1 (one workgroup per tile) or 64..65536 workgroups."""
    from paper_2006_06775_amd import bdm
    lib = bdm.lib()
    nbytes = bdm.batch_workspace_bytes(4096, 10000, 2)
    p = bdm.params()
    for cap, ok in ((0, True), (-1, True), (64, True), (65536, True), (-2, False), (1, False), (63, False),
                    (65537, False)):
        rec = bdm.BatchRec(0x100000000, nbytes, 4096, 10000, 2, cap)
        # slot 2 is outside a batch of two slots: an accepted split gets that far
        rc = lib.bdm_batch_set_slot(C.byref(rec), 2, 0, 1024, 0, 64, 1, C.byref(p), None)
        assert rc == bdm.EINVAL, cap
        msg = lib.bdm_last_error()
        assert (b"grid_cap" in msg) != ok, (cap, msg)


def test_substance_and_hull_validation_without_gpu():
    from paper_2006_06775_amd import bdm
    lib = bdm.lib()
    p = bdm.params(diff_D=100.0, dt=0.01)
    a, b, cnt = C.c_void_p(0x1000), C.c_void_p(0x100000000), C.c_void_p(0x200000000)
    for dims in ((0, 4, 4), (4, 1048561, 1), (1 << 21, 1, 1), (1024, 1024, 1025)):
        f = bdm.FieldRec(*dims, 0.0, 0.0, 0.0, 5.0, a, b, cnt)
        assert lib.bdm_diffuse(C.byref(f), C.byref(p), None) == bdm.EINVAL, dims
    f = bdm.FieldRec(8, 8, 8, 0.0, 0.0, 0.0, 5.0, a, a, cnt)  # c == c_next
    assert lib.bdm_diffuse(C.byref(f), C.byref(p), None) == bdm.EINVAL
    assert b"overlap" in lib.bdm_last_error()
    f = bdm.FieldRec(8, 8, 8, 0.0, 0.0, 0.0, 5.0, a, b, cnt)
    unstable = bdm.params(diff_D=1000.0, dt=0.01)  # D dt / h^2 = 0.4 > 1/6
    assert lib.bdm_diffuse(C.byref(f), C.byref(unstable), None) == bdm.EINVAL
    soa = bdm.Soa(10, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 0)
    assert lib.bdm_extreme_points(C.byref(soa), None, 0, None, None, None) == bdm.EINVAL
    assert lib.bdm_hull_candidates(C.byref(soa), a, 2000, 0.0, None, 0, cnt, None) == bdm.EINVAL
    assert lib.bdm_geom_step(C.byref(soa), None, C.byref(p), None, None, None) == bdm.ENOWS
