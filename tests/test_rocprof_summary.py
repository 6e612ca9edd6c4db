"""Host test of the rocprofv3 summary arithmetic behind `roofline.traffic` and the per-step byte
table: read bytes are 32, 64 and 128 times the L2's read requests of each size, write bytes are
WRITE_SIZE KiB, the first dispatch of a kernel is left out of its mean, and the copy kernel's
check takes only its large dispatches."""
import csv
import json

from paper_2006_06775_amd import rocprof_summary as rs

HEAD = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for r in rows:
            w.writerow(r)


def fixture(tmp_path):
    mech = "void bdm::k_mech<64, bdm::NoTrace, bdm::RecBuf>(...)"
    copy = "__amd_rocclr_copyBufferAligned"
    rd, wr = [], []
    # three mechanics dispatches: the first (dropped) is larger
    for d, (n32, n64, n128, wkib) in enumerate([(8, 8, 1000, 900.0), (2, 4, 100, 50.0), (4, 2, 200, 70.0)], 1):
        # a counter's instances are summed per dispatch: split one count over two rows
        rd += [(d, mech, "TCC_EA0_RDREQ_32B_sum", n32), (d, mech, "TCC_EA0_RDREQ_64B_sum", n64),
               (d, mech, "TCC_EA0_RDREQ_128B_sum", n128 - 1), (d, mech, "TCC_EA0_RDREQ_128B_sum", 1)]
        wr += [(d, mech, "WRITE_SIZE", wkib)]
    # copies: a small one (ignored by the check) and two of 1 MiB in 128-byte reads
    for d, (n128, wkib) in enumerate([(10, 1.0), (8192, 1024.0), (8192, 1024.0)], 10):
        rd += [(d, copy, "TCC_EA0_RDREQ_32B_sum", 0), (d, copy, "TCC_EA0_RDREQ_64B_sum", 0),
               (d, copy, "TCC_EA0_RDREQ_128B_sum", n128)]
        wr += [(d, copy, "WRITE_SIZE", wkib)]
    r, w = tmp_path / "read.csv", tmp_path / "write.csv"
    write_csv(r, rd)
    write_csv(w, wr)
    return str(r), str(w)


def test_bytes_from_request_sizes(tmp_path):
    r, w = fixture(tmp_path)
    tab = rs.dispatch_bytes(r, w)
    mech = next(k for k in tab if "k_mech<64" in k)
    assert tab[mech][0] == [8 * 32 + 8 * 64 + 1000 * 128, 2 * 32 + 4 * 64 + 100 * 128, 4 * 32 + 2 * 64 + 200 * 128]
    assert tab[mech][1] == [900.0 * 1024, 50.0 * 1024, 70.0 * 1024]
    rd, wr = rs.kernel_bytes(tab, "k_mech<64")
    assert rd == ((2 * 32 + 4 * 64 + 100 * 128) + (4 * 32 + 2 * 64 + 200 * 128)) / 2
    assert wr == (50.0 + 70.0) * 1024 / 2
    crd, cwr = rs.kernel_bytes(tab, "copyBuffer", largest=True)
    assert crd == 8192 * 128 and cwr == 1024 * 1024


def test_traffic_json(tmp_path):
    r, w = fixture(tmp_path)
    out = tmp_path / "t.json"
    rs.traffic(r, w, 1000, 1 << 20, str(out))
    t = json.loads(out.read_text())
    assert t["fetch_bytes"] == ((2 * 32 + 4 * 64 + 100 * 128) + (4 * 32 + 2 * 64 + 200 * 128)) / 2
    assert t["bytes_per_launch"] == t["fetch_bytes"] + t["write_bytes"]
    assert t["copy_read_ratio"] == 1.0 and t["copy_write_ratio"] == 1.0
    assert t["source_digest"] == rs.source_digest()


def test_steady_drops_only_a_first_of_several():
    assert rs.steady([5.0]) == [5.0]
    assert rs.steady([9.0, 1.0, 2.0]) == [1.0, 2.0]
