"""Host-side pieces of bench.py that turn rocprofv3 output into the committed
profile figures: the correlation byte model, the copy-calibrated HBM byte
counts, the SQ instruction summaries and the hash gate on stored traffic.
Synthetic counter files; no GPU."""
import csv
import json

import pytest

import bench

PMC_FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
PASS1 = "void fcmp::rcorr_reg_kernel<true, HIP_vector_type<float, 2u> >(fcmp::RCParams)"
PASS2 = "void fcmp::xrow_kernel<HIP_vector_type<float, 2u>, true, 1>(fcmp::XParams)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=PMC_FIELDS)
        w.writeheader()
        for i, (name, grid, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": grid,
                        "Counter_Name": counter, "Counter_Value": value})


def test_correlation_byte_model():
    """Per correlation: read r (8M) and Omega (4M), write h (8N) in complex64;
    h_0 in FP64: 16M + 4M + 16N.  At N = 65536, M = 16384 a launch pair over
    256 instances is 184,549,376 bytes, the figure the roofline divides."""
    M, N = bench.M, bench.N
    assert bench.corr_bytes(1, 1) == 16 * M + 4 * M + 16 * N
    per_pair = bench.corr_bytes(256, 2) - bench.corr_bytes(256, 1)
    assert per_pair == 256 * (8 * M + 4 * M + 8 * N) == 184_549_376


def test_pmc_copy_calibration_and_medians(tmp_path):
    """Each counter is scaled by (probe bytes) / (what it read for the probe
    copy); per pass the median over the most frequent grid is taken, other
    grids (small launches) are ignored."""
    mib256 = 256 << 20
    fetch_rows = [(COPY, 512, "FETCH_SIZE", mib256 / 2 / 1024)]      # reads half: factor 2
    write_rows = [(COPY, 512, "WRITE_SIZE", mib256 / 1024)]          # reads all: factor 1
    for v in (100.0, 300.0, 200.0):                                  # KiB per dispatch
        fetch_rows.append((PASS1, 1048576, "FETCH_SIZE", v))
        write_rows.append((PASS1, 1048576, "WRITE_SIZE", 2 * v))
        fetch_rows.append((PASS2, 1048576, "FETCH_SIZE", 3 * v))
        write_rows.append((PASS2, 1048576, "WRITE_SIZE", 1.0))
    fetch_rows.append((PASS1, 4096, "FETCH_SIZE", 1e6))              # another grid: ignored
    _write(tmp_path / "f.csv", fetch_rows)
    _write(tmp_path / "w.csv", write_rows)
    out_path = tmp_path / "traffic.json"
    out = bench.summarize_pmc(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(out_path))
    e = out["corr_c64_n65536"]
    assert e["fetch_factor"] == pytest.approx(2.0)
    assert e["write_factor"] == pytest.approx(1.0)
    assert e["pass1_read"] == 200 * 1024 * 2
    assert e["pass1_write"] == 400 * 1024
    assert e["pass2_read"] == 600 * 1024 * 2
    assert e["pass2_write"] == 1024
    assert e["bytes_per_launch"] == 200 * 2048 + 400 * 1024 + 600 * 2048 + 1024
    assert e["kernel_hash"] == bench.kernel_hash()
    assert json.load(open(out_path)) == out
    assert bench.traffic_for("corr_c64_n65536", str(out_path)) == e["bytes_per_launch"]


def test_traffic_gated_by_kernel_hash(tmp_path):
    """Stored traffic taken on other kernel sources is not reported."""
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps({"corr_c64_n65536": {"kernel_hash": "0" * 16, "bytes_per_launch": 5}}))
    assert bench.traffic_for("corr_c64_n65536", str(p)) is None
    assert bench.traffic_for("other_kind", str(p)) is None
    assert bench.traffic_for("corr_c64_n65536", str(tmp_path / "missing.json")) is None


def test_sq_ratios_and_instruction_counts(tmp_path):
    """Ratios to SQ_WAVE_CYCLES and per-dispatch instruction counts are
    medians over the kernel's most frequent grid (at least 10 dispatches);
    the VALU issue time is instructions x 4 cycles over 1024 SIMDs at
    2.4 GHz."""
    rows = []
    for d in range(11):                              # workload grid
        rows.append((d, PASS1, 1048576, [("SQ_WAVE_CYCLES", 100.0 * (d + 1)),
                                         ("SQ_WAIT_ANY", 40.0 * (d + 1)),
                                         ("SQ_INSTS_VALU", 1e6 * (d + 1))]))
    for d in range(11, 13):                          # a smaller grid: ignored
        rows.append((d, PASS1, 4096, [("SQ_WAVE_CYCLES", 1.0), ("SQ_WAIT_ANY", 1.0),
                                      ("SQ_INSTS_VALU", 1.0)]))
    path = tmp_path / "sq.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=PMC_FIELDS)
        w.writeheader()
        for d, name, grid, counters in rows:
            for c, v in counters:
                w.writerow({"Dispatch_Id": d + 1, "Kernel_Name": name, "Grid_Size": grid,
                            "Counter_Name": c, "Counter_Value": v})
    out = bench.summarize_sq(str(path))
    e = out["fcmp::rcorr_reg_kernel<true, HIP_vector_type<float, 2u> >"]
    assert e["grid"] == 1048576 and e["dispatches"] == 11
    assert e["SQ_WAIT_ANY"] == pytest.approx(0.4)
    assert e["SQ_INSTS_VALU"] == pytest.approx(1e4)
    assert e["per_dispatch"] == {"SQ_INSTS_VALU": 6_000_000}
    assert e["valu_issue_us"] == pytest.approx(round(6e6 * 4 / 1024 / 2400, 2))
