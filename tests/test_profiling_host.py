"""Host-side checks of the rocprofv3 summarisers (synthetic CSV files)."""
import csv

import pytest

from paper_2606_29129_amd import profiling


def _write(path, header, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


K3 = "void oz2::k3_gemm_i8<256, 256, 128, 0>(signed char const*, ...)"
COPY = ("void at::native::vectorized_elementwise_kernel<4, at::native::AbsFunctor<double>, "
        "std::array<char*, 2ul> >(int, at::native::AbsFunctor<double>, std::array<char*, 2ul>)")
HDR = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def test_traffic_scaling(tmp_path):
    # two K3 dispatches (one split over two rows), one copy of 1 MiB read as 2 MiB
    _write(tmp_path / "f" / "host" / "1_counter_collection.csv", HDR, [
        [1, COPY, "FETCH_SIZE", 2048.0],
        [2, K3, "FETCH_SIZE", 1000.0], [2, K3, "FETCH_SIZE", 1000.0],
        [3, K3, "FETCH_SIZE", 4000.0],
    ])
    _write(tmp_path / "w" / "host" / "1_counter_collection.csv", HDR, [
        [1, COPY, "WRITE_SIZE", 1024.0], [2, K3, "WRITE_SIZE", 10.0],
    ])
    txt = profiling.traffic_text(str(tmp_path / "f"), str(tmp_path / "w"), "cmd",
                                 "m=1 n=1 k=1 N=2", 1 << 20)
    kv = dict(l.split(": ", 1) for l in txt.splitlines() if ": " in l)
    assert kv["k3_dispatches_fetch_pass"] == "2"
    assert float(kv["fetch_scale"]) == pytest.approx(0.5)
    assert float(kv["write_scale"]) == pytest.approx(1.0)
    # mean fetch 3000 KiB scaled by 0.5, write 10 KiB
    assert float(kv["hbm_bytes_per_launch"]) == pytest.approx(1500 * 1024 + 10 * 1024)
    assert kv["kernel_code_sha256"] == profiling.source_sha()


def test_stats_markdown(tmp_path):
    _write(tmp_path / "s" / "x_kernel_stats.csv",
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"],
           [[K3, 2, 2e6, 1e6, 90.0, 0.9e6, 1.1e6], [COPY, 1, 1e5, 1e5, 10.0, 1e5, 1e5]])
    md = profiling.stats_markdown(str(tmp_path / "s"), "t", "cmd")
    assert "| `oz2::k3_gemm_i8<256, 256, 128, 0>` | 2 | 2000.0 | 1000.0 | 900.0 | 1100.0 | 90.00 |" in md
    assert "other kernels" in md


def test_bench_reads_traffic_file(tmp_path, monkeypatch):
    import bench
    f = tmp_path / "t.txt"
    f.write_text(f"kernel_code_sha256: {profiling.source_sha()}\n"
                 "workload: m=4 n=4 k=4 N=3\nhbm_bytes_per_launch: 1.5e9\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic(4, 4, 4, 3) == 1.5e9
    assert bench.load_traffic(4, 4, 4, 4) is None
    f.write_text("kernel_code_sha256: 0\nworkload: m=4 n=4 k=4 N=3\nhbm_bytes_per_launch: 1\n")
    assert bench.load_traffic(4, 4, 4, 3) is None


def test_code_hash_ignores_comments_only(tmp_path):
    a = tmp_path / "a.hpp"
    a.write_text("int f() {  // one\n  return 1; /* two */\n}\n\n")
    b = tmp_path / "b.hpp"
    b.write_text("// header\nint f() {\n    return 1;\n}\n")
    c = tmp_path / "c.hpp"
    c.write_text("int f() {\n  return 2;\n}\n")
    assert profiling.source_sha(str(a)) == profiling.source_sha(str(b))
    assert profiling.source_sha(str(a)) != profiling.source_sha(str(c))


def test_clock_by_dispatch(tmp_path):
    """Per-dispatch clock = GRBM_GUI_ACTIVE / 8 XCDs / duration and MFMA busy
    = MFMA busy cycles / (4 SIMDs x CU busy cycles), from the timestamps of
    the counter file; other kernels are ignored; labels follow the order."""
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
           "Start_Timestamp", "End_Timestamp"]
    rows = []
    for disp, ns, grbm, mfma in ((7, 10_000_000, 8 * 2.0e9 * 0.01, 0.5), (9, 5_000_000, 8 * 1.0e9 * 0.005, 0.25)):
        rows += [[disp, K3, "GRBM_GUI_ACTIVE", grbm, 100, 100 + ns],
                 [disp, K3, "SQ_BUSY_CU_CYCLES", 1000.0, 100, 100 + ns],
                 [disp, K3, "SQ_VALU_MFMA_BUSY_CYCLES", 4 * 1000.0 * mfma, 100, 100 + ns]]
    rows.append([8, COPY, "GRBM_GUI_ACTIVE", 1.0, 0, 10])
    _write(tmp_path / "p" / "1_counter_collection.csv", hdr, rows)
    md = profiling.clock_markdown(str(tmp_path / "p"), "the command", ["a", "b"])
    assert "the command" in md
    assert "| 7 | a | 10.00 | 2.000 | 0.500 |" in md
    assert "| 9 | b | 5.00 | 1.000 | 0.250 |" in md
    assert "| 8 |" not in md


def test_issue_summary(tmp_path):
    """VALU issue = wave instructions x 4 / (1024 SIMDs x clock x duration),
    clock = GRBM_GUI_ACTIVE / 8 / duration; lane-ops per unit = 64 x wave
    instructions / units; waits from the second pass."""
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
           "Start_Timestamp", "End_Timestamp"]
    k4 = "void oz2::k4_crt<4, double>(unsigned char const*, ...)"
    ns = 1_000_000                                   # 1 ms
    grbm = 8 * 2.0e9 * 1e-3                          # 2 GHz
    insts = 0.5 * 1024 * 2.0e9 * 1e-3 / 4            # issue fraction 0.5
    _write(tmp_path / "a" / "1_counter_collection.csv", hdr, [
        [3, k4, "GRBM_GUI_ACTIVE", grbm, 0, ns], [3, k4, "SQ_INSTS_VALU", insts, 0, ns]])
    _write(tmp_path / "b" / "1_counter_collection.csv", hdr, [
        [3, k4, "SQ_WAIT_ANY", 25.0, 0, ns], [3, k4, "SQ_WAVE_CYCLES", 100.0, 0, ns]])
    md = profiling.issue_markdown([str(tmp_path / "a"), str(tmp_path / "b")], "cmd",
                                  {"k4_crt": insts * 64 / 10.0})
    row = [ln for ln in md.splitlines() if "k4_crt" in ln][0]
    assert "| 1.000 | 2.00 |" in row and "| 10 | 0.50 | 0.25 |" in row
