"""The counter summary used for the roofline's traffic figure: CSV parsing,
calibration scaling and invalidation by the kernel's source hash."""
import csv

from paper_1705_06073_amd import pmc

HDR = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for r in rows:
            w.writerow(r)


def test_summary_scaling_and_hash(tmp_path):
    k = "sfls::k_schur(sfls::InstInfo const*)"
    write_csv(tmp_path / "f.csv", [[1, 1, k, "FETCH_SIZE", 100.0], [2, 2, k, "FETCH_SIZE", 300.0],
                                   [3, 3, "other", "FETCH_SIZE", 1e9]])
    write_csv(tmp_path / "w.csv", [[1, 1, k, "WRITE_SIZE", 10.0], [2, 2, k, "WRITE_SIZE", 30.0]])
    # a copy of 1 MiB counted as 512 KiB read and 1024 KiB written
    write_csv(tmp_path / "cf.csv", [[1, 1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0],
                                    [2, 2, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 1.0]])
    write_csv(tmp_path / "cw.csv", [[1, 1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0]])
    assert pmc.counter_values(str(tmp_path / "f.csv"), "k_schur", "FETCH_SIZE") == [100.0, 300.0]
    out = tmp_path / "s.md"
    pmc.main(["--kernel", "k_schur", "--fetch", str(tmp_path / "f.csv"),
              "--write", str(tmp_path / "w.csv"), "--cal-fetch", str(tmp_path / "cf.csv"),
              "--cal-write", str(tmp_path / "cw.csv"), "--cal-bytes", str(1 << 20),
              "--out", str(out)])
    # mean 200 KiB fetched x 2 + mean 20 KiB written x 1
    assert abs(pmc.traffic_bytes(str(out), "k_schur") - (400.0 + 20.0) * 1024) < 1e-6
    text = out.read_text().replace(pmc.sources_hash("k_schur"), "0" * 64)
    out.write_text(text)
    assert pmc.traffic_bytes(str(out), "k_schur") is None
    assert pmc.traffic_bytes(str(tmp_path / "missing.md"), "k_schur") is None
