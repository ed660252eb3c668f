"""The profile condenser on synthetic rocprofv3 CSV files (host logic only)."""
import csv
import json
import os

from paper_1011_4687_amd import profsum

HDR = ["Correlation_Id", "Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _pmc(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for r in rows:
            w.writerow(r)


def test_record_derives_issue_traffic_and_conflicts(tmp_path):
    d = str(tmp_path)
    _pmc(os.path.join(d, "sq.csv"), [
        (1, 1, 1024, "kpot", "SQ_INSTS_VALU", 3.0e9), (1, 1, 1024, "kpot", "SQ_ACTIVE_INST_VALU", 2.0e9),
        (1, 1, 1024, "kpot", "GRBM_GUI_ACTIVE", 1.0e7), (1, 1, 1024, "kpot", "SQ_LDS_BANK_CONFLICT", 2.56e8),
        (1, 1, 1024, "kpot", "SQ_INSTS_LDS", 1.0e8),
        (2, 2, 1024, "kpot", "SQ_INSTS_VALU", 1.0e9), (2, 2, 1024, "kpot", "SQ_ACTIVE_INST_VALU", 2.0e9),
        (2, 2, 1024, "kpot", "GRBM_GUI_ACTIVE", 1.0e7), (2, 2, 1024, "kpot", "SQ_LDS_BANK_CONFLICT", 2.56e8),
        (2, 2, 1024, "kpot", "SQ_INSTS_LDS", 1.0e8),
        (3, 3, 1024, "probe", "SQ_INSTS_VALU", 1.0e9), (3, 3, 1024, "probe", "SQ_ACTIVE_INST_VALU", 2.56e9),
        (3, 3, 1024, "probe", "GRBM_GUI_ACTIVE", 1.0e7)])
    _pmc(os.path.join(d, "fetch.csv"), [(1, 1, 1024, "kpot", "FETCH_SIZE", 100.0), (5, 5, 131072, "elementwise_copy", "FETCH_SIZE", 131072.0),
                                              (6, 6, 512, "elementwise_copy", "FETCH_SIZE", 3.0)])
    _pmc(os.path.join(d, "write.csv"), [(1, 1, 1024, "kpot", "WRITE_SIZE", 50.0), (5, 5, 131072, "elementwise_copy", "WRITE_SIZE", 262144.0),
                                              (6, 6, 512, "elementwise_copy", "WRITE_SIZE", 2.0)])
    with open(os.path.join(d, "stats.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["kpot", 2, 2e7, 1e7, 90, 1e7, 1e7, 0])
        w.writerow(["probe", 1, 2e6, 2e6, 10, 2e6, 2e6, 0])
    src = os.path.join(d, "src.txt")
    open(src, "w").write("kernel")
    out = os.path.join(d, "rec.json")
    profsum.main(["record", "--kernel", "kpot", "--probe", "probe", "--copy", "elementwise",
                  "--sq", os.path.join(d, "sq.csv"), "--fetch", os.path.join(d, "fetch.csv"),
                  "--write", os.path.join(d, "write.csv"), "--stats", os.path.join(d, "stats.csv"),
                  "--sources", "src.txt", "--root", d, "--out", out])
    rec = json.load(open(out))
    # two dispatches averaged: 2e9 VALU instructions in 10 ms against 1e9 in 2 ms
    assert rec["counters_per_dispatch"]["SQ_INSTS_VALU"] == 2.0e9
    assert abs(rec["valu_issue_vs_probe"] - (2e9 / 1e-2) / (1e9 / 2e-3)) < 1e-12
    assert abs(rec["valubusy_rocprof"] - 2e9 / 256 / (1e7 / 8)) < 1e-12
    assert abs(rec["valubusy_vs_probe"] - 2.0 / 2.56) < 1e-12
    assert abs(rec["lds_bank_conflict_rocprof"] - 0.8) < 1e-12
    # copy of 256 MiB (its small dispatch ignored): fetch reads half, write
    # reads all -> scales 2 and 1
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    assert abs(rec["traffic_bytes_per_dispatch"] - 1024 * (100 * 2 + 50)) < 1e-6
    assert len(rec["kernel_source_sha256"]) == 64
