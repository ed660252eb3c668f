"""Condense rocprofv3 output into the committed profile records.

Reads the CSV files rocprofv3 writes (``--kernel-trace --stats``:
``*_kernel_stats.csv``; ``--pmc``: ``*_counter_collection.csv``) and prints
per-kernel means per dispatch.  ``record`` writes a JSON record of one
kernel's counters (with the SHA-256 of the kernel sources it was taken from,
so a reader can tell whether the record still describes the current kernel)
and the figures derived from them:

* HBM traffic per dispatch: FETCH_SIZE and WRITE_SIZE (KiB) scaled by what
  the same counters read for a plain device copy of known size;
* VALU issue: wave-instructions per second against the FMA probe kernel
  (independent v_fma_f32 chains) measured in the same counter pass, and
  rocprof's VALUBusy (SQ_ACTIVE_INST_VALU / CU_NUM / GRBM_GUI_ACTIVE per XCD) for
  both kernels, so the potential kernel's figure is read against what a pure
  FMA stream reaches;
* LDS bank conflicts: rocprof's LDSBankConflict
  (SQ_LDS_BANK_CONFLICT / GRBM_GUI_ACTIVE / CU_NUM) and conflict cycles per
  LDS instruction.

usage:
  python -m paper_1011_4687_amd.profsum show FILE.csv [...]
  python -m paper_1011_4687_amd.profsum record --kernel NAME --probe NAME --copy NAME
         --sq SQ.csv --fetch FETCH.csv --write WRITE.csv [--stats STATS.csv]
         --copy-bytes N --sources a,b,c --out profiles/X.json
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

CU_NUM = 256
XCD_NUM = 8   # rocprofv3 sums GRBM_GUI_ACTIVE over the 8 XCDs; rocprof's derived
              # metrics take the per-XCD value (reduce(GRBM_GUI_ACTIVE, max))


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def expand(paths):
    out = []
    for p in paths:
        if os.path.isdir(p):
            out += sorted(glob.glob(os.path.join(p, "**", "*.csv"), recursive=True))
        else:
            out += sorted(glob.glob(p))
    return out


def counters(paths, min_grid=0):
    """{kernel: {counter: [value per dispatch]}} from counter-collection CSVs
    (dispatches with a grid of at least min_grid work-items)."""
    per = defaultdict(lambda: defaultdict(dict))
    for path in expand(paths):
        for r in _rows(path):
            if "Counter_Name" not in r:
                continue
            if min_grid and int(r.get("Grid_Size") or 0) < min_grid:
                continue
            k = r["Kernel_Name"]
            d = (path, r.get("Dispatch_Id") or r.get("Correlation_Id"))
            per[k][r["Counter_Name"]][d] = per[k][r["Counter_Name"]].get(d, 0.0) + float(r["Counter_Value"])
    return {k: {c: list(v.values()) for c, v in cs.items()} for k, cs in per.items()}


def durations(paths):
    """{kernel: [ns per dispatch]} from the timestamps of counter-collection CSVs."""
    per = defaultdict(dict)
    for path in expand(paths):
        for r in _rows(path):
            if "Start_Timestamp" in r and r.get("Start_Timestamp"):
                d = (path, r.get("Dispatch_Id") or r.get("Correlation_Id"))
                per[r["Kernel_Name"]][d] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    return {k: list(v.values()) for k, v in per.items()}


def stats(paths):
    """{kernel: (calls, average ns)} from kernel-stats CSVs."""
    out = {}
    for path in expand(paths):
        for r in _rows(path):
            if "AverageNs" in r:
                out[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]))
    return out


def find(names, pattern):
    hits = [k for k in names if pattern in k]
    if not hits:
        raise SystemExit(f"no kernel matching {pattern!r} among {sorted(names)[:20]}")
    return min(hits, key=len)


def mean(v):
    return sum(v) / len(v)


def sources_sha(root, sources):
    h = hashlib.sha256()
    for s in sources:
        h.update(open(os.path.join(root, s), "rb").read())
    return h.hexdigest()


def record(a):
    sq = counters([a.sq])
    kern = find(sq, a.kernel)
    probe = find(sq, a.probe)
    # durations of the counted dispatches themselves (timestamps of the same
    # counter pass); a kernel-stats file is the fallback
    du = durations([a.sq])
    if kern in du and probe in du:
        t_k, t_p = mean(du[kern]) * 1e-9, mean(du[probe]) * 1e-9
    else:
        ks = stats([a.stats])
        t_k, t_p = ks[find(ks, a.kernel)][1] * 1e-9, ks[find(ks, a.probe)][1] * 1e-9
    K = {c: mean(v) for c, v in sq[kern].items()}
    P = {c: mean(v) for c, v in sq[probe].items()}
    rec = {"kernel": kern, "probe_kernel": probe, "kernel_sources": a.sources,
           "dispatches": len(sq[kern]["SQ_INSTS_VALU"]),
           "kernel_source_sha256": sources_sha(a.root, a.sources),
           "kernel_avg_ms": t_k * 1e3, "probe_avg_ms": t_p * 1e3,
           "counters_per_dispatch": K, "probe_counters_per_dispatch": P}
    # VALU issue against the FMA probe of the same pass
    ik, ip = K["SQ_INSTS_VALU"], P["SQ_INSTS_VALU"]
    rate_k, rate_p = ik / t_k, ip / t_p
    busy_k = K["SQ_ACTIVE_INST_VALU"] / CU_NUM / (K["GRBM_GUI_ACTIVE"] / XCD_NUM)
    busy_p = P["SQ_ACTIVE_INST_VALU"] / CU_NUM / (P["GRBM_GUI_ACTIVE"] / XCD_NUM)
    nominal = 1024 * 2.4e9 / 4.0     # wave64 VALU issue: 1024 SIMDs, 4 cycles per instruction
    rec.update({
        "valu_wave_instr_per_s": rate_k, "probe_valu_wave_instr_per_s": rate_p,
        "valu_issue_vs_probe": rate_k / rate_p,
        "probe_issue_vs_nominal": rate_p / nominal,
        "valu_issue_vs_nominal": rate_k / nominal,
        "valubusy_rocprof": busy_k, "probe_valubusy_rocprof": busy_p,
        "valubusy_vs_probe": busy_k / busy_p,
    })
    if "SQ_LDS_BANK_CONFLICT" in K:
        rec["lds_bank_conflict_rocprof"] = K["SQ_LDS_BANK_CONFLICT"] / (K["GRBM_GUI_ACTIVE"] / XCD_NUM) / CU_NUM
        if K.get("SQ_INSTS_LDS"):
            rec["lds_conflict_cycles_per_lds_instr"] = K["SQ_LDS_BANK_CONFLICT"] / K["SQ_INSTS_LDS"]
    # HBM bytes against the copy kernel
    if a.fetch and a.write:
        fe, wr = counters([a.fetch]), counters([a.write])
        fk, wk = mean(fe[find(fe, a.kernel)]["FETCH_SIZE"]), mean(wr[find(wr, a.kernel)]["WRITE_SIZE"])
        # the copy reference: only the plain copy's own dispatches (a grid of
        # one work-item per 2 KiB copied: 131,072 for 256 MiB)
        fcp = counters([a.fetch], min_grid=int(a.copy_bytes // 2048))
        wcp = counters([a.write], min_grid=int(a.copy_bytes // 2048))
        fc, wc = mean(fcp[find(fcp, a.copy)]["FETCH_SIZE"]), mean(wcp[find(wcp, a.copy)]["WRITE_SIZE"])
        ref = a.copy_bytes / 1024.0
        rec.update({"fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "copy_reference_kib": ref,
                    "copy_fetch_kib": fc, "copy_write_kib": wc, "fetch_scale": ref / fc, "write_scale": ref / wc,
                    "traffic_bytes_per_dispatch": 1024.0 * (fk * ref / fc + wk * ref / wc)})
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("show")
    s.add_argument("files", nargs="+")
    r = sub.add_parser("record")
    for k in ("kernel", "probe", "sq", "out"):
        r.add_argument("--" + k, required=True)
    r.add_argument("--stats")
    r.add_argument("--copy", default="copyBuffer")
    r.add_argument("--fetch")
    r.add_argument("--write")
    r.add_argument("--copy-bytes", type=float, default=256.0 * 2 ** 20)
    r.add_argument("--sources", required=True, type=lambda v: v.split(","))
    r.add_argument("--root", default=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    a = ap.parse_args(argv)
    if a.cmd == "show":
        for k, cs in sorted(counters(a.files).items()):
            print(k)
            for c, v in sorted(cs.items()):
                print(f"  {c:28s} {mean(v):18.6g}  ({len(v)} dispatches)")
        for k, (calls, avg) in sorted(stats(a.files).items(), key=lambda kv: -kv[1][0] * kv[1][1]):
            print(f"{calls:6d} x {avg / 1e6:10.3f} ms  {k}")
    else:
        record(a)


if __name__ == "__main__":
    sys.exit(main())
