"""Summarise rocprofv3 memory-counter runs of bench.py into per-launch HBM
traffic of each step kernel.

Two counter runs of ``bench.py --copy-calibration`` (one collecting
FETCH_SIZE, one WRITE_SIZE, in KiB per dispatch) are combined.  Each counter is
divided by what it reads for the calibration copy of 256 MiB (a plain
device-to-device copy whose source was first evicted from the Infinity
Cache), which converts counter units into bytes moved.  The result is stamped
with a hash of the kernel sources and of the host code that splits their work:
bench.py reports the traffic only while both are unchanged.

    python -m paper_2205_06557_amd.pmc_summary --fetch F.csv --write W.csv \\
        --n-ions 1048576 --json profiles/step_kernels_traffic.json --md profiles/step_kernels_traffic.md
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/kernels.hpp", "csrc/device_common.hpp", "csrc/cutoff.hpp", "csrc/pairsym.hpp",
                  "csrc/worksplit.hpp", "csrc/symitems.hpp")
CALIB_BYTES = 1 << 28
KERNELS = {"pair_forces_f32": "pair", "pair_sym_kernel": "pair", "step_tail_kernel<float, ": "tail",
           "reinject_kernel<float>": "reinject"}


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _per_kernel(path):
    vals = collections.defaultdict(list)
    calib = 0.0
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        v = float(r["Counter_Value"])
        if "copyBuffer" in name:
            calib = max(calib, v)
        for key, short in KERNELS.items():
            if key in name:
                vals[short].append(v)
    return {k: sum(v) / len(v) for k, v in vals.items()}, calib


def summarise(fetch_csv, write_csv, n_ions):
    f, fc = _per_kernel(fetch_csv)
    w, wc = _per_kernel(write_csv)
    ff = fc * 1024.0 / CALIB_BYTES
    wf = wc * 1024.0 / CALIB_BYTES
    out = {"source_sha256": kernel_sources_hash(), "n_ions": n_ions,
           "calibration": {"fetch_kib": fc, "write_kib": wc, "fetch_factor": ff, "write_factor": wf},
           "kernels": {}}
    for k in sorted(set(f) | set(w)):
        fb = f.get(k, 0.0) * 1024.0 / ff
        wb = w.get(k, 0.0) * 1024.0 / wf
        out["kernels"][k] = {"fetch_kib": f.get(k), "write_kib": w.get(k), "fetch_bytes": fb,
                             "write_bytes": wb, "traffic_bytes": fb + wb}
    return out


def summarise_issue(counters_csv, n_ions, kernel="pair_sym_kernel"):
    """VALU issue accounting of `kernel` from one rocprofv3 --pmc run with
    SQ_INSTS_VALU, SQ_INSTS_VALU_TRANS_F32, SQ_ACTIVE_INST_VALU,
    SQ_ACTIVE_INST_VALU2 and GRBM_GUI_ACTIVE (per dispatch, averaged over the
    kernel's dispatches).  SQ_ACTIVE_INST_VALU counts one quad-cycle per
    ordinary and two per transcendental VALU instruction, summed over the
    SIMDs; SQ_ACTIVE_INST_VALU2 the quad-cycles in which two issued together;
    GRBM_GUI_ACTIVE the busy cycles summed over the 8 XCDs.  The issue
    fraction is (ACTIVE_INST_VALU - ACTIVE_INST_VALU2) over the quad-cycles
    the 1024 SIMDs had: 1024 * (GRBM_GUI_ACTIVE / 8) / 4."""
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(counters_csv)):
        if kernel in r["Kernel_Name"]:
            vals[r["Counter_Name"]].append(float(r["Counter_Value"]))
    m = {k: sum(v) / len(v) for k, v in vals.items()}
    quad = 1024 * m["GRBM_GUI_ACTIVE"] / 8 / 4
    steps = 0.5 * n_ions * (n_ions - 1) / 64          # wave steps of 64 unique pairs
    return {"source_sha256": kernel_sources_hash(), "n_ions": n_ions, "kernel": kernel,
            "valu_issue_frac": (m["SQ_ACTIVE_INST_VALU"] - m["SQ_ACTIVE_INST_VALU2"]) / quad,
            "valu_per_wave_step": m["SQ_INSTS_VALU"] / steps,
            "trans_per_wave_step": m.get("SQ_INSTS_VALU_TRANS_F32", 0.0) / steps,
            "dual_issue_quads_per_wave_step": m["SQ_ACTIVE_INST_VALU2"] / steps,
            "counters": m}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--issue", help="SQ/GRBM counter CSV of the pair kernel (issue accounting)")
    ap.add_argument("--n-ions", type=int, required=True)
    ap.add_argument("--json", required=True)
    ap.add_argument("--md")
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)
    if a.issue:
        s = summarise_issue(a.issue, a.n_ions)
        s["command"] = a.command
        with open(a.json, "w") as fh:
            json.dump(s, fh, indent=1)
        return
    s = summarise(a.fetch, a.write, a.n_ions)
    s["command"] = a.command
    with open(a.json, "w") as fh:
        json.dump(s, fh, indent=1)
    if a.md:
        lines = [f"# HBM traffic per launch of the step kernels, N = {a.n_ions} ions", "",
                 "Commands (repo root, MI355X):", "", "```", a.command, "```", "",
                 f"Calibration copy of {CALIB_BYTES} B: FETCH_SIZE {s['calibration']['fetch_kib']:.1f} KiB "
                 f"(factor {s['calibration']['fetch_factor']:.4f}), WRITE_SIZE "
                 f"{s['calibration']['write_kib']:.1f} KiB (factor {s['calibration']['write_factor']:.4f}).", "",
                 "| Kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | traffic (MB, calibrated) |",
                 "|---|---|---|---|"]
        for k, v in s["kernels"].items():
            lines.append(f"| {k} | {v['fetch_kib']} | {v['write_kib']} | {v['traffic_bytes'] / 1e6:.2f} |")
        lines += ["", f"Kernel sources sha256: `{s['source_sha256']}`"]
        with open(a.md, "w") as fh:
            fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
