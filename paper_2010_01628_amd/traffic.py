"""HBM traffic of a kernel from rocprofv3 counter runs.

Reads the per-dispatch CSV of two `rocprofv3 --pmc` runs of the same command
(one with FETCH_SIZE, one with WRITE_SIZE; both in KiB per dispatch), averages
them over the dispatches of the kernel named by `--kernel` (a substring), and
scales each by what the same counter reads for a plain device copy of known
size in the same run (`--copy-kernel`, the dispatch whose reading is largest,
`--copy-bytes` read and as many written).  Writes a JSON file with the
per-launch HBM bytes and the factors used.

    python -m paper_2010_01628_amd.traffic --fetch DIR1 --write DIR2 \\
        --kernel k_step_ab --algo-bytes 2550136832 --out traffic.json
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os


# what the lattice step kernels are compiled from (sources and flags)
STEP_SOURCES = ("csrc/kernels_d3q19.hip", "csrc/kernels_d3q27.hip", "csrc/lattice_kernels.hpp", "csrc/d3q19_cm.hpp",
                "csrc/d3q27_cm.hpp", "csrc/lbm_internal.hpp", "build.py")


def kernel_source_hash(root: str | None = None) -> str:
    """Hash of the step kernels' sources: counters taken on another hash
    describe another kernel."""
    pkg = os.path.dirname(os.path.abspath(__file__)) if root is None else os.path.join(root, "paper_2010_01628_amd")
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        with open(os.path.join(pkg, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_counter(d: str, counter: str):
    """[(kernel name, value)] of every dispatch in the counter CSV under d."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    rows = []
    for fn in files:
        with open(fn, newline="") as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return rows


def summarise(rows, kernel: str, copy_kernel: str, copy_bytes: float):
    vals = [v for k, v in rows if kernel in k]
    copies = [v for k, v in rows if copy_kernel in k]
    if not vals or not copies:
        raise ValueError(f"kernel '{kernel}' ({len(vals)}) or copy '{copy_kernel}' ({len(copies)}) not found")
    kib = sum(vals) / len(vals)
    factor = (copy_bytes / 1024.0) / max(copies)
    names = sorted({k for k, _ in rows if kernel in k})
    return {"dispatches": len(vals), "kib_per_dispatch": kib, "copy_kib": max(copies), "factor": factor,
            "bytes_per_dispatch": kib * 1024.0 * factor, "kernel_names": names}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--copy-kernel", default="copyBuffer")
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--algo-bytes", type=float, required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    f = summarise(read_counter(a.fetch, "FETCH_SIZE"), a.kernel, a.copy_kernel, a.copy_bytes)
    w = summarise(read_counter(a.write, "WRITE_SIZE"), a.kernel, a.copy_kernel, a.copy_bytes)
    out = {
        "kernel": a.kernel,
        "kernel_names": f["kernel_names"],
        "kernel_source_hash": kernel_source_hash(),
        "fetch": f,
        "write": w,
        "hbm_bytes_per_launch": f["bytes_per_dispatch"] + w["bytes_per_dispatch"],
        "algo_bytes_per_launch": a.algo_bytes,
        "ratio_to_algorithmic": (f["bytes_per_dispatch"] + w["bytes_per_dispatch"]) / a.algo_bytes,
        "command": a.command,
    }
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
