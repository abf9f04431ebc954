"""HBM traffic per launch of the right-hand-side kernels from hardware counters.

Reads the CSV output of two rocprofv3 counter runs of
``python3 bench.py --only-rhs`` (one with FETCH_SIZE, one with WRITE_SIZE,
both in KiB per dispatch), calibrates them with the streaming copy kernel that
the same command runs (512 MiB read and 512 MiB written per launch), and
records the bytes per launch of the default FP64 and mixed right-hand sides in
paper_1410_1764_amd/kernel_facts.json, with the hash of the kernel sources
(bench.py reports the figure only while the hash matches).

FP64 runs a pair of kernels (curvature + rest); its traffic is the sum of the
two kernels' per-dispatch means.  Usage:
  python -m paper_1410_1764_amd.counters FETCH_DIR WRITE_DIR
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys
from collections import defaultdict

from . import isa_count

COPY = "chemora::(anonymous namespace)::copy_kernel"
COPY_BYTES = 1 << 29  # read and written per launch of the calibration copy
FP64_KERNELS = ("bssn_curv_kernel<double", "bssn_rest_kernel<0, double")
MIXED_KERNELS = ("bssn_zfused_kernel<0, float",)


def per_kernel(run_dir: str, counter: str) -> dict[str, float]:
    """mean counter value (KiB) per dispatch of each kernel name"""
    sums: dict[str, float] = defaultdict(float)
    counts: dict[str, set] = defaultdict(set)
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    for path in files:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                name = row["Kernel_Name"]
                sums[name] += float(row["Counter_Value"])
                counts[name].add((path, row.get("Dispatch_Id")))
    return {k: sums[k] / len(counts[k]) for k in sums}


def lookup(table: dict[str, float], prefix: str) -> float:
    hits = [v for k, v in table.items() if prefix in k]
    if len(hits) != 1:
        raise KeyError(f"{prefix}: {len(hits)} matching kernels")
    return hits[0]


def main(fetch_dir: str, write_dir: str) -> dict:
    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    ff = COPY_BYTES / (lookup(fetch, COPY) * 1024)
    wf = COPY_BYTES / (lookup(write, COPY) * 1024)

    def traffic(prefixes):
        return sum(lookup(fetch, p) * 1024 * ff + lookup(write, p) * 1024 * wf for p in prefixes)

    out = {"fp64_bytes_per_launch": traffic(FP64_KERNELS),
           "mixed_bytes_per_launch": traffic(MIXED_KERNELS),
           "fetch_factor": ff, "write_factor": wf,
           "per_kernel_kib": {k: {"FETCH_SIZE": fetch[k], "WRITE_SIZE": write.get(k)}
                              for k in fetch},
           "source_hash": isa_count.source_hash(),
           "summary": "profiles/bssn_rhs_128cubed_counters.md"}
    facts = json.load(open(isa_count.FACTS)) if os.path.exists(isa_count.FACTS) else {}
    facts["traffic"] = out
    with open(isa_count.FACTS, "w") as f:
        json.dump(facts, f, indent=1)
    return out


if __name__ == "__main__":
    print(json.dumps(main(sys.argv[1], sys.argv[2]), indent=1))
