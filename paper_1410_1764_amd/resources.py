"""Register, scratch, LDS and occupancy table of the library's kernels.

Compiles the named sources for gfx950 with the compiler's resource-usage
remarks (``-Rpass-analysis=kernel-resource-usage``) and prints one markdown
row per kernel instance: VGPRs, AGPRs, scratch (spill) bytes per lane, LDS
bytes per workgroup and the compiler's waves-per-SIMD occupancy bound.
Usage: python -m paper_1410_1764_amd.resources bssn.hip bssn_split.hip [--filter TEXT]
"""
from __future__ import annotations

import argparse
import os
import re
import subprocess
import tempfile

from . import build as B

FIELDS = {"VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch",
          "LDS Size [bytes/block]": "lds", "Occupancy [waves/SIMD]": "occupancy"}


def remarks(src: str) -> list[dict]:
    with tempfile.TemporaryDirectory() as td:
        cmd = [B.HIPCC, *B.CFLAGS, "--offload-device-only", "-Rpass-analysis=kernel-resource-usage",
               "-c", os.path.join(B.CSRC, src), "-o", os.path.join(td, "k.o")]
        out = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
    rows, cur = [], None
    for line in out.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = {"mangled": m.group(1)}
            rows.append(cur)
            continue
        m = re.search(r"remark:\s+(.+?): (\S+) \[-Rpass-analysis", line)
        if m and cur is not None and m.group(1).strip() in FIELDS:
            cur[FIELDS[m.group(1).strip()]] = m.group(2)
    names = subprocess.run(["c++filt"], input="\n".join(r["mangled"] for r in rows),
                           capture_output=True, text=True, check=True).stdout.splitlines()
    for r, n in zip(rows, names):
        n = n.replace("chemora::(anonymous namespace)::", "").replace("void ", "")
        r["name"] = n.split("(")[0]
    return rows


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("sources", nargs="+")
    ap.add_argument("--filter", action="append", default=[],
                    help="keep kernels whose name contains this text (repeatable)")
    args = ap.parse_args()
    print("| kernel | VGPRs | AGPRs | scratch (B/lane) | LDS (B/workgroup) | waves/SIMD |")
    print("|---|---:|---:|---:|---:|---:|")
    for src in args.sources:
        for r in remarks(src):
            if args.filter and not any(f in r["name"] for f in args.filter):
                continue
            print(f"| `{r['name']}` | {r.get('vgpr', '?')} | {r.get('agpr', '?')} | "
                  f"{r.get('scratch', '?')} | {r.get('lds', '?')} | {r.get('occupancy', '?')} |")


if __name__ == "__main__":
    main()
