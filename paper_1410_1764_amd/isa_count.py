"""Static operation count of the BSSN right-hand-side kernels.

Compiles bssn.hip for gfx950 to assembly (device side only) and counts the
floating-point vector instructions of the right-hand-side-only kernels.  The
per-point code is branch-free, so the static count is the number executed
per grid point (plus a handful of index operations outside the point loop).
FLOPs: v_fma/v_fmac = 2; add, sub, mul, ldexp (a multiply by a power of two),
rcp and sqrt = 1; conversions and selects are not counted.

Counts the fused single-plane kernels (async-staged 32x8 tiles, three
buffers, no dissipation, in FP64 and in mixed precision): their count is the
method's operations per point, the numerator of the ALU roofline.  Also
counts the kernels that run by default (FP64: the split curvature + rest
pair; mixed: the z-blocked fused kernel), whose instruction counts include
what the split recomputes.  Writes paper_1410_1764_amd/kernel_facts.json,
which bench.py reads for the ALU roofline.  The same file carries the HBM traffic per launch
measured with hardware counters, keyed by a hash of the kernel sources so that
a stale figure is not reported once the kernel has changed.
Usage: python -m paper_1410_1764_amd.isa_count
"""
from __future__ import annotations

import json
import os
import re
import subprocess

from . import build as B

OPS = {
    "f64": {"v_fma_f64": 2, "v_fmac_f64": 2, "v_mul_f64": 1, "v_add_f64": 1,
            "v_rcp_f64": 1, "v_sqrt_f64": 1, "v_div_fmas_f64": 2, "v_div_scale_f64": 0,
            "v_div_fixup_f64": 0, "v_ldexp_f64": 1},
    "f32": {"v_fma_f32": 2, "v_fmac_f32": 2, "v_mul_f32": 1, "v_add_f32": 1, "v_sub_f32": 1,
            "v_subrev_f32": 1, "v_rcp_f32": 1, "v_sqrt_f32": 1, "v_fmamk_f32": 2,
            "v_fmaak_f32": 2, "v_mac_f32": 2, "v_div_fmas_f32": 2, "v_ldexp_f32": 1},
}


FACTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kernel_facts.json")
KERNEL_SOURCES = ("bssn.hip", "bssn_split.hip", "bssn_args.h", "bssn_zsrc.h", "bssn_lds.h",
                  "bssn_point.h", "internal.h")


def source_hash() -> str:
    """SHA-256 over the sources of the right-hand-side kernels."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_bodies(asm: str):
    starts = [(m.start(), m.group(1)) for m in re.finditer(r"^(_Z\S+):", asm, re.M)]
    for q, (pos, name) in enumerate(starts):
        end = starts[q + 1][0] if q + 1 < len(starts) else len(asm)
        yield name, asm[pos:end]


def count(body: str):
    res = {}
    for kind, table in OPS.items():
        n_instr = {}
        flops = 0
        for op, w in table.items():
            c = len(re.findall(r"^\s+" + op + r"(_e32|_e64|_dpp|_sdwa)?\s", body, re.M))
            if c:
                n_instr[op] = c
                flops += w * c
        res[kind] = {"instructions": n_instr, "flops_per_point": flops}
    res["global_load"] = len(re.findall(r"^\s+global_load", body, re.M))
    res["scratch"] = len(re.findall(r"^\s+scratch_", body, re.M))
    return res


def _asm(src: str) -> str:
    os.makedirs(B.BUILD, exist_ok=True)
    out_s = os.path.join(B.BUILD, src.split(".")[0] + "_device.s")
    cmd = [B.HIPCC, *B.CFLAGS, "--offload-device-only", "-S", "-o", out_s,
           os.path.join(B.CSRC, src)]
    subprocess.check_call(cmd)
    return open(out_s).read()


def main():
    asm = _asm("bssn.hip")
    result = {"source": "paper_1410_1764_amd/csrc/bssn.hip", "arch": B.ARCH,
              "command": "python -m paper_1410_1764_amd.isa_count"}
    for name, body in kernel_bodies(asm):
        if "bssn_async_kernelILi0EdLi32ELi8ELi3ELi0E" in name:
            c = count(body)
            result["fp64"] = {"kernel": name, "flops_per_point": c["f64"]["flops_per_point"],
                              "instructions": c["f64"]["instructions"],
                              "global_loads": c["global_load"], "scratch_ops": c["scratch"]}
        if "bssn_async_kernelILi0EfLi32ELi8ELi3ELi0E" in name:
            c = count(body)
            result["mixed"] = {"kernel": name, "f32_flops_per_point": c["f32"]["flops_per_point"],
                               "f64_flops_per_point": c["f64"]["flops_per_point"],
                               "instructions": {**c["f32"]["instructions"],
                                                **c["f64"]["instructions"]},
                               "global_loads": c["global_load"], "scratch_ops": c["scratch"]}
    # kernels of the default path (right-hand side only, no dissipation)
    split = {}
    for name, body in kernel_bodies(_asm("bssn_split.hip")):
        c = count(body)
        if "bssn_curv_kernelIdLi0ELi8ELi3E" in name:
            split["fp64_curv"] = {"kernel": name, **c["f64"]}
        if "bssn_rest_kernelILi0EdLi0ELi8E" in name:
            split["fp64_rest"] = {"kernel": name, **c["f64"]}
        if "bssn_zfused_kernelILi0EfLi0ELi8E" in name:
            split["mixed_zfused"] = {"kernel": name, "f32": c["f32"], "f64": c["f64"]}
    if "fp64_curv" in split and "fp64_rest" in split:
        split["fp64_pair_flops_per_point"] = (split["fp64_curv"]["flops_per_point"] +
                                              split["fp64_rest"]["flops_per_point"])
    result["default_path"] = split
    result["source_hash"] = source_hash()
    path = FACTS
    old = {}
    if os.path.exists(path):
        old = json.load(open(path))
    if "traffic" in old:
        result["traffic"] = old["traffic"]
    with open(path, "w") as f:
        json.dump(result, f, indent=1)
    print(json.dumps(result, indent=1))


if __name__ == "__main__":
    main()
