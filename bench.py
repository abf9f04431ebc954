"""Benchmark: BSSN right-hand-side grid-point updates/s at 128^3 (+3 ghosts),
FP64 and mixed, with the roofline fraction of the dominant kernel and the
CPU oracle timed beside it.

One timed step = one pass of the right-hand-side path over the 128^3 block:
periodic ghost fill + one evaluation of all 24 BSSN right-hand sides
(1+log slicing, Gamma-driver shift, gauge-wave data A = 0.1, d = 1),
inputs resident in HBM.  value = 128^3 * steps / elapsed.

Also measured (reported in the same JSON line): the mixed-precision path,
the fused RK4 step at 128^3 (FP64 and mixed), the scalar wave RK4 step at
256^3, the constraint kernel, and a streaming copy (achievable HBM
bandwidth).  Single GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "BSSN RHS grid-point updates/s at 128^3, FP64 vs mixed; % of roofline"
HBM_PEAK = 8.0e12          # B/s, MI355X HBM3E
FP64_PEAK = 78.6e12        # FLOP/s, MI355X vector FP64
FP32_PEAK = 157.3e12       # FLOP/s, MI355X vector FP32 (packed); unpacked issues at half
BSSN_BYTES_PER_PT = 24 * 8 * 2       # read every variable once, write every rhs once
# FP64 operations per point of the right-hand-side kernel are counted
# statically from its gfx950 ISA by paper_1410_1764_amd/isa_count.py (the
# kernel is branch-free per point) into profiles/bssn_rhs_flops.json.


def _flops_per_point():
    p = os.path.join(ROOT, "profiles", "bssn_rhs_flops.json")
    if os.path.exists(p):
        with open(p) as f:
            return json.load(f)
    return None


def _events_time(fn, reps):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / 1e3 / reps


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-rhs", action="store_true",
                    help="time only the FP64 right-hand side (for profiler runs)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU halo exchange is a design, not an implementation", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1410_1764_amd import chemora as C
    from paper_1410_1764_amd import inputs as I

    torch.cuda.set_device(0)
    n = args.n
    h = 1.0 / n
    y0 = I.gaugewave((n, n, n), h, A=0.1, d=1.0, axis=0)
    kw = dict(system=C.BSSN, slicing=C.SLICING_1PLUSLOG, shift=C.SHIFT_GAMMADRIVER)
    g64 = C.Grid((n, n, n), 3, h, precision=C.FP64, **kw)
    gmx = C.Grid((n, n, n), 3, h, precision=C.MIXED, **kw)
    st = g64.upload(y0)
    rhs = g64.new_state()
    g64.fill_ghosts(st)
    torch.cuda.synchronize()
    print(f"[bench] data ready: BSSN {n}^3, state {st.numel() * 8 / 1e6:.0f} MB", file=sys.stderr,
          flush=True)

    def step64():
        g64.fill_ghosts(st)
        g64.rhs(st, rhs)

    def stepmx():
        gmx.fill_ghosts(st)
        gmx.rhs(st, rhs)

    # ---- timed region: FP64 steps
    for _ in range(args.warmup):
        step64()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step64()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pts = float(n) ** 3
    value = pts * args.steps / elapsed
    print(f"[bench] fp64 step {elapsed / args.steps * 1e3:.3f} ms", file=sys.stderr, flush=True)

    # kernel-only durations (HIP events on the launch stream)
    reps = max(args.steps, 20)
    k64 = _events_time(lambda: g64.rhs(st, rhs), reps)
    kghost = _events_time(lambda: g64.fill_ghosts(st), reps)
    if args.only_rhs:
        # plus a streaming copy of known size: the calibration kernel for
        # hardware byte counters collected on this same command
        nb = 1 << 29
        a = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        kc = _events_time(lambda: C.probe_copy(b, a, nb), 2)
        print(json.dumps({"rhs_fp64_ms": k64 * 1e3, "copy_512MiB_ms": kc * 1e3}))
        return 0

    for _ in range(args.warmup):
        stepmx()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stepmx()
    torch.cuda.synchronize()
    elapsed_mx = time.perf_counter() - t0
    value_mx = pts * args.steps / elapsed_mx
    kmx = _events_time(lambda: gmx.rhs(st, rhs), reps)
    print(f"[bench] mixed step {elapsed_mx / args.steps * 1e3:.3f} ms", file=sys.stderr, flush=True)

    # constraints (FP64 in both modes)
    hm_norms = torch.zeros(4, dtype=torch.float64, device="cuda")
    cws = torch.empty(max(C.lib().chemora_constraints_workspace_bytes(g64.handle) // 8, 1),
                      dtype=torch.float64, device="cuda")
    kcons = _events_time(lambda: g64.constraints(st, norms=hm_norms, workspace=cws), reps)

    # fused RK4 step at 128^3 (4 right-hand sides + stage updates + ghosts)
    ws = g64.new_workspace()
    dt = 0.25 * h
    rk_steps = 5
    st_rk = st.clone()
    g64.rk4_step(st_rk, ws, 0.0, dt, 1)
    krk64 = _events_time(lambda: g64.rk4_step(st_rk, ws, 0.0, dt, 1), rk_steps)
    gmx.rk4_step(st_rk, ws, 0.0, dt, 1)
    krkmx = _events_time(lambda: gmx.rk4_step(st_rk, ws, 0.0, dt, 1), rk_steps)
    del ws, st_rk
    print("[bench] rk4 done", file=sys.stderr, flush=True)

    # scalar wave, 256^3 + 2 ghosts, RK4 steps (FP64 and mixed)
    nw = 256
    hw = 1.0 / nw
    gw64 = C.Grid((nw, nw, nw), 2, hw, system=C.WAVE, precision=C.FP64)
    gwmx = C.Grid((nw, nw, nw), 2, hw, system=C.WAVE, precision=C.MIXED)
    sw = gw64.upload(I.fourier_modes(nw, 16, I.SEED0 + 1))
    wsw = gw64.new_workspace()
    gw64.rk4_step(sw, wsw, 0.0, 0.25 * hw, 2)
    kw64 = _events_time(lambda: gw64.rk4_step(sw, wsw, 0.0, 0.25 * hw, 10), 2) / 10
    kwmx = _events_time(lambda: gwmx.rk4_step(sw, wsw, 0.0, 0.25 * hw, 10), 2) / 10
    del sw, wsw

    # streaming copy: achievable bandwidth and the counter calibration kernel
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    C.probe_copy(b, a, nbytes)
    kcopy = _events_time(lambda: C.probe_copy(b, a, nbytes), 10)
    copy_bw = 2 * nbytes / kcopy
    del a, b
    torch.cuda.synchronize()
    print("[bench] gpu done", file=sys.stderr, flush=True)

    # ---- roofline of the dominant kernel (right-hand side, FP64): both the
    # HBM bound (algorithmic bytes) and the FP64 ALU bound (counted flops);
    # "roofline" is the one whose ideal time is longer, i.e. the binding one
    fl = _flops_per_point()
    bytes_launch = BSSN_BYTES_PER_PT * pts
    roof_hbm = {"bound": "hbm", "achieved": bytes_launch / k64 / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": bytes_launch / k64 / HBM_PEAK, "traffic": None,
                "kernel": "bssn_stage_kernel<0,double>", "kernel_ms": k64 * 1e3,
                "bytes_per_point": BSSN_BYTES_PER_PT, "points_per_launch": pts}
    tr = (fl or {}).get("traffic_fp64_bytes_per_launch")
    if tr:
        roof_hbm["traffic"] = tr
    roof = roof_hbm
    roof_other = None
    if fl:
        f64 = fl["fp64"]["flops_per_point"]
        roof_alu = {"bound": "alu", "achieved": f64 * pts / k64 / 1e12, "peak": FP64_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": f64 * pts / k64 / FP64_PEAK,
                    "traffic": roof_hbm["traffic"], "kernel": roof_hbm["kernel"],
                    "kernel_ms": k64 * 1e3, "flops_per_point": f64, "points_per_launch": pts}
        if f64 * pts / FP64_PEAK > bytes_launch / HBM_PEAK:
            roof, roof_other = roof_alu, roof_hbm
        else:
            roof_other = roof_alu
    roof_mx = {"bound": "hbm", "achieved": bytes_launch / kmx / 1e9, "peak": HBM_PEAK / 1e9,
               "unit": "GB/s", "frac": bytes_launch / kmx / HBM_PEAK,
               "kernel": "bssn_stage_kernel<0,float>", "kernel_ms": kmx * 1e3}

    # ---- CPU baseline: the oracle on the host cores (rank 0, N = 1 only)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nc = n  # the same 128^3 workload, repeated for about 10 s of host time
        hb = 1.0 / nc
        blk = oracle.Block((nc, nc, nc), 3, hb, slicing=0, shift=1)
        yo = blk.embed(I.gaugewave((nc, nc, nc), hb, A=0.1, d=1.0, axis=0))
        oracle.fill_periodic(blk, yo)
        t0 = time.perf_counter()
        oracle.bssn_rhs(blk, yo)  # warm
        t1 = time.perf_counter()
        reps_c = max(3, min(200, int(10.0 / max(t1 - t0, 1e-3))))
        t0 = time.perf_counter()
        for _ in range(reps_c):
            oracle.bssn_rhs(blk, yo)
        tc = (time.perf_counter() - t0) / reps_c
        cpu = {"value": nc ** 3 / tc, "unit": "grid-point updates/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"BSSN RHS on the {nc}^3 + 3-ghost gauge-wave block (1+log, "
                         f"Gamma-driver), mean of {reps_c} evaluations, {tc:.3f} s each"}

    out = {
        "metric": METRIC, "value": value, "unit": "grid-point updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"BSSN right-hand side, {n}^3 interior + 3 ghost zones, "
                               "24 FP64 grid functions, periodic, 1+log slicing, Gamma-driver "
                               "shift, gauge-wave data A=0.1 d=1",
                   "global_batch": 1, "seq_len": n ** 3, "parallelism": "single-gpu"},
        "roofline": roof,
        "roofline_other_bound": roof_other,
        "cpu_baseline": cpu,
        "mixed": {"value": value_mx, "ms_per_step": elapsed_mx / args.steps * 1e3,
                  "dtype": "f32 arithmetic on f64 state", "roofline": roof_mx},
        "kernels_ms": {"bssn_rhs_fp64": k64 * 1e3, "bssn_rhs_mixed": kmx * 1e3,
                       "ghost_periodic_24var": kghost * 1e3, "constraints_fp64": kcons * 1e3,
                       "bssn_rk4_step_fp64": krk64 * 1e3, "bssn_rk4_step_mixed": krkmx * 1e3,
                       "wave256_rk4_step_fp64": kw64 * 1e3, "wave256_rk4_step_mixed": kwmx * 1e3,
                       "copy_1GiB": kcopy * 1e3},
        "derived": {"bssn_rk4_rhs_updates_per_s_fp64": 4 * pts / krk64,
                    "bssn_rk4_rhs_updates_per_s_mixed": 4 * pts / krkmx,
                    "wave256_rk4_point_steps_per_s_fp64": nw ** 3 / kw64,
                    "wave256_rk4_GBps_fp64": 272 * nw ** 3 / kw64 / 1e9,
                    "wave256_rk4_GBps_mixed": 272 * nw ** 3 / kwmx / 1e9,
                    "copy_GBps": copy_bw / 1e9},
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
