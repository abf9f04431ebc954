"""Benchmark: BSSN right-hand-side grid-point updates/s at 128^3 (+3 ghosts),
FP64 and mixed, with the roofline fraction of the dominant kernel and the
CPU oracle timed beside it.

One timed step = one pass of the right-hand-side path over the 128^3 block:
periodic ghost fill + one evaluation of all 24 BSSN right-hand sides
(1+log slicing, Gamma-driver shift, gauge-wave data A = 0.1, d = 1),
inputs resident in HBM.  value = 128^3 * steps / elapsed.

Also measured (reported in the same JSON line): the mixed-precision path,
the fused RK4 step at 128^3 (FP64 and mixed), the scalar wave RK4 step at
256^3, the constraint kernel, the batched path over 64 uneven patches
(autotuned, graph-captured; FP64 and mixed), and a streaming copy
(achievable HBM bandwidth).  Single GPU only.
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
# Floating-point operations per point of the default right-hand-side kernels
# are counted statically from their gfx950 ISA (the point code is
# branch-free) by paper_1410_1764_amd/isa_count.py into
# paper_1410_1764_amd/kernel_facts.json; the same file holds the HBM traffic
# per launch measured with hardware counters, valid only while the hash of
# the kernel sources matches.
# The right-hand side that runs by default: FP64 as a pair of kernels
# (curvature, then shift/advection/assembly; 32x8x2-point workgroups), mixed
# as one fused kernel over the same z-blocked staging.  Its roofline counts
# the method's operations (the fused FP64 kernel's static count; the pair
# executes about 1 % more, recomputing the inverse metric) over the time of
# the whole right-hand side.
# The method's own count: the oracle's right-hand-side expression traced at
# one point, common subexpressions merged (tests/flops/oracle_flops.cpp;
# 1,953 stencil + 2,295 pointwise operations at 4th order, 1+log,
# Gamma-driver), stated beside the instruction-stream count.
FLOPS_PER_POINT_EXPRESSION = 4248
KERNEL_FP64 = "bssn_curv_kernel<double,KO_OFF,8,3> + bssn_rest_kernel<0,double,KO_OFF,8>"
KERNEL_MIXED = "bssn_zfused_kernel<0,float,KO_OFF,8>"
# Mixed precision runs unpacked FP32 (packed FP32 is disabled at compile
# time), which issues at the FP64 vector rate: 256 CUs x 4 SIMDs x 16 lanes
# x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s.
UNPACKED_PEAK = 78.6e12


def _facts():
    from paper_1410_1764_amd import isa_count
    if not os.path.exists(isa_count.FACTS):
        return None
    with open(isa_count.FACTS) as f:
        facts = json.load(f)
    tr = facts.get("traffic")
    facts["traffic_valid"] = bool(tr) and tr.get("source_hash") == isa_count.source_hash()
    return facts


def _cpu_model() -> str:
    """the host CPU's model name (first processor in /proc/cpuinfo)"""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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


def _high_order_times(C, torch, n, h, y0, kw):
    """6th- and 8th-order right-hand sides at n^3 (staged high-order kernel),
    FP64 and mixed, and the FP64 constraints at those orders: milliseconds from
    HIP events, 10 launches each."""
    khi = {}
    for order in (6, 8):
        gho = order // 2 + 1
        for name, prec in (("fp64", C.FP64), ("mixed", C.MIXED)):
            go = C.Grid((n, n, n), gho, h, precision=prec, fd_order=order, **kw)
            so = go.upload(y0)
            go.fill_ghosts(so)
            ro = go.new_state()
            go.rhs(so, ro)
            khi[f"bssn_rhs_order{order}_{name}"] = _events_time(lambda: go.rhs(so, ro), 10) * 1e3
            if prec == C.FP64:
                nrm = torch.zeros(4, dtype=torch.float64, device="cuda")
                cw = torch.empty(max(C.lib().chemora_constraints_workspace_bytes(go.handle) // 8,
                                     1), dtype=torch.float64, device="cuda")
                go.constraints(so, norms=nrm, workspace=cw)
                khi[f"constraints_order{order}_fp64"] = _events_time(
                    lambda: go.constraints(so, norms=nrm, workspace=cw), 10) * 1e3
            del go, so, ro
    torch.cuda.synchronize()
    return khi


def _amr_timing(C, torch):
    """Prolongation (three coarse time levels) and restriction between a 128^3
    BSSN level and a centred 96^3 fine patch, 24 grid functions; algorithmic
    bytes: prolongation writes every fine ghost value and reads every coarse
    value some ghost stencil reaches, once per time level; restriction reads
    and writes each injected value once."""
    import numpy as np
    nc, nf, g, off = 128, 96, 3, 80
    hc = 1.0 / nc
    co = C.Grid((nc,) * 3, g, hc, system=C.BSSN, boundary=C.BC_CALLER)
    fi = C.Grid((nf,) * 3, g, hc / 2, origin=(off * hc / 2,) * 3, system=C.BSSN,
                boundary=C.BC_CALLER)
    cs = [co.new_state() for _ in range(3)]
    for q, s in enumerate(cs):
        s.fill_(1.0 + q)
    fs = fi.new_state()
    fs.zero_()
    times = [0.0, 0.5, 1.0]
    C.prolong(co, cs, fi, fs, times, 0.3)
    kp = _events_time(lambda: C.prolong(co, cs, fi, fs, times, 0.3), 20)
    C.restrict(co, cs[0], fi, fs)
    kr = _events_time(lambda: C.restrict(co, cs[0], fi, fs), 20)
    # coarse points reached: per axis, by ghost coordinates and by all coordinates
    def reach(idx):
        out = set()
        for i in idx:
            q = off + i
            b = q // 2
            out.update(range(b - 2, b + 4) if q & 1 else [b])
        return sorted(out)
    rg = np.array(reach(list(range(-g, 0)) + list(range(nf, nf + g)))) + g
    ra = np.array(reach(range(-g, nf + g))) + g
    m = np.zeros((nc + 2 * g,) * 3, dtype=bool)
    m[np.ix_(ra, ra, rg)] = True
    m[np.ix_(ra, rg, ra)] = True
    m[np.ix_(rg, ra, ra)] = True
    ghosts = (nf + 2 * g) ** 3 - nf ** 3
    pbytes = 24 * 8 * (ghosts + 3 * int(m.sum()))
    ninj = (nf // 2) ** 3
    rbytes = 24 * 8 * 2 * ninj
    # the fine patch as a batch of one, its ghosts prolongated from the three
    # coarse levels inside the persistent launches (Minkowski data), against
    # the same batch with analytic ghosts
    minkowski = (0, 1, 4, 6, 17)  # chi, gt11, gt22, gt33, alpha
    for s in cs:
        s.zero_()
        for v in minkowski:
            co.view(s, v).fill_(1.0)
    fb = C.Grid((nf,) * 3, g, hc / 2, origin=(off * hc / 2,) * 3, system=C.BSSN,
                boundary=C.BC_GAUGEWAVE, slicing=C.SLICING_HARMONIC, shift=C.SHIFT_FROZEN,
                gw_amp=0.1, gw_wavelength=1.0, gw_axis=0)
    sb = fb.new_state()
    sb.zero_()
    for v in minkowski:
        fb.view(sb, v).fill_(1.0)
    wb = fb.new_workspace()
    meta = torch.empty(C.batch_meta_bytes(1) // 8, dtype=torch.float64, device="cuda")
    dtf = 0.125 * hc
    lv = [(co, cs, times)]
    C.batch_step([fb], [sb], [wb], meta, 0.0, dtf, 1, parents=lv)
    kbp = _events_time(lambda: C.batch_step([fb], [sb], [wb], meta, 0.0, dtf, 5, parents=lv),
                       1) / 5
    C.batch_release(meta)
    C.batch_step([fb], [sb], [wb], meta, 0.0, dtf, 1)
    kba = _events_time(lambda: C.batch_step([fb], [sb], [wb], meta, 0.0, dtf, 5), 1) / 5
    C.batch_release(meta)
    del cs, fs, sb, wb, meta
    torch.cuda.synchronize()
    return {"workload": f"{nf}^3 fine patch (ghost {g}) in the {nc}^3 BSSN level, 24 grid "
                        "functions, prolongation from 3 coarse time levels",
            "prolong_ms": kp * 1e3, "prolong_bytes": pbytes,
            "prolong_GBps": pbytes / kp / 1e9, "fine_ghost_points": ghosts,
            "restrict_ms": kr * 1e3, "restrict_bytes": rbytes,
            "restrict_GBps": rbytes / kr / 1e9,
            "batch_rk4_step_prolongated_ghosts_ms": kbp * 1e3,
            "batch_rk4_step_analytic_ghosts_ms": kba * 1e3}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-patch batch timing")
    ap.add_argument("--only-wave", action="store_true",
                    help="time only the 256^3 wave RK4 steps and the copy (for profiler runs)")
    ap.add_argument("--only-amr", action="store_true",
                    help="time only prolongation and restriction (for profiler runs)")
    ap.add_argument("--only-hi", action="store_true",
                    help="time only the 6th/8th-order right-hand sides (for profiler runs)")
    ap.add_argument("--only-rhs", action="store_true",
                    help="time only the FP64 right-hand side (for profiler runs)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU halo exchange is a design, not an implementation", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1410_1764_amd import chemora as C
    from paper_1410_1764_amd import inputs as I

    torch.cuda.set_device(0)
    if args.only_amr:
        # plus the streaming copy: the calibration kernel for byte counters
        nb = 1 << 29
        a = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        C.probe_copy(b, a, nb)
        kc = _events_time(lambda: C.probe_copy(b, a, nb), 10)
        del a, b
        out = _amr_timing(C, torch)
        out["copy_512MiB_ms"] = kc * 1e3
        print(json.dumps(out))
        return 0
    if args.only_wave:
        nw = 256
        hw = 1.0 / nw
        gw64 = C.Grid((nw, nw, nw), 2, hw, system=C.WAVE, precision=C.FP64)
        sw = gw64.upload(I.fourier_modes(nw, 16, I.SEED0 + 1))
        wsw = gw64.new_workspace()
        gw64.rk4_step(sw, wsw, 0.0, 0.25 * hw, 2)
        kw64 = _events_time(lambda: gw64.rk4_step(sw, wsw, 0.0, 0.25 * hw, 5), 1) / 5
        nb = 1 << 29
        a = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        C.probe_copy(b, a, nb)
        kc = _events_time(lambda: C.probe_copy(b, a, nb), 10)
        print(json.dumps({"wave256_rk4_step_fp64_ms": kw64 * 1e3, "copy_512MiB_ms": kc * 1e3}))
        return 0
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
    if args.only_hi:
        print(json.dumps(_high_order_times(C, torch, n, h, y0, kw)))
        return 0
    if args.only_rhs:
        # plus a streaming copy of known size: the calibration kernel for
        # hardware byte counters collected on this same command
        nb = 1 << 29
        a = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        C.probe_copy(b, a, nb)
        kc = _events_time(lambda: C.probe_copy(b, a, nb), 10)
        kmx = _events_time(lambda: gmx.rhs(st, rhs), reps)
        print(json.dumps({"rhs_fp64_ms": k64 * 1e3, "rhs_mixed_ms": kmx * 1e3,
                          "copy_512MiB_ms": kc * 1e3}))
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
    # mixed right-hand side against the FP64 one on the same state, per grid
    # function (max |mixed - fp64| / max |fp64| over interior points); the
    # comparisons with the CPU oracle itself are the parity tests'
    rhs_mx = gmx.rhs(st)
    g64.rhs(st, rhs)
    mixed_err = {}
    for v in range(24):
        a64, amx = g64.view(rhs, v, ghosts=False), gmx.view(rhs_mx, v, ghosts=False)
        scale = float(a64.abs().max())
        d = float((amx - a64).abs().max())
        mixed_err[I.BSSN_NAMES[v]] = d / scale if scale else d
    del rhs_mx

    khi = _high_order_times(C, torch, n, h, y0, kw)

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

    # batch: 64 uneven patches (24..96 per axis, three refinement levels),
    # analytic gauge-wave ghosts, one graph-captured persistent launch per
    # substage, autotuned; 20 RK4 steps timed per precision
    batch = {}
    if not args.no_batch:
        import tempfile
        specs = I.patch_list(I.SEED0 + 4, 64, 24, 96)
        npts = sum(int(np.prod(p["n"])) for p in specs)
        dtb = 0.25 * min(p["h"] for p in specs)
        for name, prec in (("fp64", C.FP64), ("mixed", C.MIXED)):
            grids, states, wss = [], [], []
            for p in specs:
                g = C.Grid(p["n"], 3, p["h"], origin=p["origin"], system=C.BSSN, precision=prec,
                           boundary=C.BC_GAUGEWAVE, slicing=C.SLICING_HARMONIC,
                           shift=C.SHIFT_FROZEN, gw_amp=0.1, gw_wavelength=1.0, gw_axis=0)
                grids.append(g)
                states.append(g.upload(I.gaugewave(p["n"], p["h"], p["origin"], 0.1, 1.0, 0)))
                wss.append(g.new_workspace())
            meta = torch.empty(C.batch_meta_bytes(len(grids)) // 8, dtype=torch.float64,
                               device="cuda")
            # untuned plan first (the 32x8 staged kind), then the autotuned one
            C.batch_step(grids, states, wss, meta, 0.0, dtb, 1)
            ku = _events_time(lambda: C.batch_step(grids, states, wss, meta, dtb, dtb, 20), 1) / 20
            C.batch_release(meta)
            with tempfile.TemporaryDirectory() as td:
                tpath = os.path.join(td, "tune.json")
                C.autotune(grids, states, wss, meta, tpath)
                with open(tpath) as f:
                    table = json.load(f)
            C.batch_step(grids, states, wss, meta, 0.0, dtb, 1)
            kb = _events_time(lambda: C.batch_step(grids, states, wss, meta, dtb, dtb, 20), 1) / 20
            C.batch_release(meta)
            tk = next((v for k, v in table.items() if k.endswith("_kind")), {})
            batch[name] = {"ms_per_step": kb * 1e3, "point_steps_per_s": npts / kb,
                           "rhs_updates_per_s": 4 * npts / kb, "kernel_kind": tk.get("kind"),
                           "untuned_ms_per_step": ku * 1e3,
                           "untuned_kernel_kind": tk.get("untuned_kind"),
                           "tuner_kinds": tk.get("kinds"),
                           "tuner_kind0_tiles": {k.split("_")[-1]: v["tile"]
                                                 for k, v in table.items() if "_kind0_" in k}}
            del grids, states, wss, meta
            torch.cuda.synchronize()
        batch["points"] = npts
        batch["patches"] = len(specs)
        print("[bench] batch done", file=sys.stderr, flush=True)

    # two refinement levels: a 96^3 fine patch (ghost 3) centred in the 128^3
    # BSSN level, prolongation from three coarse time levels and restriction
    amr = _amr_timing(C, torch)
    print("[bench] amr done", file=sys.stderr, flush=True)

    # streaming copy: achievable bandwidth and the counter calibration kernel
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    C.probe_copy(b, a, nbytes)
    kcopy = _events_time(lambda: C.probe_copy(b, a, nbytes), 10)
    copy_bw = 2 * nbytes / kcopy
    del a, b
    # FMA throughput probe: the measured vector ALU rate, FP64 and unpacked FP32
    probe_out = torch.empty(C.lib().chemora_probe_fma_bytes() // 8, dtype=torch.float64,
                            device="cuda")
    alu_probe = {}
    for name, prec in (("fp64", C.FP64), ("fp32_unpacked", C.MIXED)):
        fl_probe = C.probe_fma(prec, probe_out, 4096)
        kfma = _events_time(lambda: C.probe_fma(prec, probe_out, 4096), 10)
        alu_probe[name] = fl_probe / kfma
    del probe_out
    torch.cuda.synchronize()
    print("[bench] gpu done", file=sys.stderr, flush=True)

    # ---- roofline of the dominant kernel (right-hand side, FP64): both the
    # HBM bound (algorithmic bytes) and the FP64 ALU bound (counted flops);
    # "roofline" is the one whose ideal time is longer, i.e. the binding one
    fl = _facts()
    bytes_launch = BSSN_BYTES_PER_PT * pts
    traffic64 = traffic_mx = None
    if fl and fl["traffic_valid"]:
        traffic64 = fl["traffic"].get("fp64_bytes_per_launch")
        traffic_mx = fl["traffic"].get("mixed_bytes_per_launch")
    roof_hbm = {"bound": "hbm", "achieved": bytes_launch / k64 / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": bytes_launch / k64 / HBM_PEAK, "traffic": traffic64,
                "kernel": KERNEL_FP64, "kernel_ms": k64 * 1e3,
                "bytes_per_point": BSSN_BYTES_PER_PT, "points_per_launch": pts}
    roof = roof_hbm
    roof_other = None
    roof_mx = {"bound": "hbm", "achieved": bytes_launch / kmx / 1e9, "peak": HBM_PEAK / 1e9,
               "unit": "GB/s", "frac": bytes_launch / kmx / HBM_PEAK, "traffic": traffic_mx,
               "kernel": KERNEL_MIXED, "kernel_ms": kmx * 1e3}
    if fl:
        f64 = fl["fp64"]["flops_per_point"]
        roof_alu = {"bound": "alu", "achieved": f64 * pts / k64 / 1e12, "peak": FP64_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": f64 * pts / k64 / FP64_PEAK,
                    "traffic": traffic64, "kernel": KERNEL_FP64,
                    "kernel_ms": k64 * 1e3, "flops_per_point": f64, "points_per_launch": pts,
                    "flops_per_point_expression": FLOPS_PER_POINT_EXPRESSION,
                    "probe_peak": alu_probe["fp64"] / 1e12,
                    "frac_of_probe": f64 * pts / k64 / alu_probe["fp64"]}
        if f64 * pts / FP64_PEAK > bytes_launch / HBM_PEAK:
            roof, roof_other = roof_alu, roof_hbm
        else:
            roof_other = roof_alu
        fmx = fl["mixed"]["f32_flops_per_point"] + fl["mixed"]["f64_flops_per_point"]
        if fmx * pts / UNPACKED_PEAK > bytes_launch / HBM_PEAK:
            roof_mx = {"bound": "alu", "achieved": fmx * pts / kmx / 1e12,
                       "peak": UNPACKED_PEAK / 1e12, "unit": "TFLOP/s",
                       "frac": fmx * pts / kmx / UNPACKED_PEAK, "traffic": traffic_mx,
                       "kernel": KERNEL_MIXED, "kernel_ms": kmx * 1e3,
                       "flops_per_point": fmx, "points_per_launch": pts,
                       "probe_peak": alu_probe["fp32_unpacked"] / 1e12,
                       "frac_of_probe": fmx * pts / kmx / alu_probe["fp32_unpacked"],
                       "note": "f32 (unpacked) and f64 vector operations, both at 78.6 TFLOP/s"}

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
               "cores": oracle.num_threads(), "cpu_model": _cpu_model(), "kind": "oracle",
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
                  "dtype": "f32 arithmetic on f64 state", "roofline": roof_mx,
                  "rhs_error_vs_fp64_per_gf": mixed_err,
                  "rhs_error_vs_fp64_max": max(mixed_err.values())},
        "kernels_ms": {"bssn_rhs_fp64": k64 * 1e3, "bssn_rhs_mixed": kmx * 1e3,
                       "ghost_periodic_24var": kghost * 1e3, "constraints_fp64": kcons * 1e3,
                       "bssn_rk4_step_fp64": krk64 * 1e3, "bssn_rk4_step_mixed": krkmx * 1e3,
                       "wave256_rk4_step_fp64": kw64 * 1e3, "wave256_rk4_step_mixed": kwmx * 1e3,
                       "copy_1GiB": kcopy * 1e3, **khi},
        "derived": {"bssn_rk4_rhs_updates_per_s_fp64": 4 * pts / krk64,
                    "bssn_rk4_rhs_updates_per_s_mixed": 4 * pts / krkmx,
                    "wave256_rk4_point_steps_per_s_fp64": nw ** 3 / kw64,
                    "wave256_rk4_GBps_fp64": 272 * nw ** 3 / kw64 / 1e9,
                    "wave256_rk4_GBps_mixed": 272 * nw ** 3 / kwmx / 1e9,
                    "copy_GBps": copy_bw / 1e9,
                    "fma_probe_TFLOPs_fp64": alu_probe["fp64"] / 1e12,
                    "fma_probe_TFLOPs_fp32_unpacked": alu_probe["fp32_unpacked"] / 1e12},
        "batch64": batch or None,
        "amr": amr,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
