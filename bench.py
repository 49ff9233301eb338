"""Benchmark of the hot path on one GPU.

Main line: explicit FP64 2D steps of the relaxation scheme on the periodic
2D Grass dune, 2000 x 2000 cells on [0, 1000]^2 m, A_g = 1e-3, m_g = 3,
CFL 0.5.  One step is one pass of the whole method (ghosts, projection,
interface Riemann solves, conservative update and the CFL wave-speed
reduction for the next step).

Two more legs measure the forms built on the step:
  * ensemble: 256 periodic Grass dunes of sides drawn from
    {256, 384, 512, 768, 1024} (A_g log-uniform on [1e-4, 1e-2], m_g uniform
    on [1, 4], bump amplitude uniform on [0.5, 1]), each with its own CFL dt,
    advanced in one graph-replayed persistent launch per step, against the
    same steps run member by member with the single-grid kernel;
  * adjoint: 1024 x 1024 Grass dune, 2000 fixed-dt steps, loss
    1/2 |z_b(T) - z_target|^2 with z_target from a run with a smooth +-30 %
    A_g field; gradients with respect to the initial state and the A_g field
    with sqrt(N) checkpointing, against the plain forward run.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "cell-updates/s and % HBM roofline (FP64 2D); ensemble and adjoint vs plain"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
BYTES_PER_CELL_FP64 = 64.0     # read h, hu, hv, z_b and write them once (8 B each)
O2_BYTES_PER_CELL = 160.0      # second-order step: U^n + rate (64 B), U^n + rate + U^{n+1} (96 B)
O2_BYTES_PER_CELL_FP32 = 112.0  # the same with float32 state (the rate stays FP64)
NX = NY = 2000

# HBM traffic of the fused step kernel on the main workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each
# scaled by the ratio of known bytes to the same counter on a plain
# streaming kernel (1 GiB read, 1 GiB written): FETCH_SIZE x 2.0000,
# WRITE_SIZE x 1.0000.  Valid only for the kernel sources it was taken on
# (kernel_source_hash) and the automatic tile split; otherwise the bench
# reports null.  Summary: profiles/k_fused_dune2000_fp64_hbm_traffic.md.
TRAFFIC = {"src": "36eed45562e5ce34", "rows": 0,
           "fetch_kib": 69010.4, "write_kib": 125210.3,
           "bytes_per_launch": 269.55e6}

# VALU activity of the same kernel, build and workload (rocprofv3 --pmc
# SQ_INSTS_VALU, SQ_INSTS_VALU_TRANS_F64; wavefront instructions per
# dispatch, summed over the device).  The chip issues one wave64 VALU
# instruction per SIMD every 4 cycles (16 for FP64 transcendentals):
# 256 CUs x 4 SIMDs at 2.4 GHz.  Summary: profiles/k_fused_dune2000_fp64_valu.md.
VALU = {"src": "36eed45562e5ce34", "rows": 0,
        "insts_valu": 39035198, "insts_trans_f64": 1111242}
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
# Algorithmic FP64 operations per 2D cell-update (estimate: about 110 flops,
# 3 square roots and 3 divisions per interface solve, two interfaces per
# cell, and about 30 for the Grass m_g = 3 closure), against the 78.6
# TFLOP/s FP64 vector peak.
ALG_FLOPS_PER_CELL = 2 * (110 + 3 + 3) + 30
FP64_PEAK_TFLOPS = 78.6


# What the step kernel's code and launch are built from: its sources, the
# host code that sizes its grid, and the build flags.
KERNEL_SOURCES = ("paper_1307_0491_amd/csrc/sve_api.hip", "paper_1307_0491_amd/csrc/sve_fused.hpp",
                  "paper_1307_0491_amd/csrc/sve_kernels.hpp",
                  "paper_1307_0491_amd/csrc/sve_device.hpp",
                  "paper_1307_0491_amd/csrc/sve_context.hpp", "include/sve.h",
                  "paper_1307_0491_amd/build.py")


def kernel_source_hash() -> str:
    """Hash of the files the step kernel is built and launched from (any
    change to them, comments included, invalidates the recorded counters)."""
    if os.environ.get("SVE_LIBRARY"):
        return "external"                # a library not built from these sources
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def workload():
    import workloads as W
    h, hu, hv, zb, dx, dy = W.dune2d(NX, NY)
    return h, hu, hv, zb


def cpu_baseline(nsteps: int = 20):
    """The oracle as it stands, on the host, over `nsteps` steps of the same
    2000 x 2000 grid (bounded sample of the workload)."""
    import oracle as O
    h, hu, hv, zb = workload()
    o = O.Oracle2D(h, hu, hv, zb, 1000.0 / NX, 1000.0 / NY,
                   O.Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0), (O.BC(),) * 4)
    t0 = time.perf_counter()
    o.step(nsteps, 0.5)
    el = time.perf_counter() - t0
    return {"value": NX * NY * nsteps / el, "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{nsteps} CFL steps of the full {NX}x{NY} grid, numpy FP64, one process",
            "seconds": el, "host": host_cpu()}


def cpu_baseline_order2(nsteps: int = 2):
    """The oracle's second-order variant on the same 2000 x 2000 grid over
    `nsteps` CFL steps (bounded sample of the order2 leg's workload)."""
    import oracle as O
    h, hu, hv, zb = workload()
    o = O.Oracle2D(h, hu, hv, zb, 1000.0 / NX, 1000.0 / NY,
                   O.Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0, order=2), (O.BC(),) * 4)
    t0 = time.perf_counter()
    o.step(nsteps, 0.5)
    el = time.perf_counter() - t0
    return {"value": NX * NY * nsteps / el, "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{nsteps} second-order CFL steps of the full {NX}x{NY} grid, numpy FP64, "
                      "one process",
            "seconds": el}


def cpu_baseline_1d(nsteps: int = 20000):
    """The oracle on the 1D dune (1000 cells, periodic, CFL 0.5) over the
    first `nsteps` of its 218 402 steps to T = 10000 s (bounded sample)."""
    import oracle as O
    import workloads as W
    h, hu, zb, dx = W.dune1d(1000)
    o = O.Oracle1D(h, hu, zb, dx, O.Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0),
                   (O.BC(), O.BC()))
    t0 = time.perf_counter()
    o.step(nsteps, 0.5, 10000.0)
    el = time.perf_counter() - t0
    rate = 1000.0 * nsteps / el
    return {"value": rate, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {nsteps} of the {DUNE1D_STEPS} CFL steps to T = 10000 s, "
                      "numpy FP64, one process",
            "seconds": el,
            "full_run_s_extrapolated": 1000.0 * DUNE1D_STEPS / rate}


def host_cpu():
    """CPU model and logical CPU count of the host the oracle ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "cpu_count": os.cpu_count()}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def device_warmup(torch, ms: float):
    """FP64 matrix products (4096 x 4096) on the device for `ms` milliseconds.
    During a leg's host-side set-up the GPU idles and its clock drops; it
    rises again only under sustained FP64 load, so without this the step
    kernel's first ~300 launches run about 10 % slower (98-102 against
    88-90 us at 2000^2) and a short timed run measures the clock's ramp.
    These products are not steps of the method; they run before the
    warm-up steps and outside the timed region."""
    if ms <= 0:
        return
    a = torch.randn(4096, 4096, dtype=torch.float64, device="cuda")
    b = torch.randn(4096, 4096, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(4):
            torch.matmul(a, b, out=c)
        torch.cuda.synchronize()
    del a, b, c


def main_leg(args, sve, torch):
    h, hu, hv, zb = workload()
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 4
    stream = sve.current_stream_handle()
    s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p, bcs=bcs, stream=stream)
    s.set_path({"fused": sve.PATH_FUSED, "split": sve.PATH_SPLIT,
                "residual": sve.PATH_RESIDUAL}[args.path])
    s.set_tile_rows(args.rows)
    torch.cuda.synchronize()
    device_warmup(torch, args.device_warmup_ms)
    if args.warmup:
        s.step(args.warmup, 0.5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps, 0.5)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = s.last_elapsed_ms()           # HIP events on the launch stream
    (gh, ghu, ghv, gz), t, dtl, ns = s.get_state()
    s.close()
    ok = bool(np.all(np.isfinite(gh)) and np.all(gh > 0))
    return wall, kern_ms, t, ns, ok


def copy_calibration(torch, mib: int, reps: int = 5):
    """Plain streaming kernels of a known size (read 8n bytes, write 8n
    bytes: an elementwise multiply by one), for scaling the HBM counters."""
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    return {"bytes_read": 8 * n, "bytes_written": 8 * n, "reps": reps}


def copy_peak(torch, mib: int = 1024, reps: int = 10) -> float:
    """Achieved HBM bandwidth of a plain streaming kernel (b = a * 1, float64,
    `mib` MiB read and written per launch), GB/s, timed with events on
    torch's stream, where the kernel runs."""
    n = mib * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    gbs = 16.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def mpm_leg(args, sve, torch):
    """Meyer-Peter & Mueller channel, Strickler K_s = 40, 8192 x 2048 cells on
    4000 x 1000 m, inflow (h 0.5, hu 2) and free boundaries; FP64 storage
    and FP32 storage (FP64 arithmetic)."""
    import workloads as W
    h, hu, hv, zb, dx, dy = W.mpm_channel()
    ny, nx = h.shape
    p = sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0, d_s=1e-3,
                   s=2.65, tau_cr=0.05)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE)]
    out = {"nx": nx, "ny": ny, "steps": args.mpm_steps, "warmup": args.mpm_warmup}
    for storage, bpc in (("fp64", 64.0), ("fp32", 32.0)):
        s = sve.Solver(h, hu, zb, hv, lx=4000.0, ly=1000.0, params=p, bcs=bcs, storage=storage,
                       stream=sve.current_stream_handle())
        torch.cuda.synchronize()
        device_warmup(torch, args.device_warmup_ms)
        s.step(args.mpm_warmup, 0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.mpm_steps, 0.5)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_launch = s.last_elapsed_ms() * 1e-3 / args.mpm_steps
        (gh, _, _, _), t, _, _ = s.get_state()
        s.close()
        achieved = bpc * nx * ny / per_launch / 1e9
        out[storage] = {"cell_updates_per_s": nx * ny * args.mpm_steps / wall,
                        "ms_per_step": wall * 1e3 / args.mpm_steps,
                        "avg_launch_us": per_launch * 1e6, "bytes_per_cell": bpc,
                        "hbm_achieved_GBs": achieved, "hbm_frac": achieved / HBM_PEAK_GBS,
                        "sim_time_s": t, "finite": bool(np.all(np.isfinite(gh)))}
        progress(f"mpm {storage}: {args.mpm_steps} steps in {wall:.3f} s")
    return out


# CFL-0.5 steps of the 1D dune from t = 0 to T = 10000 s, the last one
# clipped to land on T (the oracle's count; the full-size parity test checks
# that the library takes the same steps).
DUNE1D_STEPS = 218402


def dune1d_leg(args, sve, torch):
    """1D Grass dune, 1000 cells on [0, 1000] m, periodic, CFL 0.5, run to
    T = 10000 s (default path: one workgroup with the grid in LDS)."""
    import workloads as W
    h, hu, zb, dx = W.dune1d(1000)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0)
    s = sve.Solver(h, hu, zb, lx=1000.0, params=p, bcs=[sve.BC(sve.BC_PERIODIC)] * 2,
                   stream=sve.current_stream_handle())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = s.step(DUNE1D_STEPS, 0.5, 10000.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    (gh, _, _), _, dtl, _ = s.get_state()
    s.close()
    progress(f"dune1d: T = {t} s in {wall:.3f} s")
    out = {"nx": 1000, "t_end": t, "steps": DUNE1D_STEPS, "wall_s": wall,
           "cell_updates_per_s": 1000.0 * DUNE1D_STEPS / wall,
           "us_per_step": wall * 1e6 / DUNE1D_STEPS, "last_dt": dtl}
    if t != 10000.0 or not dtl > 0.0:
        out["error"] = "the run did not end on T with its last step"
    return out


# CFL-0.5 steps of the paper's 1D antidune (2400 cells) from t = 0 to T = 50 s,
# the last one clipped to land on T (the oracle's count, stored with the
# full-size parity test's reference).
ANTIDUNE_STEPS = 78010


def antidune_leg(args, sve, torch):
    """The paper's 1D antidune (subsection "1D antidune evolution"): 2400
    cells on a 24 m channel, q0 = 1.7, h0 = 0.5, Grass A_g = 1e-3, m_g = 3,
    inflow west / free east, CFL 0.5, to T = 50 s (one launch per step of
    the one-pass 1D kernel)."""
    import workloads as W
    h, hu, zb, dx = W.antidune1d(2400)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0)
    s = sve.Solver(h, hu, zb, lx=24.0, params=p,
                   bcs=[sve.BC(sve.BC_INFLOW, 0.5, 1.7, 0.0), sve.BC(sve.BC_FREE)],
                   stream=sve.current_stream_handle())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = s.step(ANTIDUNE_STEPS, 0.5, 50.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    (gh, _, gz), _, _, ns = s.get_state()
    s.close()
    x = (np.arange(2400) + 0.5) * dx
    progress(f"antidune: T = {t} s in {wall:.3f} s")
    out = {"nx": 2400, "t_end": t, "steps": int(ns), "wall_s": wall,
           "cell_updates_per_s": 2400.0 * ns / wall, "us_per_step": wall * 1e6 / ns,
           "crest_x_m": [float(x[np.argmax(zb)]), float(x[np.argmax(gz)])]}
    if t != 50.0:
        out["error"] = "the run did not end on T"
    return out


def laws_leg(args, sve, torch):
    """The other threshold laws (eqs. "FLVB", "Nielsen", "Ribberink",
    "Camenen") and the Meyer-Peter & Mueller law with the Manning and
    Darcy-Weisbach slopes, on the MPM channel (8192 x 2048, inflow / free,
    FP64): average launch time and HBM fraction of each closure's step."""
    import workloads as W
    h, hu, hv, zb, dx, dy = W.mpm_channel()
    ny, nx = h.shape
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE)]
    cases = (("MPM", "STRICKLER", 40.0), ("MPM", "MANNING", 0.025), ("MPM", "DARCY", 0.05),
             ("FLVB", "STRICKLER", 40.0), ("NIELSEN", "STRICKLER", 40.0),
             ("RIBBERINK", "STRICKLER", 40.0), ("CAMENEN", "STRICKLER", 40.0))
    out = {"nx": nx, "ny": ny, "steps": args.laws_steps}
    for law, fric, coef in cases:
        p = sve.Params(law=getattr(sve, "LAW_" + law), friction=getattr(sve, "FRIC_" + fric),
                       fric_coef=coef, d_s=1e-3, s=2.65, tau_cr=0.05)
        s = sve.Solver(h, hu, zb, hv, lx=4000.0, ly=1000.0, params=p, bcs=bcs,
                       stream=sve.current_stream_handle())
        torch.cuda.synchronize()
        device_warmup(torch, args.device_warmup_ms)
        s.step(5, 0.5)
        torch.cuda.synchronize()
        s.step(args.laws_steps, 0.5)
        per_launch = s.last_elapsed_ms() * 1e-3 / args.laws_steps
        s.close()
        out[f"{law}/{fric}"] = {"avg_launch_us": per_launch * 1e6,
                                "cell_updates_per_s": nx * ny / per_launch,
                                "hbm_frac": BYTES_PER_CELL_FP64 * nx * ny / per_launch / 1e9
                                            / HBM_PEAK_GBS}
    progress(f"laws: {len(cases)} closures x {args.laws_steps} steps")
    return out


def run_to(s, t_end, cfl=0.5, chunk=1000):
    """Advance solver s to t_end; returns the number of steps that advanced
    the time (chunks of `chunk` steps while they stay clear of t_end, then
    single steps, the last one clipped to land on t_end) and the summed
    time between the HIP events around each call's launches (ms)."""
    t = s.step(1, cfl, t_end)
    kern_ms = s.last_elapsed_ms()
    steps = 1
    dt = t
    while t < t_end:
        if t + 1.2 * chunk * dt < t_end:
            t_new = s.step(chunk, cfl)
            dt = (t_new - t) / chunk
            steps += chunk
        else:
            t_new = s.step(1, cfl, t_end)
            steps += 1
        kern_ms += s.last_elapsed_ms()
        t = t_new
    return steps, kern_ms


def paper2d_leg(args, sve, torch):
    """The paper's 2D bump cases (subsection "2D dune evolution cases"):
    4000 x 4000 cells on [0, 1000]^2 m, z_b = 0.1 + bump, h = 10 - z_b,
    hu = q0 = 10, hv = 0; inflow at x = 0 with (h, hu, hv) = (9.9, 10, 0), the
    initial state there; free flow on the other sides; Grass m_g = 3 with
    A_g = 1 to T = 500 s and A_g = 0.1 to T = 1000 s; CFL 0.5; FP64."""
    import workloads as W
    n = args.paper_n
    h, hu, hv, zb, dx, dy = W.dune2d(n, n, base=0.1)
    bcs = [sve.BC(sve.BC_INFLOW, 9.9, 10.0, 0.0), sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE)]
    out = {"nx": n, "ny": n}
    runs = ((0.1, 1000.0),) if args.paper_runs == "scaling" else ((1.0, 500.0), (0.1, 1000.0))
    for ag, t_end in runs:
        s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0,
                       params=sve.Params(law=sve.LAW_GRASS, A_g=ag, m_g=3.0), bcs=bcs,
                       stream=sve.current_stream_handle())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, kern_ms = run_to(s, t_end)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        (gh, _, _, gz), t, _, _ = s.get_state()
        s.close()
        k = int(np.argmax(gz))
        out[f"A_g={ag:g}"] = {
            "t_end": t, "steps": steps, "wall_s": wall,
            "cell_updates_per_s": n * n * steps / wall,
            "ms_per_step": wall * 1e3 / steps,
            "avg_launch_us": kern_ms * 1e3 / steps,
            "hbm_frac": BYTES_PER_CELL_FP64 * n * n * steps / (kern_ms * 1e-3) / 1e9
                        / HBM_PEAK_GBS,
            "zb_max": float(gz.max()), "zb_max_at_m": [float((k % n + 0.5) * dx),
                                                      float((k // n + 0.5) * dy)],
            "finite": bool(np.all(np.isfinite(gh)) and np.all(gh > 0))}
        progress(f"paper2d A_g={ag:g}: T = {t} s, {steps} steps in {wall:.1f} s")
    return out


def wb_leg(args, sve, torch):
    """The well-balanced variant (hydrostatic reconstruction) against the
    paper's scheme on the paper's 2D bump at 2000 x 2000 cells (inflow (9.9,
    10, 0) west, free elsewhere, Grass A_g = 0.1, m_g = 3, CFL 0.5, FP64),
    both on the default (fused) path."""
    import workloads as W
    n = 2000
    h, hu, hv, zb, dx, dy = W.dune2d(n, n, base=0.1)
    bcs = [sve.BC(sve.BC_INFLOW, 9.9, 10.0, 0.0), sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE)]
    out = {"nx": n, "ny": n, "steps": args.wb_steps}
    for name, rec in (("paper_scheme", 0), ("well_balanced", 1)):
        p = sve.Params(law=sve.LAW_GRASS, A_g=0.1, m_g=3.0, reconstruction=rec)
        s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p, bcs=bcs,
                       stream=sve.current_stream_handle())
        torch.cuda.synchronize()
        device_warmup(torch, args.device_warmup_ms)
        s.step(20, 0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.wb_steps, 0.5)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_launch = s.last_elapsed_ms() * 1e-3 / args.wb_steps
        (gh, _, _, _), t, _, _ = s.get_state()
        s.close()
        out[name] = {"cell_updates_per_s": n * n * args.wb_steps / wall,
                     "ms_per_step": wall * 1e3 / args.wb_steps,
                     "avg_launch_us": per_launch * 1e6,
                     "hbm_frac": BYTES_PER_CELL_FP64 * n * n / per_launch / 1e9 / HBM_PEAK_GBS,
                     "sim_time_s": t, "finite": bool(np.all(np.isfinite(gh)) and np.all(gh > 0))}
        progress(f"wb {name}: {args.wb_steps} steps in {wall:.3f} s")
    out["cost_vs_paper_scheme"] = (out["well_balanced"]["avg_launch_us"]
                                   / out["paper_scheme"]["avg_launch_us"])
    return out


def order2_leg(args, sve, torch):
    """The second-order variant (MUSCL-minmod, Heun; two kernels per step) on
    the main workload (periodic 2000 x 2000 Grass dune, A_g = 1e-3, m_g = 3,
    CFL 0.5, FP64), with either interface problem, against the first-order
    step on the same grid.  HBM bytes per cell-step of the two kernels: the
    first reads U^n and writes the FP64 rate (64 B), the second reads U^n
    and the rate and writes U^{n+1} (96 B)."""
    import workloads as W
    h, hu, hv, zb, dx, dy = W.dune2d(NX, NY)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 4
    out = {"nx": NX, "ny": NY, "steps": args.o2_steps, "bytes_per_cell_step": O2_BYTES_PER_CELL}
    for name, order, rec in (("first_order", 1, 0), ("second_order", 2, 0),
                             ("second_order_well_balanced", 2, 1)):
        p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0, reconstruction=rec, order=order)
        s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p, bcs=bcs,
                       stream=sve.current_stream_handle())
        torch.cuda.synchronize()
        device_warmup(torch, args.device_warmup_ms)
        s.step(20, 0.5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.o2_steps, 0.5)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_step = s.last_elapsed_ms() * 1e-3 / args.o2_steps
        (gh, _, _, gz), t, _, _ = s.get_state()
        s.close()
        bpc = BYTES_PER_CELL_FP64 if order == 1 else O2_BYTES_PER_CELL
        out[name] = {"cell_updates_per_s": NX * NY * args.o2_steps / wall,
                     "ms_per_step": wall * 1e3 / args.o2_steps,
                     "kernel_us_per_step": per_step * 1e6,
                     "hbm_frac": bpc * NX * NY / per_step / 1e9 / HBM_PEAK_GBS,
                     "sim_time_s": t, "zb_max": float(np.max(gz)),
                     "finite": bool(np.all(np.isfinite(gh)) and np.all(gh > 0))}
        progress(f"order2 {name}: {args.o2_steps} steps in {wall:.3f} s")
    for name in ("second_order", "second_order_well_balanced"):
        out[name]["cost_vs_first_order"] = (out[name]["kernel_us_per_step"]
                                            / out["first_order"]["kernel_us_per_step"])
    out["mpm_channel"] = o2_mpm_channel(args, sve, torch)
    if args.o2_dune1d:
        out["paper_1d_dune"] = o2_dune1d_accuracy(sve, torch)
    return out


def o2_mpm_channel(args, sve, torch):
    """The second-order variant on the MPM channel (8192 x 2048 cells,
    inflow / free, FP64 and FP32 storage) beside the first-order step."""
    import workloads as W
    h, hu, hv, zb, dx, dy = W.mpm_channel()
    ny, nx = h.shape
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE)]
    steps = max(1, args.o2_steps // 5)
    out = {"nx": nx, "ny": ny, "steps": steps}
    for name, order, storage, bpc in (("first_order_fp64", 1, "fp64", BYTES_PER_CELL_FP64),
                                      ("second_order_fp64", 2, "fp64", O2_BYTES_PER_CELL),
                                      ("second_order_fp32", 2, "fp32", O2_BYTES_PER_CELL_FP32)):
        p = sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0, d_s=1e-3,
                       s=2.65, tau_cr=0.05, order=order)
        s = sve.Solver(h, hu, zb, hv, lx=4000.0, ly=1000.0, params=p, bcs=bcs, storage=storage,
                       stream=sve.current_stream_handle())
        torch.cuda.synchronize()
        device_warmup(torch, args.device_warmup_ms)
        s.step(5, 0.45)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, 0.45)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_step = s.last_elapsed_ms() * 1e-3 / steps
        (gh, _, _, _), t, _, _ = s.get_state()
        s.close()
        out[name] = {"cell_updates_per_s": nx * ny * steps / wall,
                     "kernel_us_per_step": per_step * 1e6,
                     "hbm_frac": bpc * nx * ny / per_step / 1e9 / HBM_PEAK_GBS,
                     "sim_time_s": t,
                     "finite": bool(np.all(np.isfinite(gh)) and np.all(gh > 0))}
        progress(f"order2 MPM channel {name}: {steps} steps in {wall:.3f} s")
    out["second_order_cost_vs_first_order"] = (out["second_order_fp64"]["kernel_us_per_step"]
                                               / out["first_order_fp64"]["kernel_us_per_step"])
    return out


def o2_dune1d_accuracy(sve, torch):
    """The paper's 1D dune (Grass A_g = 1, m_g = 3, periodic, T = 700 s),
    where the paper finds J = 2000 cells diffusive and refines to 20000:
    J = 2000 at first and second order against J = 20000 at first order
    (averaged onto the coarse cells); L1 distance of z_b and crest."""
    import workloads as W
    res = {"t_end": 700.0}
    zs = {}
    for name, J, order in (("J20000_first_order", 20000, 1), ("J2000_first_order", 2000, 1),
                           ("J2000_second_order", 2000, 2)):
        h, hu, zb, dx = W.dune1d(J)
        p = sve.Params(law=sve.LAW_GRASS, A_g=1.0, m_g=3.0, order=order)
        s = sve.Solver(h, hu, zb, lx=1000.0, params=p, bcs=[sve.BC(sve.BC_PERIODIC)] * 2,
                       stream=sve.current_stream_handle())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            t, _, ns = s.times()
            if t >= 700.0:
                break
            s.step(20000, 0.5, t_end=700.0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        (_, _, z), t, _, ns = s.get_state()
        s.close()
        zs[name] = z
        res[name] = {"cells": J, "order": order, "wall_s": wall, "sim_time_s": t}
        progress(f"order2 1D dune {name}: T = {t} s in {wall:.2f} s")
    ref = zs["J20000_first_order"].reshape(2000, 10).mean(axis=1)
    x = W.cell_centres(2000, 1000.0)
    res["reference_crest"] = {"z": float(ref.max()), "x": float(x[np.argmax(ref)])}
    for name in ("J2000_first_order", "J2000_second_order"):
        z = zs[name]
        res[name].update({"l1_vs_J20000": float(np.mean(np.abs(z - ref))),
                          "crest_z": float(z.max()), "crest_x": float(x[np.argmax(z)])})
    return res


def ensemble_leg(args, sve, torch):
    import workloads as W
    from paper_1307_0491_amd.ensemble import Ensemble
    draw = W.ensemble_draw(args.ens_members)
    members = []
    cells = 0
    for m in draw:
        h, hu, hv, zb, dx, dy = W.ensemble_member_state(m)
        members.append(dict(h=h, hu=hu, hv=hv, zb=zb, lx=1000.0, ly=1000.0, A_g=m.Ag, m_g=m.mg))
        cells += m.n * m.n
    e = Ensemble(members, stream=sve.current_stream_handle())
    del members
    rows, mode = e.autotune(3, 0.5)
    e.step(5, 0.5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.step(args.ens_steps, 0.5)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    ms_b = e.last_elapsed_ms()
    progress(f"ensemble batched: {args.ens_steps} steps in {wall_b:.3f} s")
    t0 = time.perf_counter()
    e.step_sequential(args.ens_seq_steps, 0.5)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    ms_s = e.last_elapsed_ms()
    progress(f"ensemble sequential: {args.ens_seq_steps} steps in {wall_s:.3f} s")
    e.close()
    per_b = wall_b / args.ens_steps
    per_s = wall_s / args.ens_seq_steps
    sizes = {}
    for m in draw:
        sizes[m.n] = sizes.get(m.n, 0) + 1
    return {"members": len(draw), "cells": cells, "member_sizes": sizes,
            "schedule": {"tile_rows": rows, "mode": "queue" if mode == 0 else "grid"},
            "batched": {"steps": args.ens_steps, "ms_per_step": per_b * 1e3,
                        "kernel_ms_per_step": ms_b / args.ens_steps,
                        "cell_updates_per_s": cells / per_b},
            "sequential": {"steps": args.ens_seq_steps, "ms_per_step": per_s * 1e3,
                           "kernel_ms_per_step": ms_s / args.ens_seq_steps,
                           "cell_updates_per_s": cells / per_s},
            "speedup_vs_sequential": per_s / per_b}


def adjoint_leg(args, sve, torch):
    import workloads as W
    from paper_1307_0491_amd.adjoint import AdjointRun
    n = args.adj_n
    h, hu, hv, zb, dx, dy = W.dune2d(n, n)
    ag_true = W.adjoint_ag_field(n, n)
    ag0 = np.full((n, n), 1e-3)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 4
    stream = sve.current_stream_handle()

    def solver(ag):
        s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p, bcs=bcs, Ag=ag,
                       stream=stream)
        s.set_tile_rows(args.adj_fwd_rows)
        return s

    s = solver(ag0)
    s.step(1, 0.5)
    _, _, dt_cfl, _ = s.get_state()
    s.close()
    dt = 0.9 * dt_cfl
    steps = args.adj_steps
    s = solver(ag_true)
    s.step_fixed_dt(steps, dt)
    z_target = s.get_state_torch()[0][3].clone()
    s.close()
    # plain forward at the evaluation point
    s = solver(ag0)
    s.step_fixed_dt(5, dt)
    s.close()
    s = solver(ag0)
    torch.cuda.synchronize()
    device_warmup(torch, args.device_warmup_ms)
    t0 = time.perf_counter()
    s.step_fixed_dt(steps, dt)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    s.close()
    progress(f"adjoint: plain forward {fwd:.3f} s")
    # forward with checkpoints, then the reverse sweep.  A second gradient on
    # the same context (over the next window of `steps` steps) reuses the
    # checkpoint buffers: its time is the steady-state cost of a gradient.
    s = solver(ag0)
    run = AdjointRun(s)
    run.set_tile_rows(args.adj_rows)
    times = []
    for it in range(2):
        torch.cuda.synchronize()
        device_warmup(torch, args.device_warmup_ms)
        t0 = time.perf_counter()
        run.forward(steps, dt)
        zT = s.get_state_torch()[0][3]
        gT = torch.zeros((4, n, n), dtype=torch.float64, device="cuda")
        gT[3] = zT - z_target
        g0, gAg = run.backward(gT)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        progress(f"adjoint: forward with checkpoints + backward {times[-1]:.3f} s")
        if it == 0:
            loss = 0.5 * float(torch.sum((zT - z_target) ** 2))
            g_linf = (float(g0[3].abs().max()), float(gAg.abs().max()))
            finite = bool(torch.isfinite(g0).all() and torch.isfinite(gAg).all())
    s.close()
    every = int(np.ceil(np.sqrt(steps)))
    return {"nx": n, "ny": n, "steps": steps, "dt": dt, "checkpoint_every": every,
            "tile_rows": {"forward": args.adj_fwd_rows, "reverse": args.adj_rows},
            "forward_s": fwd, "forward_backward_s": times[-1],
            "forward_backward_first_s": times[0],
            "ratio_vs_forward": times[-1] / fwd,
            "loss": loss, "grad_zb0_linf": g_linf[0], "grad_Ag_linf": g_linf[1],
            "finite": finite}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--device-warmup-ms", type=float, default=50.0,
                    help="FP64 matrix products after each leg's set-up, before its warm-up "
                         "steps, to bring the GPU to its working clock (0: none)")
    ap.add_argument("--rows", type=int, default=0,
                    help="tile rows of the fused kernel (0: automatic)")
    ap.add_argument("--path", default="fused", choices=["fused", "split", "residual"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--cpu-1d-steps", type=int, default=20000)
    ap.add_argument("--cpu-o2-steps", type=int, default=5)
    ap.add_argument("--legs",
                    default="main,mpm,dune1d,antidune,laws,ensemble,adjoint,paper2d,wb,order2",
                    help="comma list of main, mpm, dune1d, antidune, laws, ensemble, adjoint, "
                         "paper2d, wb, order2 (antidune: the paper's 2400-cell 1D run to T = "
                         "50 s; laws: every bedload closure on the MPM channel; paper2d: the "
                         "paper's 4000x4000 bump to T; wb: the well-balanced variant against the "
                         "paper's scheme; order2: the second-order variant against the "
                         "first-order step)")
    ap.add_argument("--laws-steps", type=int, default=50)
    ap.add_argument("--wb-steps", type=int, default=1000)
    ap.add_argument("--o2-steps", type=int, default=1000)
    ap.add_argument("--o2-dune1d", type=int, default=1,
                    help="1: also the paper's 1D dune at J = 2000, first and second order, "
                         "against J = 20000")
    ap.add_argument("--paper-n", type=int, default=4000)
    ap.add_argument("--paper-runs", default="scaling", choices=["scaling", "both"],
                    help="scaling: A_g = 0.1 to T = 1000 s (the run of the paper's "
                         "performance figure, about a minute); both: also A_g = 1 to T = 500 s")
    ap.add_argument("--mpm-steps", type=int, default=200)
    ap.add_argument("--mpm-warmup", type=int, default=10)
    ap.add_argument("--ens-members", type=int, default=256)
    ap.add_argument("--ens-steps", type=int, default=1000)
    ap.add_argument("--ens-seq-steps", type=int, default=100)
    ap.add_argument("--adj-n", type=int, default=1024)
    ap.add_argument("--adj-steps", type=int, default=2000)
    ap.add_argument("--adj-rows", type=int, default=0,
                    help="tile rows of the reverse kernel (0: automatic)")
    ap.add_argument("--adj-fwd-rows", type=int, default=0,
                    help="tile rows of the forward kernel in the adjoint leg")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MiB",
                    help="also run plain device copies of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))

    import torch
    import paper_1307_0491_amd as sve
    sve.require_device()
    out = {"metric": METRIC, "value": None, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "2D Grass dune, periodic, 2000x2000 cells on [0,1000]^2 m, "
                                  "A_g=1e-3, m_g=3, CFL 0.5, FP64",
                      "nx": NX, "ny": NY, "path": args.path, "tile_rows": args.rows,
                      "device_warmup_ms": args.device_warmup_ms}}
    if args.copy_calib:
        out["copy_calibration"] = copy_calibration(torch, args.copy_calib)
    if "mpm" in legs:
        out["mpm"] = mpm_leg(args, sve, torch)
    if "dune1d" in legs:
        out["dune1d"] = dune1d_leg(args, sve, torch)
    if "antidune" in legs:
        out["antidune"] = antidune_leg(args, sve, torch)
    if "laws" in legs:
        out["laws"] = laws_leg(args, sve, torch)
    if "ensemble" in legs:
        out["ensemble"] = ensemble_leg(args, sve, torch)
    if "adjoint" in legs:
        out["adjoint"] = adjoint_leg(args, sve, torch)
    if "paper2d" in legs:
        out["paper2d"] = paper2d_leg(args, sve, torch)
    if "wb" in legs:
        out["wb"] = wb_leg(args, sve, torch)
    if "order2" in legs:
        out["order2"] = order2_leg(args, sve, torch)
    # the main leg runs last; device_warmup brings the GPU to its working clock
    if "main" in legs:
        wall, kern_ms, t, ns, ok = main_leg(args, sve, torch)
        progress(f"main: {args.steps} steps in {wall:.3f} s")
        cells = NX * NY
        per_launch_s = kern_ms * 1e-3 / args.steps
        achieved = BYTES_PER_CELL_FP64 * cells / per_launch_s / 1e9
        src = kernel_source_hash()
        traffic = None
        if TRAFFIC is not None and TRAFFIC["src"] == src and args.path == "fused" \
                and args.rows == TRAFFIC["rows"]:
            traffic = TRAFFIC["bytes_per_launch"]
        out["value"] = cells * args.steps / wall
        out["ms_per_step"] = wall * 1e3 / args.steps
        out["config"].update({"sim_time_s": t, "steps_done": ns})
        alg_tflops = ALG_FLOPS_PER_CELL * cells / per_launch_s / 1e12
        valu = {"algorithmic_flops_per_cell": ALG_FLOPS_PER_CELL,
                "algorithmic_tflops": alg_tflops,
                "fp64_peak_tflops": FP64_PEAK_TFLOPS,
                "fp64_frac": alg_tflops / FP64_PEAK_TFLOPS}
        if VALU["src"] == src and args.path == "fused" and args.rows == VALU["rows"]:
            cycles = (4 * (VALU["insts_valu"] - VALU["insts_trans_f64"])
                      + 16 * VALU["insts_trans_f64"]) / SIMDS
            issue_s = cycles / CLOCK_HZ
            valu.update({"lane_instructions_per_cell": VALU["insts_valu"] * 64 / cells,
                         "fp64_transcendental_per_cell": VALU["insts_trans_f64"] * 64 / cells,
                         "issue_us_at_2.4GHz": issue_s * 1e6,
                         "issue_busy_frac": issue_s / per_launch_s})
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "traffic_unit": "HBM bytes per launch",
                           "traffic_vs_algorithmic": (traffic / (BYTES_PER_CELL_FP64 * cells)
                                                      if traffic else None),
                           "kernel": "k_fused (update of step n + wave speeds of step n+1)",
                           "bytes_per_cell": BYTES_PER_CELL_FP64,
                           "avg_launch_us": per_launch_s * 1e6, "kernel_src": src,
                           "valu": valu}
        cp = copy_peak(torch)
        out["roofline"]["measured_copy_GBs"] = cp
        out["roofline"]["frac_of_measured_copy"] = achieved / cp
        if not ok:
            out["error"] = "non-finite or non-positive depth after the run"
    if not args.no_cpu and "main" in legs:
        progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    if not args.no_cpu and "dune1d" in legs:
        progress("cpu baseline 1D (oracle)")
        out["dune1d"]["cpu_baseline"] = cpu_baseline_1d(args.cpu_1d_steps)
    if not args.no_cpu and "order2" in legs:
        progress("cpu baseline, second order (oracle)")
        out["order2"]["cpu_baseline"] = cpu_baseline_order2(args.cpu_o2_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
