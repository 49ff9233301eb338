"""Benchmark of the hot path: explicit FP64 2D steps of the relaxation
scheme on the periodic 2D Grass dune, 2000 x 2000 cells on [0, 1000]^2 m,
A_g = 1e-3, m_g = 3, CFL 0.5 (one step = one pass of the whole method:
projection, interface Riemann solves, update and the CFL reduction of the
next step).

Prints one JSON line (cell-updates/s, HBM roofline of the step kernel, the
CPU oracle timed on a bounded sample of the same workload).
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

import numpy as np  # noqa: E402

METRIC = "cell-updates/s and % HBM roofline (FP64 2D); ensemble and adjoint vs plain"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
BYTES_PER_CELL_FP64 = 64.0     # read h, hu, hv, z_b and write them once (8 B each)
NX = NY = 2000


def workload():
    import workloads as W
    h, hu, hv, zb, dx, dy = W.dune2d(NX, NY)
    return h, hu, hv, zb


def cpu_baseline(nsteps: int = 3):
    """The oracle as it stands, on the host, over `nsteps` steps of the same
    2000 x 2000 grid (bounded sample of the workload)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
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
            "seconds": el}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--rows", type=int, default=32, help="tile rows of the fused kernel")
    ap.add_argument("--path", default="fused", choices=["fused", "split"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1307_0491_amd as sve
    sve.require_device()
    h, hu, hv, zb = workload()
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 4
    stream = sve.current_stream_handle()
    s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p, bcs=bcs, stream=stream)
    s.set_path(sve.PATH_FUSED if args.path == "fused" else sve.PATH_SPLIT)
    s.set_tile_rows(args.rows)
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
    cells = NX * NY
    value = cells * args.steps / wall
    per_launch_s = kern_ms * 1e-3 / args.steps
    achieved = BYTES_PER_CELL_FP64 * cells / per_launch_s / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D Grass dune, periodic, 2000x2000 cells on [0,1000]^2 m, "
                               "A_g=1e-3, m_g=3, CFL 0.5, FP64",
                   "nx": NX, "ny": NY, "path": args.path, "tile_rows": args.rows,
                   "sim_time_s": t, "steps_done": ns},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_fused (update of step n + wave speeds of step n+1)",
                     "bytes_per_cell": BYTES_PER_CELL_FP64,
                     "avg_launch_us": per_launch_s * 1e6},
    }
    if not np.all(np.isfinite(gh)) or not np.all(gh > 0):
        out["error"] = "non-finite or non-positive depth after the run"
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
