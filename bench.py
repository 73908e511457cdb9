"""Benchmark of the moving-mesh step on one MI355X.

Default workload: the FP64 Sod shock tube, a 256 x 64 x 64 jittered lattice
(1,048,576 cells) in a periodic 4 x 1 x 1 box, gamma = 1.4, Lagrangian mesh,
CFL 0.3.  One step is the whole path: sort, cell construction, mesh assembly,
cell states and timestep, gradient + predictor, half-step gradient, face
fluxes, update + drift.  Inputs are resident in HBM before the timed region.

Prints one JSON line (metric, value in cell-updates/s, roofline of the
dominant kernel measured with HIP events inside the timed region, per-stage
times, and the CPU oracle's rate on a bounded slab of the same workload).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
# Algorithmic cost model ("Measurement"):
TESS_FLOP_PER_CELL = 1.0e4          # FP64 flops to construct one cell
FLUX_FACE_BYTES = {"fp64": 48 + 40, "mixed": 48 + 20}      # face record + stored flux
FLUX_CELL_BYTES = {"fp64": 232, "mixed": 152}              # U_half, grad_half, c-r, w, r once per cell


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--workload", choices=["sod", "blast"], default="sod")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-depth", type=int, default=64,
                    help="z layers of the lattice in the oracle's timing slab")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 512 MiB device copy (for counter calibration under rocprofv3)")
    return ap.parse_args()


def make_workload(name):
    import workloads as W
    if name == "sod":
        return W.c2_sod()
    return W.c3_point_blast()


def cpu_baseline(args):
    """The oracle, as it is, on a slab of the workload: same spacing and
    states, fewer z layers (periodic), one step."""
    import oracle
    import workloads as W
    if args.workload == "sod":
        depth = args.cpu_sample_depth
        wl = W.c2_sod(shape=(256, 64, depth), box=(4.0, 1.0, depth / 64.0))
        sample = f"one oracle step of the Sod tube slab 256x64x{depth} (box 4 x 1 x {depth / 64:g})"
    else:
        depth = args.cpu_sample_depth
        wl = W.c3_point_blast(n_side=64)
        sample = "one oracle step of the blast at 64^3"
    p = oracle.make_params(wl.box, **wl.params)
    m = oracle.tessellate(wl.pos, wl.box)
    Q = oracle.init_charges(m, p, wl.prim)
    m.free()
    t0 = time.perf_counter()
    oracle.step(wl.pos, Q, p)
    dt = time.perf_counter() - t0
    return {"value": wl.n / dt, "unit": "cell-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": sample, "seconds": dt}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1707_05333_amd as M

    torch.cuda.set_device(0)
    wl = make_workload(args.workload)
    n = wl.n
    log(f"workload {args.workload} n={n} precision={args.precision}")
    params = M.make_params(box=wl.box, precision=args.precision, **wl.params)
    mm = M.MovingMesh(n, params)
    pos = torch.from_numpy(wl.pos.copy()).cuda()
    prim = torch.from_numpy(wl.prim.copy()).cuda()
    mm.tessellate(pos)
    Q = mm.init_charges(prim)
    if wl.energy_cells is not None:
        idx = torch.from_numpy(wl.energy_cells).cuda()
        Q[idx, 4] += wl.energy_amount
    w = torch.empty_like(pos)
    log("tessellated and charged")
    for _ in range(args.warmup):
        mm.step(pos, w, Q)
    log(f"warmup done ({args.warmup} steps)")

    mm.set_stage_timing(True)
    stage_tot = {k: 0.0 for k in M.STAGE_NAMES}
    faces_tot = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = mm.step(pos, w, Q)
        for k, v in mm.stage_ms().items():
            stage_tot[k] += v
        faces_tot += info["n_faces"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mm.set_stage_timing(False)
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    ms_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    stage_ms = {k: v / args.steps for k, v in stage_tot.items()}
    faces = faces_tot / args.steps

    if args.copy_calibration:
        a = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # Dominant kernel: cell construction (FP64 ALU, latency bound).
    t_cells = stage_ms["cells"] * 1e-3
    ach = TESS_FLOP_PER_CELL * n / t_cells / 1e12
    roofline = {"bound": "alu", "kernel": "k_tess_pass1 + k_tess_pass2", "achieved": ach,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS, "traffic": None,
                "algorithmic_flop_per_cell": TESS_FLOP_PER_CELL}
    t_flux = stage_ms["flux"] * 1e-3
    flux_bytes = faces * FLUX_FACE_BYTES[args.precision] + n * FLUX_CELL_BYTES[args.precision]
    flux_gbs = flux_bytes / t_flux / 1e9 if t_flux > 0 else float("nan")

    out = {
        "metric": "cell-updates/s (tessellate+flux)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": ("sod_256x64x64_fp64" if args.workload == "sod" else "blast_128^3")
                   + ("" if args.precision == "fp64" else "_mixed"),
                   "cells": n, "box": list(wl.box), "precision": args.precision,
                   "faces_per_step": faces},
        "roofline": roofline,
        "stage_ms": stage_ms,
        "flux_kernel": {"bound": "hbm", "achieved": flux_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": flux_gbs / PEAK_HBM_GBS, "algorithmic_bytes": flux_bytes},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args)
        log(f"cpu baseline {out['cpu_baseline']['seconds']:.1f} s")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
