"""Benchmark of the moving-mesh step on one MI355X.

Main line (the JSON "value"): the plain FP64 Sod shock tube, a 256 x 64 x 64
jittered lattice (1,048,576 cells) in a periodic 4 x 1 x 1 box, gamma = 1.4,
Lagrangian mesh, CFL 0.3.  One step is the whole path: sort, cell
construction, mesh assembly, cell states and timestep, gradient +
predictor, half-step gradient, face fluxes, update + drift.  Inputs are
resident in HBM before the timed region.

Also reported on the same line:
  roofline     the dominant kernel (cell construction) against the FP64 ALU
               peak, its duration from HIP events on the context stream over
               the timed region, and the HBM traffic of the committed counter
               summary when it was taken on the current kernel source; its
               "issue" member puts the counted VALU instructions per cell over
               the same duration against the VALU issue peak;
  stage_ms     mean per-step stage times from HIP events (stage_ms_median:
               their medians over the timed steps);
  hbm_copy_gbs achievable HBM bandwidth of a 512 MiB device copy;
  flux_kernel  the face kernel against the HBM peak (algorithmic bytes), and
               against the measured copy bandwidth;
  mixed        the point blast (128^3, 100 steps) in mixed precision against
               the FP64 path: cell-updates/s of both, relative L1 density
               error, conservation drift; with the CPU baseline also its
               error against the FP64 oracle on a 64^3 blast (vs_oracle);
  gresho       the Gresho-Chan vortex to t = 2 at 32^2, 64^2, 128^2: L1 of the
               tangential speed and its rate of convergence;
  sod_paper    the paper's Sod tube to t = 2, moving and static mesh, HLLC and
               HLL: L1 of density against the exact solution, oscillations;
  half_step    start-of-step against half-step geometry: Gresho vortex
               accuracy, angular momentum and cost; free-stream error order;
  entropy      the entropy switch against the energy equation alone: the
               paper's Sod tube and the cost of the extra column;
  serving      a Poisson stream of Kelvin-Helmholtz simulations (1e3..2e5
               points each, 20 steps, mixed) through the batch serving loop
               under an explicit device budget: throughput, p50/p99 step
               latency, turnaround;
  cpu_baseline the CPU oracle on a bounded sample of the Sod workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
# Algorithmic cost model:
TESS_FLOP_PER_CELL = 1.0e4          # FP64 flops to construct one cell
FLUX_FACE_BYTES = {"fp64": 48 + 40, "mixed": 48 + 20}      # face record + stored flux
FLUX_CELL_BYTES = {"fp64": 232, "mixed": 152}              # U_half, grad_half, c-r, w, r once per cell
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_tess_pair_sod_256x64x64_traffic.md")
TESS_SOURCE = os.path.join(ROOT, "paper_1707_05333_amd", "csrc", "k_tessellate.hip")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "k_tess_pair_sod_256x64x64_valu.md")
# VALU wave-instruction issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64
# instruction per SIMD every 4 cycles.
PEAK_VALU_WAVE_INSTR = 256 * 4 * 2.4e9 / 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)   # the Sod configuration runs 50 steps
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--workload", choices=["sod", "blast"], default="sod")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision blast object")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving object")
    ap.add_argument("--no-gresho", action="store_true", help="skip the Gresho-Chan convergence object")
    ap.add_argument("--no-sod-paper", action="store_true", help="skip the paper's Sod tube object")
    ap.add_argument("--no-half-step", action="store_true", help="skip the half-step mesh object")
    ap.add_argument("--no-entropy", action="store_true", help="skip the entropy switch object")
    ap.add_argument("--no-polytropes", action="store_true", help="skip the two-polytrope (non-uniform) object")
    ap.add_argument("--polytrope-steps", type=int, default=20)
    ap.add_argument("--mixed-steps", type=int, default=100)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-budget-gib", type=float, default=8.0)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum CPU time of the oracle sample (whole steps)")
    ap.add_argument("--only-polytropes", action="store_true",
                    help="run only the two-polytrope object (for profiling its kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 512 MiB device copy (for counter calibration under rocprofv3)")
    return ap.parse_args()


def copy_calibration(torch):
    """One 512 MiB device-to-device copy: under a counter run, the scale of
    FETCH_SIZE and WRITE_SIZE against bytes known to move."""
    a = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    import workloads as W
    if name == "sod":
        return W.c2_sod()
    return W.c3_point_blast()


def cpu_baseline(args):
    """The oracle, as it is, on the workload itself: whole steps until at
    least --cpu-seconds of wall time."""
    import oracle
    import workloads as W
    wl = W.c2_sod() if args.workload == "sod" else W.c3_point_blast(n_side=64)
    p = oracle.make_params(wl.box, **wl.params)
    m = oracle.tessellate(wl.pos, wl.box)
    Q = oracle.init_charges(m, p, wl.prim)
    m.free()
    pos = wl.pos
    steps, t0 = 0, time.perf_counter()
    while True:
        pos, Q, *_ = oracle.step(pos, Q, p)
        steps += 1
        if time.perf_counter() - t0 >= args.cpu_seconds or steps >= 20:
            break
    dt = time.perf_counter() - t0
    what = "Sod tube 256x64x64 (1,048,576 cells)" if args.workload == "sod" else "blast 64^3"
    return {"value": wl.n * steps / dt, "unit": "cell-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} whole oracle steps of the {what}", "seconds": dt, "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count()}


def mixed_vs_oracle(M, torch, n_side=64, steps=10):
    """The mixed-precision path against the FP64 oracle on the point blast
    (n_side^3 points, `steps` steps): relative L1 density error and the
    mass, momentum and energy drift of both.  Runs the oracle, so it belongs
    to the CPU-baseline leg."""
    import numpy as np
    import oracle
    import workloads as W
    wl = W.c3_point_blast(n_side=n_side)
    p = oracle.make_params(wl.box, **wl.params)
    m = oracle.tessellate(wl.pos, wl.box)
    Q0 = oracle.init_charges(m, p, wl.prim)
    Q0[wl.energy_cells, 4] += wl.energy_amount
    m.free()
    pos_o, Q_o = wl.pos.copy(), Q0.copy()
    for _ in range(steps):
        pos_o, Q_o, *_ = oracle.step(pos_o, Q_o, p)
    r_o = Q_o[:, 0] / oracle.tessellate(pos_o, wl.box).V
    mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, precision="mixed", **wl.params))
    pos, Q = torch.from_numpy(wl.pos.copy()).cuda(), torch.from_numpy(Q0.copy()).cuda()
    w = torch.empty_like(pos)
    for _ in range(steps):
        mm.step(pos, w, Q)
    mm.tessellate(pos)
    r_g = Q[:, 0].cpu().numpy() / mm.mesh_export().V.cpu().numpy()
    Qg = Q.cpu().numpy()
    mm.close()

    def drift(Qe):
        return {"mass": float(abs(Qe[:, 0].sum() - Q0[:, 0].sum()) / Q0[:, 0].sum()),
                "momentum": float(np.linalg.norm(Qe[:, 1:4].sum(0) - Q0[:, 1:4].sum(0))
                                  / max(np.linalg.norm(Qe[:, 1:4], axis=1).sum(), 1e-300)),
                "energy": float(abs(Qe[:, 4].sum() - Q0[:, 4].sum()) / Q0[:, 4].sum())}

    return {"workload": f"blast_{n_side}^3", "steps": steps,
            "l1_rho_rel_vs_oracle": float(np.abs(r_g - r_o).sum() / np.abs(r_o).sum()),
            "drift_mixed": drift(Qg), "drift_oracle": drift(Q_o)}


def hbm_copy_gbs(torch, mib=512, reps=10):
    """Achievable HBM bandwidth: a device-to-device copy of `mib` MiB, timed
    with events over `reps` copies; read plus written bytes per second."""
    a = torch.empty(mib << 17, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return 2 * (mib << 20) / sec / 1e9


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def tess_traffic(n_launch_cells):
    """HBM bytes per launch of the cell-construction kernel from the committed
    counter summary, or None when it was taken on another kernel source."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"source_sha1:\s*([0-9a-f]{40})", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    c = re.search(r"cells_per_launch:\s*([0-9]+)", text)
    if not (m and b and c):
        return None
    sha = hashlib.sha1(open(TESS_SOURCE, "rb").read()).hexdigest()
    if sha != m.group(1) or int(c.group(1)) != n_launch_cells:
        return None
    return float(b.group(1))


def tess_valu_per_cell(n_launch_cells):
    """VALU wave instructions per cell of the cell-construction kernel from the
    committed counter summary, or None when it was taken on another source."""
    try:
        text = open(VALU_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"source_sha1:\s*([0-9a-f]{40})", text)
    v = re.search(r"valu_instructions_per_cell:\s*([0-9.eE+]+)", text)
    c = re.search(r"cells_per_launch:\s*([0-9]+)", text)
    if not (m and v and c):
        return None
    sha = hashlib.sha1(open(TESS_SOURCE, "rb").read()).hexdigest()
    if sha != m.group(1) or int(c.group(1)) != n_launch_cells:
        return None
    return float(v.group(1))


def run_single(M, torch, wl, precision, steps, warmup, timing=True):
    """Steps one simulation through the one-simulation context.  Returns
    (elapsed seconds, per-stage ms, faces per step, state tensors)."""
    params = M.make_params(box=wl.box, precision=precision, **wl.params)
    mm = M.MovingMesh(wl.n, params)
    pos = torch.from_numpy(wl.pos.copy()).cuda()
    prim = torch.from_numpy(wl.prim.copy()).cuda()
    mm.tessellate(pos)
    Q = mm.init_charges(prim)
    if wl.energy_cells is not None:
        Q[torch.from_numpy(wl.energy_cells).cuda(), 4] += wl.energy_amount
    w = torch.empty_like(pos)
    for _ in range(warmup):
        mm.step(pos, w, Q)
    mm.set_stage_timing(timing)
    per_step, faces_tot = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = mm.step(pos, w, Q)
        if timing:
            per_step.append(mm.stage_ms())
        faces_tot += info["n_faces"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mm.set_stage_timing(False)
    stage_ms = {k: sum(s[k] for s in per_step) / max(len(per_step), 1) for k in M.STAGE_NAMES}
    run_single.median = {k: statistics.median([s[k] for s in per_step]) if per_step else 0.0
                         for k in M.STAGE_NAMES}
    return elapsed, stage_ms, faces_tot / max(steps, 1), (mm, pos, Q, w)


def mixed_object(M, torch, args):
    """Point blast 128^3, 100 steps: mixed precision against FP64."""
    import workloads as W
    wl = W.c3_point_blast()
    res = {}
    for prec in ("fp64", "mixed"):
        log(f"blast 128^3 {prec}, {args.mixed_steps} steps")
        elapsed, _, _, (mm, pos, Q, w) = run_single(M, torch, wl, prec, args.mixed_steps, 0, timing=False)
        rate = wl.n * args.mixed_steps / elapsed
        mm.tessellate(pos)
        V = mm.mesh_export().V
        rho, Qend = Q[:, 0] / V, Q.clone()
        # the face kernel on this workload (the mixed-precision gate is
        # stated for it): stage times of a few more steps
        mm.set_stage_timing(True)
        fl, nf = 0.0, 0
        for _ in range(5):
            info = mm.step(pos, w, Q)
            fl += mm.stage_ms()["flux"] / 5
            nf += info["n_faces"] / 5
        mm.set_stage_timing(False)
        fbytes = nf * FLUX_FACE_BYTES[prec] + wl.n * FLUX_CELL_BYTES[prec]
        res[prec] = dict(rate=rate, rho=rho, V=V, Q=Qend,
                         flux={"launch_ms": fl, "algorithmic_bytes": fbytes, "achieved": fbytes / (fl * 1e-3) / 1e9,
                               "peak": PEAK_HBM_GBS, "unit": "GB/s",
                               "frac": fbytes / (fl * 1e-3) / 1e9 / PEAK_HBM_GBS})
        mm.close()
    # Totals at the start (the same charges for both paths).
    _, _, _, (mm0, _, Q0, _) = run_single(M, torch, wl, "fp64", 0, 0, timing=False)
    tot0 = Q0.sum(dim=0)
    mm0.close()
    r64, r32, V = res["fp64"]["rho"], res["mixed"]["rho"], res["fp64"]["V"]
    l1 = float((r32 - r64).abs().sum() / r64.abs().sum())
    l1v = float(((r32 - r64).abs() * V).sum() / (r64.abs() * V).sum())

    def drift(Q):
        t = Q.sum(dim=0)
        pabs = Q[:, 1:4].norm(dim=1).sum()
        return {"mass": float((t[0] - tot0[0]).abs() / tot0[0].abs()),
                "momentum": float((t[1:4] - tot0[1:4]).norm() / pabs),
                "energy": float((t[4] - tot0[4]).abs() / tot0[4].abs())}

    return {"workload": "blast_128^3", "cells": wl.n, "steps": args.mixed_steps,
            "value": res["mixed"]["rate"], "fp64_value": res["fp64"]["rate"], "unit": "cell-updates/s",
            "speedup_vs_fp64": res["mixed"]["rate"] / res["fp64"]["rate"],
            "l1_rho_rel_vs_fp64": l1, "l1_rho_rel_volume_weighted": l1v,
            "drift_mixed": drift(res["mixed"]["Q"]), "drift_fp64": drift(res["fp64"]["Q"]),
            "flux_kernel_mixed": res["mixed"]["flux"], "flux_kernel_fp64": res["fp64"]["flux"],
            "reference": "the FP64 GPU path, which matches the FP64 oracle to 1e-10 in the parity tests"}


def polytropes_object(M, torch, args):
    """Two touching n = 1.5 polytropes in a background a million times
    thinner, 8,388,608 points (cell sizes differ ~20x in length), mixed
    precision: throughput of whole steps, where the time goes, and
    conservation."""
    import workloads as W
    wl = W.c5_polytropes()
    steps = args.polytrope_steps
    log(f"polytropes n={wl.n} mixed, {steps} steps")
    params = M.make_params(box=wl.box, precision="mixed", **wl.params)
    mm = M.MovingMesh(wl.n, params)
    pos = torch.from_numpy(wl.pos).cuda()
    info = mm.tessellate(pos)
    Q = mm.init_charges(torch.from_numpy(wl.prim).cuda())
    tot0 = Q.sum(dim=0)
    w = torch.empty_like(pos)
    mm.step(pos, w, Q)   # warm-up step
    mm.set_stage_timing(True)
    stage_tot = {k: 0.0 for k in M.STAGE_NAMES}
    floors, deferred, rebuilt, faces = [0, 0, 0, 0], 0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = mm.step(pos, w, Q)
        for k, v in mm.stage_ms().items():
            stage_tot[k] += v
        floors = [a + b for a, b in zip(floors, info["floor_hits"])]
        deferred += info["deferred_cells"]
        rebuilt += info["rebuilt_cells"]
        faces += info["n_faces"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    t = Q.sum(dim=0)
    out = {"workload": "two_polytropes_8388608_mixed", "cells": wl.n, "steps": steps,
           "value": wl.n * steps / elapsed, "unit": "cell-updates/s", "ms_per_step": 1e3 * elapsed / steps,
           "stage_ms": {k: v / steps for k, v in stage_tot.items()},
           "faces_per_step": faces / steps, "shell_pass_cells_per_step": deferred / steps,
           "one_cell_first_pass_cells_per_step": rebuilt / steps, "floor_hits_total": floors,
           "mass_drift": float((t[0] - tot0[0]).abs() / tot0[0]),
           "energy_drift": float((t[4] - tot0[4]).abs() / tot0[4]),
           "note": "energy changes only through post-update floors (floor_hits_total[3])"}
    mm.close()
    return out


def gresho_object(M, torch, args):
    """Gresho-Chan vortex to t = 2 at 32^2, 64^2, 128^2 (FP64): L1 of the
    tangential speed at the generators and its convergence rate."""
    import numpy as np
    import workloads as W
    out = {"workload": "gresho_chan_vortex_t2", "precision": "fp64", "runs": []}
    for N in (32, 64, 128):
        wl = W.gresho(N)
        mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, **wl.params))
        pos = torch.from_numpy(wl.pos.copy()).cuda()
        mm.tessellate(pos)
        Q = mm.init_charges(torch.from_numpy(wl.prim.copy()).cuda())
        w = torch.empty_like(pos)
        t, steps = 0.0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while t < 2.0 * (1 - 1e-12):
            t += mm.step(pos, w, Q, dt_max=2.0 - t)["dt"]
            steps += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        x, q = pos.cpu().numpy(), Q.cpu().numpy()
        dx, dy = x[:, 0] - 0.5, x[:, 1] - 0.5
        r = np.hypot(dx, dy)
        v = q[:, 1:3] / q[:, :1]
        vphi = (-dy * v[:, 0] + dx * v[:, 1]) / r
        l1 = float(np.mean(np.abs(vphi - W.gresho_profile(r)[1])))
        out["runs"].append({"N": N, "cells": wl.n, "steps": steps, "l1_vphi": l1,
                            "cell_updates_per_s": wl.n * steps / wall})
        mm.close()
        log(f"gresho N={N}: L1 {l1:.4e} in {steps} steps")
    l1 = [r["l1_vphi"] for r in out["runs"]]
    out["l1_slope"] = math.log(l1[0] / l1[-1]) / math.log(4.0)
    out["paper_slope"] = 0.88
    return out


def half_step_object(M, torch, args):
    """Start-of-step against half-step geometry: the Gresho vortex (64^2,
    t = 2; L1 of the tangential speed, relative change of the angular
    momentum about the vortex axis, time per step) and the free-stream
    density error of a uniform flow on a drifting 24^3 mesh at CFL 0.4 and
    0.1 (its ratio shows the order in time)."""
    import numpy as np
    import workloads as W
    out = {"workload": "gresho_64_t2 + free_stream_24^3", "precision": "fp64", "gresho": [], "free_stream": []}
    wl = W.gresho(64)
    for half in (0, 1):
        mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, half_step_mesh=half, **wl.params))
        pos = torch.from_numpy(wl.pos.copy()).cuda()
        mm.tessellate(pos)
        Q = mm.init_charges(torch.from_numpy(wl.prim.copy()).cuda())
        w = torch.empty_like(pos)

        def lz():
            x, q = pos.cpu().numpy(), Q.cpu().numpy()
            return float(np.sum((x[:, 0] - 0.5) * q[:, 2] - (x[:, 1] - 0.5) * q[:, 1]))
        L0 = lz()
        t, steps = 0.0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while t < 2.0 * (1 - 1e-12):
            t += mm.step(pos, w, Q, dt_max=2.0 - t)["dt"]
            steps += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        x, q = pos.cpu().numpy(), Q.cpu().numpy()
        dx, dy = x[:, 0] - 0.5, x[:, 1] - 0.5
        r = np.hypot(dx, dy)
        v = q[:, 1:3] / q[:, :1]
        l1 = float(np.mean(np.abs((-dy * v[:, 0] + dx * v[:, 1]) / r - W.gresho_profile(r)[1])))
        out["gresho"].append({"half_step_mesh": half, "steps": steps, "l1_vphi": l1,
                              "dLz_rel": (lz() - L0) / L0, "ms_per_step": 1e3 * wall / steps})
        mm.close()
        log(f"half-step {half}: gresho L1 {l1:.4e}, dLz {out['gresho'][-1]['dLz_rel']:.3e}")
    fpos = W.jittered_lattice((24, 24, 24), (1, 1, 1), jitter=0.2, seed=3)
    fw = W.uniform_state(fpos, (1, 1, 1), rho=1.3, vel=(0.4, -0.2, 0.1), P=0.7)
    for half in (0, 1):
        for cfl in (0.4, 0.1):
            mm = M.MovingMesh(fw.n, M.make_params(box=fw.box, half_step_mesh=half, **dict(fw.params, cfl=cfl)))
            pos = torch.from_numpy(fw.pos.copy()).cuda()
            mm.tessellate(pos)
            Q = mm.init_charges(torch.from_numpy(fw.prim.copy()).cuda())
            w = torch.empty_like(pos)
            t = 0.0
            while t < 0.05 * (1 - 1e-12):
                t += mm.step(pos, w, Q, dt_max=0.05 - t)["dt"]
            mm.tessellate(pos)
            V = mm.mesh_export().V.cpu().numpy()
            err = float(np.abs(Q[:, 0].cpu().numpy() / V - 1.3).max())
            out["free_stream"].append({"half_step_mesh": half, "cfl": cfl, "max_density_error": err})
            mm.close()
    return out


def entropy_object(M, torch, args):
    """Entropy switch (Mach threshold 1.1) against the energy equation alone:
    the paper's Sod tube to t = 2 (L1 of density against the exact solution,
    cells above the threshold), and the cost of the extra column on the 1M
    Sod step."""
    import numpy as np
    import workloads as W
    out = {"workload": "sod_paper_16x1x1_t2 + sod_256x64x64", "precision": "fp64", "sod_paper": [],
           "step_ms": {}}
    wl = W.sod_paper(k=14)
    for mth in (0.0, 1.1):
        mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, mach_threshold=mth, **wl.params))
        pos = torch.from_numpy(wl.pos.copy()).cuda()
        mm.tessellate(pos)
        prim = torch.from_numpy(wl.prim.copy()).cuda()
        Q, S = mm.init_charges(prim), mm.init_entropy(prim)
        w = torch.empty_like(pos)
        mach = torch.empty(wl.n, dtype=torch.float32, device="cuda")
        t, steps, shocked = 0.0, 0, 0
        while t < 2.0 * (1 - 1e-12):
            t += mm.step_entropy(pos, w, Q, S, mach, dt_max=2.0 - t)["dt"]
            steps += 1
        shocked = int((mach >= 1.1).sum())
        mm.tessellate(pos)
        V = mm.mesh_export().V.cpu().numpy()
        x, q = pos.cpu().numpy(), Q.cpu().numpy()
        mm.close()
        xx = x[:, 0]
        mid = (xx >= 4.0) & (xx < 12.0)
        ex = np.empty_like(xx)
        L, R = wl.meta["left"], wl.meta["right"]
        ex[mid] = _exact_riemann_rho(L, R, 1.4, (xx[mid] - 8.0) / 2.0)
        ex[~mid] = _exact_riemann_rho(R, L, 1.4, np.where(xx[~mid] < 4.0, xx[~mid], xx[~mid] - 16.0) / 2.0)
        out["sod_paper"].append({"mach_threshold": mth, "steps": steps, "cells_above_threshold_at_end": shocked,
                                 "l1_rho": float(np.mean(np.abs(q[:, 0] / V - ex)))})
        log(f"entropy switch {mth}: sod_paper L1 {out['sod_paper'][-1]['l1_rho']:.3e}")
    big = W.c2_sod()
    for mth in (0.0, 1.1):
        mm = M.MovingMesh(big.n, M.make_params(box=big.box, mach_threshold=mth, **big.params))
        pos = torch.from_numpy(big.pos.copy()).cuda()
        mm.tessellate(pos)
        prim = torch.from_numpy(big.prim.copy()).cuda()
        Q, S = mm.init_charges(prim), mm.init_entropy(prim)
        w = torch.empty_like(pos)

        def one():   # the energy equation alone goes through mm_step, without the column
            return mm.step_entropy(pos, w, Q, S) if mth > 0 else mm.step(pos, w, Q)
        for k in range(2):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(5):
            one()
        torch.cuda.synchronize()
        out["step_ms"]["entropy_column" if mth > 0 else "energy_only"] = 1e3 * (time.perf_counter() - t0) / 5
        mm.close()
    return out


def _exact_riemann_rho(left, right, gamma, xi):
    """Density of the exact ideal-gas Riemann solution at x/t = xi (the
    textbook construction: star pressure by bisection on the sum of the
    two wave curves, then the wave pattern sampled at xi)."""
    import numpy as np
    (rl, ul, pl), (rr, ur, pr) = left, right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)

    def f(p, r, pk, c):
        if p > pk:
            a, b = 2.0 / ((gamma + 1) * r), (gamma - 1) / (gamma + 1) * pk
            return (p - pk) * math.sqrt(a / (p + b))
        return 2 * c / (gamma - 1) * ((p / pk) ** ((gamma - 1) / (2 * gamma)) - 1)

    lo, hi = 1e-12, 10 * max(pl, pr)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid, rl, pl, cl) + f(mid, rr, pr, cr) + ur - ul < 0 else (lo, mid)
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (f(ps, rr, pr, cr) - f(ps, rl, pl, cl))
    g1 = (gamma - 1) / (gamma + 1)

    def side(r, p, c, sgn):   # sgn -1: left wave, +1: right wave; returns star density and wave bounds
        if ps > p:
            rs = r * (ps / p + g1) / (g1 * ps / p + 1)
            S = sgn * c * math.sqrt((gamma + 1) / (2 * gamma) * ps / p + (gamma - 1) / (2 * gamma))
            return rs, S, S
        rs = r * (ps / p) ** (1 / gamma)
        cs = c * (ps / p) ** ((gamma - 1) / (2 * gamma))
        return rs, sgn * c, us + sgn * cs

    rsl, hl, tl = side(rl, pl, cl, -1)
    rsr, hr, tr = side(rr, pr, cr, +1)
    hl += ul; hr += ur
    if ps > pl: tl = hl
    if ps > pr: tr = hr
    xi = np.asarray(xi, dtype=np.float64)
    out = np.empty_like(xi)
    for i, s in enumerate(xi):
        if s < us:
            if s < hl: out[i] = rl
            elif s > tl: out[i] = rsl
            else:
                c = 2 / (gamma + 1) * (cl + (gamma - 1) / 2 * (ul - s))
                out[i] = rl * (c / cl) ** (2 / (gamma - 1))
        else:
            if s > hr: out[i] = rr
            elif s < tr: out[i] = rsr
            else:
                c = 2 / (gamma + 1) * (cr - (gamma - 1) / 2 * (ur - s))
                out[i] = rr * (c / cr) ** (2 / (gamma - 1))
    return out


def sod_paper_object(M, torch, args):
    """The paper's Sod tube (16 x 1 x 1, rho_R = 0.25, P_R = 0.1795) to t = 2
    on the moving and the static mesh with HLLC and HLL: L1 of density
    against the exact solution and the total-variation excess of the
    x-profile (oscillations)."""
    import numpy as np
    import workloads as W
    k = 14
    runs = []
    for sm in (False, True):
        for rs in ("hllc", "hll"):
            wl = W.sod_paper(k=k, riemann=rs, static_mesh=sm)
            mm = M.MovingMesh(wl.n, M.make_params(box=wl.box, **wl.params))
            pos = torch.from_numpy(wl.pos.copy()).cuda()
            mm.tessellate(pos)
            Q = mm.init_charges(torch.from_numpy(wl.prim.copy()).cuda())
            w = torch.empty_like(pos)
            t, steps = 0.0, 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            while t < 2.0 * (1 - 1e-12):
                t += mm.step(pos, w, Q, dt_max=2.0 - t)["dt"]
                steps += 1
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            mm.tessellate(pos)
            V = mm.mesh_export().V.cpu().numpy()
            x, q = pos.cpu().numpy(), Q.cpu().numpy()
            mm.close()
            rho = q[:, 0] / V
            xx = x[:, 0]
            mid = (xx >= 4.0) & (xx < 12.0)
            ex = np.empty_like(xx)
            L, R = wl.meta["left"], wl.meta["right"]
            ex[mid] = _exact_riemann_rho(L, R, 1.4, (xx[mid] - 8.0) / 2.0)
            xe = np.where(xx[~mid] < 4.0, xx[~mid], xx[~mid] - 16.0)
            ex[~mid] = _exact_riemann_rho(R, L, 1.4, xe / 2.0)
            nb = 16 * k
            b = np.minimum((xx / 16.0 * nb).astype(int), nb - 1)
            cnt = np.maximum(np.bincount(b, minlength=nb), 1)
            tv = lambda p: float(np.abs(np.diff(np.r_[p, p[:1]])).sum())
            runs.append({"mesh": "static" if sm else "moving", "riemann": rs, "cells": wl.n, "steps": steps,
                         "l1_rho": float(np.mean(np.abs(rho - ex))),
                         "tv_excess": tv(np.bincount(b, weights=rho, minlength=nb) / cnt)
                         - tv(np.bincount(b, weights=ex, minlength=nb) / cnt),
                         "cell_updates_per_s": wl.n * steps / wall})
            log(f"sod_paper {runs[-1]['mesh']} {rs}: L1 {runs[-1]['l1_rho']:.3e} in {steps} steps")
    return {"workload": "sod_paper_16x1x1_t2", "precision": "fp64", "theta": 0.49, "runs": runs}


def serving_object(M, torch, args):
    """A Poisson stream of Kelvin-Helmholtz runs through the serving loop."""
    import numpy as np
    import workloads as W
    nreq = args.serve_requests
    log(f"serving: generating {nreq} Kelvin-Helmholtz requests")
    wls = [W.c4_kelvin_helmholtz(k) for k in range(nreq)]
    prec = "mixed"
    budget = int(args.serve_budget_gib * (1 << 30))

    def requests(arrivals, precision=prec):
        reqs = []
        for t, wl in zip(arrivals, wls):
            reqs.append(dict(arrival=float(t), params=M.make_params(box=wl.box, precision=precision, **wl.params),
                             pos=torch.from_numpy(wl.pos).cuda(), prim=torch.from_numpy(wl.prim).cuda(),
                             steps=wl.steps))
        return reqs

    # Saturated rate of the same 32 requests served in plain FP64.
    B64 = M.Batch(budget, max_sims=1024, precision="fp64")
    _, st64 = B64.serve(requests([0.0] * 32, "fp64")[:32])
    B64.close()
    # Calibration: the first 32 requests at once give the sustained rate;
    # arrivals then come at 0.8 of that rate divided by the mean request cost.
    B = M.Batch(budget, max_sims=1024, precision=prec)
    cal = requests([0.0] * 32)[:32]
    _, st = B.serve(cal)
    cost = float(np.mean([wl.n * wl.steps for wl in wls]))
    rate = 0.8 * st["cell_updates_per_s"] / cost
    arrivals = W.poisson_arrivals(nreq, rate, seed=4)
    log(f"serving: calibration {st['cell_updates_per_s']:.3e} cell-updates/s, arrival rate {rate:.1f}/s")
    reqs = requests(arrivals)
    res, stats = B.serve(reqs)
    ok = sum(1 for r in res if r["status"] == 0)
    B.close()
    return {"workload": f"kelvin_helmholtz_stream_{nreq}", "requests": nreq, "completed_ok": ok,
            "cells_total": int(sum(wl.n for wl in wls)), "steps_per_request": 20, "precision": prec,
            "hbm_budget_bytes": budget, "arrival_rate_per_s": rate,
            "saturated_value": st["cell_updates_per_s"], "saturated_fp64_value": st64["cell_updates_per_s"],
            "saturated_speedup_vs_fp64": st["cell_updates_per_s"] / st64["cell_updates_per_s"],
            "value": stats["cell_updates_per_s"], "unit": "cell-updates/s",
            "step_latency_p50_ms": stats["step_p50"], "step_latency_p99_ms": stats["step_p99"],
            "step_latency_mean_ms": stats["step_mean"],
            "turnaround_p50_s": stats["turnaround_p50"], "turnaround_p99_s": stats["turnaround_p99"],
            "batch_steps": stats["batch_steps"], "max_resident": stats["max_resident"], "wall_s": stats["wall"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_1707_05333_amd as M

    torch.cuda.set_device(0)
    if args.only_polytropes:
        obj = polytropes_object(M, torch, args)
        if args.copy_calibration:
            copy_calibration(torch)
        print(json.dumps({"polytropes": obj}))
        return
    wl = make_workload(args.workload)
    n = wl.n
    log(f"workload {args.workload} n={n} precision={args.precision}")
    elapsed, stage_ms, faces, (mm, *_rest) = run_single(M, torch, wl, args.precision, args.steps, args.warmup)
    mm.close()
    stage_median = dict(run_single.median)
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    ms_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    copy_gbs = hbm_copy_gbs(torch)
    log(f"device copy {copy_gbs:.0f} GB/s")

    if args.copy_calibration:
        copy_calibration(torch)

    # Dominant kernel: cell construction (FP64 ALU bound).
    t_cells = stage_ms["cells"] * 1e-3
    ach = TESS_FLOP_PER_CELL * n / t_cells / 1e12
    # (The stage's launches: the two-cells-per-wavefront pass over every
    # cell, then the list-driven passes, which exit at once on uniform inputs.)
    roofline = {"bound": "alu", "kernel": "k_tess_pair + k_tess_pass1_redo + k_tess_pass1_dense + k_tess_pass2",
                "achieved": ach,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS,
                "traffic": tess_traffic(n) if args.workload == "sod" else None,
                "algorithmic_flop_per_cell": TESS_FLOP_PER_CELL, "launch_ms": stage_ms["cells"]}
    vpc = tess_valu_per_cell(n) if args.workload == "sod" else None
    if vpc is not None:
        # What actually bounds the kernel: VALU issue (counted instructions
        # over the live launch time, against the issue peak).
        iss = vpc * n / t_cells
        roofline["issue"] = {"valu_instr_per_cell": vpc, "achieved": iss, "peak": PEAK_VALU_WAVE_INSTR,
                             "unit": "wave-instr/s", "frac": iss / PEAK_VALU_WAVE_INSTR}
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
        "stage_ms_median": stage_median,
        "hbm_copy_gbs": copy_gbs,
        "flux_kernel": {"bound": "hbm", "achieved": flux_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": flux_gbs / PEAK_HBM_GBS, "frac_of_copy": flux_gbs / copy_gbs,
                        "algorithmic_bytes": flux_bytes, "launch_ms": stage_ms["flux"],
                        "launch_ms_median": stage_median["flux"]},
    }
    if not args.no_mixed:
        out["mixed"] = mixed_object(M, torch, args)
        log(f"mixed: {out['mixed']['value']:.3e} vs fp64 {out['mixed']['fp64_value']:.3e}, "
            f"L1 {out['mixed']['l1_rho_rel_vs_fp64']:.2e}")
    if not args.no_polytropes:
        out["polytropes"] = polytropes_object(M, torch, args)
        log(f"polytropes: {out['polytropes']['value']:.3e} cell-updates/s, "
            f"{out['polytropes']['ms_per_step']:.1f} ms/step")
    if not args.no_gresho:
        out["gresho"] = gresho_object(M, torch, args)
    if not args.no_sod_paper:
        out["sod_paper"] = sod_paper_object(M, torch, args)
    if not args.no_half_step:
        out["half_step"] = half_step_object(M, torch, args)
    if not args.no_entropy:
        out["entropy"] = entropy_object(M, torch, args)
    if not args.no_serve:
        out["serving"] = serving_object(M, torch, args)
        log(f"serving: {out['serving']['value']:.3e} cell-updates/s, p50 {out['serving']['step_latency_p50_ms']:.2f} ms"
            f" p99 {out['serving']['step_latency_p99_ms']:.2f} ms")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args)
        log(f"cpu baseline {out['cpu_baseline']['seconds']:.1f} s")
        if "mixed" in out:
            # the oracle's run of a smaller blast is the FP64 reference of the
            # mixed path (the oracle runs only in this leg)
            out["mixed"]["vs_oracle"] = mixed_vs_oracle(M, torch)
            log(f"mixed vs oracle: L1 {out['mixed']['vs_oracle']['l1_rho_rel_vs_oracle']:.2e}")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
