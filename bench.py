"""Benchmark of the MTP tent sweep on one MI355X.

One step = one slab: every layer of the tent table from a flat front to the flat front
one slab height later (all tents: gather, SAT stages, scatter).  Inputs are resident in
HBM before the timed region.  Prints one JSON line.

Workload (default): 3D PEC cavity, unit cube 16^3 x 6 Kuhn tetrahedra (24576 tets),
P3 DG, q = 4 Taylor stages, m = 6 sub-intervals, slab height T = 1, FP64.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6   # TFLOP/s, MI355X FP64 vector and matrix
PEAK_FP32 = 157.3  # TFLOP/s, MI355X FP32 matrix


def log(*a):
    print(*a, file=sys.stderr, flush=True)


GRADE_A = 2.0 / 9.0   # x -> a x + (1-a) x^2: h_max / h_min = (2-a)/a = 8


def workload(name):
    from mtp_inputs import fields, meshes
    if name == "cavity3d_p3":
        mm = meshes.cube_kuhn(16)
        desc = "3D PEC cavity mode, unit cube 16^3x6 Kuhn tets (24576), P3, q=4, m=6, slab T=1"
        return dict(mm=mm, p=3, q=4, m=6, T=1.0, ex=fields.Cavity3D_PEC(), desc=desc, exact=True)
    if name == "graded3d_p4":
        grade = lambda g: GRADE_A * g + (1 - GRADE_A) * g * g  # noqa: E731
        mm = meshes.cube_kuhn(32, axis_map=grade)
        eps, mu = meshes.materials_split(mm)
        desc = ("3D PEC, unit cube 32^3x6 Kuhn tets (196608) graded toward one corner (h ratio 1:8), "
                "eps in {1, 2.25} split at x=0.5, Gaussian-pulse E, P4, q=5, m=8, slab T=0.05")
        return dict(mm=mm, p=4, q=5, m=8, T=0.05, ex=fields.GaussianPulse3D(seed=11030), desc=desc,
                    eps=eps, mu=mu, exact=False)
    if name == "graded3d_p4_cavity":
        grade = lambda g: GRADE_A * g + (1 - GRADE_A) * g * g  # noqa: E731
        mm = meshes.cube_kuhn(32, axis_map=grade)
        desc = ("3D PEC cavity mode, unit cube 32^3x6 Kuhn tets (196608) graded toward one corner "
                "(h ratio 1:8), eps = mu = 1, P4, q=5, m=8, slab T=0.05 (equal-error certification)")
        return dict(mm=mm, p=4, q=5, m=8, T=0.05, ex=fields.Cavity3D_PEC(), desc=desc, exact=True)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(W, budget_s):
    """The oracle as it stands, on the first tents of the same workload (layer order),
    until budget_s of CPU time; one thread."""
    from threadpoolctl import threadpool_limits

    from mtp_inputs import meshes
    from oracle.mesh import Mesh as OMesh
    from oracle.pitch import pitch as opitch
    from oracle.solve import OracleSolver
    with threadpool_limits(limits=1):
        om = OMesh(W["mm"]["coords"], W["mm"]["cells"], eps=W.get("eps"), mu=W.get("mu"))
        tents = opitch(om, W["T"], 0.5)
        O = OracleSolver(om, W["p"], W["q"], W["m"])
        O.set_nodal_u(W["ex"].u(meshes.equispaced_nodes(W["mm"], W["p"]), 0.0))
        order = np.argsort(tents["layer"], kind="stable")
        nc, npn = 6, (W["p"] + 1) * (W["p"] + 2) * (W["p"] + 3) // 6
        dofs, done = 0.0, 0
        t0 = time.perf_counter()
        for i in order:
            v = int(tents["vertex"][i])
            O.run_tent(v, float(tents["t_top"][i]))
            dofs += nc * npn * len(om.v2e[v]) * W["m"] * W["q"]
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        el = time.perf_counter() - t0
    return {"value": dofs / el, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} tents (layer order) of the same workload, {el:.1f} s, numpy FP64, 1 thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cavity3d_p3")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "fp64-valu"])
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        x = torch.ones(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": x.numel() * 8, "copies": 3}))
        return

    from mtp_inputs import meshes
    from paper_1906_11029_amd import mtp

    W = workload(args.workload)
    mm = W["mm"]
    t0 = time.perf_counter()
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=W.get("eps"), mu=W.get("mu"))
    T = mtp.Tents(M, W["T"], 0.5)
    t_pitch = time.perf_counter() - t0
    prec = {"fp64": mtp.MTP_FP64, "mixed": mtp.MTP_MIXED_FP32, "fp64-valu": mtp.MTP_FP64_VALU}[args.precision]
    S = mtp.Solver(M, T, W["p"], W["q"], W["m"], precision=prec)
    kernel_name = {0: "tent_kernel (vector-ALU FP64)", 1: "tent_mfma_kernel<double> (FP64 MFMA)",
                   2: "tent_mfma_kernel<float> (FP32 MFMA, FP64 inversion and Taylor sum)"}[S.kernel()]
    u0 = W["ex"].u(meshes.equispaced_nodes(mm, W["p"]), 0.0)
    S.set_fields(u0, 0.0)
    dof_slab, n_tents = S.slab_dof_updates()
    flops_slab = S.slab_flops()
    log(f"mesh {M.info} tents {n_tents} layers {T.n_layers} pitch {t_pitch:.2f}s")

    front = 0.0
    for _ in range(args.warmup):
        front += W["T"]
        S.advance_to(front)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    nl = T.n_layers
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):     # each step replays the captured slab graph
        front += W["T"]
        S.advance_to(front)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_s = ev0.elapsed_time(ev1) * 1e-3
    durs = np.full(args.steps * nl, gpu_s / (args.steps * nl))
    kern_avg = durs.mean()
    flops_avg = flops_slab / nl
    achieved = flops_avg / kern_avg / 1e12

    u = S.get_fields()
    err = None
    if W["exact"]:
        uex = W["ex"].u(meshes.equispaced_nodes(mm, W["p"]), front)
        err = float(np.linalg.norm(u - uex) / np.linalg.norm(uex))
    log(f"wall {wall:.3f}s for {args.steps} slabs; GPU time (events) {durs.sum():.3f}s; "
        f"nodal rel. error vs exact {err}")

    value = dof_slab * args.steps / wall
    peak = PEAK_FP32 if S.kernel() == 2 else PEAK_FP64
    out = {
        "metric": "DOF-updates/s, 3D Maxwell p=4 MTP: mixed/batched vs FP64 GPU at equal L2 error",
        "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if S.kernel() != 2 else "f32+f64", "data": "synthetic",
        "config": {"workload": W["desc"], "tets": int(M.info["ne"]), "p": W["p"], "q": W["q"], "m": W["m"],
                   "tents_per_step": int(n_tents), "layers_per_step": int(nl), "slope_fraction": 0.5,
                   "precision": args.precision, "nodal_rel_error_vs_exact": err},
        "roofline": {"bound": "alu" if S.kernel() == 0 else "mfma", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": kernel_name + ", one launch per layer, slab captured in a HIP graph",
                     "avg_launch_ms": kern_avg * 1e3, "launches": int(args.steps * nl)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
