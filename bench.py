"""Benchmark of the MTP tent sweep on one MI355X.

One step = one slab: every layer of the tent table from a flat front to the flat front
one slab height later (all tents: gather, SAT stages, scatter).  Inputs are resident in
HBM before the timed region.  Prints one JSON line.

Workload (default): 3D Maxwell on the unit cube, 32^3 x 6 Kuhn tetrahedra (196608 tets)
graded toward one corner (h ratio 1:8), eps in {1, 2.25} split at x = 0.5, Gaussian-pulse
initial E, P4 DG, q = 5 Taylor stages, m = 8 sub-intervals, slab height 0.05, mixed
precision (FP64 first stage of every sub-interval, FP32 matrix cores for the later stages).
Beside it, in the same run: the plain FP64 path on the same workload (DOF-updates/s,
speedup, relative L2 difference of the fields), the equal-error check (the graded mesh
with a closed-form PEC cavity mode, in both precisions, for as many slabs as the timed run
plus its warm-up), the roofline fraction against the FP32 matrix peak (and a blended
FP64/FP32 peak beside it), the tents' use of the slope bound, and the oracle timed on the
host's cores.
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
        return dict(name=name, mm=mm, p=3, q=4, m=6, T=1.0, ex=fields.Cavity3D_PEC(), desc=desc, exact=True)
    if name == "cavity3d_p5":
        mm = meshes.cube_kuhn(16)
        desc = "3D PEC cavity mode, unit cube 16^3x6 Kuhn tets (24576), P5, q=6, m=10, slab T=0.5"
        return dict(name=name, mm=mm, p=5, q=6, m=10, T=0.5, ex=fields.Cavity3D_PEC(), desc=desc, exact=True)
    if name == "graded3d_p4":
        grade = lambda g: GRADE_A * g + (1 - GRADE_A) * g * g  # noqa: E731
        mm = meshes.cube_kuhn(32, axis_map=grade)
        eps, mu = meshes.materials_split(mm)
        desc = ("3D PEC, unit cube 32^3x6 Kuhn tets (196608) graded toward one corner (h ratio 1:8), "
                "eps in {1, 2.25} split at x=0.5, Gaussian-pulse E, P4, q=5, m=8, slab T=0.05")
        return dict(name=name, mm=mm, p=4, q=5, m=8, T=0.05, ex=fields.GaussianPulse3D(seed=11030),
                    desc=desc, eps=eps, mu=mu, exact=False, cert="graded3d_p4_cavity")
    if name in ("delaunay3d_p4", "delaunay3d_p4_cavity"):
        # the 33^3-point lattice graded toward one corner, jittered and Delaunay-triangulated:
        # patches of 4-44 tets (61 % above 24, 410 vertices above 36: the 48-tet class)
        mm = meshes.graded_delaunay_cube()
        base = ("unit cube, 33^3-point lattice graded toward one corner (h ratio 1:8), jittered by 0.15 h and "
                "Delaunay-triangulated (226989 tets, vertex patches of up to 44 tets)")
        if name == "delaunay3d_p4":
            eps, mu = meshes.materials_split(mm)
            desc = ("3D PEC, " + base + ", eps in {1, 2.25} split at x=0.5, Gaussian-pulse E, P4, q=5, m=8, "
                    "slab T=0.01")
            return dict(name=name, mm=mm, p=4, q=5, m=8, T=0.01, ex=fields.GaussianPulse3D(seed=11030),
                        desc=desc, eps=eps, mu=mu, exact=False, cert="delaunay3d_p4_cavity")
        desc = "3D PEC cavity mode, " + base + ", eps = mu = 1, P4, q=5, m=8, slab T=0.01 (equal-error check)"
        return dict(name=name, mm=mm, p=4, q=5, m=8, T=0.01, ex=fields.Cavity3D_PEC(), desc=desc, exact=True)
    if name == "graded3d_p4_cavity":
        grade = lambda g: GRADE_A * g + (1 - GRADE_A) * g * g  # noqa: E731
        mm = meshes.cube_kuhn(32, axis_map=grade)
        desc = ("3D PEC cavity mode, unit cube 32^3x6 Kuhn tets (196608) graded toward one corner "
                "(h ratio 1:8), eps = mu = 1, P4, q=5, m=8, slab T=0.05 (equal-error certification)")
        return dict(name=name, mm=mm, p=4, q=5, m=8, T=0.05, ex=fields.Cavity3D_PEC(), desc=desc, exact=True)
    if name in ("acoustic3d_p4", "acoustic3d_p4_cavity"):
        grade = lambda g: GRADE_A * g + (1 - GRADE_A) * g * g  # noqa: E731
        mm = meshes.cube_kuhn(32, axis_map=grade)
        bc = meshes.uniform_bc(len(mm["cells"]), 3, meshes.PMC)       # rigid walls
        if name == "acoustic3d_p4":
            kappa, rho = meshes.materials_split(mm)
            desc = ("3D linear acoustics, unit cube 32^3x6 Kuhn tets (196608) graded toward one corner (h ratio "
                    "1:8), kappa in {1, 2.25} split at x=0.5, rho = 1, rigid walls, Gaussian pressure pulse, P4, "
                    "q=5, m=8, slab T=0.05")
            return dict(name=name, mm=mm, p=4, q=5, m=8, T=0.05, ex=fields.AcousticPulse(3), desc=desc, eps=kappa,
                        mu=rho, bc=bc, system="acoustic", exact=False, cert="acoustic3d_p4_cavity")
        desc = ("3D linear acoustics, rigid-wall cavity mode on the same graded mesh, kappa = rho = 1, P4, q=5, "
                "m=8, slab T=0.05 (equal-error certification)")
        return dict(name=name, mm=mm, p=4, q=5, m=8, T=0.05, ex=fields.AcousticCavity(3), desc=desc, bc=bc,
                    system="acoustic", exact=True)
    raise SystemExit(f"unknown workload {name}")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


_ORACLE = {}   # set by cpu_baseline before the worker processes fork


def _oracle_worker(args):
    """Tents w, w + P, w + 2P, ... of the layer-ordered list, one numpy thread, on this
    worker's copy of the oracle state, until `budget` seconds: (DOF-updates, seconds, tents)."""
    w, P, budget = args
    from threadpoolctl import threadpool_limits
    G = _ORACLE
    with threadpool_limits(limits=1):
        dofs, done, t0 = 0.0, 0, time.perf_counter()
        for i in G["order"][w::P]:
            v = int(G["tents"]["vertex"][i])
            G["O"].run_tent(v, float(G["tents"]["t_top"][i]))
            dofs += G["per_elem"] * len(G["om"].v2e[v])
            done += 1
            if time.perf_counter() - t0 > budget:
                break
        return dofs, time.perf_counter() - t0, done


def cpu_baseline(W, budget_s):
    """The oracle as it stands on the host's cores: the same workload (mesh, tents, fields),
    its tents taken in layer order and dealt round robin to one process per core in the
    affinity mask (at most 16), each with its own copy of the oracle state and one numpy
    thread, for budget_s seconds; then the same with one process.  The value is the
    all-core rate; the tents of a layer are independent, so the work per tent is that of a
    sequential run."""
    import multiprocessing as mp

    from mtp_inputs import meshes
    from oracle.mesh import Mesh as OMesh
    from oracle.pitch import pitch as opitch
    from oracle.solve import OracleSolver
    om = OMesh(W["mm"]["coords"], W["mm"]["cells"], eps=W.get("eps"), mu=W.get("mu"), face_bc=W.get("bc"))
    tents = opitch(om, W["T"], 0.5)
    O = OracleSolver(om, W["p"], W["q"], W["m"], system=W.get("system", "maxwell"))
    O.set_nodal_u(W["ex"].u(meshes.equispaced_nodes(W["mm"], W["p"]), 0.0))
    nc = 4 if W.get("system") == "acoustic" else 6
    npn = (W["p"] + 1) * (W["p"] + 2) * (W["p"] + 3) // 6
    _ORACLE.update(O=O, om=om, tents=tents, order=np.argsort(tents["layer"], kind="stable"),
                   per_elem=nc * npn * W["m"] * W["q"])
    cores = min(len(os.sched_getaffinity(0)), 16)
    out = {}
    for P in (cores, 1):
        with mp.get_context("fork").Pool(P) as pool:
            res = pool.map(_oracle_worker, [(w, P, budget_s) for w in range(P)])
        dofs = sum(r[0] for r in res)
        el = max(r[1] for r in res)
        out[P] = (dofs / el, sum(r[2] for r in res), el)
    _ORACLE.clear()
    v, n, el = out[cores]
    v1, n1, el1 = out[1]
    return {"value": v, "unit": "DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} tents in layer order of the same workload ({cores} processes x 1 numpy thread, "
                      f"{el:.1f} s); one process: {n1} tents in {el1:.1f} s",
            "value_1_core": v1, "cpu_model": _cpu_model(), "host_cores_in_mask": len(os.sched_getaffinity(0))}


def slope_use(mm, eps, mu, tents, sigma=0.5):
    """Mean over tents of max over the tent's patch of |grad tau| / (sigma sqrt(eps mu))
    just after the tent (1 = every tent as tall as the slope bound allows), and tents per
    vertex per slab.  Tents of a layer have element-disjoint patches whose vertices no other
    tent of the layer moves, so the slopes after a whole layer are those after each tent."""
    X = mm["coords"][mm["cells"]]
    d = X.shape[2]
    J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    Ji = np.linalg.inv(J)
    gl = np.concatenate([-Ji.sum(axis=1, keepdims=True), Ji], axis=1)   # (ne, d+1, d)
    ne, nv = len(mm["cells"]), len(mm["coords"])
    eps = np.ones(ne) if eps is None else np.asarray(eps)
    mu = np.ones(ne) if mu is None else np.asarray(mu)
    bound = sigma * np.sqrt(eps * mu)
    cells = mm["cells"].astype(np.int64)
    order = np.argsort(cells.ravel(), kind="stable")
    v2e = order // (d + 1)
    ptr = np.searchsorted(cells.ravel()[order], np.arange(nv + 1))
    tau = np.zeros(nv)
    lay = np.asarray(tents["layer"])
    vert = np.asarray(tents["vertex"])
    ttop = np.asarray(tents["t_top"])
    cuts = np.flatnonzero(np.diff(lay)) + 1
    tot = 0.0
    for sl in np.split(np.arange(len(lay)), cuts):
        vs = vert[sl]
        tau[vs] = ttop[sl]
        idx = np.concatenate([v2e[ptr[v]:ptr[v + 1]] for v in vs])
        g = np.einsum("ek,ekx->ex", tau[cells[idx]], gl[idx])
        r = np.linalg.norm(g, axis=1) / bound[idx]
        cnt = ptr[vs + 1] - ptr[vs]
        tot += np.maximum.reduceat(r, np.concatenate([[0], np.cumsum(cnt)[:-1]])).sum()
    return {"mean_slope_over_bound": tot / len(lay), "tents_per_vertex_per_slab": len(lay) / nv}


def blended_peak(prec_kernel, dof_slab, flops_slab, W):
    """Peak for the kernel's mix of units: FP64 (vector or matrix, 78.6) for everything
    except, in the mixed kernel, the contractions of stages n >= 2 (FP32 matrix, 157.3).
    Returns (peak, FP32 contraction flops per slab)."""
    if prec_kernel != 2:
        return PEAK_FP64, 0.0
    d, p, q = 3, W["p"], W["q"]
    npn = (p + 1) * (p + 2) * (p + 3) // 6
    nf = (p + 1) * (p + 2) // 2
    c32 = dof_slab * (q - 1) / q * 2 * d * (npn + nf)
    t = (flops_slab - c32) / PEAK_FP64 + c32 / PEAK_FP32
    return flops_slab / t, c32


def measured_traffic(tag):
    """HBM bytes per launch of the tent kernel from the committed FETCH_SIZE / WRITE_SIZE
    counter summary (copy-calibrated), or None once the kernel sources differ from the
    ones the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tent_mfma_graded3d_p4_traffic.json")
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["source_sha256"]:
            return None
        return rec["kernels"][tag]["hbm_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


SCHEDULES = {"layers": 0, "dag": 1}
PITCH = {"min-vertex": 0, "colour": 1, "auto": 2}   # tent pitching rules
RULE_NAME = {0: "min-vertex", 1: "colour"}          # the rule a table was pitched by
TILE_ORDERS = {0: "default", 1: "round-robin", 2: "blocked", 3: "column-major"}


def describe_tuning(t):
    return {"schedule": {0: "layers", 1: "dag"}[t["schedule"]], "tile_order": TILE_ORDERS[t["tile_order"]],
            "grid_frac": t["grid_frac"], "from_tuning_table": t.get("from_table", False)}


def run(W, precision, steps, warmup, M=None, T=None, schedule="auto", tune=0, pitch=0):
    """Set up one solver on workload W, advance `warmup` untimed and `steps` timed slabs
    (each a replay of the captured slab graph); returns timings and the final fields.
    schedule "auto": the launch choice the tuning table gives at creation (the default
    choice without an entry); tune > 0: run the tuner (tune timed slabs per candidate)
    after the warm-up and time the choice it applies."""
    import torch

    from mtp_inputs import meshes
    from paper_1906_11029_amd import mtp
    mm = W["mm"]
    if M is None:
        M = mtp.Mesh(mm["coords"], mm["cells"], eps=W.get("eps"), mu=W.get("mu"), face_bc=W.get("bc"),
                     system=mtp.MTP_SYSTEM_ACOUSTIC if W.get("system") == "acoustic" else mtp.MTP_SYSTEM_MAXWELL)
        T = mtp.Tents(M, W["T"], 0.5, rule=pitch)
    prec = {"fp64": mtp.MTP_FP64, "mixed": mtp.MTP_MIXED_FP32, "fp64-valu": mtp.MTP_FP64_VALU}[precision]
    S = mtp.Solver(M, T, W["p"], W["q"], W["m"], precision=prec)
    if schedule != "auto":
        S.set_tuning(SCHEDULES[schedule])
    S.set_fields(W["ex"].u(meshes.equispaced_nodes(mm, W["p"]), 0.0), 0.0)
    dof_slab, n_tents = S.slab_dof_updates()
    front = 0.0
    for _ in range(warmup):
        front += W["T"]
        S.advance_to(front)
    tuned = None
    if tune > 0:
        tuned = S.tune(tune)
        log(f"tuner: {tuned}")
    tuning = S.tuning()
    stream = torch.cuda.current_stream()   # the solver's stream: graphs replay on it
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        front += W["T"]
        S.advance_to(front)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_s = ev0.elapsed_time(ev1) * 1e-3
    u = S.get_fields()
    err = None
    if W["exact"]:
        uex = W["ex"].u(meshes.equispaced_nodes(mm, W["p"]), front)
        err = float(np.linalg.norm(u - uex) / np.linalg.norm(uex))
    r = dict(S=S, M=M, T=T, wall=wall, gpu_s=gpu_s, u=u, err=err, dof_slab=dof_slab, n_tents=n_tents,
             flops_slab=S.slab_flops(), kernel=S.kernel(), layers=T.n_layers, value=dof_slab * steps / wall,
             tuning=tuning, tuned=tuned, front=front)
    log(f"{precision:6s} {describe_tuning(tuning)} {W['name']}: {steps} slabs in {wall:.3f}s "
        f"(events {gpu_s:.3f}s), {r['value']:.4e} DOF-updates/s, error vs exact {err}")
    return r


def default_choice_ms(r, W, steps):
    """Time per slab of the same solver with the default launch choice (layer schedule,
    default tiles, full grid), continuing from where run() stopped; None if the applied
    choice is the default."""
    import torch
    t = r["tuning"]
    if t["schedule"] == 0 and t["tile_order"] == 0 and t["grid_frac"] == 1.0:
        return None
    S, front = r["S"], r["front"]
    S.set_tuning(0)
    front += W["T"]
    S.advance_to(front)   # captures the default choice's slab graph
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(steps):
        front += W["T"]
        S.advance_to(front)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - w0) / steps * 1e3
    S.set_tuning(t["schedule"], t["tile_order"], t["grid_frac"])
    return ms


def batch2d(args):
    """64 independent 2D TE plane-wave solves (seed 4): n ~ U{23..158} (2n^2 triangles),
    p ~ U{2..5}, q = p + 1, m = 2p, direction, k ~ U[pi, 4pi] and phase drawn from the seed,
    data faces on the whole boundary, slab 0.1 (ten slabs reach T = 1).  All 64 solves form
    one batch, which groups them by degree: one launch per (global layer index, degree), or
    one persistent launch per degree and slab.  Beside it, the same solves one by one
    with per-layer launches, and every solve's error against its exact plane wave."""
    import torch

    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp
    rng = np.random.default_rng(4)
    specs = [dict(n=int(rng.integers(23, 159)), p=int(rng.integers(2, 6)), theta=float(rng.uniform(0, 2 * np.pi)),
                  k=float(rng.uniform(np.pi, 4 * np.pi)), phase=float(rng.uniform(0, 2 * np.pi))) for _ in range(64)]
    prec = {"fp64": mtp.MTP_FP64, "mixed": mtp.MTP_MIXED_FP32}[args.precision]
    H = 0.1

    def make():
        out = []
        for sp in specs:
            mm = meshes.square_tri(sp["n"])
            ex = fields.PlaneWaveTE(direction=(np.cos(sp["theta"]), np.sin(sp["theta"])), k=sp["k"], phase=sp["phase"])
            M = mtp.Mesh(mm["coords"], mm["cells"], face_bc=meshes.uniform_bc(len(mm["cells"]), 2, meshes.DATA))
            T = mtp.Tents(M, H, 0.5, rule=PITCH[args.pitch])
            S = mtp.Solver(M, T, sp["p"], sp["p"] + 1, 2 * sp["p"], precision=prec)
            nodes = meshes.equispaced_nodes(mm, sp["p"])
            S.set_fields(ex.u(nodes, 0.0), 0.0)
            amp = np.array([-ex.d[1] * ex.amp, ex.d[0] * ex.amp, ex.amp])
            S.set_planewave_bc(amp, ex.k * ex.d, ex.omega, ex.phase)
            out.append((S, ex, nodes))
        return out
    t0 = time.perf_counter()
    solves = make()
    log(f"batch2d: 64 solves set up in {time.perf_counter() - t0:.1f}s")
    B = mtp.Batch([S for S, _, _ in solves])
    if args.schedule != "auto":
        B.set_tuning(SCHEDULES[args.schedule])
    dof = sum(S.slab_dof_updates()[0] for S, _, _ in solves)
    tents = sum(S.slab_dof_updates()[1] for S, _, _ in solves)
    B.advance(args.warmup)
    tuned = B.tune(args.tune) if args.tune > 0 else None
    if tuned:
        log(f"tuner: {tuned}")
    tuning = describe_tuning(B.tuning())
    if tuned:
        tuning["tuner"] = tuned
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    B.advance(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    value = dof * args.steps / wall
    tf = H * (args.warmup + args.steps)
    errs = [float(np.linalg.norm(S.get_fields() - ex.u(nodes, tf)) / np.linalg.norm(ex.u(nodes, tf)))
            for S, ex, nodes in solves]
    log(f"batched ({tuning}): {args.steps} slabs in {wall:.3f}s, {value:.4e} DOF-updates/s; errors max {max(errs):.2e}")
    compare = None
    if not args.no_compare:
        seq = make()
        for S, _, _ in seq:
            S.set_tuning(mtp.MTP_SCHEDULE_LAYERS)
            S.advance_to(H * args.warmup)
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        for S, _, _ in seq:
            S.advance_to(H * (args.warmup + args.steps))
        torch.cuda.synchronize()
        wseq = time.perf_counter() - w1
        same = all(np.array_equal(a.get_state(), b.get_state()) for (a, _, _), (b, _, _) in zip(solves, seq))
        compare = {"one_by_one_layers_dof_updates_per_s": dof * args.steps / wseq,
                   "speedup_batched_vs_one_by_one": wseq / wall, "bitwise_equal": bool(same)}
        log(f"one by one (layers): {wseq:.3f}s; batched speedup {wseq / wall:.2f}; bitwise equal {same}")
    out = {"metric": "DOF-updates/s, 3D Maxwell p=4 MTP: mixed/batched vs FP64 GPU at equal L2 error",
           "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
           "config": {"workload": "64 independent 2D TE plane-wave solves (seed 4), n in 23..158, p in 2..5, "
                                  "q = p+1, m = 2p, data faces, slab 0.1; one batch grouped by degree, "
                                  + ("one persistent launch per degree and slab" if tuning["schedule"] == "dag"
                                     else "one launch per global layer index and degree"),
                      "solves": 64, "tents_per_step": int(tents), "precision": args.precision, "pitch": args.pitch,
                      "pitch_applied": {r: sum(1 for S, _, _ in solves if RULE_NAME[S.tents.rule] == r)
                                        for r in RULE_NAME.values()},
                      "schedule": tuning["schedule"], "tuning": tuning,
                      "rel_l2_error_vs_exact": {"max": max(errs), "median": float(np.median(errs))},
                      "compare": compare}}
    print(json.dumps(out), flush=True)


def curved2d(args):
    """2D TE circular PEC cavity of radius 1: the disk of 96 rings (55,296 triangles), the
    576 triangles on the circle quadratic (midpoints of their boundary edges on the circle),
    P3, q = 4, m = 6, slab 0.05, initial data the TE mode J_1(k r) cos(theta) (k R = 1.8412).
    The tents whose patch holds a curved triangle run on the curved-element path (FP64 vector
    ALU, quadrature, weight-adjusted inverse mass), the others on the FP64 matrix-core kernel.
    Beside it: the same vertices with straight edges (every tent on the matrix-core kernel),
    the curved disk pitched by the other rule, and every run's error against the exact mode."""
    import torch

    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp
    ex = fields.CircularCavityTE()
    mm = meshes.disk_tri(96)
    geo = meshes.p2_geometry(mm, on_circle=1.0)
    p, q, m, H = 3, 4, 6, 0.05
    if args.pitch == "auto":   # the rule the library picks for the curved disk
        Mc = mtp.Mesh(mm["coords"], mm["cells"], curved=geo)
        args.pitch = RULE_NAME[mtp.Tents(Mc, H, 0.5, rule=PITCH["auto"]).rule]
        del Mc
    other = "min-vertex" if args.pitch == "colour" else "colour"
    runs = [("curved", geo, args.pitch), ("straight", None, args.pitch)]
    if not args.no_compare:
        runs.append(("curved_" + other.replace("-", "_") + "_pitch", geo, other))
    res = {}
    for label, g, rule in runs:
        M = mtp.Mesh(mm["coords"], mm["cells"], curved=g)
        T = mtp.Tents(M, H, 0.5, rule=PITCH[rule])
        S = mtp.Solver(M, T, p, q, m, precision=mtp.MTP_FP64)
        nodes = meshes.equispaced_nodes_p2(geo if g is not None else meshes.p2_geometry(mm), p)
        S.set_fields(ex.u(nodes, 0.0), 0.0)
        S.advance_to(H * args.warmup)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        S.advance_to(H * (args.warmup + args.steps))
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        dof, nt = S.slab_dof_updates()
        tf = H * (args.warmup + args.steps)
        u, ue = S.get_fields(), ex.u(nodes, tf)
        res[label] = {"pitch": rule, "dof_updates_per_s": dof * args.steps / wall,
                      "ms_per_step": wall / args.steps * 1e3, "tents_per_step": int(nt),
                      "layers_per_step": int(T.n_layers),
                      "rel_l2_nodal_error_vs_exact": float(np.linalg.norm(u - ue) / np.linalg.norm(ue))}
        log(f"{label}: {args.steps} slabs in {wall:.3f}s, {res[label]['dof_updates_per_s']:.4e} DOF-updates/s, "
            f"error vs exact {res[label]['rel_l2_nodal_error_vs_exact']:.3e}")
    curved_elems = int(sum(1 for e in range(len(mm["cells"]))
                           if np.any(np.abs(geo[e, 3:] - 0.5 * (geo[e, [0, 1, 0]] + geo[e, [1, 2, 2]])) > 1e-14)))
    out = {"metric": "DOF-updates/s, 3D Maxwell p=4 MTP: mixed/batched vs FP64 GPU at equal L2 error",
           "value": res["curved"]["dof_updates_per_s"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["curved"]["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "2D TE circular PEC cavity, disk of 96 rings (55296 triangles, 576 quadratic on "
                                  "the circle), P3, q=4, m=6, slab 0.05, TE mode J_1(kr) cos(theta); curved-element "
                                  "path for the tents whose patch holds a curved triangle",
                      "curved_elements": curved_elems, "pitch": args.pitch, "curved": res["curved"],
                      "straight_edges": res["straight"],
                      "curved_other_pitch": res[runs[2][0]] if len(runs) > 2 else None,
                      "curved_over_straight_time": res["curved"]["ms_per_step"] / res["straight"]["ms_per_step"]}}
    print(json.dumps(out), flush=True)


def stream3d(args):
    """A request stream of 3D PEC cavity solves, served by continuous batching: requests
    (seed 5) on Kuhn cubes n ~ U{8..16} (3,072-24,576 tets), p ~ U{3, 4, 5}, q = p + 1, m = 2p,
    eps = 1, the Gaussian pulse of the graded workload (seed per request), final time
    T ~ U[0.25, 1] in slabs of at most 0.25.  A calibration pass serves every request at once
    (batched, mixed) to measure the capacity; the stream then arrives as a Poisson process at
    0.7 of it.  Served in mixed precision with every solve in flight advancing one slab per
    step in one batch (admission FIFO while the estimated device memory fits 90 % of the free
    HBM), and beside it by the plain FP64 path one solve at a time on the same arrivals.
    Latency = arrival to fields read out, set-up (mesh, pitching, solver) included."""
    import torch

    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp, serve
    rng = np.random.default_rng(5)
    specs = [dict(n=int(rng.integers(8, 17)), p=int(rng.integers(3, 6)), T=float(rng.uniform(0.25, 1.0)),
                  seed=int(rng.integers(1 << 30))) for _ in range(args.stream_requests)]

    class GpuExecutor:
        def __init__(self, precision):
            self.prec = precision
            self.batch, self.members = None, ()

        def footprint(self, req):   # state, stage copy and tables: ~ (2 W + 1) per node value + per-tet tables
            sp = req.spec
            ne = 6 * sp["n"] ** 3
            npl = (sp["p"] + 1) * (sp["p"] + 2) * (sp["p"] + 3) // 6
            return ne * npl * 6 * 8 * 3 + ne * 2048

        def setup(self, req):
            sp = req.spec
            mm = meshes.cube_kuhn(sp["n"])
            M = mtp.Mesh(mm["coords"], mm["cells"])
            nslab = int(np.ceil(sp["T"] / 0.25))
            T = mtp.Tents(M, sp["T"] / nslab, 0.5, rule=PITCH[args.pitch])
            S = mtp.Solver(M, T, sp["p"], sp["p"] + 1, 2 * sp["p"], precision=self.prec)
            S.set_fields(fields.GaussianPulse3D(seed=sp["seed"]).u(meshes.equispaced_nodes(mm, sp["p"]), 0.0), 0.0)
            return {"rid": req.rid, "S": S, "T": sp["T"], "nslab": nslab, "dof": S.slab_dof_updates()[0] * nslab}

        def slabs(self, h):
            return h["nslab"]

        def step(self, hs):
            key = tuple(h["rid"] for h in hs)
            if key != self.members:   # the set in flight changed: a new batch over it
                self.batch = None
                self.batch = mtp.Batch([h["S"] for h in hs])
                self.members = key
            self.batch.advance(1)

        def run(self, h):
            h["S"].advance_to(h["T"])

        def finish(self, h):
            u = h["S"].get_fields()
            return {"dof": h["dof"], "finite": bool(np.isfinite(u).all())}

    budget = int(0.9 * torch.cuda.mem_get_info()[0])

    def serve_stream(arrivals, precision, batched):
        reqs = [serve.Request(i, a, sp) for i, (a, sp) in enumerate(zip(arrivals, specs))]
        ex = GpuExecutor(precision)
        recs = serve.StreamServer(ex, budget, batched=batched).run(reqs)
        ex.batch = None
        torch.cuda.synchronize()
        assert all(r.result["finite"] for r in recs)
        return serve.summarize(recs, sum(r.result["dof"] for r in recs))

    cal = serve_stream([0.0] * len(specs), mtp.MTP_MIXED_FP32, True)
    lam = 0.7 * cal["requests_per_s"]
    arrivals = serve.poisson_arrivals(len(specs), lam, np.random.default_rng(5))
    log(f"stream3d: capacity {cal['requests_per_s']:.2f} requests/s (all at once), arrivals at {lam:.2f}/s")
    mixed = serve_stream(arrivals, mtp.MTP_MIXED_FP32, True)
    log(f"batched mixed: {mixed}")
    seq = serve_stream(arrivals, mtp.MTP_FP64, False)
    log(f"one at a time, FP64: {seq}")
    out = {"metric": "DOF-updates/s, 3D Maxwell p=4 MTP: mixed/batched vs FP64 GPU at equal L2 error",
           "value": mixed["dof_updates_per_s"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": len(specs),
           "warmup": 0, "ms_per_step": mixed["makespan_s"] * 1e3 / len(specs), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": f"request stream of {len(specs)} 3D PEC cavity solves (seed 5), Kuhn cubes "
                                  "n in 8..16, p in 3..5, q = p+1, m = 2p, Gaussian pulse, T in [0.25, 1], Poisson "
                                  "arrivals at 0.7 of the measured capacity; continuous batching in mixed "
                                  "precision beside FP64 one solve at a time; ms_per_step is per request",
                      "capacity_requests_per_s": cal["requests_per_s"], "arrival_rate_per_s": lam,
                      "memory_budget_bytes": budget, "batched_mixed": mixed, "sequential_fp64": seq,
                      "speedup_throughput": mixed["dof_updates_per_s"] / seq["dof_updates_per_s"],
                      "p99_latency_ratio_fp64_over_mixed": seq["latency_p99_s"] / mixed["latency_p99_s"]}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="graded3d_p4")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed", "fp64-valu"])
    ap.add_argument("--schedule", default="auto", choices=["auto", "layers", "dag"],
                    help="one launch per layer, one persistent launch per slab over the tent DAG, or "
                         "auto (default): the launch choice of the package's tuning table")
    ap.add_argument("--pitch", default=None, choices=list(PITCH),
                    help="tent pitching rule: the minimum vertex moves, the colour classes take turns, or "
                         "auto (the table with less work; the default)")
    ap.add_argument("--stream-requests", type=int, default=200, help="requests of the stream3d workload")
    ap.add_argument("--tune", type=int, default=0,
                    help="run the tuner (this many timed slabs per candidate) before timing")
    ap.add_argument("--tune-out", default=None, help="write the tuning table here at the end")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 run of the same workload and the equal-error check")
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle work per measurement (all cores, then one core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(sharding is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.pitch is None:
        # the library's automatic choice: the colour order where it makes less work (the disk:
        # 47 layers per slab instead of 28,069; the batch's squares; the uniform Kuhn cubes),
        # the minimum vertex on the graded two-media cube, where colour turns make more tents
        args.pitch = "auto"

    import torch

    if args.copy_calibration:
        x = torch.ones(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": x.numel() * 8, "copies": 3}))
        return

    from paper_1906_11029_amd import mtp
    if args.workload == "curved2d":
        curved2d(args)
        return
    if args.workload == "stream3d":
        stream3d(args)
        return
    if args.workload == "batch2d":
        batch2d(args)
        if args.tune_out:
            mtp.mtp_tune_save(args.tune_out)
        return
    W = workload(args.workload)
    pitch = PITCH[args.pitch]
    head = run(W, args.precision, args.steps, args.warmup, schedule=args.schedule, tune=args.tune, pitch=pitch)
    M, T = head["M"], head["T"]
    log(f"mesh {M.info} tents {head['n_tents']} layers {head['layers']}")
    tuning = describe_tuning(head["tuning"])
    if head["tuned"]:
        tuning["tuner"] = head["tuned"]
    tuning["default_choice_ms_per_step"] = default_choice_ms(head, W, min(args.steps, 5))
    del head["S"]
    args.schedule = tuning["schedule"]
    kernel_name = {0: "tent_kernel (vector-ALU FP64)", 1: "tent_mfma_kernel<double> (FP64 MFMA)",
                   2: "tent_mfma_kernel<float> (FP64 first stage, FP32 MFMA later stages)"}[head["kernel"]]
    nl = head["layers"]
    per_slab = 1 if args.schedule == "dag" else nl   # tent-kernel launches per slab
    launches = args.steps * per_slab
    kern_avg = head["gpu_s"] / launches
    achieved = head["flops_slab"] / per_slab / kern_avg / 1e12
    peak_bl, c32 = blended_peak(head["kernel"], head["dof_slab"], head["flops_slab"], W)
    # the bulk contraction's pipe: FP32 matrix cores for the mixed kernel, FP64 otherwise
    peak = PEAK_FP32 if head["kernel"] == 2 else PEAK_FP64
    traffic = None
    if args.workload == "graded3d_p4" and head["kernel"] in (1, 2):
        traffic = measured_traffic(("mixed" if head["kernel"] == 2 else "fp64") + "_" + args.schedule)
    slopes = slope_use(W["mm"], W.get("eps"), W.get("mu"), T.export())

    compare = None
    if not args.no_compare and args.precision == "mixed":
        # the plain FP64 path on the same workload and inputs, and the equal-error check on
        # the same graded mesh with a closed-form solution over as many slabs as above
        ref = run(W, "fp64", args.steps, args.warmup, M=M, T=T, schedule="auto", tune=args.tune)
        diff = float(np.linalg.norm(head["u"] - ref["u"]) / np.linalg.norm(ref["u"]))
        del ref["S"]
        cert = {}
        if W.get("cert"):
            Wc = workload(W["cert"])
            nsl = args.steps + args.warmup
            for prec in ("fp64", "mixed"):
                rc = run(Wc, prec, nsl, 0, schedule="auto", tune=args.tune, pitch=pitch)
                cert[prec + "_rel_l2_error_vs_exact"] = rc["err"]
                del rc
            cert["slabs"] = nsl
            cert["final_time"] = nsl * Wc["T"]
            e64, emx = cert["fp64_rel_l2_error_vs_exact"], cert["mixed_rel_l2_error_vs_exact"]
            cert["mixed_over_fp64_error"] = emx / e64
            cert["equal_within_5pct"] = bool(abs(emx / e64 - 1) <= 0.05)
            cert["workload"] = Wc["desc"]
        compare = {"fp64_dof_updates_per_s": ref["value"], "speedup_vs_fp64": head["value"] / ref["value"],
                   "fp64_tuning": describe_tuning(ref["tuning"]),
                   "mixed_vs_fp64_rel_l2": diff, "equal_error_check": cert or None}

    out = {
        "metric": "DOF-updates/s, 3D Maxwell p=4 MTP: mixed/batched vs FP64 GPU at equal L2 error",
        "value": head["value"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["wall"] / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if head["kernel"] == 2 else "f64", "data": "synthetic",
        "config": {"workload": W["desc"], "tets": int(M.info["ne"]), "p": W["p"], "q": W["q"], "m": W["m"],
                   "tents_per_step": int(head["n_tents"]), "layers_per_step": int(nl), "slope_fraction": 0.5,
                   "pitch": args.pitch, "pitch_applied": RULE_NAME[T.rule],
                   "mean_slope_over_bound": round(float(slopes["mean_slope_over_bound"]), 4),
                   "tents_per_vertex_per_slab": round(float(slopes["tents_per_vertex_per_slab"]), 3),
                   "precision": args.precision, "schedule": args.schedule, "tuning": tuning,
                   "nodal_rel_error_vs_exact": head["err"],
                   "tent_dof_updates_per_s": head["value"] / (W["m"] * W["q"])},
        "roofline": {"bound": "alu" if head["kernel"] == 0 else "mfma", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "hbm_gbs": traffic / kern_avg / 1e9 if traffic else None,
                     "kernel": kernel_name + (", one persistent launch per slab over the tent DAG"
                                              if args.schedule == "dag" else ", one launch per layer")
                               + ", slab captured in a HIP graph",
                     "avg_launch_ms": kern_avg * 1e3, "launches": int(launches),
                     "flop_per_spacetime_dof": head["flops_slab"] / head["dof_slab"],
                     "peak_blended": peak_bl, "frac_blended": achieved / peak_bl,
                     "fp32_mfma_flop_share": c32 / head["flops_slab"]},
    }
    if compare:
        out["config"]["compare"] = compare
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_budget)
    if args.tune_out:
        mtp.mtp_tune_save(args.tune_out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
