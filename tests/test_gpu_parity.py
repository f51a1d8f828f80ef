"""GPU parity: the HIP path (through the C interface) against the FP64 oracle.

Small cases compare every nodal value: relative L2 <= 1e-10 (the FP64 bound) over the
whole array and, element by element, every nodal difference <= 1e-10 max |oracle|; the
tent lists must be bit-identical.  The full-size 3D cavity workload (16^3 Kuhn cube, P3,
q=4, m=6) compares sampled tents of a mid-slab layer, each re-run by the oracle from
the GPU's state before that layer."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

from cases import CASES, DATA, LARGE_P4_CASES, planewave_params, setup  # noqa: E402
from parity import assert_parity, rel  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-10


def gpu_solver(name, precision=0):
    from paper_1906_11029_amd import mtp
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc)
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=precision)
    S.set_fields(u0, 0.0)
    if c["kind"] == DATA:
        S.set_planewave_bc(*planewave_params(ex, dim))
    return c, S, T


def fixture(name):
    path = os.path.join(HERE, "golden", f"oracle_{name}.npz")
    if os.path.exists(path):
        return np.load(path)
    pytest.skip(f"missing oracle fixture {path}")


KERNELS = {"mfma64": 0, "valu64": 2}


# the vector-ALU kernel covers p <= 4 in 3D
PARITY_PARAMS = [(n, k) for n in CASES for k in KERNELS
                 if not (k == "valu64" and CASES[n]["p"] == 5 and CASES[n]["mesh"][0] in ("kuhn", "kuhn_graded",
                                                                                         "delaunay", "tet1"))]


@pytest.mark.parametrize("name,kernel", PARITY_PARAMS)
def test_parity_against_oracle(name, kernel):
    """FP64 paths (matrix-core and vector-ALU kernels): every nodal value, relative L2 <= 1e-10."""
    print(f"[gpu parity] {name} {kernel}", flush=True)
    ref = fixture(name)
    c, S, T = gpu_solver(name, KERNELS[kernel])
    assert S.kernel() == (1 if kernel == "mfma64" else 0)
    ex = T.export()
    for k in ("vertex", "t_top", "layer"):
        assert np.array_equal(ex[k], ref[k]), f"tent list differs in {k}"
    S.advance_to(c["slabs"] * c["T"])
    w = S.get_state()
    u = S.get_fields()
    assert_parity(w, ref["w"], TOL, f"{name} w")
    assert_parity(u, ref["u"], TOL, f"{name} u")


MIXED_TOL = 1e-6


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_fp32_against_oracle(name):
    """Mixed path against the FP64 oracle: relative L2 <= 1e-6.  FP32 matrix-core
    contractions for the stages n >= 2 of every sub-interval (acting on the small Taylor
    coefficients); FP64 first stage, inversions, fluxes and Taylor sum."""
    print(f"[gpu parity] {name} mixed", flush=True)
    ref = fixture(name)
    c, S, T = gpu_solver(name, 1)
    assert S.kernel() == 2
    S.advance_to(c["slabs"] * c["T"])
    err, el = assert_parity(S.get_state(), ref["w"], MIXED_TOL, f"{name} mixed w")
    print(f"  mixed relative L2 {err:.3e}, worst element {el:.3e}")


def test_layer_api_equals_advance_and_is_deterministic():
    name = "cav3d_p3"
    c, S1, T = gpu_solver(name)
    S1.advance_to(c["T"])
    w1 = S1.get_state()
    c, S2, T2 = gpu_solver(name)
    for l in range(T2.n_layers):
        S2.layer_advance(l)
    w2 = S2.get_state()
    assert np.array_equal(w1, w2)
    assert S2.front() == (c["T"], 0)


def test_error_paths():
    from paper_1906_11029_amd import mtp
    c, S, T = gpu_solver("cav3d_p1")
    with pytest.raises(mtp.MTPError) as e:      # layers out of order
        S.layer_advance(3)
    assert e.value.code == -7
    with pytest.raises(mtp.MTPError) as e:      # not a whole number of slabs
        S.advance_to(0.3 * c["T"])
    assert e.value.code == -7
    bad = np.zeros(S.shape)
    bad[0, 0, 0] = np.nan
    with pytest.raises(mtp.MTPError) as e:
        S.set_fields(bad)
    assert e.value.code == -5
    # data faces need a plane wave
    cc, mm, dim, eps, mu, bc, ex, u0 = setup("planewave3d_p2")
    M = mtp.Mesh(mm["coords"], mm["cells"], face_bc=bc)
    Tt = mtp.Tents(M, cc["T"])
    S2 = mtp.Solver(M, Tt, 2, 3, 4)
    S2.set_fields(u0)
    with pytest.raises(mtp.MTPError) as e:
        S2.advance_to(cc["T"])
    assert e.value.code == -7


def test_device_pointer_round_trip():
    import torch
    c, S, T = gpu_solver("cav3d_p2")
    _, _, _, _, _, _, _, u0 = setup("cav3d_p2")
    d_in = torch.from_numpy(u0).cuda()
    S.set_fields(d_in)
    out = torch.empty(S.shape, dtype=torch.float64, device="cuda")
    S.get_fields(out)
    assert np.allclose(out.cpu().numpy(), u0, rtol=0, atol=1e-14)


def _full_cavity(n=16, p=3):
    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp
    mm = meshes.cube_kuhn(n)
    ex = fields.Cavity3D_PEC()
    u0 = ex.u(meshes.equispaced_nodes(mm, p), 0.0)
    M = mtp.Mesh(mm["coords"], mm["cells"])
    T = mtp.Tents(M, 1.0, 0.5)
    S = mtp.Solver(M, T, p, p + 1, 2 * p)
    S.set_fields(u0)
    return mm, ex, u0, M, T, S


def test_full_size_cavity_sampled_tents():
    """16^3 Kuhn cube (24576 tets), P3, q=4, m=6, slab T=1: run to the middle layer,
    then compare 12 sampled tents of that layer with the oracle started from the GPU's
    state before it (same launch configuration as the benchmark)."""
    from oracle.mesh import Mesh as OMesh
    from oracle.solve import OracleSolver
    print("[gpu parity] full-size cavity sampled tents", flush=True)
    mm, ex, u0, M, T, S = _full_cavity()
    L = T.n_layers // 2
    for l in range(L):
        S.layer_advance(l)
    w_before = S.get_state()
    S.layer_advance(L)
    w_after = S.get_state()
    tl = T.export()
    tau = np.zeros(M.info["nv"])
    sel = tl["layer"] < L
    tau[tl["vertex"][sel]] = tl["t_top"][sel]      # front before layer L
    om = OMesh(mm["coords"], mm["cells"])
    O = OracleSolver(om, 3, 4, 6)
    O.set_nodal_w(w_before)
    O.tau[:] = tau
    idx = np.arange(T.layer_ptr[L], T.layer_ptr[L + 1])
    pick = np.random.default_rng(0).choice(idx, size=12, replace=False)
    for i in pick:
        O.run_tent(int(tl["vertex"][i]), float(tl["t_top"][i]))
    w_or = O.nodal_w()
    for i in pick:
        es = om.v2e[int(tl["vertex"][i])]
        assert_parity(w_after[es], w_or[es], TOL, f"tent {i}")
    # elements outside the layer's patches are untouched
    touched = np.unique(np.concatenate([om.v2e[int(v)] for v in tl["vertex"][idx]]))
    mask = np.ones(len(w_after), bool)
    mask[touched] = False
    assert np.array_equal(w_after[mask], w_before[mask])


def test_full_size_cavity_convergence():
    """Whole slabs at full size (16^3 Kuhn cube, P3, q=4, m=6, T=1) and at half resolution
    (8^3): the nodal error against the exact cavity mode falls at the rate of the P3
    discretisation, h^(p+1) (observed rate > p + 1 - 0.3), and the field stays finite."""
    from mtp_inputs import meshes
    errs = []
    for n in (8, 16):
        mm, ex, u0, M, T, S = _full_cavity(n)
        S.advance_to(1.0)
        u = S.get_fields()
        assert np.all(np.isfinite(u))
        errs.append(rel(u, ex.u(meshes.equispaced_nodes(mm, 3), 1.0)))
    rate = np.log2(errs[0] / errs[1])
    print(f"  P3 cavity errors {errs}, rate {rate:.2f}")
    assert rate > 3.7, errs


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_matches_eager_layers(precision):
    """advance_to replays one captured slab graph; three replays, with reads (eager work
    and synchronisation) between them, must equal the layer-by-layer launches bitwise."""
    name = "te_pmc_p2_two_slabs"
    c, A, TA = gpu_solver(name, precision)
    c, B, TB = gpu_solver(name, precision)
    B.set_graph(False)
    for k in range(1, 4):
        A.advance_to(k * c["T"])
        for l in range(TB.n_layers):
            B.layer_advance(l)
        wa, wb = A.get_state(), B.get_state()
        assert np.array_equal(wa, wb), f"replay {k}"
        assert A.front() == B.front() == (k * c["T"], 0)


def _pw_solver(n, p, q, m, T, theta, k, phase, precision):
    from mtp_inputs import fields, meshes
    from paper_1906_11029_amd import mtp
    mm = meshes.square_tri(n)
    bc = meshes.uniform_bc(len(mm["cells"]), 2, meshes.DATA)
    ex = fields.PlaneWaveTE(direction=(np.cos(theta), np.sin(theta)), k=k, phase=phase)
    M = mtp.Mesh(mm["coords"], mm["cells"], face_bc=bc)
    Tt = mtp.Tents(M, T, 0.5)
    S = mtp.Solver(M, Tt, p, q, m, precision=precision)
    S.set_fields(ex.u(meshes.equispaced_nodes(mm, p), 0.0))
    S.set_planewave_bc(*planewave_params(ex, 2))
    return S, ex, mm


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_solves(precision):
    """Solvers on different meshes, plane waves, q and m, advanced as one batch (one launch
    per layer index), equal the same solvers advanced one by one, bitwise."""
    from paper_1906_11029_amd import mtp
    specs = [(5, 2, 3, 4, 0.3, 0.2, 6.0, 0.1), (9, 2, 3, 4, 0.3, 1.3, 9.0, 2.0),
             (3, 2, 4, 2, 0.25, 2.9, 4.0, 0.7), (7, 2, 3, 6, 0.2, 4.4, 7.5, 5.1)]
    single = [_pw_solver(*sp, precision)[0] for sp in specs]
    batched = [_pw_solver(*sp, precision)[0] for sp in specs]
    for S, sp in zip(single, specs):
        S.advance_to(2 * sp[4])
    B = mtp.Batch(batched)
    B.advance(1)
    B.advance(1)
    for S1, S2, sp in zip(single, batched, specs):
        assert S2.front() == (2 * sp[4], 0)
        assert np.array_equal(S1.get_state(), S2.get_state())


BATCH_3D = ["cav3d_p2", "cav3d_p2_pmc_eps", "planewave3d_p2"]


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, TOL), (1, MIXED_TOL)])
def test_batch_3d_against_oracle_fixtures(precision, tol, schedule):
    """Three 3D P2 cases (PEC cavity, PMC cavity with two media, plane-wave data faces)
    advanced as one batch, in both precisions and both schedules (one launch per global
    layer index, or one persistent launch draining the three tent DAGs), against the
    oracle's fixtures: FP64 <= 1e-10, mixed <= 1e-6, element by element."""
    from paper_1906_11029_amd import mtp
    print(f"[gpu parity] 3D batch precision {precision} schedule {schedule}", flush=True)
    solvers = [gpu_solver(nm, precision)[1] for nm in BATCH_3D]
    B = mtp.Batch(solvers)
    B.set_schedule(schedule)
    B.advance(1)
    for S, nm in zip(solvers, BATCH_3D):
        assert_parity(S.get_state(), fixture(nm)["w"], tol, f"batch {nm}")


@pytest.mark.parametrize("schedule", [0, 1])
def test_batch_2d_mixed_degrees_against_oracle_fixtures(schedule):
    """2D P2 cases of different meshes, boundary kinds and q, m (plane wave, 32-fan with data
    faces, PEC cavity with two media) in one mixed-precision batch against the oracle."""
    from paper_1906_11029_amd import mtp
    names = ["te_planewave_p2", "te_fan32_p2_data", "te_pec_p2_eps"]
    print(f"[gpu parity] 2D mixed batch schedule {schedule}", flush=True)
    solvers = [gpu_solver(nm, 1)[1] for nm in names]
    B = mtp.Batch(solvers)
    B.set_schedule(schedule)
    B.advance(1)
    for S, nm in zip(solvers, names):
        assert_parity(S.get_state(), fixture(nm)["w"], MIXED_TOL, f"batch {nm}")


def test_planewave_change_between_graph_replays():
    """Boundary data changed between two advance_to calls takes effect on the next slab:
    the replayed slab graph equals eager layer launches fed the same sequence of data
    (the setter drops the captured graph, which holds the parameter block by value), and
    differs from a run that kept the first wave."""
    from mtp_inputs import fields
    print("[gpu parity] plane-wave change between graph replays", flush=True)
    name = "te_planewave_p2"
    c, A, TA = gpu_solver(name)
    c, B, TB = gpu_solver(name)
    c, K, TK = gpu_solver(name)
    B.set_graph(False)
    second = planewave_params(fields.PlaneWaveTE(direction=(1.0, -0.4), k=3.0, phase=0.7), 2)
    A.advance_to(c["T"])
    K.advance_to(c["T"])
    for l in range(TB.n_layers):
        B.layer_advance(l)
    A.set_planewave_bc(*second)
    B.set_planewave_bc(*second)
    A.advance_to(2 * c["T"])
    K.advance_to(2 * c["T"])
    for l in range(TB.n_layers):
        B.layer_advance(l)
    wa, wb, wk = A.get_state(), B.get_state(), K.get_state()
    assert np.array_equal(wa, wb)
    assert rel(wa, wk) > 1e-3


MIXED_DEGREE = {
    2: ["te_pmc_p1", "te_planewave_p2", "te_pmc_p3", "te_pec_p4_alpha025", "te_pmc_p5", "te_fan32_p2_data",
        "te_fan12_p3"],
    3: ["cav3d_p1", "cav3d_p3", "planewave3d_p2", "cav3d_p2", "delaunay3d_p3_eps", "cav3d_p4"],
}


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, TOL), (1, MIXED_TOL)])
@pytest.mark.parametrize("dim", [2, 3])
def test_batch_mixed_degrees_against_oracle(dim, precision, tol, schedule):
    """Solves of several degrees (listed out of degree order; cavities, plane-wave data
    faces, fans and a Delaunay patch) in one batch: the batch groups its solvers by degree,
    one launch per (global layer index, degree) or one persistent launch per degree; against
    the oracle's fixtures element by element, and equal to the same solves advanced one by
    one: bitwise where the batch runs a solve with the kernel of the same patch capacity
    (the group's largest patch falls in the same class as the solve's own), else to
    rounding (a kernel of another capacity is another instantiation, which the compiler
    may contract differently)."""
    from paper_1906_11029_amd import mtp
    names = MIXED_DEGREE[dim]
    print(f"[gpu parity] {dim}D mixed-degree batch precision {precision} schedule {schedule}", flush=True)
    batched = [gpu_solver(nm, precision)[1] for nm in names]
    single = [gpu_solver(nm, precision) for nm in names]
    B = mtp.Batch(batched)
    B.set_schedule(schedule)
    B.advance(1)
    cap = lambda mp: 8 if mp <= 8 else 24 if mp <= 24 else 48   # noqa: E731
    group = {}
    for S in batched:
        group[S.p] = max(group.get(S.p, 0), S.mesh.info["max_patch"])
    for S, (c, S1, _), nm in zip(batched, single, names):
        S1.advance_to(c["T"])
        w, w1 = S.get_state(), S1.get_state()
        assert_parity(w, fixture(nm)["w"], tol, f"batch {nm}")
        if cap(group[S.p]) == cap(S.mesh.info["max_patch"]):
            assert np.array_equal(w, w1), nm
        else:
            assert np.abs(w - w1).max() <= (1e-13 if precision == 0 else 1e-9) * np.abs(w1).max(), nm


LARGE_P4_SAT = [n for n, c in LARGE_P4_CASES.items()
                if "method" not in c and "system" not in c and c["mesh"][0] == "delaunay"]
# patches of 37-48 tets: the 48-tet class (F/R of the tent in device memory); the RK4
# variant runs in FP64 only
XL_P4 = [n for n, c in LARGE_P4_CASES.items() if c["mesh"][0] == "delaunay48" and "method" not in c]
XL_P4_RK4 = [n for n, c in LARGE_P4_CASES.items() if c["mesh"][0] == "delaunay48" and c.get("method") == "rk4"]
XL_PARAMS = [(n, 0, TOL) for n in XL_P4_RK4] + [(n, p, t) for n in XL_P4 for p, t in ((0, TOL), (1, MIXED_TOL))]


@pytest.mark.parametrize("precision,tol", [(0, TOL), (1, MIXED_TOL)])
@pytest.mark.parametrize("name", LARGE_P4_SAT)
def test_large_p4_patches_against_oracle(name, precision, tol):
    """P4 on the jittered Delaunay cube, whose vertex patches hold up to 36 tets: the 36-tet
    class (operator block in device memory, column-block products, Taylor sums in W) against
    the oracle, element by element: FP64 <= 1e-10, mixed <= 1e-6."""
    print(f"[gpu parity] {name} precision {precision}", flush=True)
    ref = fixture(name)
    c, S, T = gpu_solver(name, precision)
    assert S.mesh.info["max_patch"] > 24
    assert S.kernel() == (1 if precision == 0 else 2)
    ex = T.export()
    for k in ("vertex", "t_top", "layer"):
        assert np.array_equal(ex[k], ref[k]), f"tent list differs in {k}"
    S.advance_to(c["slabs"] * c["T"])
    assert_parity(S.get_state(), ref["w"], tol, f"{name} w")


def test_large_p4_patches_persistent_schedule_and_batch():
    """The 36-tet class under the persistent schedule (bit-identical to the layers) and in a
    batch of both cases (against the oracle)."""
    from paper_1906_11029_amd import mtp
    names = LARGE_P4_SAT
    print("[gpu parity] large P4 patches: persistent schedule and batch", flush=True)
    c, A, _ = gpu_solver(names[0])
    _, B, _ = gpu_solver(names[0])
    B.set_schedule(mtp.MTP_SCHEDULE_DAG)
    A.advance_to(c["T"])
    B.advance_to(c["T"])
    assert np.array_equal(A.get_state(), B.get_state())
    solvers = [gpu_solver(nm)[1] for nm in names]
    mtp.Batch(solvers).advance(1)
    for S, nm in zip(solvers, names):
        assert_parity(S.get_state(), fixture(nm)["w"], TOL, f"batch {nm}")


@pytest.mark.parametrize("name,precision,tol", [("delaunay3d_p4_rk4", 0, TOL), ("ac_delaunay3d_p4", 0, TOL),
                                                ("ac_delaunay3d_p4", 1, MIXED_TOL)])
def test_large_p4_patches_rk4_and_acoustics(name, precision, tol):
    """The 36-tet P4 class under the classical RK4 variant (FP64) and for linear acoustics
    (both precisions) against the oracle, element by element."""
    from paper_1906_11029_amd import mtp
    print(f"[gpu parity] {name} precision {precision}", flush=True)
    ref = fixture(name)
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    system = mtp.MTP_SYSTEM_ACOUSTIC if c["system"] == "acoustic" else mtp.MTP_SYSTEM_MAXWELL
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc, system=system)
    assert M.info["max_patch"] > 24
    T = mtp.Tents(M, c["T"], 0.5)
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=precision)
    if c["method"] == "rk4":
        S.set_method(mtp.MTP_METHOD_RK4)
    S.set_fields(u0, 0.0)
    S.advance_to(c["slabs"] * c["T"])
    assert_parity(S.get_state(), ref["w"], tol, f"{name} w")


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("name,precision,tol", XL_PARAMS)
def test_xl_p4_patches_against_oracle(name, precision, tol, schedule):
    """P4 on a jittered Delaunay cube with two vertex patches above 36 tets (the largest 48):
    the 48-tet class (operator block in LDS, the tent's F/R in a device-memory slot per
    workgroup, column-block products, Taylor sums in W) against the oracle, element by
    element (FP64 <= 1e-10, mixed <= 1e-6), per-layer launches and the persistent schedule;
    SAT in both precisions, the RK4 variant in FP64, Maxwell and acoustics."""
    from paper_1906_11029_amd import mtp
    print(f"[gpu parity] {name} precision {precision} schedule {schedule}", flush=True)
    ref = fixture(name)
    c, mm, dim, eps, mu, bc, ex, u0 = setup(name)
    system = mtp.MTP_SYSTEM_ACOUSTIC if c["system"] == "acoustic" else mtp.MTP_SYSTEM_MAXWELL
    M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc, system=system)
    assert M.info["max_patch"] == 48
    T = mtp.Tents(M, c["T"], 0.5)
    ex_t = T.export()
    for k in ("vertex", "t_top", "layer"):
        assert np.array_equal(ex_t[k], ref[k]), f"tent list differs in {k}"
    S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=precision)
    assert S.kernel() == (1 if precision == 0 else 2)
    if c["method"] == "rk4":
        S.set_method(mtp.MTP_METHOD_RK4)
    S.set_schedule(schedule)
    S.set_fields(u0, 0.0)
    S.advance_to(c["slabs"] * c["T"])
    assert_parity(S.get_state(), ref["w"], tol, f"{name} w")


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("precision,tol", [(0, TOL), (1, MIXED_TOL)])
def test_p4_batch_mixing_patch_classes(precision, tol, schedule):
    """A P4 group of a Kuhn cube (patches up to 24 tets: its own solver keeps the operator in
    LDS) and the jittered Delaunay cube (up to 36): the group runs in the 36-tet class, whose
    operator block the batch stages in its own workspace for every member, against the
    oracle."""
    from paper_1906_11029_amd import mtp
    names = ["cav3d_p4", "delaunay3d_p4"]
    print(f"[gpu parity] P4 batch of a 24- and a 36-tet-patch solve, precision {precision} schedule {schedule}",
          flush=True)
    refs = [fixture(n) for n in names]
    made = [gpu_solver(n, precision) for n in names]
    assert made[0][1].mesh.info["max_patch"] <= 24 < made[1][1].mesh.info["max_patch"] <= 36
    B = mtp.Batch([S for _, S, _ in made])
    B.set_schedule(schedule)
    B.advance(1)
    for (c, S, _), n, ref in zip(made, names, refs):
        assert_parity(S.get_state(), ref["w"], tol, f"batch {n}")


# batches with a degree group in the 48-tet P4 class (a 36-tet-patch solve joins the group
# and runs in its class): name, cases, precisions
XL_BATCHES = [("maxwell", ["delaunay48_p4", "delaunay48_p4_pmc_eps", "delaunay3d_p4"], (0, 1)),
              ("acoustic", ["ac_delaunay48_p4", "ac_delaunay3d_p4"], (0, 1)),
              ("rk4", ["delaunay48_p4_rk4", "delaunay3d_p4_rk4"], (0,))]
XL_BATCH_PARAMS = [(n, cs, p) for n, cs, ps in XL_BATCHES for p in ps]


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("batch,names,precision", XL_BATCH_PARAMS)
def test_xl_p4_batches_against_oracle(batch, names, precision, schedule):
    """A batch whose P4 group falls in the 48-tet class (the batch's own F/R slots, a capped
    per-layer grid striding over the layer's segments, or the persistent schedule) against
    the oracle, element by element: FP64 <= 1e-10, mixed <= 1e-6."""
    from paper_1906_11029_amd import mtp
    print(f"[gpu parity] 48-tet P4 batch {batch} precision {precision} schedule {schedule}", flush=True)
    refs = [fixture(n) for n in names]
    solvers = []
    for n in names:
        c, mm, dim, eps, mu, bc, ex, u0 = setup(n)
        system = mtp.MTP_SYSTEM_ACOUSTIC if c["system"] == "acoustic" else mtp.MTP_SYSTEM_MAXWELL
        M = mtp.Mesh(mm["coords"], mm["cells"], eps=eps, mu=mu, face_bc=bc, system=system)
        T = mtp.Tents(M, c["T"], 0.5)
        S = mtp.Solver(M, T, c["p"], c["q"], c["m"], alpha=c["alpha"], precision=precision)
        if c["method"] == "rk4":
            S.set_method(mtp.MTP_METHOD_RK4)
        S.set_fields(u0, 0.0)
        solvers.append(S)
    assert max(S.mesh.info["max_patch"] for S in solvers) > 36
    B = mtp.Batch(solvers)
    B.set_schedule(schedule)
    B.advance(1)
    tol = TOL if precision == 0 else MIXED_TOL
    for S, n, ref in zip(solvers, names, refs):
        assert_parity(S.get_state(), ref["w"], tol, f"batch {batch}: {n}")


def test_p5_3d_persistent_schedule_and_mixed_degree_batch():
    """3D P5 (operator block in device memory, column-block products) under the persistent
    schedule (bit-identical to the layers) and in a batch with P3 (two degree groups) against
    the oracle."""
    from paper_1906_11029_amd import mtp
    print("[gpu parity] 3D P5: persistent schedule and P3+P5 batch", flush=True)
    c, A, _ = gpu_solver("cav3d_p5")
    _, B, _ = gpu_solver("cav3d_p5")
    B.set_schedule(mtp.MTP_SCHEDULE_DAG)
    A.advance_to(c["T"])
    B.advance_to(c["T"])
    assert np.array_equal(A.get_state(), B.get_state())
    names = ["cav3d_p3", "cav3d_p5_pmc_eps"]
    solvers = [gpu_solver(nm)[1] for nm in names]
    mtp.Batch(solvers).advance(1)
    for S, nm in zip(solvers, names):
        assert_parity(S.get_state(), fixture(nm)["w"], TOL, f"batch {nm}")
